"""Small numpy helpers the tests use to check the oracle from the outside.

These are written from the definitions (Sec. 2 of arXiv:1412.3655) in a
vectorised form that is deliberately different from the oracle's loops.
"""

import numpy as np

import gauge_inputs as gi

PAULI = [
    np.eye(2, dtype=np.complex128),
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]
# real basis of the quaternion algebra (real span of SU(2)): 1, i s1, i s2, i s3
QBASIS = [PAULI[0], 1j * PAULI[1], 1j * PAULI[2], 1j * PAULI[3]]


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def backward_sites(dims, mu):
    c = gi.lex_coords(dims)
    n = tuple(int(d) for d in dims)
    c[:, mu] = (c[:, mu] - 1) % n[mu]
    return c[:, 0] + n[0] * (c[:, 1] + n[1] * (c[:, 2] + n[2] * c[:, 3]))


def forward_sites(dims, mu):
    c = gi.lex_coords(dims)
    n = tuple(int(d) for d in dims)
    c[:, mu] = (c[:, mu] + 1) % n[mu]
    return c[:, 0] + n[0] * (c[:, 1] + n[1] * (c[:, 2] + n[2] * c[:, 3]))


def colours(dims):
    return gi.lex_coords(dims).sum(axis=1) % 2


def K_all(links, dims):
    """K(x) for all sites, (V, 3, 3) complex."""
    u = gi.complex_view(links)
    K = np.zeros((u.shape[0], 3, 3), dtype=np.complex128)
    for mu in range(4):
        K += u[:, mu] + dag(u[backward_sites(dims, mu), mu])
    return K


def delta_from_K(links, dims):
    """Delta(x) = [(K - K^dag)/(2i)]_traceless, (V, 3, 3)."""
    K = K_all(links, dims)
    M = (K - dag(K)) / 2j
    tr = np.trace(M, axis1=1, axis2=2) / 3.0
    return M - tr[:, None, None] * np.eye(3)


def theta_F_numpy(links, dims):
    u = gi.complex_view(links)
    v = u.shape[0]
    D = delta_from_K(links, dims)
    theta = np.sum(np.abs(D) ** 2) / (3.0 * v)
    F = np.sum(np.trace(u, axis1=2, axis2=3).real) / (12.0 * v)
    return theta, F


def random_su2(rng, n):
    """Haar SU(2) as 2x2 complex matrices: unit quaternions in the QBASIS."""
    a = rng.standard_normal((n, 4))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    return np.einsum("ne,eij->nij", a, np.array(QBASIS))


def quaternion_coeffs(k):
    """Coefficients of the real-orthogonal projection of 2x2 k on QBASIS."""
    return np.array([np.real(np.trace(dag(e) @ k)) / 2.0 for e in QBASIS])


def float_exact_links(dims, seed):
    """Links whose entries are 0, +-1 or +-i (real signed cyclic permutations with det 1, and
    diag(i, -i, 1), diag(-i, i, 1)): float32 stores them exactly, every float32 product and sum
    formed from them is exact, and the imaginary diagonal of K sums to zero at every site."""
    rng = np.random.default_rng(seed)
    V = gi.volume(dims)
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], dtype=np.complex128)
    mats = []
    for k in range(3):
        Pk = np.linalg.matrix_power(P, k)
        for signs in ((1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)):
            mats.append(np.diag(signs).astype(np.complex128) @ Pk)
    mats.append(np.diag([1j, -1j, 1]))
    mats.append(np.diag([-1j, 1j, 1]))
    mats = np.array(mats)
    for m in mats:
        assert abs(np.linalg.det(m) - 1) < 1e-15
    pick = rng.integers(0, len(mats), size=(V, 4))
    return gi.to_canonical(mats[pick])


def storage_floor(u, dims):
    """theta-floor from storage alone: rows 0, 1 rounded to float32, everything else exact."""
    c = gi.complex_view(u).copy()
    c[:, :, :2, :] = c[:, :, :2, :].astype(np.complex64).astype(np.complex128)
    c[:, :, 2, :] = np.conj(np.cross(c[:, :, 0, :], c[:, :, 1, :]))
    r = gi.to_canonical(c)
    E = delta_from_K(r, dims) - delta_from_K(u, dims)
    return float(np.sum(np.abs(E) ** 2) / (3 * u.shape[0]))
