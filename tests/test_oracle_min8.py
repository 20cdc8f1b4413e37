"""Pins of the oracle's 8-real storage of SU(3) links (the minimal 8-parameter representation
that arXiv:1412.3655 Sec. 4.1 names among those cuLGT2 does not provide; the paper gives no
formulae, so the oracle defines a row-pivoted variant of the 8-real reconstruction of Clark et
al., Comput. Phys. Commun. 181 (2010) 1517: see gf_oracle.c).

A storage format is correct when decoding lands in SU(3) and decoding undoes encoding.  Checked
from outside the code under test:

* decode of arbitrary parameters of the domain (drawn directly, not by the encoder) is in SU(3)
  to rounding: U^dag U = 1 and det U = 1 (closed form of the group);
* decode(encode(U)) = U for Haar-random SU(3) (to the input's own distance from SU(3)), and
  encoding a decoded matrix returns a matrix equal to it to rounding (idempotence), over every
  branch: pivot column, which of alpha and beta is larger, and the sign of the real part behind
  each half-angle tangent;
* closed forms: the identity encodes to 8 zeros; diag(-1, -1, 1) to a single clamped tangent;
  the pivot is the largest entry of row 0 and the stored magnitudes follow from the matrix;
* special matrices (centre elements, permutations, ties between entries, embedded SU(2), links
  a 1e-9 step from the identity) round trip;
* storing the links in 8 reals after every half-sweep changes the oracle's sweep as much as
  reunitarising after every half-sweep does (2e-13 over 20 sweeps): it does not alter the method.
"""

import itertools

import numpy as np
import pytest

import gauge_inputs as gi
import oracle
from tests import lattice_np as ln


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.lib()


def canon(m):
    """complex (..., 3, 3) -> canonical (..., 3, 3, 2), C-contiguous."""
    return np.ascontiguousarray(np.stack([m.real, m.imag], axis=-1))


def cplx(u):
    return u[..., 0] + 1j * u[..., 1]


def su3_error(m):
    """max |U^dag U - 1| and max |det U - 1| over a stack of complex 3x3 matrices."""
    eye = np.eye(3)
    unit = np.abs(np.conj(np.swapaxes(m, -1, -2)) @ m - eye).max()
    det = np.abs(np.linalg.det(m) - 1.0).max()
    return unit, det


def low_bits(p):
    """(pivot k, q) from the low mantissa bits of p0, p1 and p5."""
    w = p.view(np.uint64) & np.uint64(1)
    return (w[..., 0] | (w[..., 1] << np.uint64(1))).astype(int), w[..., 5].astype(int)


def set_low_bit(v, bit):
    w = np.ascontiguousarray(v).view(np.uint64)
    w = (w & ~np.uint64(1)) | np.asarray(bit, dtype=np.uint64)
    return w.view(np.float64)


def domain_params(rng, n):
    """Parameters drawn directly in the decoder's domain: |a_i|, |a_j| <= |a_k|, |s| <= |b|,
    tangents spread over many decades including 0 and the clamp, random k and q."""
    out = np.empty((n, 8))
    i = 0
    while i < n:
        a = rng.uniform(-0.82, 0.82, 4)
        ai2, aj2 = a[0] ** 2 + a[1] ** 2, a[2] ** 2 + a[3] ** 2
        rho2 = 1.0 - ai2 - aj2
        s = rng.uniform(-0.72, 0.72, 2)
        if rho2 < max(ai2, aj2) or s @ s > 0.5:
            continue
        t = rng.choice([0.0, 1e150, -1e150, 1.0, -1.0]) if rng.random() < 0.2 else \
            rng.standard_normal() * 10.0 ** rng.integers(-8, 9)
        t2 = rng.standard_normal() * 10.0 ** rng.integers(-8, 9)
        out[i] = [a[0], a[1], a[2], a[3], t, s[0], s[1], t2]
        i += 1
    k = rng.integers(0, 3, n)
    q = rng.integers(0, 2, n)
    out[:, 0] = set_low_bit(out[:, 0], k & 1)
    out[:, 1] = set_low_bit(out[:, 1], k >> 1)
    out[:, 5] = set_low_bit(out[:, 5], q)
    return np.ascontiguousarray(out)


def test_decode_lands_in_su3():
    p = domain_params(np.random.default_rng(1), 20000)
    m = cplx(oracle.min8_decode(p))
    unit, det = su3_error(m)
    assert unit <= 2e-15 and det <= 2e-15, (unit, det)
    k, q = low_bits(p)
    # the stored entries sit where the pivot puts them, with the stored values (flag bits included)
    rows = np.arange(len(p))
    assert np.array_equal(m[rows, 0, (k + 1) % 3], p[:, 0] + 1j * p[:, 1])
    assert np.array_equal(m[rows, 0, (k + 2) % 3], p[:, 2] + 1j * p[:, 3])
    # |U_0k| follows from the other two; its phase from the half-angle tangent
    ak = m[rows, 0, k]
    rho = np.sqrt(1.0 - np.abs(p[:, 0] + 1j * p[:, 1]) ** 2 - np.abs(p[:, 2] + 1j * p[:, 3]) ** 2)
    assert np.abs(np.abs(ak) - rho).max() <= 1e-15
    # the phase is 2 atan(tangent) (the clamp 1e150 is the phase pi to 1e-150)
    assert np.abs(ak / np.abs(ak) - np.exp(2j * np.arctan(p[:, 4]))).max() <= 1e-15


def test_roundtrip_haar_every_branch():
    rng = np.random.default_rng(2)
    h = gi.haar_su3(rng, 60000)
    u = canon(h)
    p = oracle.min8_encode(u)
    back = cplx(oracle.min8_decode(p))
    own_u, own_d = su3_error(h)
    err = np.abs(back - h).max()
    assert err <= 4e-15 + 2 * max(own_u, own_d), (err, own_u, own_d)
    # idempotence: the stored matrix is reproduced to rounding
    again = cplx(oracle.min8_decode(oracle.min8_encode(canon(back))))
    assert np.abs(again - back).max() <= 1.2e-15
    # every branch of the encoder is taken and round trips
    k, q = low_bits(p)
    assert np.array_equal(k, np.argmax(np.abs(h[:, 0, :]), axis=1)) or \
        (np.abs(np.abs(h[np.arange(len(h)), 0, k]) - np.abs(h[:, 0, :]).max(axis=1)).max() <= 1e-15)
    ak = h[np.arange(len(h)), 0, k]
    n = np.sqrt(1.0 - np.abs(h[np.arange(len(h)), 0, (k + 2) % 3]) ** 2)
    seen = set()
    for kk, qq, sa, sb in itertools.product(range(3), range(2), (0, 1), (0, 1)):
        sel = (k == kk) & (q == qq) & ((ak.real >= 0) == bool(sa)) & ((np.abs(p[:, 7]) <= 1.0) == bool(sb))
        if sel.any():
            seen.add((kk, qq, sa, sb))
            assert np.abs(back[sel] - h[sel]).max() <= 4e-15 + 2 * max(own_u, own_d)
    assert len(seen) == 24, sorted(seen)
    assert n.min() >= np.sqrt(1.0 / 3.0) - 1e-15


def test_identity_and_minus_ones_closed_forms():
    eye = np.eye(3, dtype=complex)
    p = oracle.min8_encode(canon(eye[None]))
    assert np.array_equal(p, np.zeros((1, 8)))
    assert np.array_equal(cplx(oracle.min8_decode(p))[0], eye)
    d = np.diag([-1.0, -1.0, 1.0]).astype(complex)
    p = oracle.min8_encode(canon(d[None]))
    assert np.array_equal(p[0], [0, 0, 0, 0, 1e150, 0, 0, 0])
    back = cplx(oracle.min8_decode(p))[0]
    assert np.abs(back - d).max() <= 1e-149


def special_matrices():
    w = np.exp(2j * np.pi / 3)
    mats = [np.eye(3) * w, np.eye(3) * w.conjugate(), np.diag([-1.0, 1.0, -1.0]), np.diag([1.0, -1.0, -1.0]),
            np.diag(np.exp(1j * np.array([0.3, -1.9, 1.6]))), np.diag(np.exp(1j * np.array([np.pi, 0.5, -0.5 - np.pi]))),
            np.roll(np.eye(3), 1, axis=1), np.roll(np.eye(3), 2, axis=1),
            np.array([[0, 0, 1], [0, -1, 0], [1, 0, 0]], dtype=complex)]
    # ties: the discrete Fourier matrix scaled to unit determinant (all |U_ij| equal)
    f = np.array([[w ** (i * j) for j in range(3)] for i in range(3)]) / np.sqrt(3.0)
    mats.append(f / np.linalg.det(f) ** (1.0 / 3.0))
    # two equal entries in row 0, with alpha = 0 and with beta = 0
    c = np.sqrt(0.5)
    mats.append(np.array([[c, c, 0], [-c, c, 0], [0, 0, 1]], dtype=complex))
    mats.append(np.array([[c, 0, c], [0, 1, 0], [-c, 0, c]], dtype=complex))
    # embedded SU(2) and links a tiny step from the identity
    for m in gi.complex_view(gi.su2_embedded_links((2, 2, 2, 2), 3, 0.9)).reshape(-1, 3, 3)[:8]:
        mats.append(m)
    h = gi.random_traceless_hermitian(np.random.default_rng(4), 8)
    mats.extend(gi.expi_hermitian(h, 1e-9))
    return [np.asarray(m, dtype=complex) for m in mats]


@pytest.mark.parametrize("idx", range(len(special_matrices())))
def test_special_matrices_round_trip(idx):
    m = special_matrices()[idx]
    own_u, own_d = su3_error(m[None])
    assert max(own_u, own_d) <= 2e-15
    back = cplx(oracle.min8_decode(oracle.min8_encode(canon(m[None]))))[0]
    assert np.abs(back - m).max() <= 4e-15, np.abs(back - m).max()


def test_stored_sweep_equals_plain_sweep():
    """Eight-real storage after every half-sweep (what a lattice held in 8 reals does) against
    the plain oracle sweep, from links the representation holds exactly: the links differ by no
    more than reunitarising after every half-sweep makes them differ (both project the rounding
    drift of the plain sweep back onto SU(3)), and by <= 2e-13 over 20 sweeps."""
    dims = (4, 4, 4, 6)
    u = oracle.min8_store(gi.gen_links(dims, 0.8, 9))
    plain, stored, reunit = u.copy(), u.copy(), u.copy()
    for _ in range(20):
        for colour in (0, 1):
            for w in (plain, stored, reunit):
                oracle.half_sweep(w, dims, colour, 1.7)
            oracle.min8_store(stored)
            oracle.reunitarize(reunit)
    d = np.abs(stored - plain).max()
    d_reunit = np.abs(reunit - plain).max()
    assert d <= 2e-13 and d <= 3.0 * d_reunit, (d, d_reunit)
    th_p, F_p = oracle.measure(plain, dims)
    th_s, F_s = oracle.measure(stored, dims)
    assert abs(F_s - F_p) <= 1e-14 and abs(th_s - th_p) <= 1e-10 * th_p
    assert max(oracle.unitarity(stored.copy())) <= 2e-15
    assert ln.colours(dims).size == u.shape[0]
