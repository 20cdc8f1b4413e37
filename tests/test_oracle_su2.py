"""Pins of the oracle's SU(2) gauge group (arXiv:1412.3655: the abstract lists SU(2) beside
SU(3); Sec. 2 gives the maximiser g = K^dag / sqrt(det K^dag) for SU(2), exact there; Sec. 4.1
changes the group by the link parameterisation alone).

Checked from outside the code under test: the SU(3) oracle (pinned on its own) on links
diag(u, 1) reproduces the SU(2) sweep at omega = 1 and the N_c normalisations; the site update
reaches the closed-form local maximum 2 sqrt(det K) and leaves K proportional to 1; single-link
closed forms of theta, F and the plaquette; theta from K (numpy) against theta from the A_mu;
the functional is non-decreasing for omega in [1, 2); gauge invariance, SU(2) membership,
order independence within a colour, the pure-gauge maximum, convergence; Coulomb gauge's
independent timeslices; the heat bath's gauge invariance and cold limit.
"""

import math

import numpy as np
import pytest

import gauge_inputs as gi
import oracle
from tests import lattice_np as ln

SMALL = (4, 4, 4, 4)
RAGGED = (6, 4, 2, 6)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.lib()


def embed3(u2):
    """(V, 4, 2, 2, 2) SU(2) links -> (V, 4, 3, 3, 2) SU(3) links diag(u, 1)."""
    c = gi.complex_view(u2)
    out = np.zeros(c.shape[:2] + (3, 3), dtype=np.complex128)
    out[..., :2, :2] = c
    out[..., 2, 2] = 1.0
    return gi.to_canonical(out)


def numpy_K(u2, dims, ndir=4):
    u = gi.complex_view(u2)
    K = np.zeros((u.shape[0], 2, 2), dtype=np.complex128)
    for mu in range(ndir):
        K += u[:, mu] + ln.dag(u[ln.backward_sites(dims, mu), mu])
    return K


def test_embedding_in_su3_reproduces_the_sweep_and_normalisations():
    """The SU(3) site update on diag(u, 1) rotates only the (0,1) block at omega = 1 (after
    it, the (0,2) and (1,2) blocks of K are already Hermitian-positive, so their maximiser is
    1): an SU(3) sweep of the embedded links equals the SU(2) sweep.  theta and F follow the
    N_c normalisations: theta_3 = (2/3) theta_2, F_3 = (2 F_2 + 1)/3."""
    dims = SMALL
    u = gi.gen_links_su2(dims, 0.7, 1)
    e = embed3(u)
    th2, F2 = oracle.su2lat_measure(u, dims)
    th3, F3 = oracle.measure(e, dims)
    assert abs(th3 - 2.0 / 3.0 * th2) <= 1e-13 * th2
    assert abs(F3 - (2.0 * F2 + 1.0) / 3.0) < 1e-15
    oracle.su2lat_sweep(u, dims, 3, 1.0)
    oracle.sweep(e, dims, 3, 1.0)
    c3 = gi.complex_view(e)
    assert np.abs(c3[..., :2, :2] - gi.complex_view(u)).max() < 1e-13
    assert np.abs(c3[..., 2, 2] - 1.0).max() < 1e-13


@pytest.mark.parametrize("mode", [oracle.OR_EXACT, oracle.OR_BINOMIAL1])
def test_site_update_reaches_the_local_maximum(mode):
    """At omega = 1 the new K(x) = g K is 2x2 positive multiple of 1 with trace 2 sqrt(det K):
    the closed-form maximum of Re tr[g K] over SU(2); 10^4 Haar trials stay below it."""
    dims = RAGGED
    u = gi.gen_links_su2(dims, 0.9, 2)
    site = 17
    K = numpy_K(u, dims)[site]
    best = 2.0 * math.sqrt(np.linalg.det(K).real)
    gain = oracle.su2lat_site_update(u, dims, site, 1.0, mode)
    K1 = numpy_K(u, dims)[site]
    assert abs(np.trace(K1).real - best) < 1e-13 * best
    assert abs(gain - (best - np.trace(K).real)) < 1e-12 * best
    assert np.abs(K1 - np.trace(K1) / 2 * np.eye(2)).max() < 1e-13 * best
    h = gi.complex_view(gi.to_canonical(gi.haar_su2(np.random.default_rng(3), 10000)))
    trials = np.einsum("nij,ji->n", h, K).real
    assert trials.max() <= best + 1e-12


@pytest.mark.parametrize("eps", [0.1, 0.8, 2.5])
def test_single_link_closed_forms(eps):
    """Unit field except U_x(x0) = diag(e^{i eps}, e^{-i eps}): A = sin(eps) sigma_3 at x0,
    Delta(x0) = A and Delta(x0 + x^) = -A, so theta = 2 * 2 sin^2(eps) / (2V); F = 1 -
    (2 - 2 cos eps)/(8V); each of the 6 plaquettes through the link has Re tr = 2 cos eps
    (every other one 2), so P = 1 - 6 (2 - 2 cos eps) / (12 V)."""
    dims = SMALL
    v = gi.volume(dims)
    u = gi.complex_view(gi.identity_links_su2(dims)).copy()
    u[9, 0] = np.diag([np.exp(1j * eps), np.exp(-1j * eps)])
    u = gi.to_canonical(u)
    th, F = oracle.su2lat_measure(u, dims)
    assert abs(th - 2.0 * math.sin(eps) ** 2 / v) < 1e-15
    assert abs(F - (1.0 - (2.0 - 2.0 * math.cos(eps)) / (8.0 * v))) < 1e-15
    P = oracle.su2lat_plaquette(u, dims)
    assert abs(P - (1.0 - 6.0 * (2.0 - 2.0 * math.cos(eps)) / (12.0 * v))) < 1e-15


@pytest.mark.parametrize("ndir", [4, 3])
def test_theta_two_ways(ndir):
    """Delta from the A_mu (oracle) equals Delta = [(K - K^dag)/(2i)]_traceless (numpy)."""
    dims = RAGGED
    u = gi.gen_links_su2(dims, 0.7, 4)
    K = numpy_K(u, dims, ndir)
    M = (K - ln.dag(K)) / 2j
    D = M - (np.trace(M, axis1=1, axis2=2) / 2.0)[:, None, None] * np.eye(2)
    dens = np.sum(np.abs(D) ** 2, axis=(1, 2))
    got = oracle.su2lat_theta_density(u, dims, ndir)
    assert np.abs(got - dens).max() <= 1e-13 * dens.max()


@pytest.mark.parametrize("omega,mode", [(1.0, 0), (1.7, 0), (1.95, 0), (1.7, 1)])
def test_functional_non_decreasing(omega, mode):
    dims = RAGGED
    u = gi.gen_links_su2(dims, 0.9, 5)
    _, F = oracle.su2lat_measure(u, dims)
    for _ in range(15):
        oracle.su2lat_sweep(u, dims, 1, omega, mode)
        _, F2 = oracle.su2lat_measure(u, dims)
        assert F2 >= F - 1e-14
        F = F2


def test_gauge_invariance_and_membership():
    dims = RAGGED
    u = gi.gen_links_su2(dims, 1.0, 6)
    P0 = oracle.su2lat_plaquette(u, dims)
    oracle.su2lat_sweep(u, dims, 40, 1.7)
    assert abs(oracle.su2lat_plaquette(u, dims) - P0) < 1e-12
    du, dd = oracle.su2lat_unitarity(u)
    assert du < 1e-13 and dd < 1e-13


def test_order_within_a_colour_is_irrelevant():
    dims = RAGGED
    u = gi.gen_links_su2(dims, 0.8, 7)
    a = u.copy()
    oracle.su2lat_half_sweep(a, dims, 0, 1.7)
    black = np.flatnonzero(ln.colours(dims) == 0)
    c = u.copy()
    oracle.su2lat_update_sites_in_order(c, dims, np.random.default_rng(0).permutation(black), 1.7)
    assert np.array_equal(a, c)


def test_pure_gauge_and_convergence():
    dims = SMALL
    u = gi.pure_gauge_links_su2(dims, 8)
    r = oracle.su2lat_fix_until(u, dims, 1.7, 0, 1e-12, 3000, 10, 100)
    assert r["converged"] and abs(r["F"] - 1.0) < 1e-10
    dims = (8, 8, 8, 8)
    u = gi.gen_links_su2(dims, 0.6, 0)
    r = oracle.su2lat_fix_until(u, dims, 1.7, 0, 1e-12, 3000, 10, 100)
    assert r["converged"] and r["sweeps"] < 3000
    th, F = oracle.su2lat_measure(u, dims)
    assert th == r["theta"] and F == r["F"]


def test_reunitarize_projects_onto_su2():
    """Idempotent on SU(2) to 1e-15, and a perturbed link comes back into SU(2)."""
    u = gi.gen_links_su2(SMALL, 0.7, 9)
    a = u.copy()
    oracle.su2lat_reunitarize(a)
    assert np.abs(a - u).max() < 2e-15
    noisy = u + 1e-4 * np.random.default_rng(1).standard_normal(u.shape)
    oracle.su2lat_reunitarize(noisy)
    du, dd = oracle.su2lat_unitarity(noisy)
    assert du < 1e-14 and dd < 1e-14
    assert np.abs(noisy - u).max() < 1e-3


def test_coulomb_timeslices_are_independent():
    dims = SMALL
    a = gi.gen_links_su2(dims, 0.8, 10)
    b = a.copy()
    other = gi.gen_links_su2(dims, 0.5, 11)
    t = gi.lex_coords(dims)[:, 3]
    b[t == 0, :3] = other[t == 0, :3]
    b[:, 3] = other[:, 3]
    oracle.su2lat_sweep(a, dims, 4, 1.7, ndir=3)
    oracle.su2lat_sweep(b, dims, 4, 1.7, ndir=3)
    keep = t != 0
    assert np.array_equal(a[keep, :3], b[keep, :3])
    r = oracle.su2lat_fix_until(a, dims, 1.7, 0, 1e-12, 3000, 10, 100, ndir=3)
    th, F = oracle.su2lat_coulomb_measure(a, dims)
    assert r["converged"] and th.max() == r["theta"] and abs(F.mean() - r["F"]) < 1e-15


def test_heat_bath_gauge_invariance_and_cold_limit():
    dims = RAGGED
    u = gi.gen_links_su2(dims, 0.9, 12)
    P0 = oracle.su2lat_plaquette(u, dims)
    a = u.copy()
    assert oracle.su2lat_anneal(a, dims, 10, 1.25, 0.01, 5) == 0
    assert abs(oracle.su2lat_plaquette(a, dims) - P0) < 1e-12
    du, dd = oracle.su2lat_unitarity(a)
    assert du < 1e-13 and dd < 1e-13
    hb = u.copy()
    orr = u.copy()
    oracle.su2lat_anneal(hb, dims, 1, 1e-10, 1e-10, 3)
    oracle.su2lat_sweep(orr, dims, 1, 1.0)
    assert np.abs(hb - orr).max() < 1e-3


@pytest.mark.parametrize("eps", [0.3, 1.9])
def test_coulomb_measure_closed_forms(eps):
    """Unit field except U_y(x0) = diag(e^{i eps}, e^{-i eps}), x0 in timeslice 0:
    theta_C(0) = 2 * 2 sin^2(eps) / (2 V3), F_C(0) = 1 - (2 - 2 cos eps)/(6 V3), all other
    timeslices theta_C = 0, F_C = 1; a temporal link perturbed the same way enters neither."""
    dims = SMALL
    v3 = 64
    for mu, hit in ((1, True), (3, False)):
        u = gi.complex_view(gi.identity_links_su2(dims)).copy()
        u[5, mu] = np.diag([np.exp(1j * eps), np.exp(-1j * eps)])
        th, F = oracle.su2lat_coulomb_measure(gi.to_canonical(u), dims)
        if hit:
            assert abs(th[0] - 2.0 * math.sin(eps) ** 2 / v3) < 1e-15
            assert abs(F[0] - (1.0 - (2.0 - 2.0 * math.cos(eps)) / (6.0 * v3))) < 1e-15
            assert np.all(th[1:] == 0) and np.all(F[1:] == 1)
        else:
            assert np.all(th == 0) and np.all(F == 1)


def test_coulomb_heat_bath_timeslices_are_independent():
    """The Coulomb heat bath weighs each draw by K_C: other timeslices' spatial links end
    bitwise identical when timeslice 0's spatial links and all temporal links start elsewhere."""
    dims = SMALL
    a = gi.gen_links_su2(dims, 0.8, 13)
    b = a.copy()
    other = gi.gen_links_su2(dims, 0.5, 14)
    t = gi.lex_coords(dims)[:, 3]
    b[t == 0, :3] = other[t == 0, :3]
    b[:, 3] = other[:, 3]
    for u in (a, b):
        oracle.su2lat_anneal(u, dims, 3, 1.25, 0.5, 77, ndir=3)
    keep = t != 0
    assert np.array_equal(a[keep, :3], b[keep, :3])
    assert not np.array_equal(a[~keep, :3], b[~keep, :3])
