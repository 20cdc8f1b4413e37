"""Pins of the oracle's Coulomb gauge (arXiv:1412.3655, abstract and Sec. 1 list it beside
Landau gauge; the condition, functional and iteration are those of Sec. 2 with mu over the
spatial directions only, one independent problem per timeslice).

Checked from the outside: closed forms on single-link fields, a numpy evaluation of
Delta_C from K_C, monotonicity of the functional (a theorem for omega in [1, 2)),
independence of the timeslices, gauge invariance (which needs the temporal links to be
transformed too), the embedded-SU(2) special case, the pure-gauge global maximum, order
independence within a colour and convergence.
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


def _numpy_coulomb(links, dims):
    """theta_C(t), F_C(t) from K_C = sum_i [U_i(x) + U_i(x-i^)^dag] (i = x, y, z) through
    Delta_C = [(K_C - K_C^dag)/(2i)]_traceless, per timeslice."""
    u = gi.complex_view(links)
    v = u.shape[0]
    nt = int(dims[3])
    v3 = v // nt
    K = np.zeros((v, 3, 3), dtype=np.complex128)
    for i in range(3):
        K += u[:, i] + ln.dag(u[ln.backward_sites(dims, i), i])
    M = (K - ln.dag(K)) / 2j
    D = M - (np.trace(M, axis1=1, axis2=2) / 3.0)[:, None, None] * np.eye(3)
    dens = np.sum(np.abs(D) ** 2, axis=(1, 2))
    fr = np.trace(u[:, :3], axis1=2, axis2=3).real.sum(axis=1)
    t = gi.lex_coords(dims)[:, 3]
    th = np.array([dens[t == k].sum() / (3.0 * v3) for k in range(nt)])
    F = np.array([fr[t == k].sum() / (9.0 * v3) for k in range(nt)])
    return th, F, dens


def _one_link(dims, eps, site, mu):
    u = gi.complex_view(gi.identity_links(dims)).copy()
    u[site, mu] = np.diag([np.exp(1j * eps), np.exp(-1j * eps), 1.0])
    return gi.to_canonical(u)


@pytest.mark.parametrize("eps", [0.1, 0.7, 2.0])
def test_coulomb_measure_closed_forms(eps):
    """A field that is 1 except U_x(x0) = diag(e^{i eps}, e^{-i eps}, 1), x0 in timeslice 0:
    A_x(x0) = diag(sin eps, -sin eps, 0), Delta_C(x0) = A, Delta_C(x0 + x^) = -A, so
    theta_C(0) = 2 * 2 sin^2(eps) / (3 V_3) and F_C(0) = 1 - (2 - 2 cos eps) / (9 V_3); every
    other timeslice has theta_C = 0, F_C = 1.  The same perturbation on a temporal link
    enters neither: theta_C = 0 and F_C = 1 everywhere."""
    dims = SMALL
    v3 = 64
    th, F = oracle.coulomb_measure(_one_link(dims, eps, 5, 0), dims)
    assert abs(th[0] - 4 * math.sin(eps) ** 2 / (3 * v3)) < 1e-15
    assert abs(F[0] - (1 - (2 - 2 * math.cos(eps)) / (9 * v3))) < 1e-15
    assert np.all(th[1:] == 0) and np.all(F[1:] == 1)
    th, F = oracle.coulomb_measure(_one_link(dims, eps, 5, 3), dims)
    assert np.all(th == 0) and np.all(F == 1)


@pytest.mark.parametrize("dims", [SMALL, RAGGED])
def test_coulomb_measure_two_ways(dims):
    """Delta_C from the A_i (oracle) equals Delta_C from K_C (numpy), per timeslice."""
    u = gi.gen_links(dims, 0.7, 3)
    th, F = oracle.coulomb_measure(u, dims)
    th_n, F_n, _ = _numpy_coulomb(u, dims)
    assert np.abs(th - th_n).max() <= 1e-13 * th_n.max()
    assert np.abs(F - F_n).max() < 1e-14


@pytest.mark.parametrize("omega,mode", [(1.0, 0), (1.7, 0), (1.95, 0), (1.7, 1)])
def test_coulomb_functional_non_decreasing(omega, mode):
    """Every subgroup step raises Re tr[g K_C] (gain 2n(cos((1-w)phi) - cos phi) >= 0), so the
    functional of every timeslice is non-decreasing sweep by sweep."""
    dims = RAGGED
    u = gi.gen_links(dims, 0.8, 4)
    _, F = oracle.coulomb_measure(u, dims)
    for _ in range(12):
        oracle.coulomb_sweep(u, dims, 1, omega, mode)
        _, F2 = oracle.coulomb_measure(u, dims)
        assert np.all(F2 >= F - 1e-14)
        F = F2


def test_coulomb_timeslices_are_independent():
    """K_C at x holds spatial links of x's timeslice only, so what happens in one timeslice
    (its spatial links) and to the temporal links cannot change the spatial links of another:
    after sweeps, those are bitwise identical to a run where timeslice 0's spatial links and
    all temporal links started elsewhere."""
    dims = SMALL
    a = gi.gen_links(dims, 0.8, 5)
    b = a.copy()
    other = gi.gen_links(dims, 0.5, 6)
    t = gi.lex_coords(dims)[:, 3]
    b[t == 0, :3] = other[t == 0, :3]
    b[:, 3] = other[:, 3]
    oracle.coulomb_sweep(a, dims, 4, 1.7)
    oracle.coulomb_sweep(b, dims, 4, 1.7)
    keep = t != 0
    assert np.array_equal(a[keep, :3], b[keep, :3])
    assert not np.array_equal(a[~keep, :3], b[~keep, :3])


def test_coulomb_sweeps_are_gauge_transformations():
    """A gauge transformation acts on every link at x, temporal ones included; then every
    plaquette, spatial and temporal, is unchanged (a sweep that left the temporal links alone
    would change the space-time plaquettes), and the links stay in SU(3)."""
    dims = RAGGED
    u = gi.gen_links(dims, 0.9, 7)
    P0 = oracle.plaquette(u, dims)
    u0 = u.copy()
    oracle.coulomb_sweep(u, dims, 25, 1.7)
    assert abs(oracle.plaquette(u, dims) - P0) < 1e-12
    assert not np.array_equal(u[:, 3], u0[:, 3])
    du, dd = oracle.unitarity(u)
    assert du < 1e-13 and dd < 1e-13


def test_coulomb_su2_embedded_special_case():
    """Links diag(u, 1): K_C = diag(k, 6) with k in the real span of SU(2), so after the black
    half-sweep at omega = 1 K_C is Hermitian and Delta_C vanishes at every black site."""
    dims = SMALL
    u = gi.su2_embedded_links(dims, 8)
    oracle.coulomb_half_sweep(u, dims, 0, 1.0)
    _, _, dens = _numpy_coulomb(u, dims)
    black = ln.colours(dims) == 0
    assert dens[black].max() < 1e-26
    assert dens[~black].max() > 1e-6


def test_coulomb_pure_gauge_reaches_unit_functional():
    """A gauge copy of the unit field: every timeslice reaches F_C = 1 at theta_C < 1e-12."""
    dims = SMALL
    u = gi.pure_gauge_links(dims, 9)
    r = oracle.coulomb_fix_until(u, dims, 1.7, 0, 1e-12, 3000, 10, 100)
    assert r["converged"], r
    th, F = oracle.coulomb_measure(u, dims)
    assert th.max() < 1e-12 and np.abs(F - 1).max() < 1e-10


def test_coulomb_order_within_a_colour_is_irrelevant():
    dims = RAGGED
    u = gi.gen_links(dims, 0.8, 10)
    a = u.copy()
    oracle.coulomb_half_sweep(a, dims, 0, 1.7)
    black = np.flatnonzero(ln.colours(dims) == 0)
    c = u.copy()
    oracle.coulomb_update_sites_in_order(c, dims, np.random.default_rng(0).permutation(black), 1.7)
    assert np.array_equal(a, c)


def test_coulomb_fix_until_converges_8x4():
    """8^4, eps = 0.6: every timeslice below 1e-12 well inside 3000 sweeps; the reported theta
    is the largest per-timeslice value and F the mean."""
    dims = (8, 8, 8, 8)
    u = gi.gen_links(dims, 0.6, 0)
    r = oracle.coulomb_fix_until(u, dims, 1.7, 0, 1e-12, 3000, 10, 100)
    assert r["converged"] and r["sweeps"] < 3000
    th, F = oracle.coulomb_measure(u, dims)
    assert r["theta"] == th.max() and abs(r["F"] - F.mean()) < 1e-15


def test_coulomb_anneal_timeslices_are_independent():
    """The Coulomb heat bath draws each subgroup element from the block of K_C, which holds
    spatial links of the site's timeslice only, and its Philox stream is keyed by the site:
    spatial links of every other timeslice end bitwise identical when timeslice 0's spatial
    links and all temporal links start elsewhere.  (A heat bath weighted by the Landau K,
    temporal links included, fails this.)"""
    dims = SMALL
    a = gi.gen_links(dims, 0.8, 15)
    b = a.copy()
    other = gi.gen_links(dims, 0.5, 16)
    t = gi.lex_coords(dims)[:, 3]
    b[t == 0, :3] = other[t == 0, :3]
    b[:, 3] = other[:, 3]
    for u in (a, b):
        assert oracle.coulomb_anneal(u, dims, 3, 1.25, 0.5, 77) == 0
    keep = t != 0
    assert np.array_equal(a[keep, :3], b[keep, :3])
    assert not np.array_equal(a[~keep, :3], b[~keep, :3])


def test_coulomb_anneal_is_a_gauge_transformation():
    """Annealing moves along the gauge orbit: every plaquette unchanged, temporal links
    transformed, links in SU(3), and the draws differ from the Landau heat bath's."""
    dims = RAGGED
    u = gi.gen_links(dims, 0.9, 17)
    P0 = oracle.plaquette(u, dims)
    land = u.copy()
    u0 = u.copy()
    assert oracle.coulomb_anneal(u, dims, 10, 1.25, 0.01, 5) == 0
    oracle.anneal(land, dims, 10, 1.25, 0.01, 5)
    assert abs(oracle.plaquette(u, dims) - P0) < 1e-12
    assert not np.array_equal(u[:, 3], u0[:, 3])
    assert np.abs(u - land).max() > 1e-3
    du, dd = oracle.unitarity(u)
    assert du < 1e-13 and dd < 1e-13


def test_coulomb_anneal_cold_limit_is_the_maximiser():
    """At T -> 0 the subgroup weight exp(2 n r0 / T) pins r0 to 1 (1 - r0 = O(T), the
    direction off the maximiser O(sqrt(T))), so one heat-bath sweep is one omega = 1
    overrelaxation sweep of the Coulomb functional up to O(sqrt(T)) in the links and in F_C
    (later sites maximise against links already moved by O(sqrt(T)))."""
    dims = SMALL
    u = gi.gen_links(dims, 0.6, 18)
    hb = u.copy()
    orr = u.copy()
    oracle.coulomb_anneal(hb, dims, 1, 1e-10, 1e-10, 3)
    oracle.coulomb_sweep(orr, dims, 1, 1.0)
    assert np.abs(hb - orr).max() < 1e-3
    _, F_hb = oracle.coulomb_measure(hb, dims)
    _, F_or = oracle.coulomb_measure(orr, dims)
    assert np.abs(F_hb - F_or).max() < 1e-5
