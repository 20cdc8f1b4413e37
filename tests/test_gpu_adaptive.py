"""The fused estimate of the gauge condition and adaptive checks of the fix-until loop.

The paper iterates until the gauge condition holds to a given precision (Sec. 2).  A sweep
forms every site's K(x) anyway, so it can also sum tr[Delta Delta^dag] of K just before each
update (the estimate); the exact measurement, a separate pass over every link, is then needed
only where the estimate is close to a threshold that decides something.  Checked here:

* the estimate against the oracle: the black sites' terms before the black half-sweep plus the
  white sites' terms after it, relative 1e-12 (float64);
* the ratio of estimate to theta over whole runs, which the margin (100) must cover with room;
* adaptive checks give bitwise the result of exact checks (sweep count, theta, F, links) in
  float64, mixed precision and Coulomb gauge, with fewer exact measurements.
"""

import sys

import numpy as np
import pytest

import gauge_inputs as gi
import oracle
from paper_1412_3655_amd import gf
from tests import lattice_np as ln

pytestmark = pytest.mark.gpu

CFG8 = (8, 8, 8, 8)
RAGGED = (6, 10, 6, 6)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    oracle.lib()
    gf.lib()


def coulomb_density(links, dims):
    """tr[Delta_C Delta_C^dag] per site from K_C (numpy)."""
    u = gi.complex_view(links)
    K = np.zeros((u.shape[0], 3, 3), dtype=np.complex128)
    for i in range(3):
        K += u[:, i] + ln.dag(u[ln.backward_sites(dims, i), i])
    M = (K - ln.dag(K)) / 2j
    D = M - (np.trace(M, axis1=1, axis2=2) / 3.0)[:, None, None] * np.eye(3)
    return np.sum(np.abs(D) ** 2, axis=(1, 2))


@pytest.mark.parametrize("dims", [CFG8, RAGGED, (2, 4, 6, 8)])
@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
@pytest.mark.parametrize("tps", [1, 2, 8])
def test_estimate_against_oracle(dims, gauge, tps):
    say(f"estimate vs oracle dims={dims} gauge={gauge} tps={tps}")
    u = gi.gen_links(dims, 0.7, 51)
    black = ln.colours(dims) == 0
    ref = u.copy()
    dens = (oracle.theta_density if gauge == gf.GF_LANDAU else coulomb_density)
    s_black = dens(ref, dims)[black].sum()
    half = oracle.half_sweep if gauge == gf.GF_LANDAU else oracle.coulomb_half_sweep
    half(ref, dims, 0, 1.7, oracle.OR_EXACT)
    s_white = dens(ref, dims)[~black].sum()
    half(ref, dims, 1, 1.7, oracle.OR_EXACT)
    expect = (s_black + s_white) / (3.0 * u.shape[0])
    with gf.Lattice(dims, gf.GF_FP64, gauge=gauge) as lat:
        lat.set_sweep_config(tps, 128 if tps < 8 else 512, 0)
        lat.set_links(u)
        est = lat.sweep_estimate(1.7)
        got = lat.get_links()
        assert lat.counters == (0, 1)
    say(f"  estimate {est:.12e} oracle {expect:.12e}")
    assert abs(est - expect) <= 1e-12 * expect
    assert float(np.abs(got - ref).max()) <= 1e-12


def test_estimate_sweep_moves_links_like_a_plain_sweep():
    """The estimating sweep runs the same site updates: links bitwise equal to gf_sweep_or's."""
    u = gi.gen_links(RAGGED, 0.8, 52)
    outs = []
    for est in (False, True):
        with gf.Lattice(RAGGED, gf.GF_MIXED) as lat:
            lat.set_links(u)
            lat.sweep(2, 1.7)
            if est:
                lat.sweep_estimate(1.7)
            else:
                lat.sweep(1, 1.7)
            lat.promote_fp64()
            outs.append(lat.get_links())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dims,eps,sweeps", [(CFG8, 0.6, 1500), ((16, 16, 16, 16), 0.6, 600),
                                              ((16, 16, 16, 16), 0.9, 400)])
def test_estimate_to_theta_ratio(dims, eps, sweeps):
    """Over a run, the estimate of the last sweep of every 10 against theta after it: the ratio
    stays far inside the default margin of 100 (the adaptive loop measures exactly whenever
    the estimate is below 100 x a threshold, so it can miss a decision only if theta fell
    below a threshold while the estimate stayed 100 x above it)."""
    say(f"estimate / theta over {sweeps} sweeps, dims={dims} eps={eps}")
    u = gi.gen_links(dims, eps, 53)
    ratios = []
    with gf.Lattice(dims, gf.GF_FP64) as lat:
        lat.set_links(u)
        for k in range(sweeps // 10):
            lat.sweep(9, 1.7)
            est = lat.sweep_estimate(1.7)
            th, _ = lat.measure()
            ratios.append(est / th)
            if k % 10 == 9:
                lat.reunitarize()
    r = np.array(ratios)
    say(f"  est/theta: min {r.min():.3f} median {np.median(r):.3f} max {r.max():.3f}; final theta {th:.2e}")
    assert r.max() < 10.0 and r.min() > 0.0


@pytest.mark.parametrize("prec,dims,eps,gauge", [
    (gf.GF_FP64, CFG8, 0.6, gf.GF_LANDAU),
    (gf.GF_MIXED, CFG8, 0.6, gf.GF_LANDAU),
    (gf.GF_MIXED, (12, 12, 12, 12), 0.6, gf.GF_LANDAU),
    (gf.GF_FP64, RAGGED, 0.6, gf.GF_LANDAU),
    (gf.GF_FP64, CFG8, 0.6, gf.GF_COULOMB),
    (gf.GF_MIXED, CFG8, 0.6, gf.GF_COULOMB),
])
def test_adaptive_checks_equal_exact_checks(prec, dims, eps, gauge):
    say(f"adaptive vs exact checks prec={prec} dims={dims} eps={eps} gauge={gauge}")
    u = gi.gen_links(dims, eps, 54)
    kw = dict(omega=1.7, theta_target=1e-12, max_sweeps=6000, check_every=10, reunit_every=100, theta_switch=-1.0)
    out = []
    for adaptive in (False, True):
        with gf.Lattice(dims, prec, gauge=gauge) as lat:
            lat.set_links(u)
            lat.set_check_policy(adaptive)
            r = lat.fix_until(**kw)
            out.append((r, lat.get_links(), lat.counters))
    (r0, l0, c0), (r1, l1, c1) = out
    say(f"  exact: {r0.sweeps} sweeps ({r0.sweeps_fp32}/{r0.sweeps_fp64}), {c0[0]} measurements; "
        f"adaptive: {r1.sweeps}, {c1[0]} measurements + {c1[1]} estimates; theta {r1.theta:.3e}")
    assert r0.converged
    assert r1 == r0
    assert np.array_equal(l1, l0)
    assert c1[0] < c0[0] and c1[1] == r0.sweeps // 10


def test_adaptive_cap_and_arguments():
    """At the sweep cap the last check is exact (an unconverged result carries the exact theta),
    and the margin must be >= 1."""
    u = gi.gen_links(RAGGED, 0.9, 55)
    kw = dict(omega=1.7, theta_target=1e-12, max_sweeps=95, check_every=10, reunit_every=100)
    res = []
    for adaptive in (False, True):
        with gf.Lattice(RAGGED, gf.GF_FP64) as lat:
            lat.set_links(u)
            lat.set_check_policy(adaptive)
            res.append(lat.fix_until(**kw))
            th, F = lat.measure()
            assert (res[-1].theta, res[-1].F) == (th, F)
    assert res[0] == res[1] and not res[1].converged and res[1].sweeps == 95
    with gf.Lattice(RAGGED) as lat:
        for bad in (0.5, float("nan"), float("inf")):
            with pytest.raises(gf.GFError) as e:
                lat.set_check_policy(True, bad)
            assert e.value.status == gf.GF_E_ARG
