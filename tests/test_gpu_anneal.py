"""Heat-bath (simulated annealing) prelude on the GPU against the FP64 oracle.

Both sides implement Philox4x32-10 from its published definition and draw the
same counters, so in float64 every accept/reject decision is the same unless
a uniform falls within rounding (~1e-16 relative) of its threshold; links are
compared to 1e-12 max-abs.  float32 annealing is checked statistically only.
"""

import sys

import numpy as np
import pytest

import gauge_inputs as gi
import oracle
from paper_1412_3655_amd import gf

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


def gpu_anneal(dims, u, calls, prec=gf.GF_FP64, tps=4, block=256, cp=0):
    with gf.Lattice(dims, prec) as lat:
        lat.set_anneal_config(tps, block, cp)
        lat.set_links(u)
        for (n, T0, T1, seed) in calls:
            lat.anneal(n, T0, T1, seed)
        return lat.get_links(), lat.plaquette()


@pytest.mark.parametrize("dims", [CFG8, RAGGED])
def test_anneal_fp64_parity(dims):
    """5 sweeps, T 1.25 -> 0.01 (kappa crosses the Creutz / Kennedy-Pendleton boundary)."""
    say(f"anneal fp64 parity dims={dims}")
    u = gi.gen_links(dims, 1.0, 11)
    ref = u.copy()
    capped = oracle.anneal(ref, dims, 5, 1.25, 0.01, 42)
    got, P = gpu_anneal(dims, u, [(5, 1.25, 0.01, 42)])
    d = np.abs(got - ref).max()
    say(f"  max|diff| {d:.3e}, oracle capped {capped}")
    assert capped == 0
    assert d <= 1e-12
    assert abs(P - oracle.plaquette(u, dims)) < 1e-12


def test_anneal_bitwise_across_tps_and_resume():
    say("anneal bitwise across tps, resume")
    u = gi.gen_links(RAGGED, 1.0, 12)
    base, _ = gpu_anneal(RAGGED, u, [(4, 0.8, 0.8, 7)], tps=4)
    for tps, block, cp in ((1, 256, 0), (2, 256, 0), (8, 256, 0), (1, 128, 2), (2, 64, 1), (1, 64, 2)):
        got, _ = gpu_anneal(RAGGED, u, [(4, 0.8, 0.8, 7)], tps=tps, block=block, cp=cp)
        assert np.array_equal(got, base), (tps, block, cp)
    # the sweep counter continues across calls: 2 + 2 sweeps == 4 sweeps at constant T
    split, _ = gpu_anneal(RAGGED, u, [(2, 0.8, 0.8, 7), (2, 0.8, 0.8, 7)])
    assert np.array_equal(split, base)
    ref = u.copy()
    oracle.anneal(ref, RAGGED, 2, 0.8, 0.8, 7, 0)
    oracle.anneal(ref, RAGGED, 2, 0.8, 0.8, 7, 2)
    assert np.abs(split - ref).max() <= 1e-12
    # schedule endpoints are exact: 2 sweeps 1.25 -> 0.01 == one at 1.25, then one at 0.01
    two, _ = gpu_anneal(RAGGED, u, [(2, 1.25, 0.01, 7)])
    steps, _ = gpu_anneal(RAGGED, u, [(1, 1.25, 1.25, 7), (1, 0.01, 0.01, 7)])
    assert np.array_equal(two, steps)


def test_anneal_then_or_matches_oracle():
    """5 heat-bath sweeps (T 1.25 -> 0.01) within 1e-12 of the oracle, then 30 sweeps of the
    fix-until iteration within 1e-10, with the same sweep count, theta and F.  (Rounding
    differences grow about 2.7x per hot (T = 1.25) heat-bath sweep and hardly at all below
    T = 0.3: two oracle runs one ulp apart stay below 1e-13 over these 5 schedule sweeps but
    pass 1e-12 over 20, see test_heat_bath_rounding_growth_sets_parity_length, so longer
    anneals are compared through theta, F and the plaquette.)"""
    say("anneal 5 + fix_until 30 on 8^4")
    u = gi.gen_links(CFG8, 1.0, 13)
    ref = u.copy()
    oracle.anneal(ref, CFG8, 5, 1.25, 0.01, 5)
    with gf.Lattice(CFG8) as lat:
        lat.set_links(u)
        lat.anneal(5, 1.25, 0.01, 5)
        d_anneal = float(np.abs(lat.get_links() - ref).max())
        ro = oracle.fix_until(ref, CFG8, 1.7, 0, 1e-12, 30, 10, 100)
        r = lat.fix_until(omega=1.7, mode=0, theta_target=1e-12, max_sweeps=30, check_every=10, reunit_every=100)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"  after anneal {d_anneal:.2e}, after OR {d:.2e}; oracle theta {ro['theta']:.6e} gpu {r.theta:.6e}")
    assert d_anneal <= 1e-12
    assert r.converged == ro["converged"] and r.sweeps == ro["sweeps"] == 30
    assert abs(r.theta - ro["theta"]) <= 1e-8 * ro["theta"]
    assert abs(r.F - ro["F"]) <= 1e-12
    assert d <= 1e-10


def test_anneal_fp32_and_mixed_statistics():
    """float32 annealing: gauge invariance to float32 accuracy; cold annealing raises F like
    the float64 oracle's; in GF_MIXED the tracked g keeps the promoted links on the orbit."""
    say("anneal fp32 / mixed statistics")
    u = gi.gen_links(CFG8, 0.8, 14)
    P0 = oracle.plaquette(u, CFG8)
    ref = u.copy()
    oracle.anneal(ref, CFG8, 30, 1.0, 0.02, 9)
    _, F_ref = oracle.measure(ref, CFG8)
    got, P = gpu_anneal(CFG8, u, [(30, 1.0, 0.02, 9)], prec=gf.GF_FP32)
    _, F32 = oracle.measure(got, CFG8)
    say(f"  fp32: dP {abs(P - P0):.2e}, F {F32:.6f} vs oracle {F_ref:.6f}")
    assert abs(P - P0) < 1e-5
    assert abs(F32 - F_ref) < 0.01
    with gf.Lattice(CFG8, gf.GF_MIXED) as lat:
        lat.set_links(u)
        lat.anneal(30, 1.0, 0.02, 9)
        lat.promote_fp64()
        Pm = lat.plaquette()
        lm = lat.get_links()
    assert abs(Pm - P0) < 1e-12
    du, dd = oracle.unitarity(lm)
    assert du < 1e-13 and dd < 1e-13


def test_anneal_argument_checks():
    say("anneal argument checks")
    with gf.Lattice((4, 4, 4, 4)) as lat:
        lat.set_links(gi.gen_links((4, 4, 4, 4), 0.5, 0))
        for args in [(1, 0.5, 1.0, 1), (1, 1.0, 0.0, 1), (-1, 1.0, 0.5, 1), (1, float("inf"), 0.5, 1)]:
            with pytest.raises(gf.GFError) as e:
                lat.anneal(*args)
            assert e.value.status == gf.GF_E_ARG


@pytest.mark.parametrize("prec", [gf.GF_FP64, gf.GF_FP32, gf.GF_MIXED])
def test_long_anneal_stays_in_su3(prec):
    """Regression: 500 heat-bath sweeps (T 1.25 -> 0.01) keep the links in SU(3) and the
    plaquette unchanged (two-row storage must not amplify non-unitarity)."""
    say(f"long anneal prec={prec}")
    u = gi.gen_links(CFG8, 0.7, 2007)
    P0 = oracle.plaquette(u, CFG8)
    with gf.Lattice(CFG8, prec) as lat:
        lat.set_links(u)
        lat.anneal(500, 1.25, 0.01, 2007)
        if prec == gf.GF_MIXED:
            lat.promote_fp64()
        th, F = lat.measure()
        P = lat.plaquette()
        links = lat.get_links()
    du, dd = oracle.unitarity(links)
    tol_u = 1e-12 if prec != gf.GF_FP32 else 1e-5
    say(f"  theta {th:.3e} F {F:.6f} |dP| {abs(P - P0):.2e} unitarity {du:.1e} det {dd:.1e}")
    assert np.isfinite(th) and 0.0 < F <= 1.0
    assert du < tol_u and dd < tol_u
    assert abs(P - P0) < (1e-12 if prec != gf.GF_FP32 else 1e-5)
    ref = u.copy()
    oracle.anneal(ref, CFG8, 500, 1.25, 0.01, 2007)
    _, F_o = oracle.measure(ref, CFG8)
    assert abs(F - F_o) < 0.02  # same distribution; trajectories decorrelate over 500 sweeps


@pytest.mark.parametrize("prec", [gf.GF_FP64, gf.GF_FP32])
def test_anneal_checkpoint_resume(prec):
    """Links and heat-bath counter saved after 3 sweeps and restored on a fresh lattice continue
    bitwise as the uninterrupted 6-sweep run; a GF_MIXED lattice refuses."""
    say(f"anneal checkpoint/resume prec={prec}")
    u = gi.gen_links(RAGGED, 0.9, 13)
    with gf.Lattice(RAGGED, prec) as lat:
        lat.set_links(u)
        lat.anneal(3, 1.0, 1.0, 5)
        lat.anneal(3, 1.0, 1.0, 5)
        straight = lat.get_links()
    with gf.Lattice(RAGGED, prec) as lat:
        lat.set_links(u)
        lat.anneal(3, 1.0, 1.0, 5)
        saved, counter = lat.get_links(), lat.anneal_counter
    assert counter == 3
    with gf.Lattice(RAGGED, prec) as lat:
        lat.set_links(saved)
        assert lat.anneal_counter == 0
        lat.anneal_counter = counter
        lat.anneal(3, 1.0, 1.0, 5)
        assert lat.anneal_counter == 6
        resumed = lat.get_links()
    # float32 links come back as float64 values that round to themselves on upload, so the
    # restored state is the saved one in either precision
    assert np.array_equal(resumed, straight)
    with gf.Lattice(RAGGED, gf.GF_MIXED) as lat:
        lat.set_links(u)
        with pytest.raises(gf.GFError) as e:
            _ = lat.anneal_counter
        assert e.value.status == gf.GF_E_STATE
