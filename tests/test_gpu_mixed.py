"""Mixed precision (float32 bulk sweeps, float64 polish) against the FP64 oracle.

Several gauge-fixed results are correct (Gribov copies, Sec. 1 of the paper),
and float32 rounding can steer the iteration to a different copy than the
float64 oracle, so links are not compared after many sweeps; what is unique
is compared: the gauge condition theta < target, the gauge-invariant
plaquette (the promotion rebuilds the float64 links as g U0 g^dag from the
original links, so it must match the input's plaquette to float64
precision), SU(3) membership, and the functional F against the oracle's run
on the same input (reported, bounded loosely).
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


def test_mixed_bulk_sweep_equals_fp32_sweep():
    """Before promotion a GF_MIXED lattice sweeps exactly like a GF_FP32 one (g tracking
    only adds the g(x) update)."""
    say("mixed bulk == fp32 sweep, RAGGED")
    u = gi.gen_links(RAGGED, 0.8, 1)
    with gf.Lattice(RAGGED, gf.GF_FP32) as a:
        a.set_links(u)
        a.sweep(5, 1.7)
        la = a.get_links()
    with gf.Lattice(RAGGED, gf.GF_MIXED) as b:
        b.set_links(u)
        b.sweep(5, 1.7)
        lb = b.get_links()
    assert np.array_equal(la, lb)


@pytest.mark.parametrize("tps", [1, 4, 8])
def test_promotion_stays_on_gauge_orbit(tps):
    """After float32 sweeps, promotion gives g U0 g^dag: same plaquette as U0 to 1e-12,
    SU(3) to 1e-13, and within float32 accuracy of the float32 links."""
    say(f"promotion orbit tps={tps}, RAGGED")
    u = gi.gen_links(RAGGED, 0.8, 2)
    P0 = oracle.plaquette(u, RAGGED)
    with gf.Lattice(RAGGED, gf.GF_MIXED) as lat:
        lat.set_sweep_config(tps, 256)
        lat.set_links(u)
        lat.sweep(30, 1.7)
        l32 = lat.get_links()
        P32 = lat.plaquette()
        lat.promote_fp64()
        l64 = lat.get_links()
        P64 = lat.plaquette()
    say(f"  plaquette drift: fp32 links {abs(P32 - P0):.2e}, promoted {abs(P64 - P0):.2e}; "
        f"max|promoted - fp32| {np.abs(l64 - l32).max():.2e}")
    assert abs(P64 - P0) < 1e-12
    assert oracle.plaquette(l64, RAGGED) == pytest.approx(P0, abs=1e-12)
    du, dd = oracle.unitarity(l64)
    assert du < 1e-13 and dd < 1e-13
    assert np.abs(l64 - l32).max() < 1e-4


def test_mixed_fix_until_8x4():
    """8^4, eps = 0.6, seed 0: float32 bulk to theta < 1e-8, float64 polish to theta < 1e-12."""
    say("mixed fix_until 8^4")
    u = gi.gen_links(CFG8, 0.6, 0)
    P0 = oracle.plaquette(u, CFG8)
    ref = u.copy()
    ro = oracle.fix_until(ref, CFG8, 1.7, 0, 1e-12, 3000, 10, 100)
    with gf.Lattice(CFG8, gf.GF_MIXED) as lat:
        lat.set_links(u)
        r = lat.fix_until(omega=1.7, mode=0, theta_target=1e-12, max_sweeps=3000, check_every=10,
                          reunit_every=100, theta_switch=1e-8)
        P = lat.plaquette()
        links = lat.get_links()
    th_chk, F_chk = oracle.measure(links, CFG8)
    say(f"  mixed: sweeps {r.sweeps} (fp32 {r.sweeps_fp32}, fp64 {r.sweeps_fp64}) theta {r.theta:.3e} "
        f"F {r.F:.15f}; oracle fp64: sweeps {ro['sweeps']} F {ro['F']:.15f}; dF {r.F - ro['F']:.2e}")
    assert r.converged and r.theta < 1e-12
    assert r.sweeps_fp32 > 0 and r.sweeps_fp64 > 0
    assert r.sweeps_fp32 + r.sweeps_fp64 == r.sweeps
    assert abs(P - P0) < 1e-12
    assert th_chk < 1e-12 and abs(th_chk - r.theta) <= 1e-8 * r.theta + 1e-20
    assert abs(F_chk - r.F) < 1e-13
    assert abs(r.F - ro["F"]) < 1e-3


def test_mixed_stall_switch():
    """theta_switch = 0 is below the float32 floor: stall detection still promotes, and the
    float64 polish reaches a target float32 cannot (1e-20)."""
    say("mixed stall switch RAGGED")
    u = gi.gen_links(RAGGED, 0.5, 3)
    with gf.Lattice(RAGGED, gf.GF_MIXED) as lat:
        lat.set_links(u)
        r = lat.fix_until(omega=1.7, mode=0, theta_target=1e-20, max_sweeps=5000, check_every=5,
                          reunit_every=100, theta_switch=0.0)
    say(f"  sweeps {r.sweeps} fp32 {r.sweeps_fp32} fp64 {r.sweeps_fp64} theta {r.theta:.2e}")
    assert r.converged and r.sweeps_fp64 > 0


def test_fp32_floor_properties_and_the_switch():
    """gf_tune_switch: the float32 rounding floor of theta (a switch-point heuristic of the
    library; no result depends on it, the result is always the float64 one).  Checked by what
    the rounding fixes: exactly 0 on links whose entries are 0, +-1, +-i (float32 stores them and
    every float32 product and sum formed from them exactly); on generic links a few float32 units
    squared (u = 2^-24: between 1 and 30 u^2), above the floor of the storage alone (rows rounded
    to float32, everything else exact; numpy) by the float32 arithmetic of the row-2 rebuild and
    the K sums (2 to 20 times), and unchanged within 20 % by a Haar gauge rotation (a property of
    rounding, not of the gauge).  The switch point is max(target, 100 x floor)."""
    u2 = 2.0 ** -48
    for dims, eps, seed in ((CFG8, 0.2, 5), (CFG8, 0.6, 0), (RAGGED, 1.0, 4)):
        u = gi.gen_links(dims, eps, seed)
        h = gi.to_canonical(gi.haar_su3(np.random.default_rng(9), gi.volume(dims)))
        rot = oracle.gauge_transform(u.copy(), dims, h)
        floors = []
        for links in (u, rot):
            with gf.Lattice(dims, gf.GF_MIXED) as lat:
                lat.set_links(links)
                f_g, sw = lat.tune_switch(1e-12)
                f_g2, sw2 = lat.tune_switch(1e-20)
            assert sw == max(1e-12, 100.0 * f_g) and sw2 == 100.0 * f_g2 and f_g2 == f_g
            floors.append(f_g)
        s = ln.storage_floor(u, dims)
        say(f"  floor {dims} eps {eps}: {floors[0] / u2:.2f} u^2, rotated {floors[1] / u2:.2f} u^2, "
            f"storage only {s / u2:.2f} u^2")
        assert 1.0 * u2 < floors[0] < 30.0 * u2
        assert 2.0 < floors[0] / s < 20.0
        assert abs(floors[1] / floors[0] - 1.0) < 0.2
    ex = ln.float_exact_links(CFG8, 3)
    with gf.Lattice(CFG8, gf.GF_FP64) as lat:
        lat.set_links(ex)
        f_g, sw = lat.tune_switch(1e-12)
    assert f_g == 0.0 and sw == 1e-12
    with gf.Lattice(CFG8, gf.GF_FP32) as lat:
        lat.set_links(ex)
        with pytest.raises(gf.GFError):
            lat.tune_switch(1e-12)


@pytest.mark.parametrize("dims,eps,seed", [(CFG8, 0.6, 0), ((16, 16, 16, 16), 0.4, 11)])
def test_mixed_auto_switch_ends_in_float64(dims, eps, seed):
    """theta_switch < 0: the library's switch point.  Float32 sweeps run down to it and the result
    is the float64 one (links rebuilt from g and U0, theta and F measured in float64): the oracle's
    theta of the downloaded links is below the target, the plaquette is the input's, and the
    sweep count is the float64 run's (float32 converges at the float64 rate above its floor)."""
    u = gi.gen_links(dims, eps, seed)
    P0 = oracle.plaquette(u, dims)
    with gf.Lattice(dims, gf.GF_FP64) as lat:
        lat.set_links(u)
        r64 = lat.fix_until(omega=1.7, mode=0, theta_target=1e-12, max_sweeps=6000, check_every=10,
                            reunit_every=100, theta_switch=0.0)
    with gf.Lattice(dims, gf.GF_MIXED) as lat:
        lat.set_links(u)
        _, sw = lat.tune_switch(1e-12)
        r = lat.fix_until(omega=1.7, mode=0, theta_target=1e-12, max_sweeps=6000, check_every=10,
                          reunit_every=100, theta_switch=-1.0)
        P = lat.plaquette()
        links = lat.get_links()
    th_o, F_o = oracle.measure(links, dims)
    say(f"  auto switch {dims} eps {eps}: switch {sw:.2e}, sweeps {r.sweeps} ({r.sweeps_fp32}/{r.sweeps_fp64}) "
        f"vs float64 {r64.sweeps}; theta {r.theta:.3e} (oracle {th_o:.3e})")
    assert r.converged and r64.converged
    assert r.sweeps_fp32 > 0 and r.sweeps_fp32 + r.sweeps_fp64 == r.sweeps
    assert th_o < 1e-12 and abs(th_o - r.theta) <= 1e-8 * r.theta
    assert abs(F_o - r.F) < 1e-13
    assert abs(P - P0) < 1e-12
    assert abs(r.sweeps - r64.sweeps) <= 0.1 * r64.sweeps
