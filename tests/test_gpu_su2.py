"""Gauge group SU(2) on the GPU (through the C ABI) against the FP64 CPU oracle.

The abstract lists SU(2) beside SU(3); Sec. 2's maximiser K^dag / sqrt(det K^dag) is exact for
SU(2), and Sec. 4.1 changes the group by the link parameterisation alone.  The GPU stores each
link as a quaternion; the oracle holds full 2x2 complex links.  Tolerances as for SU(3): float64
links within 1e-12 after one sweep and 1e-10 after 100, theta relative 1e-12, F 1e-14, the
fix-until sweep count equal to the oracle's, heat-bath links within 1e-12 after 5 sweeps
(same Philox counters); float32 links within 5e-5.
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
EDGE = [(2, 2, 2, 2), (2, 4, 6, 8), (4, 2, 2, 6)]


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


def su2_lattice(dims, prec=gf.GF_FP64, gauge=gf.GF_LANDAU, stream=None):
    return gf.Lattice(dims, prec, stream=stream, gauge=gauge, group=2)


def ndir(gauge):
    return 3 if gauge == gf.GF_COULOMB else 4


def test_roundtrip_host_and_device():
    import torch

    u = gi.gen_links_su2(RAGGED, 0.7, 61)
    with su2_lattice(RAGGED) as lat:
        assert gf.gf_lattice_group(lat.handle) == 2
        lat.set_links(u)
        got = lat.get_links()
        assert got.shape == u.shape
        assert np.abs(got - u).max() < 1e-15
        lat.set_links(torch.from_numpy(u).cuda())
        out = torch.zeros(u.shape, dtype=torch.float64, device="cuda")
        lat.get_links(out)
        assert np.array_equal(out.cpu().numpy(), got)
        with pytest.raises(ValueError):
            lat.set_links(gi.gen_links(RAGGED, 0.7, 61))  # SU(3) links do not fit


@pytest.mark.parametrize("dims", [CFG8, RAGGED] + EDGE)
@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
@pytest.mark.parametrize("mode", [gf.GF_OR_EXACT, gf.GF_OR_BINOMIAL1])
def test_one_sweep_parity(dims, gauge, mode):
    say(f"su2 1 sweep dims={dims} gauge={gauge} mode={mode}")
    u = gi.gen_links_su2(dims, 0.7, 62)
    ref = u.copy()
    oracle.su2lat_sweep(ref, dims, 1, 1.7, mode, ndir(gauge))
    with su2_lattice(dims, gauge=gauge) as lat:
        lat.set_links(u)
        lat.sweep(1, 1.7, mode)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"  max|links - oracle| {d:.3e}")
    assert d <= 1e-12


@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
def test_100_sweeps_parity(gauge):
    u = gi.gen_links_su2(CFG8, 0.6, 0)
    ref = u.copy()
    oracle.su2lat_sweep(ref, CFG8, 100, 1.7, 0, ndir(gauge))
    with su2_lattice(CFG8, gauge=gauge) as lat:
        lat.set_links(u)
        lat.sweep(100, 1.7)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"su2 100 sweeps gauge={gauge}: max|links - oracle| {d:.3e}")
    assert d <= 1e-10


@pytest.mark.parametrize("block,nt", [(64, 0), (128, 1), (256, 2), (512, 0), (512, 2)])
def test_launch_shape_is_bitwise_irrelevant(block, nt):
    u = gi.gen_links_su2(RAGGED, 0.8, 63)
    outs = []
    for cfg in [(1, 256, 0), (1, block, nt)]:
        with su2_lattice(RAGGED) as lat:
            lat.set_sweep_config(*cfg)
            lat.set_links(u)
            lat.sweep(3, 1.7)
            outs.append(lat.get_links())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dims", [CFG8, RAGGED, (2, 4, 6, 8)])
def test_measurements(dims):
    u = gi.gen_links_su2(dims, 0.7, 64)
    th_o, F_o = oracle.su2lat_measure(u, dims)
    P_o = oracle.su2lat_plaquette(u, dims)
    tht_o, Ft_o = oracle.su2lat_coulomb_measure(u, dims)
    with su2_lattice(dims) as lat:
        lat.set_links(u)
        th, F = lat.measure()
        P = lat.plaquette()
        lat.gauge = gf.GF_COULOMB
        tht, Ft = lat.measure_timeslices()
    assert abs(th - th_o) <= 1e-12 * th_o
    assert abs(F - F_o) <= 1e-14
    assert abs(P - P_o) <= 1e-14
    assert np.abs(tht - tht_o).max() <= 1e-12 * tht_o.max()
    assert np.abs(Ft - Ft_o).max() <= 1e-14


@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
def test_fix_until_matches_oracle(gauge):
    dims = CFG8
    u = gi.gen_links_su2(dims, 0.6, 0)
    ref = u.copy()
    r_o = oracle.su2lat_fix_until(ref, dims, 1.7, 0, 1e-12, 3000, 10, 100, ndir(gauge))
    P0 = oracle.su2lat_plaquette(u, dims)
    with su2_lattice(dims, gauge=gauge) as lat:
        lat.set_links(u)
        r = lat.fix_until(omega=1.7, theta_target=1e-12, max_sweeps=3000, check_every=10, reunit_every=100)
        got = lat.get_links()
        P = lat.plaquette()
    say(f"su2 fix-until gauge={gauge}: oracle {r_o['sweeps']} sweeps, gpu {r.sweeps}; theta {r.theta:.3e}")
    assert r_o["converged"] and r.converged and r.sweeps == r_o["sweeps"]
    assert abs(r.theta - r_o["theta"]) <= 1e-6 * r_o["theta"] and abs(r.F - r_o["F"]) < 1e-13
    assert float(np.abs(got - ref).max()) <= 1e-10
    assert abs(P - P0) < 1e-12


@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
@pytest.mark.parametrize("dims", [CFG8, RAGGED])
def test_anneal_fp64_parity(gauge, dims):
    u = gi.gen_links_su2(dims, 1.0, 65)
    ref = u.copy()
    capped = oracle.su2lat_anneal(ref, dims, 5, 1.25, 0.01, 44, 0, ndir(gauge))
    with su2_lattice(dims, gauge=gauge) as lat:
        lat.set_links(u)
        lat.anneal(5, 1.25, 0.01, 44)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"su2 anneal gauge={gauge} dims={dims}: max|links - oracle| {d:.3e}")
    assert capped == 0 and d <= 1e-12


def test_fp32_sweep_and_reunitarize():
    u = gi.gen_links_su2(RAGGED, 0.7, 66)
    ref = u.copy()
    oracle.su2lat_sweep(ref, RAGGED, 1, 1.7)
    with su2_lattice(RAGGED, gf.GF_FP32) as lat:
        lat.set_links(u)
        lat.sweep(1, 1.7)
        got = lat.get_links()
    assert float(np.abs(got - ref).max()) <= 5e-5
    noisy = u + 1e-6 * np.random.default_rng(2).standard_normal(u.shape)
    ref = noisy.copy()
    oracle.su2lat_reunitarize(ref)
    with su2_lattice(RAGGED) as lat:
        lat.set_links(noisy)
        lat.reunitarize()
        got = lat.get_links()
    assert float(np.abs(got - ref).max()) <= 1e-15


def test_estimate_and_adaptive_checks():
    """The fused estimate of an SU(2) sweep against the oracle ((1/(2V)) of the black terms
    before the black half-sweep and the white terms after it), and adaptive checks equal to
    exact checks."""
    dims = CFG8
    u = gi.gen_links_su2(dims, 0.7, 67)
    black = ln.colours(dims) == 0
    ref = u.copy()
    s_b = oracle.su2lat_theta_density(ref, dims)[black].sum()
    oracle.su2lat_half_sweep(ref, dims, 0, 1.7)
    s_w = oracle.su2lat_theta_density(ref, dims)[~black].sum()
    expect = (s_b + s_w) / (2.0 * u.shape[0])
    with su2_lattice(dims) as lat:
        lat.set_links(u)
        est = lat.sweep_estimate(1.7)
    assert abs(est - expect) <= 1e-12 * expect
    u = gi.gen_links_su2(dims, 0.6, 0)
    res = []
    for adaptive in (False, True):
        with su2_lattice(dims) as lat:
            lat.set_links(u)
            lat.set_check_policy(adaptive)
            res.append((lat.fix_until(omega=1.7, theta_target=1e-12, max_sweeps=3000, check_every=10),
                        lat.get_links(), lat.counters))
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])
    assert res[1][2][0] < res[0][2][0]


def test_autotune_and_errors():
    u = gi.gen_links_su2(CFG8, 0.7, 68)
    with pytest.raises(gf.GFError) as e:
        gf.Lattice(CFG8, gf.GF_MIXED, group=2)
    assert e.value.status == gf.GF_E_ARG
    with su2_lattice(CFG8) as lat:
        lat.set_links(u)
        with pytest.raises(gf.GFError) as e:
            lat.set_sweep_config(2, 128, 0)
        assert e.value.status == gf.GF_E_ARG
        with pytest.raises(gf.GFError) as e:
            lat.tune_switch()
        assert e.value.status == gf.GF_E_STATE
        (tps, block, nt, minw), table = lat.autotune(gf.GF_FP64, n_sweeps=2)
        assert tps == 1 and minw == 0 and len(table) == 12
        before = lat.get_links()
        assert np.array_equal(before, lat.get_links())
