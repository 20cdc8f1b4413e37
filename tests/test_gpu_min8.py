"""Float64 links stored in 8 reals (gf_create_lattice_min8) on the GPU, through the C ABI,
against the FP64 CPU oracle.

arXiv:1412.3655 Sec. 4.1 names the minimal 8-parameter representation among the link
parameterisations cuLGT2 does not provide; the library stores it in the row-pivoted form the
oracle defines (oracle/gf_oracle.c, pinned in test_oracle_min8.py).  The method is unchanged:
the stored links are SU(3) to rounding, so the sweep must match the oracle's plain sweep, started
from the links the representation holds (oracle.min8_store of the input), to the tolerances of
the 12-real float64 path: 1e-12 after one sweep, 1e-10 after 100, theta relative 1e-12, F 1e-14.
The decode/encode pair itself: set_links then get_links reproduces the oracle's stored links to
4e-15.  Launch shapes give bitwise equal links.  The storage of a float64 lattice can also be
switched at run time (gf_set_storage) and chosen by timing (gf_autotune_storage).
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


def min8_lattice(dims, gauge=gf.GF_LANDAU, stream=None):
    return gf.Lattice(dims, gf.GF_FP64, stream=stream, gauge=gauge, storage=8)


def stored(u):
    return oracle.min8_store(u.copy())


def ndir(gauge):
    return 3 if gauge == gf.GF_COULOMB else 4


def oracle_sweep(ref, dims, n, omega, mode, gauge):
    if gauge == gf.GF_COULOMB:
        oracle.coulomb_sweep(ref, dims, n, omega, mode)
    else:
        oracle.sweep(ref, dims, n, omega, mode)


def test_storage_roundtrip_and_footprint():
    import torch

    u = gi.gen_links(RAGGED, 0.7, 71)
    ref = stored(u)
    with min8_lattice(RAGGED) as lat:
        assert gf.gf_lattice_storage(lat.handle) == 8
        lat.set_links(u)
        got = lat.get_links()
        d = float(np.abs(got - ref).max())
        say(f"min8 set/get vs oracle store: {d:.2e}; vs input {np.abs(got - u).max():.2e}")
        assert d <= 4e-15
        du, dd = oracle.unitarity(got.copy())
        assert du <= 2e-15 and dd <= 2e-15
        lat.set_links(torch.from_numpy(u).cuda())
        out = torch.zeros(u.shape, dtype=torch.float64, device="cuda")
        lat.get_links(out)
        assert np.array_equal(out.cpu().numpy(), got)
        # a second store of stored links changes them by rounding only
        lat.set_links(got)
        assert float(np.abs(lat.get_links() - got).max()) <= 1.2e-15
        b8 = gf.gf_lattice_info(lat.handle)[1]
    with gf.Lattice(RAGGED, gf.GF_FP64) as lat:
        assert gf.gf_lattice_storage(lat.handle) == 12
        b12 = gf.gf_lattice_info(lat.handle)[1]
    ld = -(-RAGGED[0] * RAGGED[1] * RAGGED[2] * RAGGED[3] // 2 // 64) * 64
    assert b12 - b8 == 2 * 4 * ld * 2 * 16  # two 16-byte chunks fewer per link


def test_special_links_round_trip():
    """Identity, centre elements, diag(-1, -1, 1) (a clamped tangent) and permutations survive the
    device encode/decode to rounding."""
    dims = (2, 2, 2, 2)
    w = np.exp(2j * np.pi / 3)
    mats = [np.eye(3), np.eye(3) * w, np.diag([-1.0, -1.0, 1.0]), np.diag([1.0, -1.0, -1.0]),
            np.roll(np.eye(3), 1, axis=1), np.roll(np.eye(3), 2, axis=1),
            np.array([[0, 0, 1], [0, -1, 0], [1, 0, 0]]), np.diag(np.exp(1j * np.array([np.pi, 0.5, -0.5 - np.pi])))]
    c = np.zeros((16, 4, 3, 3), dtype=complex)
    for k in range(64):
        c[k // 4, k % 4] = mats[k % len(mats)]
    u = gi.to_canonical(c)
    with min8_lattice(dims) as lat:
        lat.set_links(u)
        got = lat.get_links()
    assert float(np.abs(got - u).max()) <= 2e-15


@pytest.mark.parametrize("dims", [CFG8, RAGGED] + EDGE)
@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
@pytest.mark.parametrize("mode", [gf.GF_OR_EXACT, gf.GF_OR_BINOMIAL1])
def test_one_sweep_parity(dims, gauge, mode):
    say(f"min8 1 sweep dims={dims} gauge={gauge} mode={mode}")
    u = stored(gi.gen_links(dims, 0.7, 72))
    ref = u.copy()
    oracle_sweep(ref, dims, 1, 1.7, mode, gauge)
    with min8_lattice(dims, gauge) as lat:
        lat.set_links(u)
        lat.sweep(1, 1.7, mode)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"  max|links - oracle| {d:.3e}")
    assert d <= 1e-12


@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
def test_100_sweeps_parity(gauge):
    u = stored(gi.gen_links(CFG8, 0.6, 0))
    ref = u.copy()
    oracle_sweep(ref, CFG8, 100, 1.7, 0, gauge)
    with min8_lattice(CFG8, gauge) as lat:
        lat.set_links(u)
        lat.sweep(100, 1.7)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"min8 100 sweeps gauge={gauge}: max|links - oracle| {d:.3e}")
    assert d <= 1e-10


@pytest.mark.parametrize("tps,block,nt", [(1, 64, 0), (2, 128, 1), (4, 256, 2), (8, 512, 0), (2, 64, 2),
                                          (4, 128, 1)])
def test_launch_shape_is_bitwise_irrelevant(tps, block, nt):
    u = gi.gen_links(RAGGED, 0.8, 73)
    outs = []
    for cfg in [(4, 256, 0), (tps, block, nt)]:
        with min8_lattice(RAGGED) as lat:
            lat.set_sweep_config(*cfg)
            lat.set_links(u)
            lat.sweep(3, 1.7)
            outs.append(lat.get_links())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dims", [CFG8, RAGGED, (2, 4, 6, 8)])
def test_measurements(dims):
    u = stored(gi.gen_links(dims, 0.7, 74))
    th_o, F_o = oracle.measure(u, dims)
    P_o = oracle.plaquette(u, dims)
    tht_o, Ft_o = oracle.coulomb_measure(u, dims)
    with min8_lattice(dims) as lat:
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
def test_fix_until_against_oracle(gauge):
    """To theta < 1e-12 checked every 10 sweeps: converged, the oracle's sweep count (the links
    differ from the oracle's, reunitarised every 100 sweeps, by rounding only), and the
    gauge-invariant plaquette kept to 1e-12."""
    dims = CFG8
    u = stored(gi.gen_links(dims, 0.6, 0))
    ref = u.copy()
    fix = oracle.fix_until if gauge == gf.GF_LANDAU else oracle.coulomb_fix_until
    r_o = fix(ref, dims, 1.7, 0, 1e-12, 3000, 10, 100)
    P0 = oracle.plaquette(u, dims)
    with min8_lattice(dims, gauge) as lat:
        lat.set_links(u)
        r = lat.fix_until(omega=1.7, theta_target=1e-12, max_sweeps=3000, check_every=10, reunit_every=100)
        got = lat.get_links()
        P = lat.plaquette()
    say(f"min8 fix-until gauge={gauge}: oracle {r_o['sweeps']} sweeps, gpu {r.sweeps}; theta {r.theta:.3e}")
    assert r_o["converged"] and r.converged and r.sweeps == r_o["sweeps"]
    assert abs(r.F - r_o["F"]) < 1e-13
    assert float(np.abs(got - ref).max()) <= 1e-10
    assert abs(P - P0) < 1e-12


@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
def test_anneal_parity(gauge):
    """Five heat-bath sweeps (the same Philox counters) against the oracle: 1e-12."""
    dims = RAGGED
    u = stored(gi.gen_links(dims, 1.0, 75))
    ref = u.copy()
    anneal = oracle.anneal if gauge == gf.GF_LANDAU else oracle.coulomb_anneal
    capped = anneal(ref, dims, 5, 1.25, 0.01, 46)
    with min8_lattice(dims, gauge) as lat:
        lat.set_links(u)
        lat.anneal(5, 1.25, 0.01, 46)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"min8 anneal gauge={gauge}: max|links - oracle| {d:.3e}")
    assert capped == 0 and d <= 1e-12


def test_estimate_and_adaptive_checks():
    dims = CFG8
    u = stored(gi.gen_links(dims, 0.7, 76))
    black = ln.colours(dims) == 0
    ref = u.copy()
    s_b = oracle.theta_density(ref, dims)[black].sum()
    oracle.half_sweep(ref, dims, 0, 1.7)
    s_w = oracle.theta_density(ref, dims)[~black].sum()
    expect = (s_b + s_w) / (3.0 * u.shape[0])
    with min8_lattice(dims) as lat:
        lat.set_links(u)
        est = lat.sweep_estimate(1.7)
    assert abs(est - expect) <= 1e-12 * expect
    u = stored(gi.gen_links(dims, 0.6, 0))
    res = []
    for adaptive in (False, True):
        with min8_lattice(dims) as lat:
            lat.set_links(u)
            lat.set_check_policy(adaptive)
            res.append((lat.fix_until(omega=1.7, theta_target=1e-12, max_sweeps=3000, check_every=10),
                        lat.get_links(), lat.counters))
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])
    assert res[1][2][0] < res[0][2][0]


def test_autotune_graphs_and_errors(tmp_path):
    import torch

    u = gi.gen_links(RAGGED, 0.7, 77)
    with min8_lattice(RAGGED) as lat:
        lat.set_links(u)
        before = lat.get_links()
        lat.reunitarize()  # nothing to do: every store re-projects
        assert np.array_equal(lat.get_links(), before)
        with pytest.raises(gf.GFError) as e:
            lat.set_sweep_config(1, 128, 0, min_waves=2)
        assert e.value.status == gf.GF_E_ARG
        with pytest.raises(gf.GFError) as e:
            lat.tune_switch()
        assert e.value.status == gf.GF_E_STATE
        cache = str(tmp_path / "tune.txt")
        (tps, block, nt, minw), table = lat.autotune(gf.GF_FP64, n_sweeps=2, cache_path=cache)
        assert minw == 0 and len(table) == 15 + 9 + 9 and all(e[3] == 0 for e in table)
        assert np.array_equal(lat.get_links(), before)
        assert "-min8" in open(cache).read()
        lat.sweep(2, 1.7)
        tuned = lat.get_links()
    stream = torch.cuda.Stream()
    with min8_lattice(RAGGED, stream=stream) as lat:  # graph capture and replay
        lat.set_links(u)
        lat.sweep(2, 1.7)
        assert np.array_equal(lat.get_links(), tuned)
    with pytest.raises(ValueError):
        gf.Lattice(RAGGED, gf.GF_FP64, group=2, storage=8)


def test_full_size_32x4_one_sweep():
    """32^4, eps = 0.8, seed 0 (the bandwidth workload) in 8-real storage, in two launch shapes:
    theta/F of the stored input, then every link after one sweep against the oracle."""
    dims = (32, 32, 32, 32)
    say("min8 full size 32^4: generating")
    u = stored(gi.gen_links(dims, 0.8, 0))
    th_o, F_o = oracle.measure(u, dims)
    ref = u.copy()
    oracle.sweep(ref, dims, 1, 1.7, 0)
    th1_o, F1_o = oracle.measure(ref, dims)
    for tps, block, nt in ((4, 256, 0), (2, 128, 1)):
        say(f"min8 full size 32^4: gpu {tps}/{block}/{nt}")
        with min8_lattice(dims) as lat:
            lat.set_sweep_config(tps, block, nt)
            lat.set_links(u)
            th, F = lat.measure()
            lat.sweep(1, 1.7, 0)
            th1, F1 = lat.measure()
            got = lat.get_links()
        assert abs(th - th_o) <= 1e-12 * th_o and abs(F - F_o) <= 1e-14
        d = float(np.abs(got - ref).max())
        say(f"  max|diff| after 1 sweep: {d:.3e}")
        assert d <= 1e-12
        assert abs(th1 - th1_o) <= 1e-10 * th1_o and abs(F1 - F1_o) <= 1e-13


def test_set_storage_converts_both_ways():
    """12 -> 8 reals holds the oracle's stored links (4e-15), 8 -> 12 keeps them bitwise; sweeps
    after each conversion match the oracle from those links; graphs captured before a conversion
    are not replayed on the freed field."""
    import torch

    dims = RAGGED
    u = gi.gen_links(dims, 0.7, 78)
    stream = torch.cuda.Stream()
    with gf.Lattice(dims, gf.GF_FP64, stream=stream) as lat:
        lat.set_links(u)
        lat.sweep(2, 1.7)  # captures a graph over the 12-real field
        before = lat.get_links()
        b12 = gf.gf_lattice_info(lat.handle)[1]
        lat.storage = 8
        assert lat.storage == 8 and gf.gf_lattice_info(lat.handle)[1] < b12
        got8 = lat.get_links()
        assert float(np.abs(got8 - stored(before)).max()) <= 4e-15
        ref = got8.copy()
        oracle.sweep(ref, dims, 2, 1.7, 0)
        lat.sweep(2, 1.7)  # a new graph over the 8-real field
        after8 = lat.get_links()
        assert float(np.abs(after8 - ref).max()) <= 1e-12
        lat.storage = 12
        assert lat.storage == 12 and gf.gf_lattice_info(lat.handle)[1] == b12
        assert np.array_equal(lat.get_links(), after8)
        ref = after8.copy()
        oracle.sweep(ref, dims, 2, 1.7, 0)
        lat.sweep(2, 1.7)
        assert float(np.abs(lat.get_links() - ref).max()) <= 1e-12
        with pytest.raises(gf.GFError) as e:
            lat.storage = 9
        assert e.value.status == gf.GF_E_ARG
    for prec in (gf.GF_FP32, gf.GF_FP64):
        with gf.Lattice(dims, prec, group=2) as lat:
            with pytest.raises(gf.GFError) as e:
                lat.storage = 8
            assert e.value.status == gf.GF_E_STATE


@pytest.mark.parametrize("start", [12, 8])
def test_autotune_storage(start):
    """The tuner times both storages and keeps the faster, with its configuration; the links are
    those of the chosen storage (unchanged when the storage stays, the stored projection when it
    switches to 8 reals)."""
    dims = (16, 16, 16, 16)
    u = gi.gen_links(dims, 0.8, 79)
    with gf.Lattice(dims, gf.GF_FP64, storage=start) as lat:
        lat.set_links(u)
        before = lat.get_links()
        reals, us12, us8 = lat.autotune_storage(2)
        say(f"storage autotune from {start}: chose {reals}; 12 reals {us12:.1f} us, 8 reals {us8:.1f} us")
        assert reals in (8, 12) and lat.storage == reals and us12 > 0 and us8 > 0
        assert reals == (8 if us8 < us12 else 12)
        got = lat.get_links()
        if reals == start:
            assert np.array_equal(got, before)
        else:
            assert float(np.abs(got - stored(before)).max()) <= 4e-15
        ref = got.copy()
        oracle.sweep(ref, dims, 1, 1.7, 0)
        lat.sweep(1, 1.7)
        assert float(np.abs(lat.get_links() - ref).max()) <= 1e-12
    with gf.Lattice(dims, gf.GF_FP64, group=2) as lat:
        lat.set_links(gi.gen_links_su2(dims, 0.8, 79))
        with pytest.raises(gf.GFError) as e:
            lat.autotune_storage(2)
        assert e.value.status == gf.GF_E_STATE
