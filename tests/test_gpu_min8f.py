"""Float32 links stored in 8 reals (gf_set_storage(8) on GF_FP32 and GF_MIXED lattices) on the
GPU, through the C ABI, against the FP64 CPU oracle.

The storage is the 8-parameter representation of the float64 8-real lattices (oracle/gf_oracle.c,
pinned in test_oracle_min8.py) with the 8 values held in float32.  Packing encodes in float64 and
rounds the values; measurement and unpacking decode the float32 values in float64, so the links a
lattice holds are SU(3) to float64 rounding and the oracle's measurement of the downloaded links
is the lattice's own (1e-12 relative).  The sweeps decode and encode in float32: one sweep against
the oracle's float64 sweep from the same links is bounded as for 12-real float32 links (max-abs
5e-5, RMS 1e-6: float32 rounding of K amplified by the maximiser and omega), launch shapes give
bitwise equal links, and mixed precision ends in float64 with the float64 run's guarantees
(theta < target measured by the oracle, the input's plaquette to 1e-12).
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


def lat8(dims, prec=gf.GF_FP32, gauge=gf.GF_LANDAU, stream=None):
    return gf.Lattice(dims, prec, stream=stream, gauge=gauge, storage=8)


@pytest.mark.parametrize("prec", [gf.GF_FP32, gf.GF_MIXED])
def test_storage_roundtrip_and_footprint(prec):
    """set_links then get_links: the float32 rounding of the 8 values moves a link by < 1e-6
    from the oracle's float64 8-real store, and the downloaded links are SU(3) to float64
    rounding; the float32 field takes 2/3 of its 12-real size."""
    u = gi.gen_links(RAGGED, 0.7, 81)
    ref = oracle.min8_store(u.copy())
    with gf.Lattice(RAGGED, prec) as lat12:
        b12 = gf.gf_lattice_info(lat12.handle)[1]
    with lat8(RAGGED, prec) as lat:
        assert lat.storage == 8
        b8 = gf.gf_lattice_info(lat.handle)[1]
        lat.set_links(u)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    du, dd = oracle.unitarity(got.copy())
    V = gi.volume(RAGGED)
    say(f"min8 float32 set/get vs float64 store: {d:.2e}; unitarity {du:.1e} {dd:.1e}; bytes {b8} vs {b12}")
    assert d <= 1e-6
    assert du <= 4e-15 and dd <= 4e-15  # entries of the float64 decode within ~2 units each
    ld = -(-(V // 2) // 64) * 64  # sites per (colour, direction) plane, padded to whole 64-site tiles
    assert b12 - b8 == 2 * 4 * ld * 16  # one float4 chunk less per link


@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
@pytest.mark.parametrize("mode", [gf.GF_OR_EXACT, gf.GF_OR_BINOMIAL1])
def test_one_sweep_parity(gauge, mode):
    dims = RAGGED
    u = gi.gen_links(dims, 0.8, 82)
    with lat8(dims, gauge=gauge) as lat:
        lat.set_links(u)
        start = lat.get_links()
        lat.sweep(1, 1.7, mode)
        got = lat.get_links()
        th, F = lat.measure()
    ref = start.copy()
    if gauge == gf.GF_COULOMB:
        oracle.coulomb_sweep(ref, dims, 1, 1.7, mode)
    else:
        oracle.sweep(ref, dims, 1, 1.7, mode)
    err = np.abs(got - ref)
    say(f"min8 float32 sweep gauge={gauge} mode={mode}: max {err.max():.2e} rms {np.sqrt(np.mean(err ** 2)):.2e}")
    assert err.max() <= 5e-5 and np.sqrt(np.mean(err ** 2)) <= 1e-6
    if gauge == gf.GF_LANDAU:
        th_o, F_o = oracle.measure(got, dims)
        assert abs(th - th_o) <= 1e-12 * th_o and abs(F - F_o) <= 1e-14


@pytest.mark.parametrize("tps,block,nt", [(1, 64, 0), (2, 128, 1), (4, 256, 2), (8, 512, 0), (2, 64, 2)])
@pytest.mark.parametrize("prec", [gf.GF_FP32, gf.GF_MIXED])
def test_launch_shape_is_bitwise_irrelevant(prec, tps, block, nt):
    u = gi.gen_links(RAGGED, 0.8, 83)
    outs = []
    for cfg in [(4, 256, 0), (tps, block, nt)]:
        with lat8(RAGGED, prec) as lat:
            lat.set_sweep_config(*cfg, kernel=gf.GF_FP32)
            lat.set_links(u)
            lat.sweep(3, 1.7)
            if prec == gf.GF_MIXED:
                lat.promote_fp64()  # the float64 links g U0 g^dag: g(x) tracked bitwise too
            outs.append(lat.get_links())
    assert np.array_equal(outs[0], outs[1])


def test_mixed_bulk_equals_fp32_and_promotion_stays_on_orbit():
    """A GF_MIXED lattice's 8-real float32 sweeps are those of a GF_FP32 one (bitwise); promotion
    rebuilds g U0 g^dag from the original float64 links: the input's plaquette to 1e-12, SU(3) to
    1e-13, within float32 accuracy of the float32 links."""
    u = gi.gen_links(RAGGED, 0.8, 84)
    P0 = oracle.plaquette(u, RAGGED)
    with lat8(RAGGED, gf.GF_FP32) as a:
        a.set_links(u)
        a.sweep(30, 1.7)
        la = a.get_links()
    with lat8(RAGGED, gf.GF_MIXED) as b:
        b.set_links(u)
        b.sweep(30, 1.7)
        lb = b.get_links()
        b.promote_fp64()
        l64 = b.get_links()
        P64 = b.plaquette()
    assert np.array_equal(la, lb)
    assert abs(P64 - P0) < 1e-12
    du, dd = oracle.unitarity(l64.copy())
    assert du < 1e-13 and dd < 1e-13
    assert np.abs(l64 - lb).max() < 1e-4


@pytest.mark.parametrize("gauge", [gf.GF_LANDAU, gf.GF_COULOMB])
def test_mixed_fix_until_ends_in_float64(gauge):
    """8^4, eps = 0.6, seed 0, the library's switch point: float32 sweeps in 8 reals, then the
    float64 polish; the oracle's theta of the downloaded links is below 1e-12, the plaquette is
    the input's, F is the oracle's within the Gribov-copy slack of the 12-real mixed test, and the
    sweep count is within 10 % of the float64 run's."""
    dims = CFG8
    u = gi.gen_links(dims, 0.6, 0)
    P0 = oracle.plaquette(u, dims)
    kw = dict(omega=1.7, mode=0, theta_target=1e-12, max_sweeps=3000, check_every=10, reunit_every=100)
    with gf.Lattice(dims, gf.GF_FP64, gauge=gauge) as lat:
        lat.set_links(u)
        r64 = lat.fix_until(theta_switch=0.0, **kw)
    with lat8(dims, gf.GF_MIXED, gauge=gauge) as lat:
        lat.set_links(u)
        floor, sw = lat.tune_switch(1e-12)
        r = lat.fix_until(theta_switch=-1.0, **kw)
        P = lat.plaquette()
        links = lat.get_links()
    if gauge == gf.GF_LANDAU:
        th_o, F_o = oracle.measure(links, dims)
    else:
        tht, Ft = oracle.coulomb_measure(links, dims)
        th_o, F_o = float(tht.max()), float(Ft.mean())
    say(f"min8 float32 mixed gauge={gauge}: floor {floor:.2e} switch {sw:.2e}; sweeps {r.sweeps} "
        f"({r.sweeps_fp32}/{r.sweeps_fp64}) vs float64 {r64.sweeps}; theta {r.theta:.3e} (oracle {th_o:.3e})")
    assert r.converged and r64.converged
    assert r.sweeps_fp32 > 0 and r.sweeps_fp64 > 0 and r.sweeps_fp32 + r.sweeps_fp64 == r.sweeps
    assert th_o < 1e-12 and abs(th_o - r.theta) <= 1e-8 * r.theta
    assert abs(F_o - r.F) < 1e-13 and abs(r.F - r64.F) < 1e-3
    assert abs(P - P0) < 1e-12
    assert abs(r.sweeps - r64.sweeps) <= 0.1 * r64.sweeps


def test_fp32_floor_of_the_8_real_storage():
    """gf_tune_switch on an 8-real GF_MIXED lattice gives the floor of links rounded through the
    8-real float32 storage: a few float32 units squared (u = 2^-24: between 1 and 60 u^2),
    unchanged within 20 % by a Haar gauge rotation, and the switch point max(target, 100 x floor)."""
    u2 = 2.0 ** -48
    for dims, eps, seed in ((CFG8, 0.6, 0), (RAGGED, 1.0, 4)):
        u = gi.gen_links(dims, eps, seed)
        h = gi.to_canonical(gi.haar_su3(np.random.default_rng(9), gi.volume(dims)))
        rot = oracle.gauge_transform(u.copy(), dims, h)
        floors = []
        for links in (u, rot):
            with lat8(dims, gf.GF_MIXED) as lat:
                lat.set_links(links)
                f8, sw = lat.tune_switch(1e-12)
            assert sw == max(1e-12, 100.0 * f8)
            floors.append(f8)
        with gf.Lattice(dims, gf.GF_MIXED) as lat:
            lat.set_links(u)
            f12, _ = lat.tune_switch(1e-12)
        say(f"  floor {dims} eps {eps}: 8 reals {floors[0] / u2:.2f} u^2 (rotated {floors[1] / u2:.2f}), "
            f"12 reals {f12 / u2:.2f} u^2")
        assert 1.0 * u2 < floors[0] < 60.0 * u2
        assert abs(floors[1] / floors[0] - 1.0) < 0.2


@pytest.mark.parametrize("prec", [gf.GF_FP32, gf.GF_MIXED])
def test_anneal_keeps_the_orbit(prec):
    """Heat-bath sweeps on 8-real float32 links: links SU(3) (float64 decode), the plaquette of the
    float32 links within float32 accuracy of the input's; GF_MIXED tracks g(x), so the promoted
    float64 links g U0 g^dag hold it to 1e-12."""
    dims = RAGGED
    u = gi.gen_links(dims, 0.6, 85)
    P0 = oracle.plaquette(u, dims)
    with lat8(dims, prec) as lat:
        lat.set_links(u)
        F0 = lat.measure()[1]
        lat.anneal(20, 1.25, 0.5, 47)
        P32 = lat.plaquette()
        F1 = lat.measure()[1]
        links = lat.get_links()
        if prec == gf.GF_MIXED:
            lat.promote_fp64()
            P64 = lat.plaquette()
    du, dd = oracle.unitarity(links.copy())
    say(f"min8 float32 anneal prec={prec}: F {F0:.6f} -> {F1:.6f}; plaquette drift {abs(P32 - P0):.2e}")
    assert du <= 4e-15 and dd <= 4e-15  # entries of the float64 decode within ~2 units each
    assert abs(P32 - P0) < 1e-5
    assert F1 != F0
    if prec == gf.GF_MIXED:
        assert abs(P64 - P0) < 1e-12


def test_estimate_and_adaptive_checks():
    """The estimating sweep sums tr[Delta Delta^dag] of the float32 K before each update: within
    float32 rounding of the oracle's sum over the downloaded links; adaptive checks give bitwise the
    fix-until result of exact checks with fewer exact measurements."""
    dims = CFG8
    u = gi.gen_links(dims, 0.7, 86)
    black = ln.colours(dims) == 0
    with lat8(dims) as lat:
        lat.set_links(u)
        start = lat.get_links()
        est = lat.sweep_estimate(1.7)
    ref = start.copy()
    s_b = oracle.theta_density(ref, dims)[black].sum()
    oracle.half_sweep(ref, dims, 0, 1.7)
    s_w = oracle.theta_density(ref, dims)[~black].sum()
    expect = (s_b + s_w) / (3.0 * u.shape[0])
    assert abs(est - expect) <= 1e-3 * expect
    u = gi.gen_links(dims, 0.6, 0)
    res = []
    for adaptive in (False, True):
        with lat8(dims, gf.GF_MIXED) as lat:
            lat.set_links(u)
            lat.set_check_policy(adaptive)
            res.append((lat.fix_until(omega=1.7, theta_target=1e-12, max_sweeps=3000, check_every=10,
                                      theta_switch=-1.0), lat.get_links(), lat.counters))
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])
    assert res[1][2][0] < res[0][2][0]


def test_set_storage_converts_both_ways_and_autotune(tmp_path):
    """GF_FP32: 12 -> 8 reals holds the float64 8-real store of the links to float32 rounding,
    8 -> 12 the decoded rows rounded to float32; a GF_MIXED lattice converts its float32 links only;
    the tuner times 8-real float32 sweeps under their own cache key and gf_autotune_storage keeps
    the faster storage."""
    import torch

    dims = RAGGED
    u = gi.gen_links(dims, 0.7, 87)
    stream = torch.cuda.Stream()
    with gf.Lattice(dims, gf.GF_FP32, stream=stream) as lat:
        lat.set_links(u)
        lat.sweep(2, 1.7)  # a graph over the 12-real field
        before = lat.get_links()
        lat.storage = 8
        assert lat.storage == 8
        got8 = lat.get_links()
        assert float(np.abs(got8 - oracle.min8_store(before.copy())).max()) <= 1e-6
        lat.sweep(2, 1.7)  # a new graph over the 8-real field
        after8 = lat.get_links()
        lat.storage = 12
        got12 = lat.get_links()
        assert float(np.abs(got12 - after8).max()) <= 1e-6
        lat.reunitarize()
    with gf.Lattice(dims, gf.GF_MIXED) as lat:
        lat.set_links(u)
        b12 = gf.gf_lattice_info(lat.handle)[1]
        lat.storage = 8
        assert gf.gf_lattice_info(lat.handle)[1] < b12
        lat.sweep(3, 1.7)
        lat.promote_fp64()
        P = lat.plaquette()
        assert abs(P - oracle.plaquette(u, dims)) < 1e-12
        cache = str(tmp_path / "tune.txt")
        lat.storage = 12
        lat.storage = 8
        (tps, block, nt, minw), table = lat.autotune(gf.GF_FP32, n_sweeps=2, cache_path=cache)
        assert len(table) == 15 + 9 + 9 and minw == 0
        with pytest.raises(gf.GFError) as e:
            lat.set_sweep_config(1, 128, 0, min_waves=2, kernel=gf.GF_FP32)
        assert e.value.status == gf.GF_E_ARG
    assert "fp32g" in open(cache).read() and "-min8" in open(cache).read()
    with gf.Lattice((16, 16, 16, 16), gf.GF_MIXED) as lat:
        lat.set_links(gi.gen_links((16, 16, 16, 16), 0.8, 88))
        reals, us12, us8 = lat.autotune_storage(2)
        say(f"float32 storage autotune: chose {reals}; 12 reals {us12:.1f} us, 8 reals {us8:.1f} us")
        assert lat.storage == reals == (8 if us8 < us12 else 12) and us12 > 0 and us8 > 0


def test_flags_add_no_drift():
    """The pivot and q flags ride in the lowest bits of three float32 values; setting them must not
    bias those values (clearing or setting the bit shrinks or grows them by half a unit on average
    at every store, which 1500 sweeps compound into a plaquette drift of the float32 links of
    ~1e-5 on this input).  Unbiased flags leave the drift at the level of plain float32 rounding:
    below 3e-6 here, where the 12-real float32 links drift 4.5e-7."""
    dims = (16, 16, 16, 16)
    u = gi.gen_links(dims, 0.8, 0)
    P0 = oracle.plaquette(u, dims)
    drift = {}
    for storage in (12, 8):
        with gf.Lattice(dims, gf.GF_MIXED, storage=storage) as lat:
            lat.set_links(u)
            lat.sweep(1500, 1.7)
            lat.reunitarize()
            drift[storage] = lat.plaquette() - P0
    say(f"float32 plaquette drift after 1500 sweeps: 12 reals {drift[12]:+.2e}, 8 reals {drift[8]:+.2e}")
    assert abs(drift[8]) < 3e-6
