"""Full-size checks at the workloads' real shapes, in the launch configuration the
benchmark uses (tuned: 2 lanes per site, 128-thread blocks, non-temporal accesses
for float64; 2 lanes, 64-thread blocks for float32).

48^3 x 96 (10,616,832 sites, eps = 1.0, seed 0): one float64 sweep and two
heat-bath sweeps compared with the FP64 oracle link by link (1e-12), theta/F
of the input, one float64 sweep with links in 12 and in 8 reals in the
autotuner's launch configuration against the oracle, then the mixed-precision pipeline of that workload (2000 float32
heat-bath sweeps T 1.25 -> 0.01 tracking g, overrelaxation with float32 bulk
and float64 polish, reunitarisation every 100 sweeps) checked through what
holds at any size: gauge invariance of the plaquette (1e-12 after the float64
rebuild), SU(3) membership, theta/F recomputed by the oracle from the
downloaded links, and F not lower than after the anneal.
"""

import sys

import numpy as np
import pytest

import gauge_inputs as gi
import oracle
from paper_1412_3655_amd import gf

pytestmark = pytest.mark.gpu

BIG = (48, 48, 48, 96)
CFG64 = (2, 128, 1)
CFG32 = (2, 64, 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big_links():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    oracle.lib()
    gf.lib()
    say("48^3x96: generating eps=1.0 seed 0")
    return gi.gen_links(BIG, 1.0, 0)


@pytest.mark.timeout(900)
def test_48x96_fp64_sweep_and_heat_bath_parity(big_links):
    u = big_links
    say("48^3x96: oracle theta/F")
    th_o, F_o = oracle.measure(u, BIG)
    say("48^3x96: oracle sweep")
    ref = u.copy()
    oracle.sweep(ref, BIG, 1, 1.7, oracle.OR_EXACT)
    say("48^3x96: gpu sweep")
    with gf.Lattice(BIG) as lat:
        lat.set_sweep_config(*CFG64)
        lat.set_links(u)
        th, F = lat.measure()
        lat.sweep(1, 1.7, gf.GF_OR_EXACT)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"  theta {th:.6e} (oracle {th_o:.6e}), F {F:.15f} (oracle {F_o:.15f}), max|diff| after 1 sweep {d:.2e}")
    assert abs(th - th_o) <= 1e-12 * th_o
    assert abs(F - F_o) <= 1e-14
    assert d <= 1e-12
    del got, ref
    say("48^3x96: heat bath, 2 sweeps")
    ref = u.copy()
    capped = oracle.anneal(ref, BIG, 2, 1.25, 0.8, 99)
    with gf.Lattice(BIG) as lat:
        lat.set_sweep_config(*CFG64)
        lat.set_links(u)
        lat.anneal(2, 1.25, 0.8, 99)
        got = lat.get_links()
    d = float(np.abs(got - ref).max())
    say(f"  heat bath max|diff| {d:.2e}, oracle capped {capped}")
    assert capped == 0
    assert d <= 1e-12


@pytest.mark.timeout(900)
def test_48x96_autotuned_fp64_sweep_parity(big_links):
    """One float64 sweep with links in 12 and in 8 reals, each in the launch configuration the
    autotuner picks on this GPU (what the benchmark times), against the oracle link by link.  As
    in the 8-real parity tests, the oracle sweeps the links the 8-real representation holds
    (oracle.min8_store of the input): on this rough input some sites have nearly degenerate
    subgroup blocks, where the sweep magnifies a rounding-level change of its input links."""
    for storage in (12, 8):
        u = big_links if storage == 12 else oracle.min8_store(big_links.copy())
        say(f"48^3x96 autotuned, {storage} reals: oracle sweep")
        ref = u.copy()
        oracle.sweep(ref, BIG, 1, 1.7, oracle.OR_EXACT)
        with gf.Lattice(BIG, storage=storage) as lat:
            lat.set_links(u)
            chosen, _ = lat.autotune(gf.GF_FP64, n_sweeps=3)
            lat.sweep(1, 1.7, gf.GF_OR_EXACT)
            got = lat.get_links()
        d = float(np.abs(got - ref).max())
        say(f"  {storage} reals, tuned {chosen}: max|diff| after 1 sweep {d:.2e}")
        assert d <= 1e-12
        del got, ref, u


@pytest.mark.timeout(900)
def test_48x96_mixed_pipeline_invariants(big_links):
    u = big_links
    P0 = oracle.plaquette(u, BIG)
    say("48^3x96: mixed pipeline (anneal 2000 float32 sweeps, then OR)")
    with gf.Lattice(BIG, gf.GF_MIXED) as lat:
        lat.set_sweep_config(*CFG32, kernel=gf.GF_FP32)
        lat.set_sweep_config(*CFG64, kernel=gf.GF_FP64)
        lat.set_links(u)
        lat.anneal(2000, 1.25, 0.01, 0)
        th_a, F_a = lat.measure()
        r = lat.fix_until(omega=1.7, mode=0, theta_target=1e-13, max_sweeps=3000, check_every=10,
                          reunit_every=100, theta_switch=1e-9)
        lat.promote_fp64()  # no-op if the iteration already switched to float64
        P = lat.plaquette()
        th_g, F_g = lat.measure()
        links = lat.get_links()
    say(f"  after anneal theta {th_a:.3e} F {F_a:.6f}; after OR sweeps {r.sweeps} ({r.sweeps_fp32}/{r.sweeps_fp64}) "
        f"theta {th_g:.3e} F {F_g:.9f} converged {r.converged}; |dP| {abs(P - P0):.2e}")
    assert abs(P - P0) < 1e-12
    assert F_g >= F_a - 1e-6
    # this eps = 1.0 input is one of the rough ones that do not reach 1e-13 within the cap (the
    # design notes' input section); the iteration must still have reduced theta by 3 decades
    assert th_g < 1e-3 * th_a
    du, dd = oracle.unitarity(links)
    assert du < 1e-12 and dd < 1e-12
    th_o, F_o = oracle.measure(links, BIG)
    assert abs(th_o - th_g) <= 1e-6 * th_g + 1e-20
    assert abs(F_o - F_g) < 1e-13
