"""The C-ABI library loads and exports every entry point include/gf.h declares.

CPU only: no device work is started; the calls below fail argument checks
before any HIP call.
"""

import os
import re
import subprocess

import pytest

from paper_1412_3655_amd import gf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gf_status|const char\*|double)\s+(gf_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gf_create_lattice", "gf_sweep_or", "gf_anneal", "gf_measure_theta_F", "gf_fix_until",
                     "gf_reunitarize"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(gf.LIB_PATH), "libgf.so must be built (__graft_entry__.build())"
    out = subprocess.run(["nm", "-D", "--defined-only", gf.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s+(gf_\w+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = gf.lib()
    for n in declared_functions():
        assert hasattr(L, n)


def test_binding_covers_declared_symbols():
    assert sorted(gf.exported_symbols()) == declared_functions()


def test_version_and_argument_checks_without_device():
    assert "gfx950" in gf.gf_version()
    for dims in [(4, 4, 3, 4), (0, 4, 4, 4), (4, 4, 4, 1), (4, -2, 4, 4)]:
        with pytest.raises(gf.GFError) as e:
            gf.gf_create_lattice(dims)
        assert e.value.status == gf.GF_E_ARG
    with pytest.raises(gf.GFError) as e:
        gf.gf_create_lattice((4, 4, 4, 4), prec=7)
    assert e.value.status == gf.GF_E_ARG
    with pytest.raises(gf.GFError) as e:
        gf.gf_create_lattice((65536, 65536, 2, 2))
    assert e.value.status == gf.GF_E_ARG
    for name in ("gf_sweep_or", "gf_measure_theta_F", "gf_reunitarize", "gf_plaquette", "gf_get_links"):
        fn = getattr(gf.lib(), name)
        args = {"gf_sweep_or": (None, 1, 1.5, 0), "gf_measure_theta_F": (None, None, None),
                "gf_reunitarize": (None,), "gf_plaquette": (None, None), "gf_get_links": (None, None)}[name]
        assert fn(*args) == gf.GF_E_ARG
    assert "null" in gf.gf_last_error()
    assert gf.lib().gf_destroy_lattice(None) == gf.GF_OK


def test_bench_rejects_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and a message, before any
    device work."""
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_bench_cpu_baseline_fields():
    """bench.py's cpu_baseline: the oracle on all host threads and on one core, with the thread count
    restored afterwards (a 4^4 lattice, a fraction of a second each)."""
    import sys

    import numpy as np

    import gauge_inputs as gi
    import oracle

    sys.path.insert(0, ROOT)
    import bench

    dims = (4, 4, 4, 4)
    u = gi.gen_links(dims, 0.6, 3)
    before = oracle.num_threads()
    cb = bench.cpu_baseline(u, dims, 1.7, 0, 0.05, 0.05)
    assert oracle.num_threads() == before
    assert cb["kind"] == "oracle" and cb["unit"] == "site-updates/s" and cb["cores"] == before
    assert cb["value"] > 0 and cb["one_core"]["cores"] == 1 and cb["one_core"]["value"] > 0
    assert "4x4x4x4" in cb["sample"]
    # the timing copies the input: the caller's links are untouched
    assert np.array_equal(u, gi.gen_links(dims, 0.6, 3))


def test_pool_job_bytes_by_storage():
    """gf_pool_job_bytes is host arithmetic: a GF_MIXED job whose float32 links take 8 reals holds
    one float4 chunk less per link than with 12 (2 colours x 4 directions x ld sites x 16 B, ld the
    half volume padded to whole 64-site tiles); a GF_FP64 job has no float32 links to store in 8."""
    for dims in [(4, 4, 4, 4), (6, 10, 6, 6), (16, 16, 16, 32)]:
        V = 1
        for d in dims:
            V *= d
        ld = -(-(V // 2) // 64) * 64
        b12 = gf.gf_pool_job_bytes(dims, gf.GF_MIXED)
        assert gf.gf_pool_job_bytes(dims, gf.GF_MIXED, 0) == b12
        assert b12 - gf.gf_pool_job_bytes(dims, gf.GF_MIXED, 8) == 2 * 4 * ld * 16
    for prec, reals in ((gf.GF_FP64, 8), (gf.GF_MIXED, 10)):
        with pytest.raises(gf.GFError) as e:
            gf.gf_pool_job_bytes((4, 4, 4, 4), prec, reals)
        assert e.value.status == gf.GF_E_ARG
