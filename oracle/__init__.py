"""FP64 CPU oracle for SU(3) Landau gauge fixing by checkerboard overrelaxation.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_1412_3655_amd``) never imports, links or calls it, and the
two share no code: the oracle is plain C99 (``gf_oracle.c``), built with gcc,
FP contraction off, no fast-math.

Links are canonical float64 arrays ``(V, 4, 3, 3, 2)`` (see ``gauge_inputs``).
Every function that changes links works in place on a C-contiguous float64
array and returns it.  Citations (H. Vogt, M. Schroeck, arXiv:1412.3655) are in
the C source next to each function.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

__all__ = [
    "OR_EXACT",
    "OR_BINOMIAL1",
    "build",
    "lib",
    "num_threads",
    "set_num_threads",
    "su2_project",
    "su2_maximiser",
    "su2_overrelax",
    "site_update",
    "half_sweep",
    "update_sites_in_order",
    "sweep",
    "measure",
    "theta_density",
    "plaquette",
    "unitarity",
    "reunitarize",
    "gauge_transform",
    "fix_until",
    "philox4x32_10",
    "anneal",
    "hb_sample_r0",
    "hb_sample_su2",
    "hb_subgroup_draws",
    "coulomb_half_sweep",
    "coulomb_sweep",
    "coulomb_update_sites_in_order",
    "coulomb_measure",
    "coulomb_fix_until",
    "coulomb_anneal",
    "su2lat_site_update",
    "su2lat_half_sweep",
    "su2lat_sweep",
    "su2lat_update_sites_in_order",
    "su2lat_theta_density",
    "su2lat_measure",
    "su2lat_coulomb_measure",
    "su2lat_plaquette",
    "su2lat_unitarity",
    "su2lat_reunitarize",
    "su2lat_fix_until",
    "su2lat_anneal",
    "min8_encode",
    "min8_decode",
    "min8_store",
]

OR_EXACT = 0
OR_BINOMIAL1 = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_CFLAGS = ["-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile gf_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def _declare(L):
    L.oracle_su2_project.argtypes = [_dp, _dp]
    L.oracle_su2_maximiser.argtypes = [_dp, _dp]
    L.oracle_su2_maximiser.restype = ctypes.c_int
    L.oracle_su2_overrelax.argtypes = [_dp, ctypes.c_double, ctypes.c_int, _dp]
    L.oracle_site_update.argtypes = [_dp, _ip, ctypes.c_int64, ctypes.c_double, ctypes.c_int]
    L.oracle_site_update.restype = ctypes.c_double
    L.oracle_half_sweep.argtypes = [_dp, _ip, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    L.oracle_update_sites_in_order.argtypes = [_dp, _ip, _i64p, ctypes.c_int64, ctypes.c_double, ctypes.c_int]
    L.oracle_sweep.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double, ctypes.c_int]
    L.oracle_theta_density.argtypes = [_dp, _ip, _dp]
    L.oracle_measure.argtypes = [_dp, _ip, _dp, _dp]
    L.oracle_plaquette.argtypes = [_dp, _ip]
    L.oracle_plaquette.restype = ctypes.c_double
    L.oracle_unitarity.argtypes = [_dp, ctypes.c_int64, _dp, _dp]
    L.oracle_reunitarize.argtypes = [_dp, ctypes.c_int64]
    L.oracle_gauge_transform.argtypes = [_dp, _ip, _dp]
    L.oracle_fix_until.argtypes = [_dp, _ip, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, _ip, _dp, _dp, _dp, _ip]
    L.oracle_fix_until.restype = ctypes.c_int
    L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.oracle_anneal.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                ctypes.c_int32]
    L.oracle_anneal.restype = ctypes.c_int64
    L.oracle_hb_sample_r0.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, _dp]
    L.oracle_hb_sample_r0.restype = ctypes.c_int64
    L.oracle_hb_sample_su2.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, _dp]
    L.oracle_hb_sample_su2.restype = ctypes.c_int64
    L.oracle_coulomb_half_sweep.argtypes = [_dp, _ip, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    L.oracle_coulomb_sweep.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double, ctypes.c_int]
    L.oracle_coulomb_update_sites_in_order.argtypes = [_dp, _ip, _i64p, ctypes.c_int64, ctypes.c_double,
                                                       ctypes.c_int]
    L.oracle_coulomb_measure.argtypes = [_dp, _ip, _dp, _dp]
    L.oracle_coulomb_fix_until.argtypes = [_dp, _ip, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _ip, _dp, _dp]
    L.oracle_coulomb_fix_until.restype = ctypes.c_int
    L.oracle_coulomb_anneal.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_uint64, ctypes.c_int32]
    L.oracle_coulomb_anneal.restype = ctypes.c_int64
    L.oracle_su2lat_site_update.argtypes = [_dp, _ip, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    L.oracle_su2lat_site_update.restype = ctypes.c_double
    L.oracle_su2lat_half_sweep.argtypes = [_dp, _ip, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    L.oracle_su2lat_sweep.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    L.oracle_su2lat_update_sites_in_order.argtypes = [_dp, _ip, _i64p, ctypes.c_int64, ctypes.c_double,
                                                      ctypes.c_int, ctypes.c_int]
    L.oracle_su2lat_theta_density.argtypes = [_dp, _ip, ctypes.c_int, _dp]
    L.oracle_su2lat_measure.argtypes = [_dp, _ip, _dp, _dp]
    L.oracle_su2lat_coulomb_measure.argtypes = [_dp, _ip, _dp, _dp]
    L.oracle_su2lat_plaquette.argtypes = [_dp, _ip]
    L.oracle_su2lat_plaquette.restype = ctypes.c_double
    L.oracle_su2lat_unitarity.argtypes = [_dp, ctypes.c_int64, _dp, _dp]
    L.oracle_su2lat_reunitarize.argtypes = [_dp, ctypes.c_int64]
    L.oracle_su2lat_fix_until.argtypes = [_dp, _ip, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int, _ip, _dp, _dp]
    L.oracle_su2lat_fix_until.restype = ctypes.c_int
    L.oracle_su2lat_anneal.argtypes = [_dp, _ip, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                       ctypes.c_int32, ctypes.c_int]
    L.oracle_su2lat_anneal.restype = ctypes.c_int64
    L.oracle_hb_subgroup_draws.argtypes = [_dp, ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, _dp]
    L.oracle_hb_subgroup_draws.restype = ctypes.c_int64
    L.oracle_min8_encode.argtypes = [_dp, ctypes.c_int64, _dp]
    L.oracle_min8_decode.argtypes = [_dp, ctypes.c_int64, _dp]
    L.oracle_min8_store.argtypes = [_dp, ctypes.c_int64]
    L.oracle_num_threads.restype = ctypes.c_int
    L.oracle_set_num_threads.argtypes = [ctypes.c_int]


def _links(u: np.ndarray) -> np.ndarray:
    if not (isinstance(u, np.ndarray) and u.dtype == np.float64 and u.flags.c_contiguous):
        raise TypeError("links must be a C-contiguous float64 numpy array")
    if u.shape[-4:] != (4, 3, 3, 2):
        raise ValueError("links must have shape (V, 4, 3, 3, 2)")
    return u


def _dims(dims, u=None):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (4,) or np.any(d < 2) or np.any(d % 2):
        raise ValueError("extents must be four even integers >= 2")
    if u is not None and int(np.prod(d.astype(np.int64))) != u.shape[0]:
        raise ValueError("links do not match the extents")
    return d


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing control; results do not depend on it)."""
    lib().oracle_set_num_threads(int(n))


def _c2(m) -> np.ndarray:
    """2x2 complex -> 8 contiguous doubles."""
    m = np.ascontiguousarray(np.asarray(m, dtype=np.complex128).reshape(2, 2))
    return m.view(np.float64).reshape(8).copy()


def _to_c2(a: np.ndarray) -> np.ndarray:
    return a.view(np.complex128).reshape(2, 2).copy()


def su2_project(k) -> np.ndarray:
    a = _c2(k)
    out = np.empty(8)
    lib().oracle_su2_project(_p(a), _p(out))
    return _to_c2(out)


def su2_maximiser(k):
    """(g, ok): the SU(2) maximiser of Re tr[g k]; ok is False when det q = 0."""
    a = _c2(k)
    out = np.empty(8)
    ok = lib().oracle_su2_maximiser(_p(a), _p(out))
    return _to_c2(out), bool(ok)


def su2_overrelax(g, omega: float, mode: int = OR_EXACT) -> np.ndarray:
    a = _c2(g)
    out = np.empty(8)
    lib().oracle_su2_overrelax(_p(a), float(omega), int(mode), _p(out))
    return _to_c2(out)


def site_update(u, dims, site: int, omega: float, mode: int = OR_EXACT) -> float:
    """Overrelax one site in place; returns the change of Re tr K at that site."""
    u = _links(u)
    d = _dims(dims, u)
    return float(lib().oracle_site_update(_p(u), _p(d, _ip), int(site), float(omega), int(mode)))


def half_sweep(u, dims, colour: int, omega: float, mode: int = OR_EXACT):
    u = _links(u)
    d = _dims(dims, u)
    lib().oracle_half_sweep(_p(u), _p(d, _ip), int(colour), float(omega), int(mode))
    return u


def update_sites_in_order(u, dims, sites, omega: float, mode: int = OR_EXACT):
    u = _links(u)
    d = _dims(dims, u)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    lib().oracle_update_sites_in_order(_p(u), _p(d, _ip), _p(s, _i64p), s.size, float(omega), int(mode))
    return u


def sweep(u, dims, nsweeps: int, omega: float, mode: int = OR_EXACT):
    u = _links(u)
    d = _dims(dims, u)
    lib().oracle_sweep(_p(u), _p(d, _ip), int(nsweeps), float(omega), int(mode))
    return u


def measure(u, dims):
    """(theta, F)."""
    u = _links(u)
    d = _dims(dims, u)
    th = ctypes.c_double()
    f = ctypes.c_double()
    lib().oracle_measure(_p(u), _p(d, _ip), ctypes.byref(th), ctypes.byref(f))
    return th.value, f.value


def theta_density(u, dims) -> np.ndarray:
    """tr[Delta(x) Delta(x)^dag] for every site."""
    u = _links(u)
    d = _dims(dims, u)
    out = np.empty(u.shape[0])
    lib().oracle_theta_density(_p(u), _p(d, _ip), _p(out))
    return out


def plaquette(u, dims) -> float:
    u = _links(u)
    d = _dims(dims, u)
    return float(lib().oracle_plaquette(_p(u), _p(d, _ip)))


def unitarity(u):
    """(max ||U^dag U - 1||_F, max |det U - 1|) over all links."""
    a = np.ascontiguousarray(u, dtype=np.float64)
    n = a.size // 18
    mu = ctypes.c_double()
    md = ctypes.c_double()
    lib().oracle_unitarity(_p(a), n, ctypes.byref(mu), ctypes.byref(md))
    return mu.value, md.value


def reunitarize(u):
    if not (u.dtype == np.float64 and u.flags.c_contiguous) or u.size % 18:
        raise TypeError("need a C-contiguous float64 array of 3x3 complex matrices")
    lib().oracle_reunitarize(_p(u), u.size // 18)
    return u


def gauge_transform(u, dims, g):
    """U_mu(x) <- g(x) U_mu(x) g(x+mu^)^dag; g is (V, 3, 3, 2) float64."""
    u = _links(u)
    d = _dims(dims, u)
    ga = np.ascontiguousarray(g, dtype=np.float64)
    if ga.shape != (u.shape[0], 3, 3, 2):
        raise ValueError("gauge field must have shape (V, 3, 3, 2)")
    lib().oracle_gauge_transform(_p(u), _p(d, _ip), _p(ga))
    return u


def fix_until(u, dims, omega: float = 1.7, mode: int = OR_EXACT, theta_target: float = 1e-12,
              max_sweeps: int = 3000, check_every: int = 1, reunit_every: int = 100):
    """Returns dict(converged, sweeps, theta, F, theta_hist)."""
    u = _links(u)
    d = _dims(dims, u)
    ce = max(1, int(check_every))
    hist = np.empty(int(max_sweeps) // ce + 3)
    sw = ctypes.c_int32()
    th = ctypes.c_double()
    f = ctypes.c_double()
    nc = ctypes.c_int32()
    conv = lib().oracle_fix_until(_p(u), _p(d, _ip), float(omega), int(mode), float(theta_target),
                                  int(max_sweeps), ce, int(reunit_every), ctypes.byref(sw),
                                  ctypes.byref(th), ctypes.byref(f), _p(hist), ctypes.byref(nc))
    return dict(converged=bool(conv), sweeps=sw.value, theta=th.value, F=f.value,
                theta_hist=hist[: nc.value].copy())


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.empty(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def anneal(u, dims, nsweeps: int, T0: float, T1: float, seed: int, sweep_offset: int = 0) -> int:
    """Heat-bath sweeps in place; returns the count of rejection-capped subgroup updates."""
    u = _links(u)
    d = _dims(dims, u)
    return int(lib().oracle_anneal(_p(u), _p(d, _ip), int(nsweeps), float(T0), float(T1),
                                   int(seed) & 0xFFFFFFFFFFFFFFFF, int(sweep_offset)))


def hb_sample_r0(kappa: float, seed: int, n: int):
    out = np.empty(int(n))
    capped = lib().oracle_hb_sample_r0(float(kappa), int(seed), int(n), _p(out))
    return out, int(capped)


def hb_sample_su2(kappa: float, seed: int, n: int):
    """n heat-bath SU(2) draws as quaternions (r0, r1, r2, r3)."""
    out = np.empty((int(n), 4))
    capped = lib().oracle_hb_sample_su2(float(kappa), int(seed), int(n), _p(out))
    return out, int(capped)


def hb_subgroup_draws(k, T: float, seed: int, n: int):
    """n heat-bath subgroup elements (2x2 complex) drawn for the fixed 2x2 block k at
    temperature T, by the same code path as the annealing sweep."""
    kk = np.ascontiguousarray(np.asarray(k, dtype=np.complex128).reshape(2, 2))
    out = np.empty((int(n), 2, 2), dtype=np.complex128)
    capped = lib().oracle_hb_subgroup_draws(_p(kk.view(np.float64)), float(T), int(seed), int(n),
                                            _p(out.view(np.float64)))
    return out, int(capped)


# ------------------------------------------------------------- Coulomb gauge --


def coulomb_half_sweep(u, dims, colour: int, omega: float, mode: int = OR_EXACT):
    """Coulomb-gauge overrelaxation over the sites of one colour (in place)."""
    u = _links(u)
    d = _dims(dims, u)
    lib().oracle_coulomb_half_sweep(_p(u), _p(d, _ip), int(colour), float(omega), int(mode))
    return u


def coulomb_sweep(u, dims, nsweeps: int, omega: float, mode: int = OR_EXACT):
    u = _links(u)
    d = _dims(dims, u)
    lib().oracle_coulomb_sweep(_p(u), _p(d, _ip), int(nsweeps), float(omega), int(mode))
    return u


def coulomb_update_sites_in_order(u, dims, sites, omega: float, mode: int = OR_EXACT):
    u = _links(u)
    d = _dims(dims, u)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    lib().oracle_coulomb_update_sites_in_order(_p(u), _p(d, _ip), _p(s, _i64p), len(s), float(omega), int(mode))
    return u


def coulomb_measure(u, dims):
    """(theta_C(t), F_C(t)) per timeslice t, as two arrays of Nt."""
    u = _links(u)
    d = _dims(dims, u)
    th = np.empty(int(d[3]))
    fr = np.empty(int(d[3]))
    lib().oracle_coulomb_measure(_p(u), _p(d, _ip), _p(th), _p(fr))
    return th, fr


def coulomb_fix_until(u, dims, omega: float = 1.7, mode: int = OR_EXACT, theta_target: float = 1e-12,
                      max_sweeps: int = 3000, check_every: int = 10, reunit_every: int = 100) -> dict:
    """Coulomb fix-until in place: theta = max over timeslices, F = mean over timeslices."""
    u = _links(u)
    d = _dims(dims, u)
    sw = ctypes.c_int32()
    th = ctypes.c_double()
    f = ctypes.c_double()
    conv = lib().oracle_coulomb_fix_until(_p(u), _p(d, _ip), float(omega), int(mode), float(theta_target),
                                          int(max_sweeps), int(check_every), int(reunit_every),
                                          ctypes.byref(sw), ctypes.byref(th), ctypes.byref(f))
    return dict(converged=bool(conv), sweeps=sw.value, theta=th.value, F=f.value)



def coulomb_anneal(u, dims, nsweeps: int, T0: float, T1: float, seed: int, sweep_offset: int = 0) -> int:
    """Heat-bath sweeps of the Coulomb functional in place (K over x, y, z); returns the
    count of rejection-capped subgroup updates."""
    u = _links(u)
    d = _dims(dims, u)
    return int(lib().oracle_coulomb_anneal(_p(u), _p(d, _ip), int(nsweeps), float(T0), float(T1),
                                           int(seed) & 0xFFFFFFFFFFFFFFFF, int(sweep_offset)))


# --------------------------------------------------------- SU(2) gauge group --
# Links are canonical float64 arrays (V, 4, 2, 2, 2); ndir = 4 (Landau) or 3 (Coulomb).


def _links2(u: np.ndarray) -> np.ndarray:
    if not (isinstance(u, np.ndarray) and u.dtype == np.float64 and u.flags.c_contiguous):
        raise TypeError("links must be a C-contiguous float64 numpy array")
    if u.shape[-4:] != (4, 2, 2, 2):
        raise ValueError("SU(2) links must have shape (V, 4, 2, 2, 2)")
    return u


def su2lat_site_update(u, dims, site: int, omega: float, mode: int = OR_EXACT, ndir: int = 4) -> float:
    """Overrelax one site in place; returns the change of Re tr K at that site."""
    u = _links2(u)
    d = _dims(dims, u)
    return float(lib().oracle_su2lat_site_update(_p(u), _p(d, _ip), int(site), float(omega), int(mode), int(ndir)))


def su2lat_half_sweep(u, dims, colour: int, omega: float, mode: int = OR_EXACT, ndir: int = 4):
    u = _links2(u)
    d = _dims(dims, u)
    lib().oracle_su2lat_half_sweep(_p(u), _p(d, _ip), int(colour), float(omega), int(mode), int(ndir))
    return u


def su2lat_sweep(u, dims, nsweeps: int, omega: float, mode: int = OR_EXACT, ndir: int = 4):
    u = _links2(u)
    d = _dims(dims, u)
    lib().oracle_su2lat_sweep(_p(u), _p(d, _ip), int(nsweeps), float(omega), int(mode), int(ndir))
    return u


def su2lat_update_sites_in_order(u, dims, sites, omega: float, mode: int = OR_EXACT, ndir: int = 4):
    u = _links2(u)
    d = _dims(dims, u)
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    lib().oracle_su2lat_update_sites_in_order(_p(u), _p(d, _ip), _p(s, _i64p), s.size, float(omega), int(mode),
                                              int(ndir))
    return u


def su2lat_theta_density(u, dims, ndir: int = 4) -> np.ndarray:
    u = _links2(u)
    d = _dims(dims, u)
    out = np.empty(u.shape[0])
    lib().oracle_su2lat_theta_density(_p(u), _p(d, _ip), int(ndir), _p(out))
    return out


def su2lat_measure(u, dims):
    """(theta, F) of Landau gauge, N_c = 2."""
    u = _links2(u)
    d = _dims(dims, u)
    th = ctypes.c_double()
    f = ctypes.c_double()
    lib().oracle_su2lat_measure(_p(u), _p(d, _ip), ctypes.byref(th), ctypes.byref(f))
    return th.value, f.value


def su2lat_coulomb_measure(u, dims):
    """(theta_C(t), F_C(t)) per timeslice, N_c = 2."""
    u = _links2(u)
    d = _dims(dims, u)
    th = np.empty(int(d[3]))
    fr = np.empty(int(d[3]))
    lib().oracle_su2lat_coulomb_measure(_p(u), _p(d, _ip), _p(th), _p(fr))
    return th, fr


def su2lat_plaquette(u, dims) -> float:
    u = _links2(u)
    d = _dims(dims, u)
    return float(lib().oracle_su2lat_plaquette(_p(u), _p(d, _ip)))


def su2lat_unitarity(u):
    a = np.ascontiguousarray(u, dtype=np.float64)
    mu = ctypes.c_double()
    md = ctypes.c_double()
    lib().oracle_su2lat_unitarity(_p(a), a.size // 8, ctypes.byref(mu), ctypes.byref(md))
    return mu.value, md.value


def su2lat_reunitarize(u):
    if not (u.dtype == np.float64 and u.flags.c_contiguous) or u.size % 8:
        raise TypeError("need a C-contiguous float64 array of 2x2 complex matrices")
    lib().oracle_su2lat_reunitarize(_p(u), u.size // 8)
    return u


def su2lat_fix_until(u, dims, omega: float = 1.7, mode: int = OR_EXACT, theta_target: float = 1e-12,
                     max_sweeps: int = 3000, check_every: int = 10, reunit_every: int = 100, ndir: int = 4) -> dict:
    u = _links2(u)
    d = _dims(dims, u)
    sw = ctypes.c_int32()
    th = ctypes.c_double()
    f = ctypes.c_double()
    conv = lib().oracle_su2lat_fix_until(_p(u), _p(d, _ip), float(omega), int(mode), float(theta_target),
                                         int(max_sweeps), int(check_every), int(reunit_every), int(ndir),
                                         ctypes.byref(sw), ctypes.byref(th), ctypes.byref(f))
    return dict(converged=bool(conv), sweeps=sw.value, theta=th.value, F=f.value)


def su2lat_anneal(u, dims, nsweeps: int, T0: float, T1: float, seed: int, sweep_offset: int = 0,
                  ndir: int = 4) -> int:
    u = _links2(u)
    d = _dims(dims, u)
    return int(lib().oracle_su2lat_anneal(_p(u), _p(d, _ip), int(nsweeps), float(T0), float(T1),
                                          int(seed) & 0xFFFFFFFFFFFFFFFF, int(sweep_offset), int(ndir)))


def _mats(u: np.ndarray) -> np.ndarray:
    if not (isinstance(u, np.ndarray) and u.dtype == np.float64 and u.flags.c_contiguous):
        raise TypeError("links must be a C-contiguous float64 numpy array")
    if u.shape[-3:] != (3, 3, 2):
        raise ValueError(f"links must end in (3, 3, 2), got {u.shape}")
    return u


def min8_encode(u) -> np.ndarray:
    """8 reals per SU(3) link (the row-pivoted minimal representation; see
    gf_oracle.c): shape (..., 3, 3, 2) -> (..., 8)."""
    u = _mats(u)
    out = np.empty(u.shape[:-3] + (8,), dtype=np.float64)
    lib().oracle_min8_encode(_p(u), u.size // 18, _p(out))
    return out


def min8_decode(p) -> np.ndarray:
    """The SU(3) links of 8-real parameters: shape (..., 8) -> (..., 3, 3, 2)."""
    if not (isinstance(p, np.ndarray) and p.dtype == np.float64 and p.flags.c_contiguous and p.shape[-1] == 8):
        raise TypeError("parameters must be a C-contiguous float64 array ending in 8")
    out = np.empty(p.shape[:-1] + (3, 3, 2), dtype=np.float64)
    lib().oracle_min8_decode(_p(p), p.size // 8, _p(out))
    return out


def min8_store(u):
    """In place: the links a lattice stored in 8 reals per link holds after u was written to it."""
    u = _mats(u)
    lib().oracle_min8_store(_p(u), u.size // 18)
    return u
