"""ctypes binding of libgf (C ABI in include/gf.h).

Argument marshalling only: every step of the gauge-fixing path runs in the
HIP kernels of libgf.so.  PyTorch is used for device memory (canonical link
arrays on the GPU) and streams.  If the library is not built, loading fails
loudly; there is no fallback of any kind.

Function names match the C entry points.  Host link arrays are canonical
float64 ``(V, 4, 3, 3, 2)`` numpy arrays; device ones are float64 torch
tensors of the same shape on a HIP device.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf.so")

GF_OK, GF_E_ARG, GF_E_NOMEM, GF_E_HIP, GF_E_STATE, GF_E_NUMERIC, GF_E_FULL, GF_E_CANCELLED = range(8)
GF_FP64, GF_FP32, GF_MIXED = 0, 1, 2
GF_OR_EXACT, GF_OR_BINOMIAL1 = 0, 1
GF_LANDAU, GF_COULOMB = 0, 1

_STATUS_NAMES = {
    GF_OK: "GF_OK",
    GF_E_ARG: "GF_E_ARG",
    GF_E_NOMEM: "GF_E_NOMEM",
    GF_E_HIP: "GF_E_HIP",
    GF_E_STATE: "GF_E_STATE",
    GF_E_NUMERIC: "GF_E_NUMERIC",
    GF_E_FULL: "GF_E_FULL",
    GF_E_CANCELLED: "GF_E_CANCELLED",
}


class GFError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class gf_fix_params(ctypes.Structure):
    _fields_ = [
        ("omega", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("theta_target", ctypes.c_double),
        ("max_sweeps", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("reunit_every", ctypes.c_int32),
        ("theta_switch", ctypes.c_double),
    ]


class gf_fix_result(ctypes.Structure):
    _fields_ = [
        ("converged", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("sweeps_fp32", ctypes.c_int32),
        ("sweeps_fp64", ctypes.c_int32),
        ("theta", ctypes.c_double),
        ("F", ctypes.c_double),
    ]


class gf_tune_entry(ctypes.Structure):
    _fields_ = [("tps", ctypes.c_int32), ("block", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("min_waves", ctypes.c_int32), ("us_per_sweep", ctypes.c_double)]


class gf_pool_config(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("max_slots", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("tps32", ctypes.c_int32),
        ("block32", ctypes.c_int32),
        ("tps64", ctypes.c_int32),
        ("block64", ctypes.c_int32),
        ("reals32", ctypes.c_int32),
        ("cache32", ctypes.c_int32),
        ("cache64", ctypes.c_int32),
    ]


class gf_pool_done(ctypes.Structure):
    _fields_ = [
        ("job_id", ctypes.c_uint64),
        ("result", gf_fix_result),
        ("status", ctypes.c_int32),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


@dataclass
class FixResult:
    converged: bool
    sweeps: int
    sweeps_fp32: int
    sweeps_fp64: int
    theta: float
    F: float


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)

# C entry points: name -> argtypes (all return gf_status unless listed in _RESTYPES)
_SIGNATURES = {
    "gf_create_lattice": [ctypes.POINTER(_i32), ctypes.c_int, _vp, ctypes.POINTER(_vp)],
    "gf_destroy_lattice": [_vp],
    "gf_create_lattice_su2": [ctypes.POINTER(_i32), ctypes.c_int, _vp, ctypes.POINTER(_vp)],
    "gf_lattice_group": [_vp, ctypes.POINTER(_i32)],
    "gf_create_lattice_min8": [ctypes.POINTER(_i32), _vp, ctypes.POINTER(_vp)],
    "gf_lattice_storage": [_vp, ctypes.POINTER(_i32)],
    "gf_set_storage": [_vp, _i32],
    "gf_autotune_storage": [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double)],
    "gf_lattice_info": [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "gf_set_sweep_config": [_vp, ctypes.c_int, _i32, _i32, _i32, _i32],
    "gf_set_anneal_config": [_vp, ctypes.c_int, _i32, _i32, _i32, _i32],
    "gf_get_anneal_counter": [_vp, ctypes.POINTER(ctypes.c_uint32)],
    "gf_set_anneal_counter": [_vp, ctypes.c_uint32],
    "gf_promote_fp64": [_vp],
    "gf_autotune_anneal": [_vp, ctypes.c_int, _i32, ctypes.c_char_p, ctypes.POINTER(gf_tune_entry), _i32,
                           ctypes.POINTER(_i32), ctypes.POINTER(gf_tune_entry)],
    "gf_autotune": [_vp, ctypes.c_int, _i32, ctypes.c_char_p, ctypes.POINTER(gf_tune_entry), _i32,
                    ctypes.POINTER(_i32), ctypes.POINTER(gf_tune_entry)],
    "gf_set_links": [_vp, _dp],
    "gf_set_links_device": [_vp, _vp],
    "gf_get_links": [_vp, _dp],
    "gf_get_links_device": [_vp, _vp],
    "gf_sweep_or": [_vp, _i32, ctypes.c_double, ctypes.c_int],
    "gf_half_sweep_or": [_vp, _i32, ctypes.c_double, ctypes.c_int],
    "gf_anneal": [_vp, _i32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64],
    "gf_measure_theta_F": [_vp, _dp, _dp],
    "gf_measure_theta_F_noalloc": [ctypes.POINTER(_i32), _vp, _vp, _vp],
    "gf_fix_until": [_vp, ctypes.POINTER(gf_fix_params), ctypes.POINTER(gf_fix_result)],
    "gf_tune_switch": [_vp, ctypes.c_double, _dp, _dp],
    "gf_set_check_policy": [_vp, _i32, ctypes.c_double],
    "gf_sweep_estimate": [_vp, ctypes.c_double, ctypes.c_int, _dp],
    "gf_lattice_counters": [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "gf_set_gauge": [_vp, ctypes.c_int],
    "gf_get_gauge": [_vp, ctypes.POINTER(ctypes.c_int)],
    "gf_measure_timeslices": [_vp, _dp, _dp],
    "gf_reunitarize": [_vp],
    "gf_plaquette": [_vp, _dp],
    "gf_pool_create": [ctypes.POINTER(gf_pool_config), _vp, ctypes.POINTER(_vp)],
    "gf_pool_destroy": [_vp],
    "gf_pool_job_bytes": [ctypes.POINTER(_i32), _i32, _i32, ctypes.POINTER(ctypes.c_int64)],
    "gf_pool_admit": [_vp, ctypes.c_uint64, ctypes.POINTER(_i32), _dp, ctypes.POINTER(gf_fix_params), _i32,
                      ctypes.c_double, ctypes.c_double, ctypes.c_uint64],
    "gf_pool_step": [_vp],
    "gf_pool_step_async": [_vp],
    "gf_pool_sync": [_vp],
    "gf_pool_poll": [_vp, ctypes.POINTER(gf_pool_done), _i32, ctypes.POINTER(_i32)],
    "gf_pool_fetch_links": [_vp, ctypes.c_uint64, _dp],
    "gf_pool_release": [_vp, ctypes.c_uint64],
    "gf_pool_cancel": [_vp, ctypes.c_uint64],
    "gf_pool_stats": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_int64)],
    "gf_pool_autotune": [_vp, _i32, _i32, ctypes.c_size_t, ctypes.POINTER(gf_tune_entry), _i32,
                         ctypes.POINTER(_i32), ctypes.POINTER(gf_tune_entry)],
    "gf_pool_get_cache": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "gf_pool_get_shape": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                          ctypes.POINTER(_i32)],
    "gf_clock": [],
    "gf_probe_copy": [ctypes.c_size_t, _i32, _i32, _i32, _dp],
    "gf_last_error": [],
    "gf_version": [],
}
_RESTYPES = {"gf_last_error": ctypes.c_char_p, "gf_version": ctypes.c_char_p, "gf_clock": ctypes.c_double}


def _check_single_hip_runtime():
    """libgf must share the process's HIP runtime with torch (one libamdhip64)."""
    try:
        with open("/proc/self/maps") as fh:
            paths = {line.split()[-1] for line in fh if "libamdhip64" in line}
    except OSError:
        return
    real = {os.path.realpath(p) for p in paths}
    if len(real) > 1:
        raise RuntimeError(f"two HIP runtimes are loaded in this process: {sorted(real)}")


def lib() -> ctypes.CDLL:
    """Load libgf.so (after torch, whose HIP runtime it shares)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    import torch  # noqa: F401  (loads the HIP runtime first)

    L = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = _RESTYPES.get(name, ctypes.c_int)
    _check_single_hip_runtime()
    _lib = L
    return L


def exported_symbols():
    return list(_SIGNATURES)


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != GF_OK:
        raise GFError(st, lib().gf_last_error().decode(errors="replace"))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _host_links(u: np.ndarray, volume: int, per_site: int = 72) -> np.ndarray:
    if not (isinstance(u, np.ndarray) and u.dtype == np.float64 and u.flags.c_contiguous):
        raise TypeError("host links must be a C-contiguous float64 numpy array")
    if u.size != volume * per_site:
        raise ValueError(f"host links hold {u.size} doubles, the lattice needs {volume * per_site}")
    return u


def _is_device_tensor(x) -> bool:
    try:
        import torch
    except ImportError:
        return False
    return isinstance(x, torch.Tensor) and x.is_cuda


def _device_links(t, volume: int, per_site: int = 72):
    import torch

    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("device links must be a contiguous float64 tensor")
    if t.numel() != volume * per_site:
        raise ValueError(f"device links hold {t.numel()} doubles, the lattice needs {volume * per_site}")
    return t


# ----------------------------------------------------------- entry points --


def gf_version() -> str:
    return lib().gf_version().decode()


def gf_last_error() -> str:
    return lib().gf_last_error().decode(errors="replace")


# hip stream handle of each live lattice (None = the default stream), so that the
# device-array calls can order the lattice's stream against torch's
_LATTICE_STREAM = {}


def gf_create_lattice(dims, prec: int = GF_FP64, stream=None, group: int = 3, storage: int = 12) -> ctypes.c_void_p:
    """group 3: SU(3) (gf_create_lattice); group 2: SU(2) (gf_create_lattice_su2).
    storage 8: SU(3) links of the sweeping precision in 8 reals (GF_FP64: gf_create_lattice_min8;
    GF_FP32 / GF_MIXED: gf_create_lattice, then gf_set_storage(8) before any links exist)."""
    d = (_i32 * 4)(*[int(x) for x in dims])
    out = _vp()
    h = _stream_handle(stream)
    if group not in (2, 3):
        raise ValueError("group must be 2 (SU(2)) or 3 (SU(3))")
    if storage not in (8, 12) or (storage == 8 and group != 3):
        raise ValueError("storage 8 is for SU(3) lattices; otherwise 12")
    if storage == 8 and prec == GF_FP64:
        _call("gf_create_lattice_min8", d, h, ctypes.byref(out))
    else:
        _call("gf_create_lattice_su2" if group == 2 else "gf_create_lattice", d, int(prec), h, ctypes.byref(out))
        if storage == 8:
            st = lib().gf_set_storage(out, 8)
            if st != GF_OK:
                err = GFError(st, lib().gf_last_error().decode(errors="replace"))
                lib().gf_destroy_lattice(out)
                raise err
    _LATTICE_STREAM[out.value] = h
    return out


def gf_lattice_storage(lat) -> int:
    """Reals stored per link of the sweeping precision: 12, 8 or 4 (SU(2))."""
    n = _i32()
    _call("gf_lattice_storage", lat, ctypes.byref(n))
    return n.value


def gf_set_storage(lat, reals_per_link: int) -> None:
    _call("gf_set_storage", lat, int(reals_per_link))


def gf_autotune_storage(lat, n_sweeps: int = 3):
    """(reals per link chosen, us per sweep with 12 reals, with 8 reals)."""
    n = _i32()
    a = ctypes.c_double()
    b = ctypes.c_double()
    _call("gf_autotune_storage", lat, int(n_sweeps), ctypes.byref(n), ctypes.byref(a), ctypes.byref(b))
    return n.value, a.value, b.value


def gf_lattice_group(lat) -> int:
    """N_c of the lattice's gauge group (2 or 3)."""
    n = _i32()
    _call("gf_lattice_group", lat, ctypes.byref(n))
    return n.value


def gf_destroy_lattice(lat) -> None:
    _call("gf_destroy_lattice", lat)
    _LATTICE_STREAM.pop(getattr(lat, "value", lat), None)


def _lattice_stream(lat, tensor):
    """(torch's current stream on the tensor's device, the lattice's stream as a torch
    stream), or None when the two are the same stream."""
    import torch

    cur = torch.cuda.current_stream(tensor.device)
    h = _LATTICE_STREAM.get(getattr(lat, "value", lat))
    if (h or 0) == int(cur.cuda_stream):
        return None
    ls = torch.cuda.ExternalStream(h, device=tensor.device) if h else torch.cuda.default_stream(tensor.device)
    return cur, ls


def _before_lattice_reads(lat, tensor) -> None:
    """The lattice's stream waits for torch's current stream (which produced the
    tensor), and the caching allocator keeps the tensor's memory until the lattice's
    stream has used it."""
    pair = _lattice_stream(lat, tensor)
    if pair is not None:
        cur, ls = pair
        ls.wait_stream(cur)
        tensor.record_stream(ls)


def _after_lattice_writes(lat, tensor) -> None:
    """Torch's current stream waits for the lattice's stream (which wrote the tensor)."""
    pair = _lattice_stream(lat, tensor)
    if pair is not None:
        cur, ls = pair
        tensor.record_stream(ls)
        cur.wait_stream(ls)


def gf_lattice_info(lat):
    v = ctypes.c_int64()
    b = ctypes.c_int64()
    _call("gf_lattice_info", lat, ctypes.byref(v), ctypes.byref(b))
    return v.value, b.value


def gf_set_sweep_config(lat, kernel: int, tps: int, block: int, nontemporal: int = 0, min_waves: int = 0) -> None:
    _call("gf_set_sweep_config", lat, int(kernel), int(tps), int(block), int(nontemporal), int(min_waves))


def gf_get_anneal_counter(lat) -> int:
    c = ctypes.c_uint32()
    _call("gf_get_anneal_counter", lat, ctypes.byref(c))
    return c.value


def gf_set_anneal_counter(lat, sweeps_done: int) -> None:
    _call("gf_set_anneal_counter", lat, int(sweeps_done))


def gf_set_anneal_config(lat, kernel: int, tps: int, block: int, nontemporal: int = 0, min_waves: int = 0) -> None:
    _call("gf_set_anneal_config", lat, int(kernel), int(tps), int(block), int(nontemporal), int(min_waves))


def _tune(name, lat, kernel, n_sweeps, cache_path):
    cap = 64
    buf = (gf_tune_entry * cap)()
    n = _i32()
    ch = gf_tune_entry()
    cp = None if cache_path is None else os.fsencode(cache_path)
    _call(name, lat, int(kernel), int(n_sweeps), cp, buf, cap, ctypes.byref(n), ctypes.byref(ch))
    table = [(buf[i].tps, buf[i].block, buf[i].nontemporal, buf[i].min_waves, buf[i].us_per_sweep)
             for i in range(n.value)]
    return (ch.tps, ch.block, ch.nontemporal, ch.min_waves), table


def gf_autotune(lat, kernel: int, n_sweeps: int = 5, cache_path=None):
    """Returns (chosen, table): chosen = (tps, block, nontemporal), table = list of
    (tps, block, nontemporal, us_per_sweep) (empty when the cache answered)."""
    return _tune("gf_autotune", lat, kernel, n_sweeps, cache_path)


def gf_autotune_anneal(lat, kernel: int, n_sweeps: int = 5, cache_path=None):
    """As gf_autotune, for the heat-bath sweep of gf_anneal."""
    return _tune("gf_autotune_anneal", lat, kernel, n_sweeps, cache_path)


def gf_promote_fp64(lat) -> None:
    _call("gf_promote_fp64", lat)


def gf_set_links(lat, links) -> None:
    volume, _ = gf_lattice_info(lat)
    nc = gf_lattice_group(lat)
    per_site = 4 * 2 * nc * nc
    if _is_device_tensor(links):
        t = _device_links(links, volume, per_site)
        _before_lattice_reads(lat, t)
        _call("gf_set_links_device", lat, t.data_ptr())
    else:
        u = _host_links(links, volume, per_site)
        _call("gf_set_links", lat, u.ctypes.data_as(_dp))


def gf_set_links_device(lat, dev_ptr: int) -> None:
    _call("gf_set_links_device", lat, int(dev_ptr))


def gf_get_links(lat, out=None):
    """Links as a canonical array: into `out` (numpy or device tensor) or a new numpy array."""
    volume, _ = gf_lattice_info(lat)
    nc = gf_lattice_group(lat)
    per_site = 4 * 2 * nc * nc
    if out is None:
        out = np.empty((volume, 4, nc, nc, 2), dtype=np.float64)
    if _is_device_tensor(out):
        t = _device_links(out, volume, per_site)
        _before_lattice_reads(lat, t)  # earlier torch work on `out` completes first
        _call("gf_get_links_device", lat, t.data_ptr())
        _after_lattice_writes(lat, t)
    else:
        u = _host_links(out, volume, per_site)
        _call("gf_get_links", lat, u.ctypes.data_as(_dp))
    return out


def gf_get_links_device(lat, dev_ptr: int) -> None:
    _call("gf_get_links_device", lat, int(dev_ptr))


def gf_sweep_or(lat, n_sweeps: int, omega: float, mode: int = GF_OR_EXACT) -> None:
    _call("gf_sweep_or", lat, int(n_sweeps), float(omega), int(mode))


def gf_half_sweep_or(lat, colour: int, omega: float, mode: int = GF_OR_EXACT) -> None:
    _call("gf_half_sweep_or", lat, int(colour), float(omega), int(mode))


def gf_anneal(lat, n_sweeps: int, T_start: float, T_end: float, seed: int) -> None:
    _call("gf_anneal", lat, int(n_sweeps), float(T_start), float(T_end), int(seed) & 0xFFFFFFFFFFFFFFFF)


def gf_measure_theta_F(lat):
    th = ctypes.c_double()
    f = ctypes.c_double()
    _call("gf_measure_theta_F", lat, ctypes.byref(th), ctypes.byref(f))
    return th.value, f.value


def gf_measure_theta_F_noalloc(dims, dev_links, dev_out, stream=None) -> None:
    """theta, F of canonical device links into dev_out[0:2] (device float64), enqueued on
    `stream` (default: torch's current stream) without allocating; async."""
    import torch

    d = [int(x) for x in dims]
    volume = int(np.prod(d))
    t = _device_links(dev_links, volume)
    if dev_out.dtype != torch.float64 or not dev_out.is_cuda or not dev_out.is_contiguous() or dev_out.numel() < 2:
        raise TypeError("dev_out must be a contiguous float64 device tensor of at least 2 elements")
    h = _stream_handle(stream) if stream is not None else int(torch.cuda.current_stream().cuda_stream)
    _call("gf_measure_theta_F_noalloc", (_i32 * 4)(*d), t.data_ptr(), dev_out.data_ptr(), h)


def gf_fix_until(lat, omega: float = 1.7, mode: int = GF_OR_EXACT, theta_target: float = 1e-12,
                 max_sweeps: int = 3000, check_every: int = 10, reunit_every: int = 100,
                 theta_switch: float = -1.0) -> FixResult:
    """theta_switch < 0: the library picks the float32 -> float64 switch point (gf_tune_switch)."""
    p = gf_fix_params(float(omega), int(mode), float(theta_target), int(max_sweeps), int(check_every),
                      int(reunit_every), float(theta_switch))
    r = gf_fix_result()
    _call("gf_fix_until", lat, ctypes.byref(p), ctypes.byref(r))
    return FixResult(bool(r.converged), r.sweeps, r.sweeps_fp32, r.sweeps_fp64, r.theta, r.F)


def gf_tune_switch(lat, theta_target: float = 1e-12):
    """(float32 rounding floor of theta, chosen switch point) for the lattice's float64 links."""
    fl = ctypes.c_double()
    sw = ctypes.c_double()
    _call("gf_tune_switch", lat, float(theta_target), ctypes.byref(fl), ctypes.byref(sw))
    return fl.value, sw.value


def gf_set_check_policy(lat, adaptive: bool, margin: float = 100.0) -> None:
    _call("gf_set_check_policy", lat, int(bool(adaptive)), float(margin))


def gf_sweep_estimate(lat, omega: float, mode: int = GF_OR_EXACT) -> float:
    th = ctypes.c_double()
    _call("gf_sweep_estimate", lat, float(omega), int(mode), ctypes.byref(th))
    return th.value


def gf_lattice_counters(lat):
    """(exact measurements, fused estimates) taken on the lattice."""
    m = ctypes.c_int64()
    e = ctypes.c_int64()
    _call("gf_lattice_counters", lat, ctypes.byref(m), ctypes.byref(e))
    return m.value, e.value


def gf_set_gauge(lat, gauge: int) -> None:
    _call("gf_set_gauge", lat, int(gauge))


def gf_get_gauge(lat) -> int:
    g = ctypes.c_int()
    _call("gf_get_gauge", lat, ctypes.byref(g))
    return g.value


def gf_measure_timeslices(lat, nt: int):
    """Coulomb gauge: (theta_C(t), F_C(t)) as two float64 arrays of nt = Nt."""
    th = np.empty(int(nt))
    fr = np.empty(int(nt))
    _call("gf_measure_timeslices", lat, th.ctypes.data_as(_dp), fr.ctypes.data_as(_dp))
    return th, fr


def gf_reunitarize(lat) -> None:
    _call("gf_reunitarize", lat)


def gf_plaquette(lat) -> float:
    p = ctypes.c_double()
    _call("gf_plaquette", lat, ctypes.byref(p))
    return p.value


class Lattice:
    """Owning wrapper: ``with Lattice(dims, GF_FP64) as lat: ...``."""

    def __init__(self, dims, prec: int = GF_FP64, stream=None, gauge: int = GF_LANDAU, group: int = 3,
                 storage: int = 12):
        self.dims = tuple(int(d) for d in dims)
        self.prec = prec
        self.group = group
        self.handle = gf_create_lattice(self.dims, prec, stream, group, storage)
        if gauge != GF_LANDAU:
            gf_set_gauge(self.handle, gauge)

    @property
    def volume(self) -> int:
        return gf_lattice_info(self.handle)[0]

    @property
    def storage(self) -> int:
        """Reals stored per link (12, 8 or 4); assign 8 or 12 to convert a float64 SU(3) lattice."""
        return gf_lattice_storage(self.handle)

    @storage.setter
    def storage(self, reals_per_link: int):
        gf_set_storage(self.handle, reals_per_link)

    def autotune_storage(self, n_sweeps: int = 3):
        return gf_autotune_storage(self.handle, n_sweeps)

    def close(self):
        if self.handle is not None and self.handle.value:
            gf_destroy_lattice(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_links(self, links):
        gf_set_links(self.handle, links)

    def get_links(self, out=None):
        return gf_get_links(self.handle, out)

    def sweep(self, n: int, omega: float, mode: int = GF_OR_EXACT):
        gf_sweep_or(self.handle, n, omega, mode)

    def half_sweep(self, colour: int, omega: float, mode: int = GF_OR_EXACT):
        gf_half_sweep_or(self.handle, colour, omega, mode)

    def anneal(self, n: int, T_start: float, T_end: float, seed: int):
        gf_anneal(self.handle, n, T_start, T_end, seed)

    def measure(self):
        return gf_measure_theta_F(self.handle)

    @property
    def gauge(self) -> int:
        return gf_get_gauge(self.handle)

    @gauge.setter
    def gauge(self, g: int):
        gf_set_gauge(self.handle, g)

    def set_check_policy(self, adaptive: bool, margin: float = 100.0):
        gf_set_check_policy(self.handle, adaptive, margin)

    def sweep_estimate(self, omega: float, mode: int = GF_OR_EXACT) -> float:
        return gf_sweep_estimate(self.handle, omega, mode)

    @property
    def counters(self):
        return gf_lattice_counters(self.handle)

    def measure_timeslices(self):
        """Coulomb gauge: (theta_C(t), F_C(t)) per timeslice."""
        return gf_measure_timeslices(self.handle, self.dims[3])

    def fix_until(self, **kw) -> FixResult:
        return gf_fix_until(self.handle, **kw)

    def tune_switch(self, theta_target: float = 1e-12):
        return gf_tune_switch(self.handle, theta_target)

    def reunitarize(self):
        gf_reunitarize(self.handle)

    def plaquette(self) -> float:
        return gf_plaquette(self.handle)

    def set_sweep_config(self, tps: int, block: int, nontemporal: int = 0, kernel=None, min_waves: int = 0):
        """Configure the sweep kernel of `kernel` precision (default: the lattice's own;
        GF_MIXED configures both)."""
        kinds = [kernel] if kernel is not None else (
            [GF_FP32, GF_FP64] if self.prec == GF_MIXED else [self.prec])
        for k in kinds:
            gf_set_sweep_config(self.handle, k, tps, block, nontemporal, min_waves)

    def promote_fp64(self):
        gf_promote_fp64(self.handle)

    def autotune(self, kernel=None, n_sweeps: int = 5, cache_path=None):
        k = kernel if kernel is not None else (GF_FP32 if self.prec != GF_FP64 else GF_FP64)
        return gf_autotune(self.handle, k, n_sweeps, cache_path)

    @property
    def anneal_counter(self) -> int:
        return gf_get_anneal_counter(self.handle)

    @anneal_counter.setter
    def anneal_counter(self, sweeps_done: int):
        gf_set_anneal_counter(self.handle, sweeps_done)

    def set_anneal_config(self, tps: int, block: int, nontemporal: int = 0, kernel=None, min_waves: int = 0):
        kinds = [kernel] if kernel is not None else (
            [GF_FP32, GF_FP64] if self.prec == GF_MIXED else [self.prec])
        for k in kinds:
            gf_set_anneal_config(self.handle, k, tps, block, nontemporal, min_waves)

    def autotune_anneal(self, kernel=None, n_sweeps: int = 5, cache_path=None):
        k = kernel if kernel is not None else (GF_FP32 if self.prec != GF_FP64 else GF_FP64)
        return gf_autotune_anneal(self.handle, k, n_sweeps, cache_path)


# ----------------------------------------------------------------- pool --


def gf_probe_copy(nbytes: int, reps: int = 10, nontemporal: bool = False, blocks: int = 4096) -> float:
    g = ctypes.c_double()
    _call("gf_probe_copy", int(nbytes), int(reps), int(bool(nontemporal)), int(blocks), ctypes.byref(g))
    return g.value


def gf_clock() -> float:
    return float(lib().gf_clock())


def gf_pool_job_bytes(dims, prec: int = GF_MIXED, reals32: int = 12) -> int:
    d = (_i32 * 4)(*[int(x) for x in dims])
    b = ctypes.c_int64()
    _call("gf_pool_job_bytes", d, int(prec), int(reals32), ctypes.byref(b))
    return b.value


def gf_pool_create(hbm_budget: int, max_slots: int, prec: int = GF_MIXED, check_every: int = 10,
                   mode: int = GF_OR_EXACT, tps32: int = 0, block32: int = 0, tps64: int = 0, block64: int = 0,
                   stream=None, reals32: int = 12, cache32: int = 0, cache64: int = 0):
    cfg = gf_pool_config(int(hbm_budget), int(max_slots), int(prec), int(check_every), int(mode), int(tps32),
                         int(block32), int(tps64), int(block64), int(reals32), int(cache32), int(cache64))
    out = _vp()
    _call("gf_pool_create", ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(out))
    return out


def gf_pool_destroy(pool) -> None:
    _call("gf_pool_destroy", pool)


def gf_pool_admit(pool, job_id: int, dims, links: np.ndarray, omega: float = 1.7, mode: int = GF_OR_EXACT,
                  theta_target: float = 1e-12, max_sweeps: int = 3000, check_every: int = 10,
                  reunit_every: int = 100, theta_switch: float = -1.0, anneal_sweeps: int = 0,
                  T_start: float = 1.25, T_end: float = 0.01, seed: int = 0) -> bool:
    """Admit a job; returns False (nothing changed) when the pool is full."""
    d = (_i32 * 4)(*[int(x) for x in dims])
    v = 1
    for x in dims:
        v *= int(x)
    u = _host_links(links, v)
    p = gf_fix_params(float(omega), int(mode), float(theta_target), int(max_sweeps), int(check_every),
                      int(reunit_every), float(theta_switch))
    st = lib().gf_pool_admit(pool, int(job_id), d, u.ctypes.data_as(_dp), ctypes.byref(p), int(anneal_sweeps),
                             float(T_start), float(T_end), int(seed) & 0xFFFFFFFFFFFFFFFF)
    if st == GF_E_FULL:
        return False
    if st != GF_OK:
        raise GFError(st, gf_last_error())
    return True


def gf_pool_step(pool) -> None:
    _call("gf_pool_step", pool)


def gf_pool_step_async(pool) -> None:
    _call("gf_pool_step_async", pool)


def gf_pool_sync(pool) -> None:
    _call("gf_pool_sync", pool)


def gf_pool_poll(pool, cap: int = 256):
    """Finished jobs since the last poll: list of dicts."""
    buf = (gf_pool_done * cap)()
    n = _i32()
    _call("gf_pool_poll", pool, buf, int(cap), ctypes.byref(n))
    out = []
    for i in range(n.value):
        d = buf[i]
        r = d.result
        out.append(dict(job_id=int(d.job_id), status=int(d.status), t_admit=d.t_admit, t_done=d.t_done,
                        result=FixResult(bool(r.converged), r.sweeps, r.sweeps_fp32, r.sweeps_fp64, r.theta, r.F)))
    return out


def gf_pool_fetch_links(pool, job_id: int, dims) -> np.ndarray:
    v = 1
    for x in dims:
        v *= int(x)
    out = np.empty((v, 4, 3, 3, 2), dtype=np.float64)
    _call("gf_pool_fetch_links", pool, int(job_id), out.ctypes.data_as(_dp))
    return out


def gf_pool_release(pool, job_id: int) -> None:
    _call("gf_pool_release", pool, int(job_id))


def gf_pool_cancel(pool, job_id: int) -> None:
    _call("gf_pool_cancel", pool, int(job_id))


def gf_pool_stats(pool):
    a = _i32()
    f = _i32()
    b = ctypes.c_int64()
    _call("gf_pool_stats", pool, ctypes.byref(a), ctypes.byref(f), ctypes.byref(b))
    return a.value, f.value, b.value


def gf_pool_autotune(pool, kernel: int, n_sweeps: int = 3, scratch_bytes: int = 8 << 30):
    """((tps, block, nontemporal), table of (tps, block, nontemporal, us_per_sweep)) of the pool's
    sweep of `kernel` (GF_FP32 / GF_FP64), timed on copies of the resident jobs (nontemporal: 0
    plain, 1 non-temporal link accesses)."""
    table = (gf_tune_entry * 32)()
    n = _i32()
    best = gf_tune_entry()
    _call("gf_pool_autotune", pool, int(kernel), int(n_sweeps), int(scratch_bytes), table, 32, ctypes.byref(n),
          ctypes.byref(best))
    rows = [(table[i].tps, table[i].block, table[i].nontemporal, table[i].us_per_sweep) for i in range(n.value)]
    return (best.tps, best.block, best.nontemporal), rows


def gf_pool_get_cache(pool):
    """(cache32, cache64) of the pool's overrelaxation sweeps: 1 plain, 2 non-temporal."""
    v = [_i32() for _ in range(2)]
    _call("gf_pool_get_cache", pool, *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)


def gf_pool_get_shape(pool):
    """(tps32, block32, tps64, block64) of the pool's sweeps."""
    v = [_i32() for _ in range(4)]
    _call("gf_pool_get_shape", pool, *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)


class Pool:
    """Owning wrapper of a gf_pool."""

    def __init__(self, hbm_budget: int, max_slots: int, prec: int = GF_MIXED, check_every: int = 10,
                 mode: int = GF_OR_EXACT, tps32: int = 0, tps64: int = 0, stream=None, block32: int = 0,
                 block64: int = 0, reals32: int = 12, cache32: int = 0, cache64: int = 0):
        """reals32 = 8: the float32 links of a GF_MIXED pool in 8 reals (gf_set_storage).
        cache32 / cache64: cache policy of the overrelaxation sweeps (1 plain, 2 non-temporal, 0 default)."""
        self.check_every = int(check_every)
        self.mode = int(mode)
        self.handle = gf_pool_create(hbm_budget, max_slots, prec, check_every, mode, tps32, block32, tps64, block64,
                                     stream, reals32, cache32, cache64)
        self.dims = {}

    def autotune(self, kernel: int, n_sweeps: int = 3, scratch_bytes: int = 8 << 30):
        return gf_pool_autotune(self.handle, kernel, n_sweeps, scratch_bytes)

    @property
    def shape(self):
        return gf_pool_get_shape(self.handle)

    @property
    def cache(self):
        return gf_pool_get_cache(self.handle)

    def admit(self, job_id, dims, links, **kw) -> bool:
        kw.setdefault("check_every", self.check_every)
        kw.setdefault("mode", self.mode)
        ok = gf_pool_admit(self.handle, job_id, dims, links, **kw)
        if ok:
            self.dims[int(job_id)] = tuple(int(x) for x in dims)
        return ok

    def step(self):
        gf_pool_step(self.handle)

    def step_async(self):
        """Complete the step in flight, launch the next and return without waiting for it."""
        gf_pool_step_async(self.handle)

    def sync(self):
        gf_pool_sync(self.handle)

    def poll(self, cap: int = 256):
        return gf_pool_poll(self.handle, cap)

    def fetch_links(self, job_id):
        out = gf_pool_fetch_links(self.handle, job_id, self.dims[int(job_id)])
        self.dims.pop(int(job_id), None)
        return out

    def release(self, job_id):
        gf_pool_release(self.handle, job_id)
        self.dims.pop(int(job_id), None)

    def cancel(self, job_id):
        gf_pool_cancel(self.handle, job_id)

    def stats(self):
        return gf_pool_stats(self.handle)

    def close(self):
        if self.handle is not None and self.handle.value:
            gf_pool_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
