"""Python binding of libslh (include/slh.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts numpy
inputs to the C structs, hands PyTorch's current HIP stream (and, optionally,
its caching allocator) to the library, and copies results back.  There is no
fallback: if libslh.so is missing or cannot be loaded, every entry point
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SLH_LIB: another build of the library (the host-sanitized one of build.py
# --sanitize-host); by default the in-tree libslh.so
LIB_PATH = os.environ.get("SLH_LIB") or os.path.join(_HERE, "libslh.so")

SLH_ABI_VERSION = 9
SLH_OK, SLH_E_INVALID_ARG, SLH_E_OUT_OF_MEMORY, SLH_E_DEVICE, SLH_E_NOT_CONVERGED, \
    SLH_E_NUMERIC, SLH_E_REJECTED, SLH_E_STATE = range(8)
SLH_FP64, SLH_FP32_TRACK = 0, 1
SLH_SOBOL_OWEN, SLH_PRNG, SLH_HALTON = 0, 1, 2
SLH_REFLECT_X_LO, SLH_REFLECT_X_HI, SLH_REFLECT_Y_LO, SLH_REFLECT_Y_HI = 1, 2, 4, 8
SLH_SI_NORM_COLLIDED, SLH_SI_NORM_TOTAL = 0, 1
SLH_CLOSE_SN, SLH_CLOSE_DIFFUSION = 0, 1
SLH_ACCEL_NONE, SLH_ACCEL_DSA = 0, 1
SLH_FLUX_REMAP, SLH_FLUX_PRE, SLH_FLUX_POST, SLH_FLUX_COLLIDED_NODAL = range(4)

STATUS_NAMES = ["SLH_OK", "SLH_E_INVALID_ARG", "SLH_E_OUT_OF_MEMORY", "SLH_E_DEVICE",
                "SLH_E_NOT_CONVERGED", "SLH_E_NUMERIC", "SLH_E_REJECTED", "SLH_E_STATE"]


class slh_problem(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("x_lo", C.c_double), ("x_hi", C.c_double), ("y_lo", C.c_double),
                ("y_hi", C.c_double), ("sigma_s", C.c_void_p), ("sigma_a", C.c_void_p),
                ("q", C.c_void_p), ("c", C.c_double), ("dt", C.c_double), ("n_s", C.c_int32),
                ("n_particles", C.c_int64), ("census_cap", C.c_int64),
                ("sn_order", C.c_int32), ("time_closure", C.c_double), ("si_tol", C.c_double),
                ("si_max_iter", C.c_int32), ("w_cut_rel", C.c_double), ("seed", C.c_uint64),
                ("points", C.c_int32), ("precision", C.c_int32), ("n_s_cell", C.c_void_p),
                ("boundary", C.c_int32), ("steady", C.c_int32), ("horizon", C.c_double),
                ("si_norm", C.c_int32), ("closure", C.c_int32), ("si_accel", C.c_int32),
                ("census_qmc", C.c_int32), ("inflow", C.c_void_p)]


class slh_balance(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("emitted", "absorbed", "scattered", "leaked",
                                          "census", "cutoff", "source_w", "census_in_w")] + \
               [("segments", C.c_uint64), ("particles", C.c_uint64),
                ("majorant_sum", C.c_double), ("weight_quantum", C.c_double),
                ("source_particles", C.c_uint64), ("killed", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class slh_stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("si_iterations", C.c_int32), ("si_residual", C.c_double),
                ("si_converged", C.c_int32), ("census_alive", C.c_int64),
                ("census_kept", C.c_int64), ("thin_factor", C.c_double),
                ("segments_total", C.c_uint64), ("ms_mc", C.c_double), ("ms_dg", C.c_double),
                ("ms_remap", C.c_double), ("ms_census", C.c_double),
                ("ms_kernel_mc_total", C.c_double), ("ms_kernel_remap_total", C.c_double),
                ("seg_mc_total", C.c_uint64), ("seg_remap_total", C.c_uint64),
                ("census_in_total", C.c_uint64), ("census_out_total", C.c_uint64),
                ("steps_total", C.c_uint64), ("thin_overflow_total", C.c_uint64),
                ("graph_launches_total", C.c_uint64), ("host_waits_total", C.c_uint64),
                ("killed_total", C.c_uint64), ("dsa_corrections", C.c_int32),
                ("dsa_iterations", C.c_int32), ("dsa_unconverged", C.c_int32),
                ("numeric_flags", C.c_int32), ("si_unconverged_total", C.c_uint64),
                ("si_batch", C.c_int32), ("pad0", C.c_int32), ("si_restarts_total", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class slh_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("n_streams", C.c_int32)]


class slh_latency(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("submit_s", "admit_s", "done_s", "queue_ms",
                                          "run_ms", "latency_ms")] + [("segments", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

EXPORTS = ["slh_create", "slh_create_static", "slh_advance", "slh_set_graphs", "slh_set_timing",
           "slh_set_si_batch",
           "slh_synchronize", "slh_get_flux", "slh_get_flux_device",
           "slh_get_balance", "slh_get_stats", "slh_get_census", "slh_save", "slh_load",
           "slh_footprint_bytes", "slh_destroy", "slh_last_error", "slh_qmc_points",
           "slh_server_create", "slh_server_submit", "slh_server_poll", "slh_server_result",
           "slh_server_destroy"]

_lib = None


def lib():
    """Loads libslh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libslh.so is not built (run __graft_entry__.build() or "
                           "python paper_2511_16821_amd/build.py); there is no fallback")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
    sig = {
        "slh_create": ([C.POINTER(slh_problem), vp, ALLOC_FN, FREE_FN, vp, C.POINTER(vp)], i32),
        "slh_create_static": ([C.POINTER(slh_problem), vp, C.POINTER(vp)], i32),
        "slh_advance": ([vp, i32], i32),
        "slh_set_graphs": ([vp, i32], i32),
        "slh_set_timing": ([vp, i32], i32),
        "slh_set_si_batch": ([vp, i32], i32),
        "slh_synchronize": ([vp], i32),
        "slh_get_flux": ([vp, i32, vp], i32),
        "slh_get_flux_device": ([vp, i32, vp], i32),
        "slh_get_balance": ([vp, i32, C.POINTER(slh_balance)], i32),
        "slh_get_stats": ([vp, C.POINTER(slh_stats)], i32),
        "slh_get_census": ([vp, C.POINTER(i64), vp, vp, vp, vp, vp, vp, vp], i32),
        "slh_save": ([vp, vp, C.POINTER(C.c_size_t)], i32),
        "slh_load": ([vp, vp, C.c_size_t], i32),
        "slh_footprint_bytes": ([C.POINTER(slh_problem)], C.c_size_t),
        "slh_destroy": ([vp], None),
        "slh_last_error": ([], C.c_char_p),
        "slh_qmc_points": ([u64, u64, u32, u32, u64, u32, u32, u32, u32, i32, vp, vp], i32),
        "slh_server_create": ([C.POINTER(slh_server_cfg), C.POINTER(vp)], i32),
        "slh_server_submit": ([vp, C.POINTER(slh_problem), i32, C.POINTER(u64)], i32),
        "slh_server_poll": ([vp, u64, C.POINTER(i32)], i32),
        "slh_server_result": ([vp, u64, vp, C.POINTER(slh_balance), C.POINTER(slh_latency)],
                              i32),
        "slh_server_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class SlhError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().slh_last_error()
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES[status] if 0 <= status < 8
                                          else status, msg.decode() if msg else ""))


def _check(st, where, allow=(SLH_OK,)):
    if st not in allow:
        raise SlhError(st, where)
    return st


def _f64(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != n:
        raise ValueError("field has %d entries, expected %d" % (a.size, n))
    return a


def make_problem(p: dict):
    """slh_problem from a problem dict (see paper_2511_16821_amd.workloads).
    Returns (struct, keep-alive list)."""
    nx, ny = int(p["nx"]), int(p["ny"])
    ss, sa, q = (_f64(p[k], nx * ny) for k in ("sigma_s", "sigma_a", "q"))
    s = slh_problem()
    s.abi_version = SLH_ABI_VERSION
    s.nx, s.ny = nx, ny
    s.x_lo, s.x_hi, s.y_lo, s.y_hi = (float(p[k]) for k in ("x_lo", "x_hi", "y_lo", "y_hi"))
    s.sigma_s, s.sigma_a, s.q = (a.ctypes.data for a in (ss, sa, q))
    s.c = float(p.get("c", 1.0))
    s.dt = float(p.get("dt", 0.0))
    s.n_s = int(p["n_s"])
    s.n_particles = int(p["n_particles"])
    s.census_cap = int(p.get("census_cap", 0))
    s.sn_order = int(p["sn_order"])
    s.time_closure = float(p.get("time_closure", 2.0))
    s.si_tol = float(p.get("si_tol", 1e-12))
    s.si_max_iter = int(p.get("si_max_iter", 200))
    s.w_cut_rel = float(p.get("w_cut_rel", 1e-8))
    s.seed = int(p.get("seed", 0)) & (2 ** 64 - 1)
    s.points = int(p.get("points", 0))
    s.precision = int(p.get("precision", 0))
    s.boundary = int(p.get("boundary", 0))
    s.steady = int(bool(p.get("steady", False)))
    s.horizon = float(p.get("horizon", 0.0))
    s.si_norm = int(p.get("si_norm", 0))
    s.closure = int(p.get("closure", 0))
    s.si_accel = int(p.get("si_accel", 0))
    s.census_qmc = int(p.get("census_qmc", 0))
    keep = [ss, sa, q]
    if p.get("n_s_cell") is not None:
        nsc = np.ascontiguousarray(p["n_s_cell"], dtype=np.int32).reshape(-1)
        if nsc.size != nx * ny:
            raise ValueError("n_s_cell must have nx*ny entries")
        s.n_s_cell = nsc.ctypes.data
        keep.append(nsc)
    if p.get("inflow") is not None:
        g = np.ascontiguousarray(p["inflow"], dtype=np.float64).reshape(-1)
        if g.size != 2 * (nx + ny):
            raise ValueError("inflow must have 2 (nx + ny) entries")
        s.inflow = g.ctypes.data
        keep.append(g)
    return s, keep


def slh_footprint_bytes(p: dict) -> int:
    s, keep = make_problem(p)
    return int(lib().slh_footprint_bytes(C.byref(s)))


def _torch_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.stream = stream
        self.live = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            p = self.torch.cuda.caching_allocator_alloc(int(nbytes), stream=self.stream)
        except Exception:  # out of memory -> NULL, the library reports it
            return None
        self.live[p] = nbytes
        return p

    def _free(self, ptr, ctx):
        if ptr in self.live:
            del self.live[ptr]
            self.torch.cuda.caching_allocator_delete(ptr)


class Solver:
    """One hybrid solve resident on the GPU (slh_create ... slh_destroy)."""

    def __init__(self, problem: dict, stream=None, torch_allocator: bool = True,
                 static: bool = False):
        """static: slh_create_static (device memory from the library's static
        scratch, no allocator)."""
        self.problem = problem
        self.nx, self.ny = int(problem["nx"]), int(problem["ny"])
        st, self._keep = make_problem(problem)
        if stream is None:
            stream = _torch_stream()
        self.stream = stream
        self._alloc = _TorchAllocator(torch_stream_obj()) if torch_allocator and not static \
            else None
        h = C.c_void_p()
        if static:
            r = lib().slh_create_static(C.byref(st), C.c_void_p(stream), C.byref(h))
        elif self._alloc is not None:
            r = lib().slh_create(C.byref(st), C.c_void_p(stream), self._alloc.alloc_cb,
                                 self._alloc.free_cb, None, C.byref(h))
        else:
            r = lib().slh_create(C.byref(st), C.c_void_p(stream), ALLOC_FN(0), FREE_FN(0), None,
                                 C.byref(h))
        _check(r, "slh_create")
        self.h = h

    def slh_advance(self, n_steps=1, allow_not_converged=False):
        allow = (SLH_OK, SLH_E_NOT_CONVERGED) if allow_not_converged else (SLH_OK,)
        return _check(lib().slh_advance(self.h, int(n_steps)), "slh_advance", allow)

    advance = slh_advance

    def slh_set_graphs(self, enable):
        _check(lib().slh_set_graphs(self.h, 1 if enable else 0), "slh_set_graphs")

    set_graphs = slh_set_graphs

    def slh_set_timing(self, enable):
        _check(lib().slh_set_timing(self.h, 1 if enable else 0), "slh_set_timing")

    set_timing = slh_set_timing

    def slh_set_si_batch(self, n):
        _check(lib().slh_set_si_batch(self.h, int(n)), "slh_set_si_batch")

    set_si_batch = slh_set_si_batch

    def slh_synchronize(self, allow_not_converged=False):
        allow = (SLH_OK, SLH_E_NOT_CONVERGED) if allow_not_converged else (SLH_OK,)
        return _check(lib().slh_synchronize(self.h), "slh_synchronize", allow)

    synchronize = slh_synchronize

    def slh_get_flux(self, which=SLH_FLUX_REMAP):
        n = self.nx * self.ny * (4 if which == SLH_FLUX_COLLIDED_NODAL else 1)
        out = np.zeros(n)
        _check(lib().slh_get_flux(self.h, int(which), out.ctypes.data), "slh_get_flux")
        return out

    get_flux = slh_get_flux

    def slh_get_flux_device(self, which, dev_ptr):
        _check(lib().slh_get_flux_device(self.h, int(which), C.c_void_p(dev_ptr)),
               "slh_get_flux_device")

    def slh_get_balance(self, pss):
        b = slh_balance()
        _check(lib().slh_get_balance(self.h, int(pss), C.byref(b)), "slh_get_balance")
        return b.as_dict()

    get_balance = slh_get_balance

    def slh_get_stats(self):
        s = slh_stats()
        _check(lib().slh_get_stats(self.h, C.byref(s)), "slh_get_stats")
        return s.as_dict()

    get_stats = slh_get_stats

    def slh_get_census(self):
        n = C.c_int64(0)
        _check(lib().slh_get_census(self.h, C.byref(n), None, None, None, None, None, None,
                                    None), "slh_get_census")
        k = n.value
        arrs = dict(x=np.zeros(k), y=np.zeros(k), ox=np.zeros(k), oy=np.zeros(k),
                    w=np.zeros(k), cell=np.zeros(k, dtype=np.int32),
                    hid=np.zeros(k, dtype=np.uint64))
        if k:
            _check(lib().slh_get_census(self.h, C.byref(n), *(arrs[f].ctypes.data for f in
                                                              ("x", "y", "ox", "oy", "w",
                                                               "cell", "hid"))),
                   "slh_get_census")
        return arrs

    get_census = slh_get_census

    def slh_save(self) -> bytes:
        ln = C.c_size_t(0)
        _check(lib().slh_save(self.h, None, C.byref(ln)), "slh_save")
        buf = C.create_string_buffer(ln.value)
        _check(lib().slh_save(self.h, buf, C.byref(ln)), "slh_save")
        return buf.raw[:ln.value]

    save = slh_save

    def slh_load(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        _check(lib().slh_load(self.h, buf, len(data)), "slh_load")

    load = slh_load

    def slh_destroy(self):
        if getattr(self, "h", None):
            lib().slh_destroy(self.h)
            self.h = None

    destroy = slh_destroy

    def __del__(self):
        try:
            self.slh_destroy()
        except Exception:
            pass


def torch_stream_obj():
    import torch
    return torch.cuda.current_stream()


def slh_qmc_points(seed, step, pss, population, cohort, dim0, n_dims, index0, n, points=0):
    """Point words from the device generator as a numpy array [n, n_dims]."""
    import torch
    out = torch.empty(max(1, n * n_dims), dtype=torch.int32, device="cuda")
    _check(lib().slh_qmc_points(seed & (2 ** 64 - 1), step, pss, population, cohort, dim0,
                                n_dims, index0, n, points, C.c_void_p(out.data_ptr()),
                                C.c_void_p(_torch_stream())), "slh_qmc_points")
    torch.cuda.synchronize()
    return out[: n * n_dims].cpu().numpy().view(np.uint32).reshape(n, n_dims)


class Server:
    """Continuous-batching server (slh_server_*)."""

    def __init__(self, hbm_budget_bytes=0, max_slots=0, n_streams=0):
        cfg = slh_server_cfg(hbm_budget_bytes, max_slots, n_streams)
        h = C.c_void_p()
        _check(lib().slh_server_create(C.byref(cfg), C.byref(h)), "slh_server_create")
        self.h = h
        self._keep = {}

    def slh_server_submit(self, problem: dict, n_steps: int) -> int:
        st, keep = make_problem(problem)
        t = C.c_uint64(0)
        _check(lib().slh_server_submit(self.h, C.byref(st), int(n_steps), C.byref(t)),
               "slh_server_submit")
        self._keep[t.value] = (problem["nx"] * problem["ny"])
        return t.value

    submit = slh_server_submit

    def slh_server_poll(self, ticket: int) -> bool:
        d = C.c_int32(0)
        _check(lib().slh_server_poll(self.h, ticket, C.byref(d)), "slh_server_poll")
        return bool(d.value)

    poll = slh_server_poll

    def slh_server_result(self, ticket: int):
        n = self._keep.pop(ticket)
        flux = np.zeros(n)
        bal = slh_balance()
        lat = slh_latency()
        _check(lib().slh_server_result(self.h, ticket, flux.ctypes.data, C.byref(bal),
                                       C.byref(lat)), "slh_server_result")
        return flux, bal.as_dict(), lat.as_dict()

    result = slh_server_result

    def slh_server_destroy(self):
        if getattr(self, "h", None):
            lib().slh_server_destroy(self.h)
            self.h = None

    destroy = slh_server_destroy

    def __del__(self):
        try:
            self.slh_server_destroy()
        except Exception:
            pass
