"""CPU oracle for the scatter-limited hybrid (Q)MC / DG-S_N method.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the device library never imports,
links or runs anything here, and this module never touches the device library.

The heavy loops live in ``slh_oracle.c`` (plain sequential C, FP64,
``-ffp-contract=off``).  This module
  * builds and loads that C file,
  * obtains the Sobol' direction numbers through scipy's public API
    (``scipy.stats.qmc.Sobol``, Joe & Kuo numbers) -- the oracle's own
    extraction, independent of the device library's,
  * obtains the Gauss-Legendre polar nodes from ``numpy.polynomial.legendre``,
  * and drives one time step as steps 1-4 of Sec. 2.2 of the paper:
      1. scatter-limited (Q)MC leg (<= N_s scatters, pre/post tallies),
      2. DG S_N collided solve with source sigma_s/(4 pi) phi_post (or a
         cell-centred diffusion solve, the alternative closing stage),
      3. remap: scatter-free (Q)MC from Q + sigma_s (phi_pre + phi_post + phi_c),
      4. the remap census is the state at t_{n+1}.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99",
          "-D_GNU_SOURCE"]


_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the C oracle into oracle/liboracle.so (gcc); sanitize: into
    oracle/liboracle_san.so with AddressSanitizer and UBSan.  With
    SLH_ORACLE_SANITIZED=1 in the environment the sanitized build is the one
    loaded (the process must then preload the gcc sanitizer runtimes)."""
    if os.environ.get("SLH_ORACLE_SANITIZED") == "1":
        sanitize = True
    out = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, *(SAN_FLAGS if sanitize else []), _SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, out)
    return out


class _Mesh(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int),
                ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("y_lo", C.c_double), ("y_hi", C.c_double),
                ("sig_s", C.c_void_p), ("sig_a", C.c_void_p),
                ("c", C.c_double), ("dt", C.c_double), ("ns_cell", C.c_void_p),
                ("bc", C.c_int), ("steady", C.c_int), ("horizon", C.c_double),
                ("census_qmc", C.c_int), ("inflow", C.c_void_p)]


class _Points(C.Structure):
    _fields_ = [("mode", C.c_int), ("sobol_dims", C.c_int), ("V", C.c_void_p)]


class _BankIn(C.Structure):
    _fields_ = [("n_in", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("ox", C.c_void_p), ("oy", C.c_void_p),
                ("w", C.c_void_p), ("cell", C.c_void_p), ("hid", C.c_void_p)]


class _BankOut(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("ox", C.c_void_p), ("oy", C.c_void_p),
                ("w", C.c_void_p), ("cell", C.c_void_p), ("hid", C.c_void_p),
                ("alive", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.or_mix64.restype = C.c_uint64
        L.or_mix64.argtypes = [C.c_uint64]
        L.or_stream_seed.restype = C.c_uint64
        L.or_stream_seed.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64]
        L.or_nested_scramble.restype = C.c_uint32
        L.or_nested_scramble.argtypes = [C.c_uint32, C.c_uint32]
        L.or_sobol_word.restype = C.c_uint32
        L.or_sobol_word.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32]
        L.or_point_u32.restype = C.c_uint32
        L.or_point_u32.argtypes = [C.POINTER(_Points), C.c_uint64, C.c_uint32, C.c_uint32]
        L.or_u01.restype = C.c_double
        L.or_u01.argtypes = [C.c_uint32]
        L.or_mc_pass.restype = C.c_int64
        L.or_mc_pass.argtypes = [C.POINTER(_Mesh), C.POINTER(_Points), C.c_int, C.c_int,
                                 C.c_void_p, C.c_void_p, C.c_double, C.POINTER(_BankIn),
                                 C.c_uint64,
                                 C.c_uint64, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.POINTER(_BankOut)]
        L.or_thin.restype = C.c_int64
        L.or_thin.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64,
                              C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.or_thin_prob.restype = None
        L.or_thin_prob.argtypes = [C.c_int64, C.c_int64, C.POINTER(C.c_double),
                                   C.POINTER(C.c_int), C.POINTER(C.c_uint64)]
        L.or_pow2_ceil.restype = C.c_double
        L.or_pow2_ceil.argtypes = [C.c_double]
        L.or_face_majorants.restype = None
        L.or_face_majorants.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double,
                                        C.c_double, C.c_void_p]
        L.or_cell_majorants.restype = None
        L.or_cell_majorants.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_void_p]
        L.or_halton_u32.restype = C.c_uint32
        L.or_halton_u32.argtypes = [C.c_uint32, C.c_uint32]
        L.or_quantum.restype = C.c_double
        L.or_quantum.argtypes = [C.c_double]
        L.or_emission_counts.restype = C.c_int64
        L.or_emission_counts.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.c_int64,
                                         C.POINTER(_Points), C.c_uint64, C.c_uint64, C.c_int,
                                         C.c_void_p, C.POINTER(C.c_double)]
        L.or_history_id.restype = C.c_uint64
        L.or_history_id.argtypes = [C.c_uint64, C.c_int64, C.c_uint32]
        L.or_dg_sweep.restype = C.c_int
        L.or_dg_sweep.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_dg_one_iteration.restype = C.c_int
        L.or_dg_one_iteration.argtypes = [C.POINTER(_Mesh), C.c_void_p, C.c_int, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p]
        L.or_dg_sigma_e.restype = None
        L.or_dg_sigma_e.argtypes = [C.POINTER(_Mesh), C.c_double, C.c_void_p]
        L.or_dg_collided.restype = C.c_int
        L.or_dg_collided.argtypes = [C.POINTER(_Mesh), C.c_double, C.c_int, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                     C.c_void_p, C.POINTER(C.c_double)]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# ----------------------------------------------------------------------------
# Point generator inputs
# ----------------------------------------------------------------------------

SOBOL_DIMS = 32
_dirs_cache = {}


_N_READ = 20


def _sobol_recurrence_fit(v):
    """Find the degree s and inner coefficients a_1..a_{s-1} of the primitive
    polynomial for which the Sobol' recurrence on 32-bit words,
        v_k = a_1 v_{k-1} ^ ... ^ a_{s-1} v_{k-s+1} ^ v_{k-s} ^ (v_{k-s} >> s),
    reproduces every word v_s..v_{n-1} given; None if no (s, a) does."""
    n = len(v)
    for s in range(1, n - 4):
        for a in range(1 << (s - 1)):
            ok = True
            for k in range(s, n):
                x = v[k - s] ^ (v[k - s] >> s)
                for i in range(1, s):
                    if (a >> (s - 1 - i)) & 1:
                        x ^= v[k - i]
                if x != v[k]:
                    ok = False
                    break
            if ok:
                return s, a
    return None


def sobol_direction_numbers(ndim: int = SOBOL_DIMS) -> np.ndarray:
    """Direction numbers v[d][j] (32-bit words, bit 31 = first digit) of
    scipy's unscrambled Sobol' sequence (Joe & Kuo numbers).

    scipy enumerates in Gray-code order, so its point number 2^(j+1) - 1 is the
    single direction number v_j.  scipy's fast_forward is linear in the skip,
    so v_0..v_19 are read off the points and the rest follow from the Sobol'
    recurrence of each dimension's primitive polynomial, which is identified
    from the words read (dimension 0 is the van der Corput identity)."""
    if ndim in _dirs_cache:
        return _dirs_cache[ndim]
    from scipy.stats import qmc
    V = np.zeros((ndim, 32), dtype=np.uint32)
    for j in range(_N_READ):
        s = qmc.Sobol(d=ndim, scramble=False, bits=32)
        s.fast_forward(2 ** (j + 1) - 1)
        V[:, j] = np.rint(s.random(1)[0] * 2.0 ** 32).astype(np.uint64).astype(np.uint32)
    for j in range(32):
        if j >= _N_READ:
            V[0, j] = np.uint32(1 << (31 - j))
        elif int(V[0, j]) != 1 << (31 - j):
            raise RuntimeError("dimension 0 is not the van der Corput sequence")
    for d in range(1, ndim):
        v = [int(x) for x in V[d, :_N_READ]]
        fit = _sobol_recurrence_fit(v)
        if fit is None:
            raise RuntimeError("no Sobol' recurrence reproduces dimension %d" % d)
        s, a = fit
        for k in range(_N_READ, 32):
            x = v[k - s] ^ (v[k - s] >> s)
            for i in range(1, s):
                if (a >> (s - 1 - i)) & 1:
                    x ^= v[k - i]
            v.append(x)
        V[d, :] = np.array(v, dtype=np.uint64).astype(np.uint32)
    _dirs_cache[ndim] = V
    return V


class Points:
    """The oracle's point function P(stream, dim, index) -> uint32."""

    def __init__(self, mode: int = 0, ndim: int = SOBOL_DIMS):
        self.V = np.ascontiguousarray(sobol_direction_numbers(ndim))
        self.s = _Points(mode, ndim, _p(self.V))

    def u32(self, stream: int, dim: int, index: int) -> int:
        return lib().or_point_u32(C.byref(self.s), stream, dim, index)

    def block(self, stream: int, dims, indices) -> np.ndarray:
        out = np.zeros((len(indices), len(dims)), dtype=np.uint32)
        L = lib()
        for a, k in enumerate(indices):
            for b, d in enumerate(dims):
                out[a, b] = L.or_point_u32(C.byref(self.s), stream, d, int(k))
        return out


def stream_seed(seed, step, pss, pop, cohort=0) -> int:
    return lib().or_stream_seed(seed, step, pss, pop, cohort)


# ----------------------------------------------------------------------------
# Angular quadrature (product S_N: Gauss-Legendre polar levels x equal azimuths)
# ----------------------------------------------------------------------------

def quadrature(order: int):
    """Product set for x-y geometry: the N/2 positive Gauss-Legendre nodes of
    order N for Oz (weights doubled for the mirrored -Oz, which has the same
    in-plane components) times 2N equally spaced azimuths (m + 1/2) pi / N.
    Returns (ox, oy, w), N^2 directions, sum(w) = 4 pi."""
    if order < 2 or order % 2:
        raise ValueError("S_N order must be even and >= 2")
    mu, a = np.polynomial.legendre.leggauss(order)
    sel = mu > 0
    mu, a = mu[sel], a[sel]
    naz = 2 * order
    phi = (np.arange(naz) + 0.5) * np.pi / order
    ox, oy, w = [], [], []
    for k in range(len(mu)):
        s = np.sqrt(1.0 - mu[k] ** 2)
        for m in range(naz):
            ox.append(s * np.cos(phi[m]))
            oy.append(s * np.sin(phi[m]))
            w.append(2.0 * a[k] * np.pi / order)
    return np.array(ox), np.array(oy), np.array(w)


# ----------------------------------------------------------------------------
# Passes and solves
# ----------------------------------------------------------------------------

BAL_NAMES = ["emitted", "absorbed", "scattered", "leaked", "census", "cutoff",
             "source_w", "census_in_w"]


class Bank:
    """Census bank (SoA), particles at the start of a step."""

    def __init__(self, n=0):
        self.x = np.zeros(n); self.y = np.zeros(n)
        self.ox = np.zeros(n); self.oy = np.zeros(n); self.w = np.zeros(n)
        self.cell = np.zeros(n, dtype=np.int32)
        self.hid = np.zeros(n, dtype=np.uint64)

    @property
    def n(self):
        return len(self.w)

    def take(self, idx, factor=1.0):
        b = Bank(0)
        for f in ("x", "y", "ox", "oy", "w", "cell", "hid"):
            setattr(b, f, np.ascontiguousarray(getattr(self, f)[idx]))
        b.w = b.w * factor
        return b


class Mesh:
    def __init__(self, prob):
        self.nx, self.ny = int(prob["nx"]), int(prob["ny"])
        self.x_lo, self.x_hi, self.y_lo, self.y_hi = (float(prob[k]) for k in
                                                      ("x_lo", "x_hi", "y_lo", "y_hi"))
        self.sig_s = np.ascontiguousarray(prob["sigma_s"], dtype=np.float64).ravel()
        self.sig_a = np.ascontiguousarray(prob["sigma_a"], dtype=np.float64).ravel()
        self.c = float(prob.get("c", 1.0))
        self.dt = float(prob.get("dt", 0.0))
        # steady state (one infinite time step): histories end at a path
        # horizon, by default ln(1/w_cut_rel) / min sigma_a, the length after
        # which every weight is below the cutoff
        self.steady = bool(prob.get("steady", False))
        self.horizon = float(prob.get("horizon", 0.0))
        if self.steady and not self.horizon > 0.0:
            if not np.min(self.sig_a) > 0.0:
                raise ValueError("steady state with sigma_a = 0 somewhere needs a horizon")
            self.horizon = math.log(1.0 / float(prob.get("w_cut_rel", 1e-8))) / float(
                np.min(self.sig_a))
        ns = prob.get("n_s_cell")
        self.ns_cell = None if ns is None else np.ascontiguousarray(ns, dtype=np.int32).ravel()
        self.bc = int(prob.get("boundary", 0))  # reflective sides: 1 x_lo, 2 x_hi, 4 y_lo, 8 y_hi
        # prescribed isotropic inflow G on the boundary faces (Sec. 2.1):
        # 2 ny + 2 nx values, x_lo faces, x_hi faces, y_lo faces, y_hi faces
        g = prob.get("inflow")
        self.inflow = None if g is None else np.ascontiguousarray(g, dtype=np.float64).ravel()
        if self.inflow is not None:
            ny_, nx_ = self.ny, self.nx
            if self.inflow.size != 2 * (nx_ + ny_):
                raise ValueError("inflow needs 2 (nx + ny) values")
            sides = (self.inflow[:ny_], self.inflow[ny_:2 * ny_], self.inflow[2 * ny_:2 * ny_ + nx_],
                     self.inflow[2 * ny_ + nx_:])
            for bit, v in zip((1, 2, 4, 8), sides):
                if (self.bc & bit) and np.any(v != 0.0):
                    raise ValueError("inflow on a reflective side")
        self.s = _Mesh(self.nx, self.ny, self.x_lo, self.x_hi, self.y_lo, self.y_hi,
                       _p(self.sig_s), _p(self.sig_a), self.c, self.dt,
                       None if self.ns_cell is None else _p(self.ns_cell), self.bc,
                       int(self.steady), self.horizon, int(prob.get("census_qmc", 0)),
                       None if self.inflow is None else _p(self.inflow))
        self.ncell = self.nx * self.ny
        self.area = ((self.x_hi - self.x_lo) / self.nx) * ((self.y_hi - self.y_lo) / self.ny)
        # tallies per unit time (steady) or per step: phi = T / adt
        self.adt = self.area if self.steady else self.area * self.dt
        self.hx = (self.x_hi - self.x_lo) / self.nx
        self.hy = (self.y_hi - self.y_lo) / self.ny
        self.tdt = 1.0 if self.steady else self.dt


def mc_pass(mesh: Mesh, pts: Points, kind: int, n_s: int, q_nodal, n_src: int,
            bank: Bank, seed: int, step: int, w_cut_rel: float, want_census: bool):
    """One (Q)MC pass (Sec. 2.3) emitting the plan of ``emission_plan``.
    Returns (T_a, T_b, balance dict, segments, census-out candidates or None).
    T are raw track-length sums."""
    q_nodal = np.ascontiguousarray(q_nodal, dtype=np.float64).reshape(-1)
    assert q_nodal.size == 4 * mesh.ncell
    plan = emission_plan(q_nodal, mesh.adt, n_src, pts, seed, step, kind, mesh)
    counts = np.ascontiguousarray(plan["counts"], dtype=np.int64)
    if counts.size == 0:
        counts = np.zeros(1, dtype=np.int64)
    Ta = np.zeros(mesh.ncell); Tb = np.zeros(mesh.ncell); bal = np.zeros(len(BAL_NAMES))
    bin_ = _BankIn(bank.n, _p(bank.x), _p(bank.y), _p(bank.ox), _p(bank.oy), _p(bank.w),
                   _p(bank.cell), _p(bank.hid))
    out = None
    bout_p = None
    if want_census:
        ncand = bank.n + plan["n_emit"]
        out = Bank(ncand)
        out.alive = np.zeros(ncand, dtype=np.uint8)
        bout = _BankOut(_p(out.x), _p(out.y), _p(out.ox), _p(out.oy), _p(out.w),
                        _p(out.cell), _p(out.hid), _p(out.alive))
        bout_p = C.byref(bout)
    seg = lib().or_mc_pass(C.byref(mesh.s), C.byref(pts.s), kind, n_s, _p(q_nodal),
                           _p(counts), plan["w_q"], C.byref(bin_), seed, step, w_cut_rel,
                           _p(Ta), _p(Tb), _p(bal), bout_p)
    balance = dict(zip(BAL_NAMES, bal))
    balance.update(majorant_sum=plan["total"], weight_quantum=plan["w_q"],
                   source_particles=plan["n_emit"])
    return Ta, Tb, balance, int(seg), out


def cell_majorants(q_nodal, adt):
    """M_i = adt * (largest corner |q_i| rounded up to a power of two)."""
    q_nodal = np.ascontiguousarray(q_nodal, dtype=np.float64).reshape(-1)
    n = q_nodal.size // 4
    M = np.zeros(max(n, 1))
    lib().or_cell_majorants(_p(q_nodal), n, adt, _p(M))
    return M[:n]


def face_majorants(mesh: "Mesh"):
    """M_f of the boundary faces with an inflow (see slh_oracle.c:
    or_face_majorants), or an empty array."""
    if mesh.inflow is None:
        return np.zeros(0)
    M = np.zeros(mesh.inflow.size)
    lib().or_face_majorants(_p(mesh.inflow), mesh.nx, mesh.ny, mesh.hx, mesh.hy, mesh.tdt,
                            _p(M))
    return M


def emission_plan(q_nodal, adt, n_src, pts: Points, seed: int, step: int, kind: int,
                  mesh: "Mesh" = None):
    """The source particles of one pass (Sec. 2.3, birth in proportion to the
    source; with an inflow also the particles entering through the boundary,
    Sec. 2.1): the emitters' majorants M_i (the cells, then the boundary
    faces), their correctly rounded sum (math.fsum), the weight quantum
    w_q = quantum(sum / n_src) and the counts floor(M_i / w_q) +
    [u_i < frac(M_i / w_q)] (see slh_oracle.c: or_emission_counts)."""
    M = cell_majorants(q_nodal, adt)
    if mesh is not None and mesh.inflow is not None:
        M = np.concatenate([M, face_majorants(mesh)])
    total = math.fsum(M.tolist())
    counts = np.zeros(max(M.size, 1), dtype=np.int64)
    wq = C.c_double(0.0)
    n_emit = lib().or_emission_counts(_p(np.ascontiguousarray(M)), M.size, total, n_src,
                                      C.byref(pts.s), seed, step, kind, _p(counts),
                                      C.byref(wq))
    return dict(M=M, total=total, w_q=wq.value, counts=counts[:M.size], n_emit=int(n_emit))


def history_id(step: int, cell: int, l: int) -> int:
    return int(lib().or_history_id(step, cell, l))


def thin(cand: Bank, cap: int, thin_stream: int):
    """Census population control (see slh_oracle.c: or_thin).  Returns the
    kept bank, the weight factor and the overflow flag.  The bank at t_{n+1}
    holds the kept candidates ordered by cell, those of one cell in slot
    order: the census cohorts of the next step (each cell's census particles
    take the points of that cell's census stream in this order)."""
    keep = np.zeros(cand.n, dtype=np.uint8)
    fac = C.c_double(1.0)
    ovf = C.c_int(0)
    lib().or_thin(cand.n, _p(cand.alive), _p(cand.hid), cap, thin_stream, _p(keep),
                  C.byref(fac), C.byref(ovf))
    idx = np.nonzero(keep)[0]
    idx = idx[np.argsort(cand.cell[idx], kind="stable")]
    return cand.take(idx, fac.value), fac.value, bool(ovf.value)


def thin_prob(count: int, cap: int):
    p = C.c_double(0.0)
    sh = C.c_int(0)
    mant = C.c_uint64(0)
    lib().or_thin_prob(count, cap, C.byref(p), C.byref(sh), C.byref(mant))
    return p.value, sh.value, mant.value


def dg_sweep(nx, ny, box, sig_e, a, b, src, in_x=None, in_y=None):
    psi = np.zeros(4 * nx * ny)
    sig_e = np.ascontiguousarray(sig_e, dtype=np.float64)
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1)
    in_x = None if in_x is None else np.ascontiguousarray(in_x, dtype=np.float64)
    in_y = None if in_y is None else np.ascontiguousarray(in_y, dtype=np.float64)
    rc = lib().or_dg_sweep(nx, ny, box[0], box[1], box[2], box[3], _p(sig_e), a, b,
                           _p(src), _p(in_x), _p(in_y), _p(psi))
    if rc != 0:
        raise RuntimeError("singular DG cell system")
    return psi.reshape(ny, nx, 4)


def mirror_indices(quad):
    """For each direction, the index of its mirror image in x (Ox -> -Ox) and
    in y (Oy -> -Oy) within the same set."""
    ox, oy, _ = quad
    n = len(ox)
    rx, ry = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
    for m in range(n):
        rx[m] = int(np.argmin(np.abs(ox + ox[m]) + np.abs(oy - oy[m])))
        ry[m] = int(np.argmin(np.abs(ox - ox[m]) + np.abs(oy + oy[m])))
        assert abs(ox[rx[m]] + ox[m]) + abs(oy[rx[m]] - oy[m]) < 1e-12
        assert abs(ox[ry[m]] - ox[m]) + abs(oy[ry[m]] + oy[m]) < 1e-12
    return rx, ry


def dg_collided(mesh: Mesh, quad, phi_post, tau=2.0, tol=1e-12, max_iter=200, phi_pre=None):
    """Source iteration for the collided flux (see slh_oracle.c: or_dg_collided);
    with phi_pre the stopping test is relative to phi_c + phi_pre + phi_post."""
    ox, oy, w = (np.ascontiguousarray(v, dtype=np.float64) for v in quad)
    rx, ry = mirror_indices((ox, oy, w))
    phi = np.zeros(4 * mesh.ncell)
    res = C.c_double(0.0)
    phi_post = np.ascontiguousarray(phi_post, dtype=np.float64)
    phi_pre = None if phi_pre is None else np.ascontiguousarray(phi_pre, dtype=np.float64)
    it = lib().or_dg_collided(C.byref(mesh.s), tau, len(w), _p(ox), _p(oy), _p(w), _p(rx),
                              _p(ry), _p(phi_post), _p(phi_pre), tol, max_iter, _p(phi),
                              C.byref(res))
    if it < 0:
        raise RuntimeError("DG sweep failed")
    return phi.reshape(mesh.ncell, 4), it, res.value


def diffusion_matrix(mesh: Mesh, tau=2.0, vacuum_sides=False):
    """Cell-centred finite-volume diffusion operator of the collided flux, the
    alternative closing stage (a P1 reading of the collided equation with the
    step closure of the S_N stage):
        (sigma_a + tau/(c dt)) phi_c - div(D grad phi_c) = sigma_s phi_post,
        D = 1 / (3 (sigma_t + tau/(c dt)))   (no tau/(c dt) in steady state).
    Interior faces carry D_f (phi_i - phi_j)/h with the harmonic mean
    D_f = 2 D_i D_j / (D_i + D_j); a vacuum side has zero incoming partial
    current (Marshak), which gives the outflow 2 D_i phi_i / (h + 4 D_i) per
    unit face length; a reflective side has none (vacuum_sides: every side
    takes the vacuum condition).  Returns the sparse matrix (per unit cell
    area, so that A phi = sigma_s phi_post)."""
    from scipy.sparse import lil_matrix
    nx, ny = mesh.nx, mesh.ny
    hx = (mesh.x_hi - mesh.x_lo) / nx
    hy = (mesh.y_hi - mesh.y_lo) / ny
    tt = 0.0 if mesh.steady else tau / (mesh.c * mesh.dt)
    A = lil_matrix((nx * ny, nx * ny))
    for j in range(ny):
        for i in range(nx):
            k = j * nx + i
            sr = mesh.sig_a[k] + tt
            D = 1.0 / (3.0 * (mesh.sig_a[k] + mesh.sig_s[k] + tt))
            A[k, k] += sr
            for di, dj, h, side in ((-1, 0, hx, 1), (1, 0, hx, 2), (0, -1, hy, 4), (0, 1, hy, 8)):
                ii, jj = i + di, j + dj
                if 0 <= ii < nx and 0 <= jj < ny:
                    kk = jj * nx + ii
                    Dn = 1.0 / (3.0 * (mesh.sig_a[kk] + mesh.sig_s[kk] + tt))
                    c = 2.0 * D * Dn / (D + Dn) / (h * h)
                    A[k, k] += c
                    A[k, kk] -= c
                elif vacuum_sides or not (mesh.bc & side):
                    A[k, k] += 2.0 * D / (h * (h + 4.0 * D))
    return A.tocsr()


def diffusion_exact(mesh: Mesh, phi_post, tau=2.0):
    """The exact solution of the diffusion closing stage's finite-volume
    system (a sparse direct solve), per cell."""
    from scipy.sparse.linalg import spsolve
    A = diffusion_matrix(mesh, tau)
    b = mesh.sig_s * np.asarray(phi_post, dtype=np.float64).ravel()
    return np.asarray(spsolve(A, b)) if np.any(b != 0.0) else np.zeros(mesh.ncell)


def diffusion_collided(mesh: Mesh, phi_post, tau=2.0, tol=1e-12, max_iter=200):
    """The collided flux of the diffusion closing stage as the method computes
    it: Jacobi-preconditioned conjugate gradients on the finite-volume system
    from phi = 0, stopping after the first iteration with
    ||r||_2 <= tol ||b||_2 (or at max_iter).  Returns nodal values (equal at
    the four nodes of a cell, like the DG solution), the iteration count and
    ||r|| / ||b||.  (The iterate agrees with diffusion_exact to about
    cond(A) tol in norm; in cells where the flux is many orders below its
    peak only the iteration itself fixes the low digits.)"""
    A = diffusion_matrix(mesh, tau)
    b = mesh.sig_s * np.asarray(phi_post, dtype=np.float64).ravel()
    x, it, resid = _pcg(A, b, tol, max_iter)
    return np.repeat(x.reshape(-1, 1), 4, axis=1), it, resid


def _pcg(A, b, tol, max_iter):
    """Jacobi-preconditioned conjugate gradients from x = 0, stopping after the
    first iteration with ||r||_2 <= tol ||b||_2 (or at max_iter).  Returns
    x, the iteration count and ||r|| / ||b||."""
    d = A.diagonal()
    x = np.zeros(len(b))
    bb = float(b @ b)
    it, rr = 0, bb
    if bb > 0.0 and max_iter > 0:
        r = b.copy()
        z = r / d
        p = z.copy()
        rz = float(r @ z)
        while True:
            q = A @ p
            alpha = rz / float(p @ q)
            x = x + alpha * p
            r = r - alpha * q
            z = r / d
            rz_new = float(r @ z)
            rr = float(r @ r)
            it += 1
            if rr <= tol * tol * bb or it >= max_iter or not np.isfinite(rr):
                break
            p = z + (rz_new / rz) * p
            rz = rz_new
    return x, it, (math.sqrt(rr / bb) if bb > 0.0 else 0.0)


DSA_TOL, DSA_MAX_ITER = 1e-2, 32


def dg_collided_dsa(mesh: Mesh, quad, phi_post, tau=2.0, tol=1e-12, max_iter=200,
                    phi_pre=None):
    """Source iteration with diffusion synthetic acceleration: after each
    transport sweep (phi^{k+1/2}), the correction delta solves the diffusion
    system of diffusion_matrix for the source sigma_s times the cell average
    of phi^{k+1/2} - phi^k (conjugate gradients to DSA_TOL, at most
    DSA_MAX_ITER steps), and phi^{k+1} = phi^{k+1/2} + delta at every node of
    the cell.  The correction takes the vacuum condition on every side: the
    sweep's reflected inflow lags one iteration, and a zero-current condition
    there makes the corrected iteration diverge (a closed box does).  The
    stopping test is that of dg_collided, on phi^{k+1} - phi^k.  Returns (phi
    nodal, sweeps, residual)."""
    ox, oy, w = (np.ascontiguousarray(v, dtype=np.float64) for v in quad)
    rx, ry = mirror_indices((ox, oy, w))
    n, nd = mesh.ncell, len(w)
    sig_e = np.zeros(n)
    lib().or_dg_sigma_e(C.byref(mesh.s), tau, _p(sig_e))
    if not np.all(sig_e > 0.0):
        raise ValueError("the diffusion correction needs sigma_t + tau/(c dt) > 0 everywhere")
    out_x = np.zeros(nd * 2 * mesh.ny)
    out_y = np.zeros(nd * 2 * mesh.nx)
    A = diffusion_matrix(mesh, tau, vacuum_sides=True)
    phi_post = np.ascontiguousarray(phi_post, dtype=np.float64)
    phi = np.zeros(4 * n)
    it, resid = 0, 0.0
    while it < max_iter:
        acc = np.zeros(4 * n)
        if lib().or_dg_one_iteration(C.byref(mesh.s), _p(sig_e), nd, _p(ox), _p(oy), _p(w),
                                     _p(rx), _p(ry), _p(phi_post), _p(phi), _p(out_x),
                                     _p(out_y), _p(acc)) != 0:
            raise RuntimeError("DG sweep failed")
        it += 1
        dnode = (acc - phi).reshape(n, 4)
        b = mesh.sig_s * (0.25 * ((dnode[:, 0] + dnode[:, 1]) + (dnode[:, 2] + dnode[:, 3])))
        delta, _, _ = _pcg(A, b, DSA_TOL, DSA_MAX_ITER)
        new = acc.reshape(n, 4) + delta[:, None]
        d = dnode + delta[:, None]
        ref = new if phi_pre is None else new + (phi_pre + phi_post)[:, None]
        dn = math.sqrt(float(np.sum(d * d)))
        nrm = math.sqrt(float(np.sum(ref * ref)))
        phi = new.ravel()
        resid = dn / nrm if nrm > 0.0 else 0.0
        if dn <= tol * nrm:
            break
    return phi.reshape(n, 4), it, resid


# ----------------------------------------------------------------------------
# Time stepping (Sec. 2.2, steps 1-4)
# ----------------------------------------------------------------------------

PASS_MC, PASS_REMAP = 1, 2
POP_SOURCE, POP_CENSUS, POP_THIN = 0, 1, 2


class HybridOracle:
    """Plain sequential hybrid solver, one call to ``step`` per time step."""

    def __init__(self, prob: dict):
        self.prob = prob
        self.mesh = Mesh(prob)
        self.q = np.ascontiguousarray(prob["q"], dtype=np.float64).ravel()
        self.n_s = int(prob["n_s"])
        self.n_p = int(prob["n_particles"])
        self.cap = int(prob.get("census_cap", 0)) or self.n_p
        self.seed = int(prob.get("seed", 0)) & (2 ** 64 - 1)
        self.tau = float(prob.get("time_closure", 2.0))
        self.si_tol = float(prob.get("si_tol", 1e-12))
        self.si_max = int(prob.get("si_max_iter", 200))
        self.w_cut_rel = float(prob.get("w_cut_rel", 1e-8))
        self.si_norm_total = int(prob.get("si_norm", 0)) == 1
        self.diffusion = int(prob.get("closure", 0)) == 1
        self.dsa = not self.diffusion and int(prob.get("si_accel", 0)) == 1
        ns = prob.get("n_s_cell")
        # steady pure MC (no limit in any cell): no collided solve, no remap
        # (Sec. 3: relabeling is unnecessary there), phi_R = phi_pre
        self.skip_remap = self.mesh.steady and (
            self.n_s < 0 if ns is None else bool(np.all(np.asarray(ns) < 0)))
        self.points = Points(int(prob.get("points", 0)))
        self.quad = quadrature(int(prob["sn_order"]))
        self.bank = Bank(0)
        self.step_index = 0

    def step(self) -> dict:
        m = self.mesh
        n = self.step_index
        adt = m.adt
        q4 = np.repeat(self.q, 4)
        # step 1: scatter-limited leg from Q and the census (initial data)
        Tpre, Tpost, bal1, seg1, _ = mc_pass(m, self.points, PASS_MC, self.n_s, q4, self.n_p,
                                             self.bank, self.seed, n, self.w_cut_rel, False)
        phi_pre, phi_post = Tpre / adt, Tpost / adt
        if self.skip_remap:
            self.step_index += 1
            zero = dict(zip(BAL_NAMES, np.zeros(len(BAL_NAMES))))
            return dict(step=n, phi_R=phi_pre.copy(), phi_pre=phi_pre, phi_post=phi_post,
                        phi_c=np.zeros((m.ncell, 4)), T_pre=Tpre, T_post=Tpost, T_R=Tpre.copy(),
                        bal_mc=bal1, bal_remap=zero, segments=seg1, seg_mc=seg1, seg_remap=0,
                        si_iters=0, si_resid=0.0, census_alive=0, census_kept=0,
                        thin_factor=1.0, thin_overflow=False, q_remap=None)
        # step 2: collided S_N-DG solve, zero initial/boundary data (or the
        # diffusion closing stage by conjugate gradients)
        if self.diffusion:
            phi_c, iters, resid = diffusion_collided(m, phi_post, self.tau, self.si_tol,
                                                     self.si_max)
        else:
            solve = dg_collided_dsa if self.dsa else dg_collided
            phi_c, iters, resid = solve(m, self.quad, phi_post, self.tau, self.si_tol,
                                        self.si_max, phi_pre if self.si_norm_total else None)
        # step 3: remap source Q + sigma_s (phi_pre + phi_post + phi_c), scatter-free leg
        qR = (self.q + m.sig_s * (phi_pre + phi_post))[:, None] + m.sig_s[:, None] * phi_c
        _, TR, bal2, seg2, cand = mc_pass(m, self.points, PASS_REMAP, self.n_s, qR, self.n_p,
                                          self.bank, self.seed, n, self.w_cut_rel,
                                          not m.steady)
        # step 4: the remap census is the state at t_{n+1} (capped); steady
        # state carries none (the weight at the horizon is only booked)
        if m.steady:
            n_alive, factor, overflow = 0, 1.0, False
            self.bank = Bank(0)
        else:
            thin_stream = stream_seed(self.seed, n, PASS_REMAP, POP_THIN, 0)
            n_alive = int(cand.alive.sum())
            self.bank, factor, overflow = thin(cand, self.cap, thin_stream)
        self.step_index += 1
        return dict(step=n, phi_R=TR / adt, phi_pre=phi_pre, phi_post=phi_post, phi_c=phi_c,
                    T_pre=Tpre, T_post=Tpost, T_R=TR, bal_mc=bal1, bal_remap=bal2,
                    segments=seg1 + seg2, seg_mc=seg1, seg_remap=seg2, si_iters=iters,
                    si_resid=resid, census_alive=n_alive, census_kept=self.bank.n,
                    thin_factor=factor, thin_overflow=overflow, q_remap=qR)

    def run(self, n_steps: int):
        return [self.step() for _ in range(n_steps)]
