"""Seeded synthetic problem generators.

This module only builds inputs (mesh, cross-section and source fields, run
parameters) as plain numpy arrays; it holds none of the transport method's
arithmetic.  Both the device path and the CPU oracle consume its output.

The paper's own test problems (a 1-D slab benchmark and a 2-D duct problem)
are specified only in figures that are not available, so the configurations
below are synthetic stand-ins with the structure of a heterogeneous 2-D
transport problem: localised sources, absorber/scatterer contrasts, optically
thick regions with voids and random block materials, and for the steady
state a multi-region slab and a bent duct.

Fields are row-major with shape (ny, nx): cell (i, j) is element [j, i].
"""
from __future__ import annotations

import numpy as np

DEFAULTS = dict(c=1.0, time_closure=2.0, si_tol=1e-12, si_max_iter=200, w_cut_rel=1e-8,
                seed=20251116, points=0, precision=0, census_cap=0)


def _problem(nx, ny, box, sig_s, sig_a, q, **kw):
    p = dict(DEFAULTS)
    p.update(nx=nx, ny=ny, x_lo=box[0], x_hi=box[1], y_lo=box[2], y_hi=box[3],
             sigma_s=np.ascontiguousarray(sig_s, dtype=np.float64),
             sigma_a=np.ascontiguousarray(sig_a, dtype=np.float64),
             q=np.ascontiguousarray(q, dtype=np.float64))
    p.update(kw)
    return p


def homogeneous_box(n=20, L=2.0, sig_s=1.0, sig_a=0.1, src_cells=((9, 11), (9, 11)), **kw):
    """C1 family: homogeneous square with a central source block."""
    ss = np.full((n, n), sig_s)
    sa = np.full((n, n), sig_a)
    q = np.zeros((n, n))
    (i0, i1), (j0, j1) = src_cells
    q[j0:j1, i0:i1] = 1.0
    kw.setdefault("n_s", 0)
    kw.setdefault("n_particles", 10_000)
    kw.setdefault("dt", 0.1)
    kw.setdefault("n_steps", 10)
    kw.setdefault("sn_order", 8)
    return _problem(n, n, (0.0, L, 0.0, L), ss, sa, q, **kw)


def c1(**kw):
    """[0,2]^2, 20x20 cells, sigma_s = 1, sigma_a = 0.1, Q = 1 in the central
    2x2 cells, N_s = 0, 1e4 particles per pass, dt = 0.1, 10 steps, S_8."""
    return homogeneous_box(**kw)


def checkerboard(blocks=7, cells_per_block=20, n_s=2, **kw):
    """C2 family: blocks x blocks unit blocks; block (I, J) with I + J even is
    a pure scatterer (sigma_s = 1, sigma_a = 0), odd a pure absorber
    (sigma_a = 10, sigma_s = 0); unit source in the centre block."""
    n = blocks * cells_per_block
    I = np.arange(n) // cells_per_block
    even = ((I[None, :] + I[:, None]) % 2) == 0
    ss = np.where(even, 1.0, 0.0)
    sa = np.where(even, 0.0, 10.0)
    q = np.zeros((n, n))
    cb = blocks // 2
    sl = slice(cb * cells_per_block, (cb + 1) * cells_per_block)
    q[sl, sl] = 1.0
    kw.setdefault("n_particles", 1_000_000)
    kw.setdefault("dt", 0.05)
    kw.setdefault("n_steps", 40)
    kw.setdefault("sn_order", 12)
    return _problem(n, n, (0.0, float(blocks), 0.0, float(blocks)), ss, sa, q, n_s=n_s, **kw)


def c2(n_s=2, **kw):
    """7x7 checkerboard of unit blocks on 140x140 cells, N_s in {1, 2},
    1e6 particles per pass, dt = 0.05, 40 steps, S_12."""
    return checkerboard(n_s=n_s, **kw)


def thick_with_voids(n=256, L=10.0, n_s=0, void_frac=0.2, src_half=16, void_seed=7, **kw):
    """C3 family: optically thick diffusive medium (sigma_s = 100,
    sigma_a = 0.01) with seeded, cell-aligned rectangular voids (sigma_t = 0.1)
    added until they cover >= void_frac of the area; unit source on the
    central (2 src_half)^2 cells."""
    rng = np.random.default_rng(void_seed)
    void = np.zeros((n, n), dtype=bool)
    lo_side, hi_side = max(1, n // 64), max(2, n // 8)
    while void.mean() < void_frac:
        w, h = rng.integers(lo_side, hi_side + 1, size=2)
        i0 = rng.integers(0, n - w + 1)
        j0 = rng.integers(0, n - h + 1)
        void[j0:j0 + h, i0:i0 + w] = True
    ss = np.where(void, 0.09, 100.0)
    sa = np.full((n, n), 0.01)
    q = np.zeros((n, n))
    c = n // 2
    q[c - src_half:c + src_half, c - src_half:c + src_half] = 1.0
    kw.setdefault("n_particles", 10_000_000)
    kw.setdefault("dt", 0.01)
    kw.setdefault("n_steps", 20)
    kw.setdefault("sn_order", 8)
    return _problem(n, n, (0.0, L, 0.0, L), ss, sa, q, n_s=n_s, **kw)


def c3(n_s=0, **kw):
    return thick_with_voids(n_s=n_s, **kw)


def random_blocks(n=1024, L=10.0, blocks=32, lo=0.01, hi=20.0, n_s=3, mat_seed=11, **kw):
    """C5 family: sigma_s and sigma_a i.i.d. uniform on [lo, hi] per block of
    (n/blocks)^2 cells; unit source in the central 2x2 blocks."""
    rng = np.random.default_rng(mat_seed)
    cb = n // blocks
    bs = rng.uniform(lo, hi, size=(blocks, blocks))
    ba = rng.uniform(lo, hi, size=(blocks, blocks))
    ss = np.kron(bs, np.ones((cb, cb)))
    sa = np.kron(ba, np.ones((cb, cb)))
    q = np.zeros((n, n))
    h = blocks // 2
    q[(h - 1) * cb:(h + 1) * cb, (h - 1) * cb:(h + 1) * cb] = 1.0
    kw.setdefault("n_particles", 100_000_000)
    kw.setdefault("dt", 0.05)
    kw.setdefault("n_steps", 50)
    kw.setdefault("sn_order", 16)
    return _problem(n, n, (0.0, L, 0.0, L), ss, sa, q, n_s=n_s, **kw)


def c5(**kw):
    return random_blocks(**kw)


def c5_subproblem(**kw):
    """Seeded 128^2 subproblem of the large resident solve: same recipe,
    4x4-cell blocks on [0, 1.25]^2, 1e6 particles, 10 steps."""
    kw.setdefault("n_particles", 1_000_000)
    kw.setdefault("n_steps", 10)
    return random_blocks(n=128, L=1.25, blocks=32, **kw)


def lognormal_blocks(n, L=10.0, blocks=8, rng=None, **kw):
    """C4 request family: sigma_s, sigma_a i.i.d. lognormal (median 1,
    sigma 1) on blocks x blocks blocks; unit source on the central 2x2 blocks."""
    rng = rng if rng is not None else np.random.default_rng(0)
    cb = max(1, n // blocks)
    bs = rng.lognormal(0.0, 1.0, size=(blocks, blocks))
    ba = rng.lognormal(0.0, 1.0, size=(blocks, blocks))
    ss = np.kron(bs, np.ones((cb, cb)))[:n, :n]
    sa = np.kron(ba, np.ones((cb, cb)))[:n, :n]
    q = np.zeros((n, n))
    h = blocks // 2
    q[(h - 1) * cb:(h + 1) * cb, (h - 1) * cb:(h + 1) * cb] = 1.0
    kw.setdefault("dt", 0.05)
    kw.setdefault("sn_order", 8)
    return _problem(n, n, (0.0, L, 0.0, L), ss, sa, q, **kw)


def slab_regions(nx=80, ny=1, L=8.0, height=1.0, **kw):
    """Steady 1-D multi-region slab (stand-in with the structure of the
    paper's slab benchmark; the values are our own): along x a strongly
    absorbing source region, a pure absorber, a void, a scattering region with
    a source and a scattering region without; uniform in y with reflective
    y sides (an infinite slab), reflective at x = 0, vacuum at x = L.  The
    void needs an explicit path horizon."""
    x = (np.arange(nx) + 0.5) * (L / nx)
    edges = np.array([0.0, 1.5, 3.0, 4.5, 6.0, L]) * (L / 8.0)
    region = np.searchsorted(edges, x, side="right") - 1
    sa_r = np.array([20.0, 3.0, 0.0, 0.2, 0.05])
    ss_r = np.array([0.0, 0.0, 0.0, 0.8, 0.95])
    q_r = np.array([20.0, 0.0, 0.0, 1.0, 0.0])
    row = lambda v: np.tile(v[region], (ny, 1))
    kw.setdefault("n_s", 0)
    kw.setdefault("n_particles", 64_000)
    kw.setdefault("sn_order", 4)
    kw.setdefault("horizon", 200.0)
    kw.setdefault("si_max_iter", 1000)
    kw.setdefault("boundary", 1 | 4 | 8)
    return _problem(nx, ny, (0.0, L, 0.0, height), row(ss_r), row(sa_r), row(q_r),
                    steady=True, **kw)


def duct(nx=30, ny=50, **kw):
    """Steady 2-D duct (stand-in with the structure of the paper's duct
    problem; geometry and values are our own): a near-vacuum duct with two
    bends (sigma_s = sigma_a = 1e-4) through a scattering, absorbing medium
    (sigma_s = 0.9, sigma_a = 0.1) on [0,3] x [0,5], with a unit source in the
    first 0.5 x 0.5 of the duct; vacuum sides.  The duct needs an explicit
    path horizon."""
    hx, hy = 3.0 / nx, 5.0 / ny
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(xc, yc)
    duct = ((X < 0.5) & (Y < 2.0)) | ((Y >= 1.5) & (Y < 2.0) & (X < 2.0)) | \
           ((X >= 1.5) & (X < 2.0) & (Y >= 1.5))
    ss = np.where(duct, 1e-4, 0.9)
    sa = np.where(duct, 1e-4, 0.1)
    q = np.where((X < 0.5) & (Y < 0.5), 1.0, 0.0)
    kw.setdefault("n_s", 0)
    kw.setdefault("n_particles", 64_000)
    kw.setdefault("sn_order", 4)
    kw.setdefault("horizon", 200.0)
    kw.setdefault("si_max_iter", 1000)
    return _problem(nx, ny, (0.0, 3.0, 0.0, 5.0), ss, sa, q, steady=True, **kw)


def request_stream(n_req=256, rho=1.0, mean_service_s=None, seed=4, sides=(32, 64, 128, 256, 512),
                   np_range=(1e4, 1e7), steps_range=(5, 50), n_s_set=(0, 1, 2, 4)):
    """C4: a Poisson-arrival stream of solve requests.  Returns a list of
    (arrival_offset_s, problem) with arrival rate rho / mean_service_s (the
    arrival times are filled in by the caller when mean_service_s is None)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        n = int(rng.choice(sides))
        n_s = int(rng.choice(n_s_set))
        n_p = int(np.exp(rng.uniform(np.log(np_range[0]), np.log(np_range[1]))))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        prec = int(rng.integers(0, 2))
        p = lognormal_blocks(n, rng=rng, n_s=n_s, n_particles=n_p, n_steps=steps,
                             precision=prec, seed=1000 + r)
        reqs.append(p)
    gaps = rng.exponential(1.0, size=n_req)
    if mean_service_s is not None:
        gaps = gaps * mean_service_s / rho
    arrivals = np.cumsum(gaps) - gaps[0]
    return list(zip(arrivals.tolist(), reqs))


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c5": c5, "c5_sub": c5_subproblem}
