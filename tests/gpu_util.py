"""Helpers shared by the GPU tests: run the device path and the oracle on the
same seeded problem and compare."""
import sys

import numpy as np

FP64_TOL = 1e-10   # relative, L2 and max norm, per tally array
FP32_TOL = 1e-4    # relative L2 of the FP32-tracking path against the FP64 oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(got, want):
    got = np.asarray(got, dtype=np.float64).ravel()
    want = np.asarray(want, dtype=np.float64).ravel()
    nw = np.linalg.norm(want)
    if nw == 0.0:
        return float(np.linalg.norm(got))
    return float(np.linalg.norm(got - want) / nw)


def rel_max(got, want):
    got = np.asarray(got, dtype=np.float64).ravel()
    want = np.asarray(want, dtype=np.float64).ravel()
    m = np.max(np.abs(want)) if want.size else 0.0
    if m == 0.0:
        return float(np.max(np.abs(got))) if got.size else 0.0
    return float(np.max(np.abs(got - want)) / m)


FLUXES = (("phi_R", 0), ("phi_pre", 1), ("phi_post", 2), ("phi_c", 3))


def compare_step(S, solver, ref, tol=FP64_TOL, what=FLUXES, l2_only=False):
    errs = {}
    for key, kind in what:
        got = solver.get_flux(kind)
        want = np.asarray(ref[key]).ravel()
        e2 = rel_l2(got, want)
        em = rel_max(got, want)
        errs[key] = (e2, em)
        assert e2 <= tol, ("step", ref["step"], key, e2, em)
        if not l2_only:
            assert em <= tol, ("step", ref["step"], key, e2, em)
    return errs


def compare_balance(solver, ref, tol=1e-10):
    for pss, key in ((1, "bal_mc"), (2, "bal_remap")):
        b = solver.get_balance(pss)
        r = ref[key]
        scale = max(abs(r["emitted"]), 1e-300)
        for f in ("emitted", "absorbed", "scattered", "leaked", "census", "cutoff", "source_w",
                  "census_in_w"):
            assert abs(b[f] - r[f]) <= tol * scale, (pss, f, b[f], r[f])
        out = b["absorbed"] + b["scattered"] + b["leaked"] + b["census"] + b["cutoff"]
        assert abs(b["emitted"] - out) <= 1e-13 * scale + 1e-300, (pss, b)
        if "majorant_sum" in r:
            # the emission plan: the correctly rounded majorant sum, w_q and
            # the particle count are exact on both sides
            assert b["majorant_sum"] == r["majorant_sum"], (pss, b["majorant_sum"], r)
            assert b["weight_quantum"] == r["weight_quantum"], (pss, b, r)
            assert b["source_particles"] == r["source_particles"], (pss, b, r)
        assert b["killed"] == 0, (pss, b)
