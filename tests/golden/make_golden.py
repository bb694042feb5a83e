#!/usr/bin/env python3
"""Writes the stored expected values of tests/test_gpu_golden.py.

CPU only: every value comes from the oracle (oracle/), run on the seeded
synthetic problems of paper_2511_16821_amd/workloads.py at sizes where the
oracle takes minutes rather than seconds, so the values are computed once
here and stored:

  c5_sub   the 128x128 subproblem of the large resident solve at its stated
           size: 4x4-cell random blocks, N_s = 3, 1e6 particles per pass,
           S_16, 10 steps;
  c2       the 140x140 checkerboard, N_s = 2, 1e6 particles per pass, S_12,
           the first 5 of its 40 steps;
  mesh1024 the 1024x1024 random-block mesh of the large solve with 2e5
           particles per pass and S_2 for 3 steps: a mesh on which the
           device's private tally copies take the layout of the large solve;
  c3_small the 256x256 thick medium with voids of the precision form, N_s = 2,
           with 1e5 particles per pass for 3 steps (its whole phi_R is
           stored: the FP32-tracking path is compared with it).

For every step the file holds, per flux (phi_R, phi_pre, phi_post and the
nodal phi_c): its L2 norm, maximum and sum over the whole mesh, and its
values at a fixed sample of cells (seeded, plus the cell of the maximum);
both passes' balance; the step's segment and source-iteration counts; and
the census bank's size, an order-sensitive hash of its (history id, cell)
sequence and the sums of its weights and of their squares.

    python tests/golden/make_golden.py [case ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_SAMPLE = 2048
MASK64 = (1 << 64) - 1


def cases():
    from paper_2511_16821_amd import workloads as W
    return {
        "c5_sub": (W.c5_subproblem(), 10),
        "c2": (W.c2(n_s=2), 5),
        "mesh1024": (W.c5(n_particles=200_000, sn_order=2), 3),
        "c3_small": (W.c3(n_s=2, n_particles=100_000), 3),
    }


# cases whose whole phi_R is stored (the FP32 comparison takes the full L2)
FULL_PHI_R = ("c3_small",)


def mix64(z):
    """SplitMix64 output function (Steele, Lea & Flood 2014) on a numpy
    uint64 array (arithmetic modulo 2^64)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def census_hash(hid, cell):
    """Order-sensitive 64-bit hash of the census bank's (history id, cell)
    sequence: the sum modulo 2^64 of a mix of each entry with its position."""
    hid = np.asarray(hid, dtype=np.uint64)
    cell = np.asarray(cell, dtype=np.int64).astype(np.uint64)
    pos = np.arange(hid.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        terms = mix64(hid ^ mix64(cell ^ (pos << np.uint64(32))))
        return int(np.sum(terms, dtype=np.uint64))


def sample_cells(n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(N_SAMPLE, n), replace=False))


FLUXES = ("phi_R", "phi_pre", "phi_post", "phi_c")
BAL = ("emitted", "absorbed", "scattered", "leaked", "census", "cutoff", "source_w",
       "census_in_w")


def run_case(name, p, steps):
    from oracle import oracle as O
    O.build()
    o = O.HybridOracle(p)
    n = int(p["nx"]) * int(p["ny"])
    idx = sample_cells(n, 1234)
    out = {"steps": np.array(steps), "sample_cells": idx}
    t0 = time.perf_counter()
    for k in range(steps):
        r = o.step()
        for key in FLUXES:
            v = np.asarray(r[key], dtype=np.float64).reshape(n, -1)
            flat = v.ravel()
            cells = np.union1d(idx, [int(np.argmax(np.abs(v).max(axis=1)))])
            out["%s_%d_cells" % (key, k)] = cells
            out["%s_%d_values" % (key, k)] = v[cells]
            out["%s_%d_norms" % (key, k)] = np.array(
                [np.linalg.norm(flat), np.max(np.abs(flat)), flat.sum()])
        if name in FULL_PHI_R:
            out["phi_R_full_%d" % k] = np.asarray(r["phi_R"], dtype=np.float64).ravel()
        for pss, bk in ((1, "bal_mc"), (2, "bal_remap")):
            b = r[bk]
            out["bal%d_%d" % (pss, k)] = np.array([b[f] for f in BAL])
            out["plan%d_%d" % (pss, k)] = np.array([b.get("majorant_sum", 0.0),
                                                    b.get("weight_quantum", 0.0),
                                                    float(b.get("source_particles", 0))])
        out["counts_%d" % k] = np.array([r["segments"], r["si_iters"], r["census_alive"],
                                         r["census_kept"]], dtype=np.int64)
        bank = o.bank
        out["census_%d" % k] = np.array([census_hash(bank.hid, bank.cell)], dtype=np.uint64)
        out["census_w_%d" % k] = np.array([bank.w.sum(), (bank.w * bank.w).sum(),
                                           np.abs(bank.w).sum()])
        print("%s: step %d done (%.0f s)" % (name, k, time.perf_counter() - t0), flush=True)
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **out)
    print("wrote", path, os.path.getsize(path), "bytes", flush=True)


def main():
    todo = sys.argv[1:] or list(cases())
    cs = cases()
    for name in todo:
        p, steps = cs[name]
        run_case(name, p, steps)


if __name__ == "__main__":
    main()
