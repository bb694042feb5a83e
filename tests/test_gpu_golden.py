"""The device path against oracle results stored by tests/golden/make_golden.py
at the configurations' stated sizes (oracle minutes, not seconds): the
128x128 subproblem of the large solve (1e6 particles per pass, S_16, 10
steps), the checkerboard benchmark (1e6 particles, S_12, 5 steps), the
1024x1024 mesh of the large solve (the device's tally-copy layout of that
solve) and the thick medium with voids, in FP64 at 1e-10 and, for the last,
with FP32 tracking within 1e-4 of the FP64 oracle.

Every step: each flux at a fixed sample of cells (and the cell of its
maximum) element by element, and its L2 norm, maximum and sum over the whole
mesh; both passes' balances; the emission plans bitwise; the segment,
source-iteration and census counts exactly; the census bank's (history id,
cell) sequence by an order-sensitive hash and its weight sums; and no history
stopped by the segment guard."""
import os
import sys

import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if GOLD not in sys.path:
    sys.path.insert(0, GOLD)
import make_golden as G  # noqa: E402

TOL = 1e-10
BAL = G.BAL
KINDS = (("phi_R", 0), ("phi_pre", 1), ("phi_post", 2), ("phi_c", 3))


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_16821_amd import slh
    slh.lib()
    return slh


def _check_step(S, s, g, k, n, tol):
    for key, kind in KINDS:
        got = s.get_flux(kind).reshape(n, -1)
        cells = g["%s_%d_cells" % (key, k)]
        want = g["%s_%d_values" % (key, k)]
        nrm = g["%s_%d_norms" % (key, k)]
        scale = max(float(nrm[1]), 1e-300)
        err = float(np.max(np.abs(got[cells] - want))) / scale
        assert err <= tol, (k, key, err)
        flat = got.ravel()
        assert abs(np.linalg.norm(flat) - nrm[0]) <= tol * max(float(nrm[0]), 1e-300), (k, key)
        assert abs(np.max(np.abs(flat)) - nrm[1]) <= tol * scale, (k, key)
        assert abs(flat.sum() - nrm[2]) <= tol * float(nrm[0]) * np.sqrt(flat.size) + 1e-300
    for pss in (1, 2):
        b = s.get_balance(pss)
        want = g["bal%d_%d" % (pss, k)]
        sc = max(abs(float(want[0])), 1e-300)
        for f, w in zip(BAL, want):
            assert abs(b[f] - w) <= tol * sc, (k, pss, f, b[f], w)
        plan = g["plan%d_%d" % (pss, k)]
        if plan[1] > 0.0:
            assert b["majorant_sum"] == plan[0] and b["weight_quantum"] == plan[1], (k, pss)
            assert b["source_particles"] == int(plan[2]), (k, pss)
        assert b["killed"] == 0
    st = s.get_stats()
    seg, it, alive, kept = (int(v) for v in g["counts_%d" % k])
    assert st["segments_total"] == seg, (k, st["segments_total"], seg)
    assert st["si_iterations"] == it, (k, st["si_iterations"], it)
    assert st["census_alive"] == alive and st["census_kept"] == kept, (k, st)
    c = s.get_census()
    assert G.census_hash(c["hid"], c["cell"]) == int(g["census_%d" % k][0]), k
    cw = g["census_w_%d" % k]
    for got, want in ((c["w"].sum(), cw[0]), ((c["w"] ** 2).sum(), cw[1]),
                      (np.abs(c["w"]).sum(), cw[2])):
        assert abs(got - want) <= 1e-12 * max(abs(float(cw[2])), 1e-300), k


@pytest.mark.parametrize("name", ["c5_sub", "c2", "mesh1024", "c3_small"])
def test_fp64_against_stored_oracle(S, name):
    g = np.load(os.path.join(GOLD, name + ".npz"))
    p, steps = G.cases()[name]
    assert int(g["steps"]) == steps
    n = int(p["nx"]) * int(p["ny"])
    log("golden case", name, p["nx"], p["ny"], "N_p", p["n_particles"], "S_%d" % p["sn_order"],
        "steps", steps)
    s = S.Solver(p)
    for k in range(steps):
        s.advance(1)
        _check_step(S, s, g, k, n, TOL)
        log("  step", k, "ok")
    assert s.get_stats()["killed_total"] == 0
    s.destroy()


def test_fp32_against_stored_oracle(S):
    """FP32 tracking (FP64 tallies) on the thick medium with voids against
    the FP64 oracle: relative L2 of phi_R below 1e-4 every step."""
    name = "c3_small"
    g = np.load(os.path.join(GOLD, name + ".npz"))
    p, steps = G.cases()[name]
    s = S.Solver(dict(p, precision=1))
    for k in range(steps):
        s.advance(1)
        want = g["phi_R_full_%d" % k]
        got = s.get_flux(0)
        e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        log("  fp32 step", k, "rel-L2 vs the FP64 oracle %.2e" % e)
        assert e < 1e-4, (k, e)
    s.destroy()
