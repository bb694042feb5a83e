"""FP32-tracking path (geometry, distance sampling and attenuation in FP32;
tallies, balance totals, emission trees and the DG solve in FP64) against
the FP64 oracle on the same seeded inputs: relative L2 <= 1e-4 for every
tally array at every step."""
import numpy as np
import pytest

from gpu_util import FP32_TOL, log, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_16821_amd import slh
    slh.lib()
    return slh


def _run(S, oracle, p, steps):
    log("fp32 case", p["nx"], p["ny"], "n_s", p["n_s"], "N_p", p["n_particles"], "steps", steps)
    p32 = dict(p)
    p32["precision"] = 1
    o = oracle.HybridOracle(p)
    s = S.Solver(p32)
    worst = 0.0
    for k in range(steps):
        r = o.step()
        s.advance(1)
        for key, kind in (("phi_R", 0), ("phi_pre", 1), ("phi_post", 2), ("phi_c", 3)):
            e = rel_l2(s.get_flux(kind), r[key])
            worst = max(worst, e)
            assert e <= FP32_TOL, (k, key, e)
        for pss in (1, 2):
            b = s.get_balance(pss)
            out = b["absorbed"] + b["scattered"] + b["leaked"] + b["census"] + b["cutoff"]
            assert abs(b["emitted"] - out) <= 1e-6 * abs(b["emitted"]) + 1e-300
    log("  worst rel-L2 %.2e" % worst)
    s.destroy()
    return worst


def test_fp32_c1(S, oracle):
    from paper_2511_16821_amd import workloads as W
    _run(S, oracle, W.c1(), 10)


def test_fp32_checkerboard(S, oracle):
    from paper_2511_16821_amd import workloads as W
    p = W.checkerboard(blocks=7, cells_per_block=4, n_s=2, n_particles=50000, dt=0.05,
                       sn_order=6)
    _run(S, oracle, p, 6)


def test_fp32_thick_voids(S, oracle):
    from paper_2511_16821_amd import workloads as W
    p = W.thick_with_voids(n=32, n_s=4, n_particles=40000, dt=0.01, src_half=4, sn_order=4)
    _run(S, oracle, p, 4)


def test_fp32_with_halton_cellwise_limit_and_reflective_sides(S, oracle):
    """FP32 tracking with the options beyond the paper's examples at once:
    Halton points, a material-dependent N_s(x) and reflective x_lo / y_hi."""
    from paper_2511_16821_amd import workloads as W
    p = W.checkerboard(blocks=5, cells_per_block=4, n_s=2, n_particles=20000, dt=0.1,
                       sn_order=6, points=2, boundary=9)
    ss = np.asarray(p["sigma_s"], dtype=np.float64).ravel()
    p["n_s_cell"] = np.where(ss > 0, 3, 0).astype(np.int32)
    _run(S, oracle, p, 3)
