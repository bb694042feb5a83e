"""Steady-state mode (one infinite time step, the setting of the paper's runs
in Sec. 3) on the device against the CPU oracle: FP64 to 1e-10 relative for
every tally array, equal balances, source-iteration counts and segment
counts; FP32 tracking to 1e-4 relative L2."""
import numpy as np
import pytest

from gpu_util import FP32_TOL, compare_balance, compare_step, log, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_16821_amd import slh
    slh.lib()
    return slh


def _run_pair(S, oracle, p, steps, name):
    log("steady case", name, p["nx"], p["ny"], "n_s", p["n_s"], "N_p", p["n_particles"],
        "si_norm", p.get("si_norm", 0), "horizon", p.get("horizon", 0.0))
    o = oracle.HybridOracle(p)
    s = S.Solver(p)
    for k in range(steps):
        r = o.step()
        s.advance(1)
        errs = compare_step(S, s, r)
        compare_balance(s, r)
        st = s.get_stats()
        assert st["si_iterations"] == r["si_iters"], (st["si_iterations"], r["si_iters"])
        assert st["segments_total"] == r["segments"], (st["segments_total"], r["segments"])
        if p.get("steady", False):
            assert st["census_alive"] == 0 and st["census_kept"] == 0
            assert len(s.get_census()["w"]) == 0
        else:
            assert st["census_kept"] == r["census_kept"]
        log("  step", k, "si", r["si_iters"], {kk: "%.1e" % v[0] for kk, v in errs.items()})
    s.destroy()


@pytest.mark.parametrize("n_s", [0, 2, -1])
def test_steady_box(S, oracle, n_s):
    """Homogeneous box with a central source, vacuum sides, default horizon;
    two steps (independent steady solves with their own points)."""
    from paper_2511_16821_amd import workloads as W
    p = W.c1(n_s=n_s, steady=True, n_particles=10000, si_max_iter=400)
    _run_pair(S, oracle, p, 2, "box")


def test_steady_slab_and_duct(S, oracle):
    """The multi-region slab (void, reflective sides, explicit horizon) and
    the bent duct, with both stopping tests and pure MC (no remap)."""
    from paper_2511_16821_amd import workloads as W
    _run_pair(S, oracle, W.slab_regions(n_s=5, n_particles=20000, si_norm=1, si_tol=1e-8),
              1, "slab")
    _run_pair(S, oracle, W.slab_regions(n_s=0, n_particles=12000), 1, "slab")
    _run_pair(S, oracle, W.duct(n_s=0, n_particles=20000, si_norm=1, si_tol=1e-8), 1, "duct")
    _run_pair(S, oracle, W.duct(n_s=-1, n_particles=20000), 2, "duct")


def test_steady_horizon(S, oracle):
    """Histories cut by the horizon: a void box closed on every side (all of
    the weight reaches the horizon) and a weakly absorbing box whose horizon
    ends part of the histories."""
    from paper_2511_16821_amd import workloads as W
    n = 6
    p = W._problem(n, n, (0.0, 1.5, 0.0, 1.5), np.zeros((n, n)), np.zeros((n, n)),
                   np.full((n, n), 3.0), n_s=0, n_particles=3000, sn_order=4, steady=True,
                   boundary=15, horizon=7.5)
    _run_pair(S, oracle, p, 1, "void box")
    q = W.homogeneous_box(n=12, L=3.0, sig_s=0.5, sig_a=0.05, src_cells=((4, 8), (4, 8)),
                          n_s=1, n_particles=8000, sn_order=4, steady=True, horizon=3.0,
                          boundary=5)
    _run_pair(S, oracle, q, 1, "short horizon")


def test_steady_reflective_box_with_cell_limits(S, oracle):
    """Closed checkerboard (an infinite periodic medium) with N_s(x)."""
    from paper_2511_16821_amd import workloads as W
    p = W.checkerboard(blocks=3, cells_per_block=4, n_s=1, n_particles=12000, sn_order=4,
                       steady=True, boundary=15, si_max_iter=600,
                       horizon=100.0)
    ss = np.asarray(p["sigma_s"], dtype=np.float64).ravel()
    p["n_s_cell"] = np.where(ss > 0, 2, 0).astype(np.int32)
    _run_pair(S, oracle, p, 1, "closed checkerboard")


def test_steady_fp32(S, oracle):
    from paper_2511_16821_amd import workloads as W
    for name, p in (("slab", W.slab_regions(n_s=5, n_particles=20000)),
                    ("duct", W.duct(n_s=0, n_particles=20000)),
                    ("box", W.c1(n_s=2, steady=True, n_particles=10000, si_max_iter=400))):
        log("steady fp32 case", name)
        o = oracle.HybridOracle(p)
        s = S.Solver(dict(p, precision=1))
        r = o.step()
        s.advance(1)
        for key, kind in (("phi_R", 0), ("phi_pre", 1), ("phi_post", 2), ("phi_c", 3)):
            e = rel_l2(s.get_flux(kind), r[key])
            log("  ", key, "%.2e" % e)
            assert e <= FP32_TOL, (name, key, e)
        s.destroy()


def test_steady_and_diffusion_degenerate_cases(S, oracle):
    """No source (all zero, no iterations for the diffusion stage), one cell,
    no particles, and pure MC with the diffusion closure selected (no
    collided source, so the stage is skipped)."""
    from paper_2511_16821_amd import workloads as W
    for extra in (dict(steady=True), dict(closure=1), dict(steady=True, closure=1)):
        p = dict(W.c1(n_particles=1000), **extra)
        p["q"] = np.zeros_like(p["q"])
        s = S.Solver(p)
        s.advance(2)
        assert np.all(s.get_flux(0) == 0.0) and np.all(s.get_flux(3) == 0.0)
        st = s.get_stats()
        assert st["census_kept"] == 0
        if extra.get("closure"):
            assert st["si_iterations"] == 0
        s.destroy()
        q = dict(W.c1(n_particles=0), **extra)
        s = S.Solver(q)
        s.advance(1)
        assert np.all(s.get_flux(0) == 0.0)
        s.destroy()
    one = W.homogeneous_box(n=1, L=1.0, src_cells=((0, 1), (0, 1)), n_particles=3000, n_s=2,
                            sn_order=2, steady=True)
    _run_pair(S, oracle, one, 2, "one cell")
    _run_pair(S, oracle, dict(one, closure=1, si_tol=1e-13), 1, "one cell, diffusion")
    _run_pair(S, oracle, dict(W.c1(n_s=-1, n_particles=4000), closure=1), 2, "pure MC, diffusion")
