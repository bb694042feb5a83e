"""slh_create_static, the entry point for callers that cannot allocate: the
solver's device memory comes from the library's static scratch.  Checked
through the C ABI against slh_create on the same problems, bitwise, for two
solvers in a row (the second smaller, reusing the scratch), and its limits."""
import numpy as np
import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_16821_amd import slh
    slh.lib()
    return slh


def _compare(S, p, steps):
    log("static vs allocated", p["nx"], p["ny"], "N_p", p["n_particles"], "steps", steps)
    a = S.Solver(p)
    b = S.Solver(p, static=True)
    for k in range(steps):
        a.advance(1)
        b.advance(1)
        for kind in (S.SLH_FLUX_REMAP, S.SLH_FLUX_PRE, S.SLH_FLUX_POST,
                     S.SLH_FLUX_COLLIDED_NODAL):
            assert np.array_equal(a.get_flux(kind), b.get_flux(kind)), (k, kind)
        for pss in (1, 2):
            assert a.get_balance(pss) == b.get_balance(pss), (k, pss)
        ca, cb = a.get_census(), b.get_census()
        for f in ca:
            assert np.array_equal(ca[f], cb[f]), (k, f)
        sa, sb = a.get_stats(), b.get_stats()
        for f in ("si_iterations", "segments_total", "census_kept", "step"):
            assert sa[f] == sb[f], (k, f)
        log("  step", k, "segments", sb["segments_total"])
    a.destroy()
    b.destroy()


def test_static_solver_matches_allocated(S):
    from paper_2511_16821_amd import workloads as W
    big = W.checkerboard(blocks=5, cells_per_block=4, n_s=2, n_particles=20000, dt=0.05,
                         sn_order=6, census_cap=15000)
    small = W.checkerboard(blocks=3, cells_per_block=4, n_s=1, n_particles=3000, dt=0.1,
                           sn_order=4)
    assert S.slh_footprint_bytes(small) < S.slh_footprint_bytes(big) <= 64 << 20
    _compare(S, big, 3)
    _compare(S, small, 2)


def test_static_solver_limits(S):
    from paper_2511_16821_amd import workloads as W
    p = W.checkerboard(blocks=3, cells_per_block=4, n_s=1, n_particles=3000, dt=0.1,
                       sn_order=4)
    a = S.Solver(p, static=True)
    # one static solver per device at a time
    with pytest.raises(S.SlhError) as e:
        S.Solver(p, static=True)
    assert e.value.status == S.SLH_E_STATE
    with pytest.raises(S.SlhError) as e:
        a.set_graphs(True)
    assert e.value.status == S.SLH_E_STATE
    a.advance(1)
    a.destroy()
    # above the scratch: rejected before anything is touched
    big = W.c2(n_s=2)
    assert S.slh_footprint_bytes(big) > 64 << 20
    with pytest.raises(S.SlhError) as e:
        S.Solver(big, static=True)
    assert e.value.status == S.SLH_E_REJECTED
    # the scratch is free again
    b = S.Solver(p, static=True)
    b.advance(1)
    b.destroy()
