"""Serving (continuous batching on one GPU): every request's result is the
same alone and in the mix (bitwise: all sums are order-independent fixed
point), across time-dependent and steady requests, both closing stages, with
and without DSA, both precisions and per-cell scatter limits; admission never exceeds the HBM
budget, and requests that can never fit are rejected."""
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


def _mix(n=10, seed=3):
    from paper_2511_16821_amd import workloads as W
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n):
        side = int(rng.choice([16, 24, 32, 48]))
        p = W.lognormal_blocks(side, L=4.0, blocks=8, rng=rng, n_s=int(rng.choice([0, 1, 2, 4])),
                               n_particles=int(rng.choice([3000, 12000, 40000])),
                               precision=int(rng.integers(0, 2)), seed=100 + r, sn_order=4)
        if r % 4 == 1:  # per-cell scatter limits travel with the request
            p["n_s_cell"] = rng.choice([-1, 0, 1, 3], size=side * side).astype(np.int32)
        if r % 4 == 2:  # steady-state requests, with the whole-flux stopping test
            p.update(steady=True, si_norm=1, si_tol=1e-9, si_max_iter=400)
        if r % 4 == 3:  # the diffusion closing stage
            p.update(closure=1, si_max_iter=1000)
        if r % 5 == 4:  # diffusion synthetic acceleration of the S_N iteration
            p.update(si_accel=1)
        out.append((p, int(rng.integers(2, 6))))
    return out


def _alone(S, p, steps):
    s = S.Solver(p)
    s.advance(steps, allow_not_converged=True)
    f = s.get_flux(0)
    b = s.get_balance(2)
    s.destroy()
    return f, b


def test_results_same_alone_and_in_mix(S):
    reqs = _mix()
    srv = S.Server(hbm_budget_bytes=2 << 30, max_slots=4)
    tickets = [srv.submit(p, k) for p, k in reqs]
    got = [srv.result(t) for t in tickets]
    srv.destroy()
    for (p, k), (flux, bal, lat) in zip(reqs, got):
        f, b = _alone(S, p, k)
        assert np.array_equal(flux, f), (p["nx"], p["n_s"], p["precision"],
                                         p.get("steady", False), p.get("closure", 0))
        assert bal["census"] == b["census"] and bal["segments"] == b["segments"]
        assert lat["latency_ms"] >= lat["run_ms"] > 0
    log("mix of", len(reqs), "requests matches the standalone runs bitwise")


def test_admission_respects_budget(S):
    reqs = _mix(6, seed=9)
    fps = [S.slh_footprint_bytes(p) for p, _ in reqs]
    budget = max(fps) + (1 << 20)  # room for one request at a time
    srv = S.Server(hbm_budget_bytes=budget, max_slots=4)
    tickets = [srv.submit(p, k) for p, k in reqs]
    lats = [srv.result(t)[2] for t in tickets]
    srv.destroy()
    iv = sorted((l["admit_s"], l["done_s"], fp) for l, fp in zip(lats, fps))
    for a in range(len(iv)):
        for b in range(a + 1, len(iv)):
            overlap = iv[a][1] > iv[b][0] and iv[b][1] > iv[a][0]
            if overlap:
                assert iv[a][2] + iv[b][2] <= budget


def test_reject_and_invalid(S):
    from paper_2511_16821_amd import workloads as W
    srv = S.Server(hbm_budget_bytes=64 << 20, max_slots=2)
    with pytest.raises(S.SlhError) as e:
        srv.submit(W.c1(n_particles=2_000_000), 2)
    assert e.value.status == S.SLH_E_REJECTED
    bad = W.c1()
    bad["dt"] = -1.0
    with pytest.raises(S.SlhError) as e:
        srv.submit(bad, 1)
    assert e.value.status == S.SLH_E_INVALID_ARG
    t = srv.submit(W.c1(n_particles=2000), 1)
    flux, bal, lat = srv.result(t)
    assert flux.sum() > 0
    srv.destroy()


def test_large_request_is_not_starved(S):
    """A request that cannot share the arena with the one running waits at
    the head of the queue; at most four later (small) requests are admitted
    ahead of it, and the rest of them wait until it has been admitted."""
    from paper_2511_16821_amd import workloads as W
    big = W.homogeneous_box(n=128, n_particles=200_000, n_s=2)
    small = W.checkerboard(blocks=2, cells_per_block=8, n_s=1, n_particles=3000, dt=0.1,
                           sn_order=2)
    fb, fs = S.slh_footprint_bytes(big), S.slh_footprint_bytes(small)
    assert fb > 8 * fs
    srv = S.Server(hbm_budget_bytes=2 * fb - 4096, max_slots=4)
    first = srv.submit(big, 40)        # long: holds its block
    waiting = srv.submit(big, 2)       # cannot fit beside the first
    smalls = [srv.submit(small, 2) for _ in range(10)]
    lat_first = srv.result(first)[2]
    lat_wait = srv.result(waiting)[2]
    lat_small = [srv.result(t)[2] for t in smalls]
    srv.destroy()
    ahead = sum(1 for x in lat_small if x["admit_s"] < lat_wait["admit_s"])
    log("small requests admitted ahead of the waiting one:", ahead,
        "its queue ms %.1f, the first one's run ms %.1f" % (lat_wait["queue_ms"],
                                                            lat_first["run_ms"]))
    assert ahead <= 4
    assert lat_wait["admit_s"] >= lat_first["done_s"] - 1e-3
