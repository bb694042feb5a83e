"""Failure paths of the C ABI on the device, each forced from the host so
that every kernel still exits normally: an allocator that runs out of memory
part-way through slh_create, one that returns a misaligned block, a source
iteration stopped at its limit, a
source too large for the fixed-point bounds, and a checkpoint written for
another mesh."""
import ctypes as C

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


def _small():
    from paper_2511_16821_amd import workloads as W
    return W.checkerboard(blocks=3, cells_per_block=4, n_s=1, n_particles=3000, dt=0.1,
                          sn_order=4)


def test_allocator_failure_releases_everything(S):
    """An allocator that returns NULL on its k-th request: slh_create reports
    SLH_E_OUT_OF_MEMORY, hands back no solver, and returns every block it had
    obtained before the failure (no leak), for every k up to the last request."""
    import torch
    p = _small()
    st, keep = S.make_problem(p)
    stream = torch.cuda.current_stream()

    class Counting:
        def __init__(self, fail_at):
            self.fail_at, self.calls, self.live = fail_at, 0, {}
            self.a = S.ALLOC_FN(self._alloc)
            self.f = S.FREE_FN(self._free)

        def _alloc(self, n, ctx):
            self.calls += 1
            if self.calls == self.fail_at:
                return None
            ptr = torch.cuda.caching_allocator_alloc(int(n), stream=stream)
            self.live[ptr] = n
            return ptr

        def _free(self, ptr, ctx):
            assert ptr in self.live
            del self.live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

    # how many requests a good create makes
    ok = Counting(0)
    h = C.c_void_p()
    assert S.lib().slh_create(C.byref(st), C.c_void_p(stream.cuda_stream), ok.a, ok.f, None,
                              C.byref(h)) == S.SLH_OK
    n_req = ok.calls
    S.lib().slh_destroy(h)
    assert not ok.live and n_req > 10
    log("allocations of a create", n_req)
    for k in sorted({1, 2, 5, n_req // 2, n_req - 1, n_req}):
        a = Counting(k)
        h = C.c_void_p()
        r = S.lib().slh_create(C.byref(st), C.c_void_p(stream.cuda_stream), a.a, a.f, None,
                               C.byref(h))
        assert r == S.SLH_E_OUT_OF_MEMORY, (k, r)
        assert not h.value
        assert b"allocation failed" in S.lib().slh_last_error()
        assert not a.live, (k, len(a.live))
    torch.cuda.synchronize()


def test_misaligned_allocator_block_is_rejected(S):
    """An allocator whose k-th block is not aligned to 256 bytes: slh_create
    reports SLH_E_INVALID_ARG (the kernels' vector loads need the alignment),
    hands the block back to free_fn with every other one, and returns no
    solver."""
    import torch
    p = _small()
    st, keep = S.make_problem(p)
    stream = torch.cuda.current_stream()

    class Skewed:
        def __init__(self, skew_at):
            self.skew_at, self.calls, self.live = skew_at, 0, {}
            self.a = S.ALLOC_FN(self._alloc)
            self.f = S.FREE_FN(self._free)

        def _alloc(self, n, ctx):
            self.calls += 1
            base = torch.cuda.caching_allocator_alloc(int(n) + 256, stream=stream)
            ptr = base + 16 if self.calls == self.skew_at else base
            self.live[ptr] = base
            return ptr

        def _free(self, ptr, ctx):
            torch.cuda.caching_allocator_delete(self.live.pop(ptr))

    for k in (1, 7):
        a = Skewed(k)
        h = C.c_void_p()
        r = S.lib().slh_create(C.byref(st), C.c_void_p(stream.cuda_stream), a.a, a.f, None,
                               C.byref(h))
        assert r == S.SLH_E_INVALID_ARG, (k, r)
        assert not h.value
        assert b"aligned" in S.lib().slh_last_error()
        assert not a.live, (k, len(a.live))
    torch.cuda.synchronize()


def test_source_iteration_limit_reports_not_converged(S):
    """si_max_iter = 1 on a scattering problem: slh_advance returns at once
    (SLH_OK), slh_synchronize reports SLH_E_NOT_CONVERGED for the steps
    since the last call (and SLH_OK after that), the steps are still
    completed (step counter, fluxes), and the stats count the steps whose
    iteration stopped at the limit."""
    p = _small()
    p["si_max_iter"] = 1
    s = S.Solver(p)
    assert s.advance(2) == S.SLH_OK
    assert s.synchronize(allow_not_converged=True) == S.SLH_E_NOT_CONVERGED
    assert "si_max_iter" in S.lib().slh_last_error().decode()
    assert s.synchronize() == S.SLH_OK
    st = s.get_stats()
    assert st["step"] == 2 and st["steps_total"] == 2
    assert st["si_iterations"] == 1 and st["si_converged"] == 0
    assert st["si_unconverged_total"] == 2
    assert np.all(np.isfinite(s.get_flux(0))) and s.get_flux(0).sum() > 0
    s.destroy()


def test_overflowing_source_reports_numeric(S):
    """A source so large that a cell majorant overflows (q = 1e308 rounds up
    to 2^1024): no particle is emitted from it, and slh_synchronize returns
    SLH_E_NUMERIC with a message that names the majorant."""
    from paper_2511_16821_amd import workloads as W
    n = 4
    q = np.zeros((n, n))
    q[1, 2] = 1e308
    p = W._problem(n, n, (0.0, 4.0, 0.0, 4.0), np.full((n, n), 0.5), np.full((n, n), 0.5), q,
                   n_s=0, n_particles=1000, sn_order=2, dt=0.1)
    s = S.Solver(p)
    assert s.advance(1) == S.SLH_OK
    with pytest.raises(S.SlhError) as e:
        s.synchronize()
    assert e.value.status == S.SLH_E_NUMERIC
    assert "majorant" in str(e.value)
    assert s.get_stats()["numeric_flags"] & 1
    s.destroy()


def test_checkpoint_of_another_mesh_is_rejected(S):
    """slh_load checks the recorded mesh, seed and particles before anything
    reaches the device: a checkpoint of another mesh or seed, or one whose
    particles were altered, is SLH_E_INVALID_ARG and leaves the solver usable."""
    from paper_2511_16821_amd import workloads as W
    a = S.Solver(W.c1(n_particles=2000))
    a.advance(2)
    blob = a.save()
    b = S.Solver(W.checkerboard(blocks=3, cells_per_block=4, n_s=1, n_particles=2000, dt=0.1,
                                sn_order=4))
    with pytest.raises(S.SlhError) as e:
        b.load(blob)
    assert e.value.status == S.SLH_E_INVALID_ARG and "another mesh" in str(e.value)
    c = S.Solver(dict(W.c1(n_particles=2000), seed=99))
    with pytest.raises(S.SlhError) as e:
        c.load(blob)
    assert "another seed" in str(e.value)
    # a particle moved off the mesh (its cell index beyond nx*ny)
    d = S.Solver(W.c1(n_particles=2000))
    raw = bytearray(blob)
    cnt = int(np.frombuffer(raw[32:40], dtype=np.uint64)[0])
    assert cnt > 0
    cell_off = 80 + 5 * 8 * cnt + 8 * cnt
    raw[cell_off:cell_off + 4] = np.array([400], dtype=np.int32).tobytes()
    with pytest.raises(S.SlhError) as e:
        d.load(bytes(raw))
    assert "not valid" in str(e.value)
    # the rejected solvers still run, and the genuine checkpoint still loads
    d.load(blob)
    d.advance(1)
    b.advance(1)
    for s in (a, b, c, d):
        s.destroy()
