"""The prescribed isotropic inflow G (boundary data of Sec. 2.1, applied in
both MC legs) on the device against the oracle: time steps with a source
and inflows on two sides (census, balances, fluxes, emission plans every
step), FP32 tracking, a steady half-space against its closed form, and a
server request with an inflow."""
import numpy as np
import pytest
from scipy.special import expn

from gpu_util import log
from test_gpu_parity import _run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_16821_amd import slh
    slh.lib()
    return slh


@pytest.fixture(scope="module")
def oracle():
    from oracle import oracle as O
    O.build()
    return O


def _time_problem(**kw):
    from paper_2511_16821_amd import workloads as W
    p = W.checkerboard(blocks=3, cells_per_block=6, n_s=1, n_particles=20000, dt=0.05,
                       sn_order=4, **kw)
    n = p["nx"]
    g = np.zeros(4 * n)
    g[:n] = 1.0                       # x_lo
    g[3 * n:] = 0.3 + 0.01 * np.arange(n)  # y_hi, varying along the side
    p["inflow"] = g
    return p


def test_inflow_time_steps(S, oracle):
    _run_pair(S, oracle, _time_problem(), 4)


def test_inflow_with_reflective_sides(S, oracle):
    p = _time_problem(boundary=2 | 4)  # x_hi and y_lo reflect; the inflow sides are vacuum
    _run_pair(S, oracle, p, 3)


def test_inflow_fp32(S, oracle):
    p = _time_problem()
    o = oracle.HybridOracle(p)
    s = S.Solver(dict(p, precision=1))
    for k in range(3):
        r = o.step()
        s.advance(1)
        got, want = s.get_flux(0), r["phi_R"].ravel()
        e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        log("  fp32 step", k, "rel-L2 %.2e" % e)
        assert e < 1e-4, (k, e)
    s.destroy()


def test_inflow_steady_half_space(S, oracle):
    """Steady, purely absorbing, inflow on x_lo, reflective y sides: the
    oracle's closed-form case (2 pi G (E_3 - E_3) / (sigma h) per cell), on
    the device and against the oracle."""
    from paper_2511_16821_amd import workloads as W
    nx, ny, G = 20, 4, 2.0
    p = W.homogeneous_box(n=4, L=2.0, n_s=-1, n_particles=200_000, steady=True, sn_order=2)
    p.update(nx=nx, ny=ny, x_hi=2.0, y_hi=0.4, boundary=4 | 8)
    p["sigma_s"] = np.zeros((ny, nx))
    p["sigma_a"] = np.ones((ny, nx))
    p["q"] = np.zeros((ny, nx))
    g = np.zeros(2 * (nx + ny))
    g[:ny] = G
    p["inflow"] = g
    _run_pair(S, oracle, p, 1, check_census=False)
    s = S.Solver(p)
    s.advance(1)
    phi = s.get_flux(0).reshape(ny, nx).mean(axis=0)
    s.destroy()
    d = np.linspace(0.0, 2.0, nx + 1)
    exact = 2 * np.pi * G * (expn(3, d[:-1]) - expn(3, d[1:])) / 0.1
    assert np.max(np.abs(phi / exact - 1.0)) < 1e-3


def test_inflow_request_in_server(S):
    """A request with an inflow gives the same result through the server as
    alone (its inflow array travels with it)."""
    p = _time_problem()
    srv = S.Server(hbm_budget_bytes=1 << 30, max_slots=2)
    t = srv.submit(p, 3)
    flux, bal, lat = srv.result(t)
    srv.destroy()
    s = S.Solver(p)
    s.advance(3)
    assert np.array_equal(flux, s.get_flux(0))
    s.destroy()
