"""Pins of the oracle's prescribed inflow (Sec. 2.1 boundary data G, applied
in the MC legs of Sec. 2.2 steps 1 and 3): particles entering through the
boundary faces with the cosine law about the inward normal and weights that
carry the partial current pi G per unit length.

Closed form: an isotropic inflow G on one side of a purely absorbing
half-space (the other two sides reflective, so the problem is 1D) gives the
scalar flux 2 pi G E_2(sigma d) at depth d, whose average over a cell
[a, b] of depth is 2 pi G (E_3(sigma a) - E_3(sigma b)) / (sigma (b - a))."""
import numpy as np
import pytest
from scipy.special import expn

from oracle import oracle as O


def _slab(side, n_long=20, n_wide=4, G=2.0, sig=1.0, depth=2.0):
    from paper_2511_16821_amd import workloads as W
    nx, ny = (n_long, n_wide) if side < 2 else (n_wide, n_long)
    w = depth * n_wide / n_long
    p = W.homogeneous_box(n=4, L=2.0, n_s=-1, n_particles=200_000, steady=True, sn_order=2)
    p.update(nx=nx, ny=ny, x_hi=depth if side < 2 else w, y_hi=w if side < 2 else depth,
             boundary=(4 | 8) if side < 2 else (1 | 2))
    p["sigma_s"] = np.zeros((ny, nx))
    p["sigma_a"] = np.full((ny, nx), sig)
    p["q"] = np.zeros((ny, nx))
    g = np.zeros(2 * (nx + ny))
    start = {0: 0, 1: ny, 2: 2 * ny, 3: 2 * ny + nx}[side]
    g[start:start + (ny if side < 2 else nx)] = G
    p["inflow"] = g
    return p, w


@pytest.mark.parametrize("side", [0, 1, 2, 3])
def test_inflow_half_space_closed_form(side):
    O.build()
    G, sig, depth, n_long = 2.0, 1.0, 2.0, 20
    p, width = _slab(side, n_long=n_long, G=G, sig=sig, depth=depth)
    r = O.HybridOracle(p).step()
    phi = r["phi_R"].reshape(p["ny"], p["nx"])
    prof = phi.mean(axis=0) if side < 2 else phi.mean(axis=1)  # along the depth axis
    if side in (1, 3):
        prof = prof[::-1]  # depth measured from the side with the inflow
    d = np.linspace(0.0, depth, n_long + 1)
    exact = 2 * np.pi * G * (expn(3, sig * d[:-1]) - expn(3, sig * d[1:])) / (sig * (d[1] - d[0]))
    assert np.max(np.abs(prof / exact - 1.0)) < 1e-3, (side, prof / exact - 1.0)
    # the emitted weight is the partial current pi G times the side's length,
    # within one weight quantum per face (the counts' randomized rounding)
    b = r["bal_mc"]
    n_faces = len(p["inflow"])
    assert abs(b["source_w"] - np.pi * G * width) <= n_faces * b["weight_quantum"]


def test_inflow_on_a_reflective_side_is_rejected():
    p, _ = _slab(0)
    p["boundary"] = 1  # x_lo reflective, where the inflow is
    with pytest.raises(ValueError):
        O.HybridOracle(p)
