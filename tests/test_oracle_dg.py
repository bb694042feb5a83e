"""Pins of the oracle's DG S_N collided solve (step 2 of Sec. 2.2; bilinear
discontinuous Galerkin in space, Sec. 1 abstract; Gauss-Legendre S_N
estimator of <Psi>, Sec. 2.2)."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("order", [2, 4, 8, 12, 16])
def test_quadrature_moments(oracle, order):
    ox, oy, w = oracle.quadrature(order)
    assert len(w) == order * order
    assert w.sum() == pytest.approx(4 * math.pi, rel=1e-14)
    assert abs((w * ox).sum()) < 1e-13 and abs((w * oy).sum()) < 1e-13
    assert (w * ox * ox).sum() == pytest.approx(4 * math.pi / 3, rel=1e-13)
    assert (w * oy * oy).sum() == pytest.approx(4 * math.pi / 3, rel=1e-13)
    assert abs((w * ox * oy).sum()) < 1e-13
    if order >= 4:
        assert (w * ox ** 4).sum() == pytest.approx(4 * math.pi / 5, rel=1e-13)
    assert np.all(np.abs(ox) > 0) and np.all(np.abs(oy) > 0)


@pytest.mark.parametrize("a,b", [(0.7, 0.3), (-0.45, 0.8), (0.2, -0.9), (-0.6, -0.55)])
def test_manufactured_bilinear_solution_is_exact(oracle, a, b):
    """psi = c0 + c1 x + c2 y + c3 x y lies in Q1 on every cell and its
    source a psi_x + b psi_y + sig psi is in Q1 too, so upwind DG with the exact
    inflow trace must reproduce psi at every node (consistency)."""
    nx, ny, box = 5, 4, (0.0, 1.5, -0.5, 1.5)
    c0, c1, c2, c3 = 0.3, -1.2, 0.8, 2.1
    rng = np.random.default_rng(2)
    sig = rng.uniform(0.1, 5.0, size=nx * ny)
    hx, hy = (box[1] - box[0]) / nx, (box[3] - box[2]) / ny

    def psi(x, y):
        return c0 + c1 * x + c2 * y + c3 * x * y

    src = np.zeros((ny, nx, 4))
    ref = np.zeros((ny, nx, 4))
    for j in range(ny):
        for i in range(nx):
            for k in range(4):
                x = box[0] + (i + (k & 1)) * hx
                y = box[2] + (j + (k >> 1)) * hy
                ref[j, i, k] = psi(x, y)
                src[j, i, k] = a * (c1 + c3 * y) + b * (c2 + c3 * x) + sig[j * nx + i] * psi(x, y)
    xb = box[0] if a > 0 else box[1]
    yb = box[2] if b > 0 else box[3]
    in_x = np.array([[psi(xb, box[2] + (j + t) * hy) for t in (0, 1)] for j in range(ny)])
    in_y = np.array([[psi(box[0] + (i + t) * hx, yb) for t in (0, 1)] for i in range(nx)])
    got = oracle.dg_sweep(nx, ny, box, sig, a, b, src, in_x.ravel(), in_y.ravel())
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_collided_infinite_medium_interior(oracle):
    """Uniform phi_post far from the boundary: sig_e psi = sig_s/(4 pi)
    (phi_c + phi_post) with sig_e = sig_t + tau/(c dt) gives
    phi_c = sig_s phi_post / (sig_a + tau/(c dt))."""
    ss, sa, dt, tau = 1.0, 0.1, 0.1, 2.0
    n, L = 20, 2.0
    prob = dict(nx=n, ny=n, x_lo=0, x_hi=L, y_lo=0, y_hi=L, sigma_s=np.full((n, n), ss),
                sigma_a=np.full((n, n), sa), dt=dt, c=1.0)
    m = oracle.Mesh(prob)
    phi_post = np.full(n * n, 3.0)
    phi, it, res = oracle.dg_collided(m, oracle.quadrature(8), phi_post, tau, 1e-13, 100)
    exact = ss * 3.0 / (sa + tau / dt)
    centre = phi.reshape(n, n, 4)[n // 2, n // 2]
    np.testing.assert_allclose(centre, exact, rtol=1e-7)
    rho = ss / (ss + sa + tau / dt)
    assert it <= math.ceil(math.log(1e-13) / math.log(rho)) + 2
    assert res <= 1e-13


def test_zero_source_gives_zero(oracle):
    n = 4
    prob = dict(nx=n, ny=n, x_lo=0, x_hi=1, y_lo=0, y_hi=1, sigma_s=np.ones((n, n)),
                sigma_a=np.ones((n, n)), dt=0.1, c=1.0)
    phi, it, res = oracle.dg_collided(oracle.Mesh(prob), oracle.quadrature(4), np.zeros(n * n))
    assert np.all(phi == 0.0) and it == 1


def test_si_converges_to_fixed_point(oracle):
    """The SI fixed point satisfies phi = sum_m w_m psi_m[phi] to the
    tolerance: one extra sweep from the returned phi changes it by <= tol."""
    from paper_2511_16821_amd import workloads as W
    p = W.checkerboard(blocks=3, cells_per_block=3, n_s=1, dt=0.5)
    m = oracle.Mesh(p)
    rng = np.random.default_rng(4)
    phi_post = rng.uniform(0, 1, size=m.ncell)
    quad = oracle.quadrature(4)
    phi, it, res = oracle.dg_collided(m, quad, phi_post, 2.0, 1e-12, 500)
    phi2, it2, _ = oracle.dg_collided(m, quad, phi_post, 2.0, 1e-14, 500)
    assert it2 >= it
    assert np.linalg.norm(phi - phi2) <= 1e-11 * np.linalg.norm(phi2)


def test_reflective_box_is_infinite_medium(oracle):
    """Reflective sides on all four faces: a uniform phi_post gives the
    infinite-medium value sig_s phi_post / (sig_a + tau/(c dt)) in every cell,
    not only far from the boundary."""
    ss, sa, dt, tau = 1.0, 0.1, 0.1, 2.0
    n, L = 6, 0.6
    prob = dict(nx=n, ny=n, x_lo=0, x_hi=L, y_lo=0, y_hi=L, sigma_s=np.full((n, n), ss),
                sigma_a=np.full((n, n), sa), dt=dt, c=1.0, boundary=15)
    phi, it, res = oracle.dg_collided(oracle.Mesh(prob), oracle.quadrature(6), np.full(n * n, 3.0),
                                      tau, 1e-13, 400)
    np.testing.assert_allclose(phi, ss * 3.0 / (sa + tau / dt), rtol=1e-11)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_reflective_side_is_a_symmetry_plane(oracle, axis):
    """A problem mirror-symmetric about x = L/2 (or y = L/2) solved on the full
    mesh with vacuum sides, and on one half with the cut side reflective:
    the half solution is the full solution restricted to that half."""
    rng = np.random.default_rng(12)
    n, L = 8, 1.6
    half = rng.uniform(0.2, 3.0, size=(n, n // 2))
    ss = np.concatenate([half, half[:, ::-1]], axis=1)
    sa = np.concatenate([half[::-1, :] * 0.3, (half[::-1, :] * 0.3)[:, ::-1]], axis=1)
    post = rng.uniform(0.0, 2.0, size=(n, n // 2))
    pp = np.concatenate([post, post[:, ::-1]], axis=1)
    if axis == "y":
        ss, sa, pp = ss.T.copy(), sa.T.copy(), pp.T.copy()
    full = dict(nx=n, ny=n, x_lo=0, x_hi=L, y_lo=0, y_hi=L, sigma_s=ss, sigma_a=sa, dt=0.2,
                c=1.0)
    quad = oracle.quadrature(6)
    phi_f, _, _ = oracle.dg_collided(oracle.Mesh(full), quad, pp.ravel(), 2.0, 1e-14, 500)
    phi_f = phi_f.reshape(n, n, 4)
    if axis == "x":
        hp = dict(full, nx=n // 2, x_hi=L / 2, sigma_s=ss[:, :n // 2], sigma_a=sa[:, :n // 2],
                  boundary=2)
        phi_h, _, _ = oracle.dg_collided(oracle.Mesh(hp), quad, pp[:, :n // 2].ravel(), 2.0,
                                         1e-14, 500)
        want = phi_f[:, :n // 2]
        phi_h = phi_h.reshape(n, n // 2, 4)
    else:
        hp = dict(full, ny=n // 2, y_hi=L / 2, sigma_s=ss[:n // 2], sigma_a=sa[:n // 2],
                  boundary=8)
        phi_h, _, _ = oracle.dg_collided(oracle.Mesh(hp), quad, pp[:n // 2].ravel(), 2.0,
                                         1e-14, 500)
        want = phi_f[:n // 2]
        phi_h = phi_h.reshape(n // 2, n, 4)
    assert np.linalg.norm(phi_h - want) <= 1e-11 * np.linalg.norm(want)


def _dsa_cases():
    from paper_2511_16821_amd import workloads as W
    return [("duct", W.duct(n_s=0, n_particles=6000)),
            ("closed box", W.c1(n_s=0, steady=True, n_particles=6000, boundary=15)),
            ("quarter box", W.c1(n_s=1, steady=True, n_particles=6000, boundary=5)),
            ("checkerboard", W.checkerboard(blocks=5, cells_per_block=4, n_s=1,
                                            n_particles=8000, dt=0.05, sn_order=6))]


@pytest.mark.parametrize("case", range(4))
def test_dsa_reaches_the_source_iteration_fixed_point(oracle, case):
    """Diffusion synthetic acceleration changes the iteration, not its fixed
    point: at a tight tolerance both give the same collided flux, and the
    accelerated one needs fewer sweeps (vacuum or reflective sides)."""
    name, p = _dsa_cases()[case]
    p = dict(p, si_tol=1e-13, si_max_iter=1000)
    a = oracle.HybridOracle(p).step()
    b = oracle.HybridOracle(dict(p, si_accel=1)).step()
    assert np.array_equal(a["phi_post"], b["phi_post"])
    err = np.linalg.norm(b["phi_c"] - a["phi_c"]) / np.linalg.norm(a["phi_c"])
    assert err <= 1e-10, (name, err)
    assert b["si_iters"] < a["si_iters"], (name, a["si_iters"], b["si_iters"])


def test_dsa_closed_box_closed_form(oracle):
    """In a closed homogeneous box with a uniform collided source the
    accelerated iteration still converges to sigma_s phi_post / sigma_a."""
    from paper_2511_16821_amd import workloads as W
    n, ss, sa = 6, 0.9, 0.1
    p = W.homogeneous_box(n=n, L=3.0, sig_s=ss, sig_a=sa, src_cells=((0, n), (0, n)), n_s=0,
                          n_particles=1, sn_order=4, steady=True, boundary=15)
    m = oracle.Mesh(p)
    phi_post = np.full(n * n, 2.0)
    phi, it, res = oracle.dg_collided_dsa(m, oracle.quadrature(4), phi_post, tol=1e-13,
                                          max_iter=2000)
    assert np.allclose(phi, ss * 2.0 / sa, rtol=1e-10, atol=0)
    _, it0, _ = oracle.dg_collided(m, oracle.quadrature(4), phi_post, tol=1e-13, max_iter=2000)
    assert it < it0


def test_dsa_reduction_factor_matches_fourier_analysis(oracle):
    """In a thick, scattering-dominated medium of optically thin cells, the
    error of diffusion-synthetic-accelerated source iteration falls per sweep
    by about 0.2247 c, the Fourier-analysis factor of DSA in an infinite
    medium (Alcouffe 1977; Larsen 1982), where plain source iteration
    approaches c.  Here c = 0.99, sigma_t h = 0.25."""
    from paper_2511_16821_amd import workloads as W
    n = 24
    p = W.homogeneous_box(n=n, L=1.2, sig_s=4.95, sig_a=0.05, src_cells=((8, 16), (8, 16)),
                          n_s=0, n_particles=1, sn_order=4, steady=True)
    m = oracle.Mesh(p)
    phi_post = np.zeros(n * n)
    phi_post.reshape(n, n)[8:16, 8:16] = 1.0

    def ratios(solve):
        r = [solve(m, oracle.quadrature(4), phi_post, tol=1e-300, max_iter=k)[2]
             for k in range(1, 12)]
        return np.array(r[1:]) / np.array(r[:-1])

    si, dsa = ratios(oracle.dg_collided), ratios(oracle.dg_collided_dsa)
    assert si[-1] > 0.8
    assert np.all(dsa[3:] > 0.15) and np.all(dsa[3:] < 0.25), dsa


@pytest.mark.parametrize("n_s", [0, 5])
def test_whole_flux_stopping_rule(oracle, n_s):
    """The whole-flux test stops at the first sweep whose change is within
    tol of the nodal norm of phi_c + phi_pre + phi_post, recomputed here from
    the iterates (N_s = 0: the uncollided part is all post-limit; 5: mostly
    pre-limit)."""
    from paper_2511_16821_amd import workloads as W
    tol = 1e-6
    p = W.duct(n_s=n_s, n_particles=8000)
    r = oracle.HybridOracle(p).step()
    m, quad = oracle.Mesh(p), oracle.quadrature(4)
    pre, post = r["phi_pre"], r["phi_post"]
    it = oracle.dg_collided(m, quad, post, 2.0, tol, 1000, phi_pre=pre)[1]

    def iterate(k):
        return oracle.dg_collided(m, quad, post, 2.0, 0.0, k, phi_pre=pre)[0]

    def rule(k):
        a, b = iterate(k), iterate(k - 1)
        ref = a + (pre + post)[:, None]
        return np.linalg.norm(a - b) <= tol * np.linalg.norm(ref)

    assert it >= 3 and rule(it) and not rule(it - 1)
