"""Pins of the oracle's census: the bank at t_{n+1} holds the kept
candidates ordered by cell, those of a cell in slot order; with census_qmc
the census particles of a cell (a cohort) draw the points of that cell's
census stream at their ranks, a low-discrepancy point set: for identical
particles the variance of the estimate over scramblings falls much faster
than 1/N (reading of Sec. 2.4: the census histories of a step sampled like
its source particles, per cell, from one QMC point set); without it each
history draws from its own stream and the variance falls as 1/N."""
import numpy as np

from oracle import oracle as O


def _cands(n, n_cells, seed):
    rng = np.random.default_rng(seed)
    c = O.Bank(n)
    c.cell[:] = rng.integers(0, n_cells, size=n).astype(np.int32)
    c.hid[:] = (np.arange(n) + 1000).astype(np.uint64)
    c.w[:] = rng.uniform(0.5, 1.5, size=n)
    c.alive = (rng.uniform(size=n) < 0.7).astype(np.uint8)
    return c


def _check_order(cand, bank):
    # ordered by cell; within a cell, the kept candidates in slot order
    assert np.all(np.diff(bank.cell) >= 0)
    slot = {int(h): k for k, h in enumerate(cand.hid)}
    pos = np.array([slot[int(h)] for h in bank.hid])
    for c in np.unique(bank.cell):
        s = pos[bank.cell == c]
        assert np.all(np.diff(s) > 0), c
    assert np.all(cand.alive[pos] == 1)
    assert np.array_equal(bank.cell, cand.cell[pos])


def test_census_bank_ordered_by_cell_in_slot_order():
    O.build()
    cand = _cands(600, 23, 1)
    bank, fac, ovf = O.thin(cand, 10 ** 6, 12345)
    assert fac == 1.0 and not ovf and bank.n == int(cand.alive.sum())
    _check_order(cand, bank)
    # with the cap below the count: the kept subset in the same order
    bank, fac, ovf = O.thin(cand, 200, 12345)
    assert fac > 1.0 and bank.n <= 200
    _check_order(cand, bank)
    assert np.allclose(bank.w, cand.w[[int(h) - 1000 for h in bank.hid]] * fac)


def _identical_census_variance(census_qmc):
    from paper_2511_16821_amd import workloads as W
    O.build()
    p = W.homogeneous_box(n=4, L=2.0, n_s=1, n_particles=1, dt=1.0, sn_order=2,
                          census_qmc=census_qmc)
    p["sigma_s"] = np.full((4, 4), 1.0)
    p["sigma_a"] = np.full((4, 4), 0.5)
    p["q"] = np.zeros((4, 4))
    mesh, pts = O.Mesh(p), O.Points(0)

    def est(n, seed):
        b = O.Bank(n)
        b.x[:] = 0.25
        b.y[:] = 0.25
        b.ox[:] = 0.6
        b.oy[:] = 0.8
        b.w[:] = 1.0
        b.cell[:] = 5
        b.hid[:] = np.arange(n, dtype=np.uint64) + 7
        Ta, Tb, bal, seg, _ = O.mc_pass(mesh, pts, 1, 1, np.zeros(64), 0, b, seed, 3, 1e-8,
                                        False)
        assert abs(bal["census_in_w"] - n) < 1e-9
        return (Ta.sum() + Tb.sum()) / n

    v = {}
    for n in (64, 1024):
        xs = [est(n, 1000 + r) for r in range(32)]
        v[n] = np.var(xs, ddof=1)
    return v


def test_census_cohort_is_a_low_discrepancy_set():
    """N identical census particles in one cell (no source, one scatter
    allowed, scattering and absorbing medium): the mean track length per
    particle over 32 scramblings of the cohort stream.  Plain MC would
    shrink its variance 16-fold from N = 64 to N = 1024; the cohort's
    scrambled Sobol' points shrink it more than 64-fold."""
    v = _identical_census_variance(1)
    assert v[64] > 0.0 and v[64] / v[1024] > 64.0, v


def test_census_streams_per_history_are_plain_mc():
    """The same particles drawing from a stream each (census_qmc = 0): the
    variance falls about 16-fold (1/N), within the sampling error of 32
    runs."""
    v = _identical_census_variance(0)
    assert 6.0 < v[64] / v[1024] < 40.0, v
