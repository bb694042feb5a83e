"""Pins of the oracle's point generator (Sec. 2.4: low-discrepancy points in
place of pseudo-random draws) against things other than itself: scipy's own
Sobol' enumeration, the van der Corput sequence, digital-net stratification,
the nested-scramble property and the published SplitMix64 output."""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def test_splitmix64_published_outputs(oracle):
    # SplitMix64 from state 0: its first two outputs are the published
    # reference values 0xE220A8397B1DCDAF and 0x6E789E6AA1B965F4.
    L = oracle.lib()
    assert L.or_mix64(0) == 0xE220A8397B1DCDAF
    assert L.or_mix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_dim0_is_van_der_corput(oracle):
    V = oracle.sobol_direction_numbers()
    L = oracle.lib()
    for k in list(range(2048)) + [2 ** 31 - 1, 2 ** 32 - 1, 123456789, 3 ** 20]:
        rev = int(format(k, "032b")[::-1], 2)
        assert L.or_sobol_word(V.ctypes.data, 0, k) == rev


def _gray(i):
    return i ^ (i >> 1)


def test_unscrambled_matches_scipy_sequence(oracle):
    """scipy enumerates Sobol' points in Gray-code order; the oracle's natural
    order point gray(i) must be scipy's point i, in all 32 dimensions."""
    from scipy.stats import qmc
    V = oracle.sobol_direction_numbers()
    L = oracle.lib()
    s = qmc.Sobol(d=32, scramble=False, bits=32)
    ref = np.rint(s.random(1024) * 2.0 ** 32).astype(np.uint64)
    for i in range(1024):
        g = _gray(i)
        got = [L.or_sobol_word(V.ctypes.data, d, g) for d in range(32)]
        assert np.array_equal(np.array(got, dtype=np.uint64), ref[i]), i
    # far indices exercise the recurrence-extended direction numbers
    for k in (2 ** 21 + 77, 2 ** 23 + 4097, 3 * 2 ** 22 + 5):
        s = qmc.Sobol(d=32, scramble=False, bits=32)
        s.fast_forward(k)
        ref = np.rint(s.random(1)[0] * 2.0 ** 32).astype(np.uint64)
        got = [L.or_sobol_word(V.ctypes.data, d, _gray(k)) for d in range(32)]
        assert np.array_equal(np.array(got, dtype=np.uint64), ref), k


def _points(oracle, stream, dims, n, mode=0):
    P = oracle.Points(mode)
    return P.block(stream, dims, range(n)).astype(np.uint64)


@pytest.mark.parametrize("stream", [None, 0x1234ABCD5678EF01])
def test_first_two_dims_form_0m2_net(oracle, stream):
    """The first 2^m points of dims (0, 1) put exactly one point in every
    elementary interval of area 2^-m, unscrambled and scrambled."""
    m = 10
    n = 2 ** m
    if stream is None:
        V = oracle.sobol_direction_numbers()
        L = oracle.lib()
        X = np.array([[L.or_sobol_word(V.ctypes.data, d, k) for d in (0, 1)] for k in range(n)],
                     dtype=np.uint64)
    else:
        X = _points(oracle, stream, (0, 1), n)
    for a in range(m + 1):
        b = m - a
        cx = X[:, 0] >> np.uint64(32 - a) if a else np.zeros(n, dtype=np.uint64)
        cy = X[:, 1] >> np.uint64(32 - b) if b else np.zeros(n, dtype=np.uint64)
        cells = cx * np.uint64(2 ** b) + cy
        assert len(np.unique(cells)) == n, (a, b)


def test_every_dim_is_stratified_after_scrambling(oracle):
    """Each 1-D projection of the first 2^m points hits every dyadic interval
    of length 2^-m exactly once (a (0, m, 1)-net), scrambled or not."""
    m = 9
    X = _points(oracle, 0xDEADBEEF, range(32), 2 ** m)
    for d in range(32):
        assert len(np.unique(X[:, d] >> np.uint64(32 - m))) == 2 ** m, d


def test_scramble_is_nested_bijection(oracle):
    """Digit k of the output depends only on input digits 1..k, and the map is
    a bijection on every digit prefix."""
    L = oracle.lib()
    rng = np.random.default_rng(3)
    for s in rng.integers(0, 2 ** 32, size=4):
        s = int(s)
        for _ in range(200):
            x = int(rng.integers(0, 2 ** 32))
            k = int(rng.integers(1, 32))
            low = int(rng.integers(0, 2 ** (32 - k)))
            y = ((x >> (32 - k)) << (32 - k)) | low
            assert (L.or_nested_scramble(x, s) >> (32 - k)) == (L.or_nested_scramble(y, s) >> (32 - k))
        outs = {L.or_nested_scramble(v << 20, s) >> 20 for v in range(4096)}
        assert len(outs) == 4096


def test_u01_open_interval(oracle):
    L = oracle.lib()
    assert L.or_u01(0) == 0.5 * 2.0 ** -32
    assert L.or_u01(0xFFFFFFFF) == 1.0 - 0.5 * 2.0 ** -32
    assert 0.0 < L.or_u01(0) and L.or_u01(0xFFFFFFFF) < 1.0


def test_prng_mode_uniform_and_distinct(oracle):
    X = _points(oracle, 42, (0, 1, 7), 4096, mode=1).astype(np.float64) / 2 ** 32
    for d in range(3):
        # Kolmogorov-Smirnov distance for n = 4096: 1.63/sqrt(n) ~ 0.025 at 1%
        xs = np.sort(X[:, d])
        ks = np.max(np.abs(xs - (np.arange(1, 4097) - 0.5) / 4096))
        assert ks < 0.03
    assert abs(np.corrcoef(X[:, 0], X[:, 1])[0, 1]) < 0.06


def test_sobol_dims_beyond_table_use_hash(oracle):
    P = oracle.Points(0)
    a = P.block(99, (40,), range(8))
    b = P.block(99, (41,), range(8))
    assert not np.array_equal(a, b)


def _radical_inverse_word(b, i):
    """floor(phi_b(i) 2^32) from the definition, in exact rational arithmetic."""
    from fractions import Fraction
    phi, scale = Fraction(0), Fraction(1, b)
    while i > 0:
        phi += (i % b) * scale
        i //= b
        scale /= b
    return int(phi * 2 ** 32)


def test_halton_is_the_radical_inverse(oracle):
    """Halton coordinate d of point i is the radical inverse of i in the d-th
    prime base (Sec. 2.4, Halton 1960): checked against the definition in
    exact arithmetic for every base, small indices and indices near 2^32."""
    primes = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71, 73,
              79, 83, 89, 97, 101, 103, 107, 109, 113, 127, 131]
    rng = np.random.default_rng(3)
    idx = list(range(0, 40)) + [int(v) for v in rng.integers(0, 2 ** 32, size=40)] + [2 ** 32 - 1]
    L = oracle.lib()
    for d, b in enumerate(primes):
        for i in idx:
            assert L.or_halton_u32(d, i) == _radical_inverse_word(b, i), (d, i)
    assert L.or_halton_u32(0, 1) == 2 ** 31 and L.or_halton_u32(0, 3) == 3 * 2 ** 30
    assert L.or_halton_u32(1, 1) == (2 ** 32) // 3


@pytest.mark.parametrize("stream", [1, 0xDEADBEEF])
def test_shifted_halton_stays_stratified(oracle, stream):
    """A shift modulo 1 keeps the van der Corput stratification: the first b^k
    points of a base-b coordinate put exactly one point in each interval
    [j / b^k, (j + 1) / b^k)."""
    P = oracle.Points(2)
    for d, b, k in [(0, 2, 10), (1, 3, 6), (2, 5, 4), (6, 17, 2), (31, 131, 1)]:
        n = b ** k
        u = (P.block(stream, [d], range(n))[:, 0].astype(np.float64) + 0.5) / 2 ** 32
        counts = np.bincount(np.floor(u * n).astype(np.int64), minlength=n)
        assert np.all(counts == 1), (d, b)
