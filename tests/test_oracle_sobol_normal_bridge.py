"""Pins for the oracle's point set, inverse normal and Brownian bridge.

Each check compares the oracle with something other than itself: SciPy's and
PyTorch's independent Sobol implementations, the closed-form van der Corput
sequence, SciPy's ``ndtri`` within Moro's published accuracy, and the
covariance of Brownian motion.
"""
import numpy as np
import pytest


def _scipy_sobol_ints(d, count, skip=0):
    import scipy.stats.qmc as q
    e = q.Sobol(d=d, scramble=False, bits=32)
    if skip:
        e.fast_forward(skip)
    pts = e.random(count)
    ints = np.rint(pts * 2.0 ** 32).astype(np.uint64)
    assert ints.max() < 2 ** 32
    return ints.astype(np.uint32)


@pytest.mark.parametrize("d,count", [(1, 4097), (50, 16385), (100, 4097), (252, 2049), (365, 1025)])
def test_sobol_matches_scipy_bit_exact(orc, d, count):
    ours = orc.sobol_block(d, 0, count)
    assert np.array_equal(ours, _scipy_sobol_ints(d, count))


def test_sobol_matches_scipy_far_index(orc):
    # positions around 2^20 (fast_forward walks the Gray code, so keep it modest)
    first = (1 << 20) - 3
    ours = orc.sobol_block(8, first, 7)
    assert np.array_equal(ours, _scipy_sobol_ints(8, 7, skip=first))


def test_sobol_matches_torch_30bit(orc):
    import torch
    eng = torch.quasirandom.SobolEngine(dimension=40, scramble=False)
    t = eng.draw(2049, dtype=torch.float64).numpy()
    tint = np.rint(t * 2.0 ** 30).astype(np.uint64)
    ours = orc.sobol_block(40, 0, 2049).astype(np.uint64) >> 2
    assert np.array_equal(ours, tint)


def _bitrev32(v):
    return int(f"{v:032b}"[::-1], 2)


def test_sobol_first_dimension_is_van_der_corput_in_gray_order(orc):
    # closed form: dimension 1 is the radical inverse of the Gray code
    n = np.arange(0, 3000, dtype=np.uint64)
    ours = orc.sobol_block(1, 0, len(n))[:, 0]
    want = [_bitrev32(int(k ^ (k >> 1))) for k in n]
    assert np.array_equal(ours, np.array(want, dtype=np.uint32))


def test_sobol_net_property(orc):
    # (0, m, 1)-net: each block of 2^m points aligned at a multiple of 2^m puts
    # exactly one point in each dyadic interval of length 2^-m, in every dim
    m = 6
    pts = orc.sobol_block(20, 64 * 5, 64)
    for j in range(20):
        top = np.sort(pts[:, j] >> (32 - m))
        assert np.array_equal(top, np.arange(64))


def test_inverse_normal_within_moro_bound(orc):
    from scipy.special import ndtri
    u = np.concatenate([np.linspace(1e-10, 1 - 1e-10, 20001),
                        np.geomspace(1e-10, 0.08, 2000), 1 - np.geomspace(1e-10, 0.08, 2000)])
    ours = np.array([orc.inv_normal(x) for x in u])
    err = np.abs(ours - ndtri(u))
    # Moro (1995) quotes a maximum absolute error of about 3e-9 on [1e-10, 1-1e-10]
    assert err.max() < 3.2e-9
    # the rational central part is far more accurate near the median
    c = np.abs(u - 0.5) < 0.4
    assert err[c].max() < 3.2e-9


def test_inverse_normal_integer_odd_symmetry(orc):
    rng = np.random.default_rng(7)
    xs = rng.integers(1, 2 ** 32, size=5000, dtype=np.uint64)
    for x in xs[:2000]:
        x = int(x)
        assert orc.inv_normal_u32(x) == -orc.inv_normal_u32((1 << 32) - x)
    assert orc.inv_normal_u32(1 << 31) == 0.0


def test_inverse_normal_monotone(orc):
    xs = np.unique(np.concatenate([np.linspace(1, 2 ** 32 - 1, 30001).astype(np.uint64),
                                   np.arange(1, 3000, dtype=np.uint64)]))
    z = np.array([orc.inv_normal_u32(int(x)) for x in xs])
    assert np.all(np.diff(z) > 0)


def test_inverse_normal_u32_matches_real_argument(orc):
    # u = x 2^-32 is exact in binary64, so both entry points must agree bitwise
    rng = np.random.default_rng(5)
    xs = [1, 12345, 1 << 20, 0x40000000, 0x7FFFFFFF, 0x80000001, 0xC0000000, 0xFFFFFFFF]
    xs += [int(v) for v in rng.integers(1, 2 ** 32, size=4000, dtype=np.uint64)]
    for x in xs:
        assert orc.inv_normal_u32(x) == orc.inv_normal(x / 2.0 ** 32)


@pytest.mark.parametrize("M", [1, 2, 3, 7, 50, 100, 252, 365])
def test_bridge_covariance_is_brownian(orc, M):
    T = 1.7
    B = np.zeros((M, M))
    for q in range(M):
        e = np.zeros(M)
        e[q] = 1.0
        B[:, q] = orc.bridge_apply(M, T, e)[1:]
    t = np.arange(1, M + 1) * T / M
    cov = B @ B.T
    assert np.abs(cov - np.minimum.outer(t, t)).max() < 1e-12


@pytest.mark.parametrize("M", [1, 2, 5, 50, 365])
def test_bridge_nodes_cover_each_date_once(orc, M):
    m, left, right = orc.bridge_nodes(M)
    assert m[0] == M and left[0] == 0
    assert sorted(m.tolist()) == list(range(1, M + 1))
    # breadth-first: a node's parents were set by earlier nodes (or are 0 / M)
    pos = {int(v): i for i, v in enumerate(m)}
    for q in range(1, M):
        assert left[q] < m[q] < right[q]
        for par in (left[q], right[q]):
            assert par == 0 or pos[int(par)] < q
        assert m[q] == (left[q] + right[q]) // 2


def test_bridge_single_date_is_scaled_normal(orc):
    W = orc.bridge_apply(1, 2.25, np.array([0.7]))
    assert W[0] == 0.0 and W[1] == 1.5 * 0.7


def test_bridge_first_dimension_drives_terminal_value(orc):
    # W(T) must depend on dimension 1 only (the bridge's defining property)
    M, T = 37, 1.3
    rng = np.random.default_rng(3)
    z = rng.standard_normal(M)
    z2 = z.copy()
    z2[1:] = rng.standard_normal(M - 1)
    assert orc.bridge_apply(M, T, z)[M] == orc.bridge_apply(M, T, z2)[M]


def test_sobol_tail_points_per_wave_are_bounded(orc):
    # the path generator stages at most 13 tail points (|u - 1/2| >= 0.42) per
    # dimension and wave of 64 paths (Sobol indices 64w + 1 .. 64w + 64): the
    # leading 6 x 6 block of every dimension's generator matrix is triangular
    # with unit diagonal (one point per interval of length 1/64 in each
    # aligned block), and the tails meet 12 such intervals.  Checked on the
    # matrices of all 640 dimensions and by counting points
    V = orc.directions(640).astype(np.uint64)
    for b in range(6):
        # the 6 leading bits of direction number b hold 2^-1 .. 2^-(b+1):
        # 2^-(b+1) set (odd m_b), nothing below it
        top = V[:, b] >> np.uint64(26)
        assert np.all((top >> np.uint64(5 - b)) & np.uint64(1) == 1), b
        assert np.all(top & np.uint64((1 << (5 - b)) - 1) == 0), b
    lo, hi = 0.08 * 2.0 ** 32, 0.92 * 2.0 ** 32
    worst = 0
    for first in (1, 64 * 37 + 1, (1 << 18) + 1):
        pts = orc.sobol_block(640, first, 64 * 8).astype(np.float64)
        for w in range(8):
            blk = pts[64 * w:64 * (w + 1)]
            worst = max(worst, int(((blk <= lo) | (blk >= hi)).sum(axis=0).max()))
    assert worst <= 13
