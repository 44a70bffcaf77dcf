"""Energy-series statistics: the oracle's blocking analysis and correlated-
sampling difference pinned to closed forms and exact properties, and the C-ABI
host implementation (afqmc_reblock, afqmc_cs_difference) against the oracle on
seeded series.  CPU only."""
import os

import numpy as np
import pytest

from oracle import cs_difference, reblock

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ar1(n, rho, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0]
    c = np.sqrt(1.0 - rho * rho)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + c * e[t]
    return x


def _lib():
    from paper_1804_03310_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libafqmc.so is not built; run __graft_entry__.build()")
    import paper_1804_03310_amd as afq
    return afq


# -- oracle pins -------------------------------------------------------------

def test_reblock_uncorrelated_series_matches_sigma_over_sqrt_n():
    """iid N(0, 1): the error of the mean is 1/sqrt(n) at every level."""
    n = 1 << 14
    x = np.random.default_rng(3).standard_normal(n)
    mean, sems, plateau = reblock(x)
    assert plateau >= 0
    assert abs(sems[plateau] * np.sqrt(n) - 1.0) < 0.05
    assert abs(mean) < 4.0 / np.sqrt(n)


@pytest.mark.parametrize("rho", [0.8, 0.95])
def test_reblock_ar1_plateau_matches_closed_form(rho):
    """AR(1) with unit variance: n Var(mean) -> (1 + rho) / (1 - rho); the
    naive level-0 error underestimates it by sqrt((1 - rho) / (1 + rho))."""
    n = 1 << 16
    x = _ar1(n, rho, seed=11)
    _, sems, plateau = reblock(x)
    exact = np.sqrt((1.0 + rho) / ((1.0 - rho) * n))
    assert plateau > 0
    assert abs(sems[plateau] / exact - 1.0) < 0.25
    assert abs(sems[0] * np.sqrt(n) - 1.0) < 0.05


def test_reblock_repeated_values_reach_the_underlying_series_at_level_j():
    """Each value of an iid series repeated 2^j times: level j is that series
    exactly, so its error is the series' own level-0 error."""
    y = np.random.default_rng(5).standard_normal(1 << 10)
    j = 3
    x = np.repeat(y, 1 << j)
    _, sx, _ = reblock(x)
    _, sy, _ = reblock(y)
    assert np.allclose(sx[j:], sy[:len(sx) - j], rtol=1e-12, atol=0)
    assert sx[0] < sx[j]


def test_reblock_shift_and_scale():
    x = _ar1(4096, 0.5, seed=2)
    m0, s0, p0 = reblock(x)
    m1, s1, p1 = reblock(-3.0 * x + 7.0)
    assert abs(m1 - (-3.0 * m0 + 7.0)) < 1e-12
    assert np.allclose(s1, 3.0 * np.asarray(s0), rtol=1e-10)
    assert p1 == p0


def test_cs_difference_constant_offset_has_zero_error():
    a = np.random.default_rng(1).standard_normal((8, 50)) - 100.0
    mean, sem = cs_difference(a, a + 0.25)
    assert np.allclose(mean, 0.25, atol=1e-12)
    assert np.allclose(sem, 0.0, atol=1e-12)


def test_cs_difference_independent_noise_closed_form():
    """Independent N(0, s^2) noise on both series: the cumulative average of
    the difference after t + 1 steps has variance 2 s^2 / (t + 1), so the
    error over R repeats is sqrt(2 s^2 / ((t + 1) R))."""
    R, T, s = 400, 40, 0.3
    rng = np.random.default_rng(9)
    a = s * rng.standard_normal((R, T))
    b = 1.5 + s * rng.standard_normal((R, T))
    mean, sem = cs_difference(a, b)
    t = np.arange(T)
    exact = np.sqrt(2 * s * s / ((t + 1) * R))
    assert np.all(np.abs(sem / exact - 1.0) < 0.15)
    assert np.all(np.abs(mean - 1.5) < 5 * exact)


def test_cs_difference_first_and_missing_steps():
    a = np.zeros((2, 6))
    b = np.array([[1, 2, np.nan, 4, 5, 6], [1, 2, np.nan, 4, 5, 6]], dtype=float)
    mean, sem = cs_difference(a, b, first=1)
    assert np.isnan(mean[0])
    assert mean[1] == 2.0 and mean[2] == 2.0  # the missing step leaves the average
    assert mean[3] == 3.0 and mean[5] == (2 + 4 + 5 + 6) / 4
    assert np.all(sem[1:] == 0.0)
    m1, s1 = cs_difference(a[:1], b[:1])
    assert np.all(np.isnan(s1))


# -- C ABI vs oracle ---------------------------------------------------------

@pytest.mark.parametrize("n,rho", [(2, 0.0), (1001, 0.3), (1 << 13, 0.9)])
def test_reblock_abi_matches_oracle(n, rho):
    afq = _lib()
    x = _ar1(n, rho, seed=n) + 5.0
    m_o, s_o, p_o = reblock(x)
    m_c, s_c, p_c = afq.reblock(x)
    assert abs(m_c - m_o) <= 1e-12 * abs(m_o)
    assert len(s_c) == len(s_o)
    assert np.allclose(s_c, s_o, rtol=1e-12, atol=0)
    assert p_c == p_o


def test_reblock_abi_rejects_bad_input():
    afq = _lib()
    with pytest.raises(afq.AfqmcError):
        afq.reblock([1.0])
    with pytest.raises(afq.AfqmcError):
        afq.reblock([1.0, np.nan, 2.0])


@pytest.mark.parametrize("R,T,first", [(1, 7, 0), (16, 200, 10), (5, 33, 32)])
def test_cs_difference_abi_matches_oracle(R, T, first):
    afq = _lib()
    rng = np.random.default_rng(R * T)
    a = rng.standard_normal((R, T)) - 40.0
    b = a + 0.3 + 0.05 * rng.standard_normal((R, T))
    a[:, ::7] = np.nan  # steps without a measurement
    b[:, ::7] = np.nan
    m_o, s_o = cs_difference(a, b, first)
    m_c, s_c = afq.cs_difference(a, b, first)
    assert np.array_equal(np.isnan(m_c), np.isnan(m_o))
    assert np.array_equal(np.isnan(s_c), np.isnan(s_o))
    f = np.isfinite(m_o)
    assert np.allclose(m_c[f], m_o[f], rtol=1e-12, atol=1e-14)
    g = np.isfinite(s_o)
    assert np.allclose(s_c[g], s_o[g], rtol=1e-10, atol=1e-15)
