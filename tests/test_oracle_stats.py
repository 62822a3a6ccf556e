"""Pins for the oracle's statistics (the sample-size and burn-in formulas of Sec. 3.1, Alg. 3, Skart-P pieces).

* Gelman-Rubin: a worked-by-hand example (golden file) and the identical-chains
  case R = sqrt(1 - 1/psi) (B = 0).
* N: the binomial special case alpha + beta = 1 (N = q(1-q) z^2 / r^2, 9604 at
  q = 1/2, r = 0.01, s = 0.95) and the asymptotic variance of the sample mean of
  a simulated two-state chain.
* M: the 2x2 transition matrix raised to the M-th power is within eps of its
  limit, and not yet at M-1.
* Quantiles against scipy; the skewness adjustment inverts Willink's cubic.
* Skart statistics from exact integer batch sums: the textbook moments of the
  batch means, the t interval when one batch per chain carries no skewness,
  degenerate and correlated cases, and the exact skewness decision on 0-1 data
  against scipy.
* Alg. 4 control flow on a scripted 0-1 process worked by hand (golden file).
"""
import math
import os

import numpy as np
import pytest
from scipy import stats as sst

from oracle import drivers, stats

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            out[k] = v
    return out


def test_gr_hand_example():
    g = _golden("gr_hand_example.txt")
    x = np.array([[int(ch) for ch in c] for c in g["chains"]])
    assert abs(stats.psrf(x) ** 2 - float(g["rhat2"][0])) < 1e-12


@pytest.mark.parametrize("psi", [4, 16, 100])
def test_gr_identical_chains(psi):
    rng = np.random.default_rng(psi)
    row = rng.integers(0, 2, psi)
    row[0], row[1] = 0, 1
    x = np.tile(row, (5, 1))
    assert abs(stats.psrf(x) - math.sqrt(1 - 1 / psi)) < 1e-12


def test_gr_constant_window_not_converged():
    assert stats.psrf(np.ones((3, 8))) == math.inf


def test_N_binomial_case():
    z = stats.z_of_confidence(0.95)
    assert math.ceil(stats.sample_size_N(0.5, 0.5, z, 0.01)) == 9604
    for a in (0.1, 0.3, 0.77):
        b = 1 - a
        q = a / (a + b)
        assert abs(stats.sample_size_N(a, b, z, 0.02) - q * (1 - q) * z * z / 0.02 ** 2) < 1e-6
    # worked sequence 0 0 1 1 0: every pair type once -> alpha = beta = 1/2
    cnt = stats.transition_counts(np.array([[0, 0, 1, 1, 0]]))
    assert cnt == (1, 1, 1, 1)
    assert stats.alpha_beta(cnt) == (0.5, 0.5)
    assert stats.burn_in_M(0.5, 0.5, 1e-10) == 0


def test_N_matches_two_state_variance():
    # N z^-2 r^2 is the asymptotic variance of the sample mean times the length.
    rng = np.random.default_rng(5)
    a, b, L, reps = 0.05, 0.15, 4000, 1500
    x = np.zeros((reps, L), np.int8)
    x[:, 0] = rng.random(reps) < a / (a + b)
    u = rng.random((reps, L))
    for t in range(1, L):
        prev = x[:, t - 1]
        x[:, t] = np.where(prev == 1, u[:, t] >= b, u[:, t] < a)
    var_emp = x.mean(axis=1).var(ddof=1) * L
    var_formula = stats.sample_size_N(a, b, 1.0, 1.0)
    assert abs(var_emp / var_formula - 1) < 0.12


@pytest.mark.parametrize("a,b", [(0.05, 0.15), (0.3, 0.01), (0.9, 0.8), (0.002, 0.004)])
def test_M_reaches_eps(a, b):
    eps = 1e-10
    M = stats.burn_in_M(a, b, eps)
    P = np.array([[1 - a, a], [b, 1 - b]])
    pi = np.array([b, a]) / (a + b)

    def dev(m):
        Pm = np.linalg.matrix_power(P, m)
        return np.abs(Pm - pi[None, :]).max()
    assert dev(M) <= eps * (1 + 1e-6)
    assert dev(M - 1) > eps * (1 - 1e-6)


def test_quantiles_vs_scipy():
    for s in (0.5, 0.9, 0.95, 0.99, 0.999999):
        z = stats.z_of_confidence(s)
        assert abs(z - sst.norm.ppf(0.5 * (1 + s))) <= 1e-15 * max(1, abs(z)) * 4
    for p in (1e-300, 1e-20, 1e-5, 0.02, 0.3, 0.7, 0.98):
        assert abs(stats.normal_quantile(p) - sst.norm.ppf(p)) <= 1e-14 * abs(sst.norm.ppf(p))
    assert stats.z_of_confidence(0.95) == pytest.approx(1.959963984540054, rel=1e-15)
    for nu in (100, 500, 1279, 10000):
        for p in (0.975, 0.995, 0.025, 0.9):
            err = 1e-9 if nu < 1000 else 1e-12
            assert abs(stats.t_quantile(p, nu) - sst.t.ppf(p, nu)) < err


def test_willink_inverts_cubic():
    for beta in (1e-4, 0.01, 0.05, -0.03):
        for zeta in (-2.5, -1.96, 0.3, 1.96, 2.8):
            g = stats.willink_G(zeta, beta)
            b2 = 2 * beta
            h = g + b2 * g * g + b2 * b2 * g ** 3 / 3          # Willink's transform with skew 2 beta
            assert abs(h - (zeta - beta)) < 1e-12
    assert stats.willink_G(1.7, 0.0) == 1.7


def test_ci_reduces_to_t_interval():
    # one batch per chain (no lag pairs) and no skewness adjustment: the textbook t interval
    rng = np.random.default_rng(2)
    K = 1000
    b = rng.binomial(K, 0.3, size=(2000, 1))
    Y = b / K
    mu, lo, hi = stats.adjusted_ci(b, K, 0.05)
    assert mu == b.sum() / (K * b.size)
    se = Y.std(ddof=1) / math.sqrt(Y.size)
    tlo, thi = sst.t.interval(0.95, Y.size - 1, loc=Y.mean(), scale=se)
    skew = sst.skew(Y.ravel())
    # the skewness shift is about beta (1 + 2 t^2) se with beta = skew/(6 sqrt(p)); bound it
    slack = abs(skew) / (6 * math.sqrt(Y.size)) * 12.0 * se + 1e-12
    assert abs(lo - tlo) < slack and abs(hi - thi) < slack
    # symmetric batch sums (each b beside K - b): skewness exactly 0, the t interval itself
    bs = np.concatenate([b, K - b])
    Ys = bs / K
    mu, lo, hi = stats.adjusted_ci(bs, K, 0.05)
    assert mu == 0.5
    se = Ys.std(ddof=1) / math.sqrt(Ys.size)
    tlo, thi = sst.t.interval(0.95, Ys.size - 1, loc=Ys.mean(), scale=se)
    assert abs(lo - tlo) < 1e-11 and abs(hi - thi) < 1e-11


def _textbook(b, K):
    """The batch-mean statistics from their definitions, in floating point:
    mean, sum of squared deviations, third central sum, lag-1 products and the
    von Neumann numerator over within-chain neighbours."""
    Y = np.asarray(b, dtype=np.float64) / K
    mu = Y.mean()
    d = Y - mu
    ss = float(np.sum(d * d))
    s3 = float(np.sum(d * d * d))
    lag = float(np.sum(d[:, 1:] * d[:, :-1]))
    dn = float(np.sum((Y[:, 1:] - Y[:, :-1]) ** 2))
    return mu, ss, s3, lag, dn


@pytest.mark.parametrize("omega,m,K,seed", [(64, 20, 16, 1), (3, 200, 1, 2), (500, 3, 1000, 3),
                                            (1500, 1, 77, 4), (7, 90, 1 << 20, 5)])
def test_batch_moments_match_definitions(omega, m, K, seed):
    """The exact integer aggregates equal the textbook moments of the batch means
    (mean, squared and cubed deviations, lag-1 products, squared successive
    differences) within rounding, on skewed and autocorrelated batch sums."""
    rng = np.random.default_rng(seed)
    walk = np.cumsum(rng.normal(size=(omega, m)), axis=1)               # autocorrelated within chains
    q = 1.0 / (1.0 + np.exp(-walk / 3.0 - 1.5))                           # skewed towards 1
    b = rng.binomial(K, q)
    g = stats.batch_moments(b)
    mu, ss, s3, lag, dn = _textbook(b, K)
    P = omega * m
    assert g["P"] == P and g["pairs"] == omega * (m - 1)
    assert math.isclose(g["S1"] / (K * P), mu, rel_tol=1e-13)
    assert math.isclose(g["Q2"] / (K * K * P), ss, rel_tol=1e-10)
    assert math.isclose(g["Q3"] / (K ** 3 * P * P), s3, rel_tol=1e-8, abs_tol=1e-12 * abs(ss) ** 1.5)
    assert math.isclose(g["QL"] / (K * K * P * P), lag, rel_tol=1e-9, abs_tol=1e-12 * ss)
    assert math.isclose(g["D2"] / (K * K), dn, rel_tol=1e-12, abs_tol=1e-300)
    # the interval itself against one built from the textbook moments
    mu2, lo, hi = stats.adjusted_ci(b, K, 0.05)
    if m >= 2:
        phi = (lag / (omega * (m - 1))) / (ss / P)
    else:
        phi = 0.0
    A = (1 + phi) / (1 - phi) if phi > 0 else 1.0
    se = math.sqrt(A * ss / (P - 1) / P)
    beta = ((s3 / P) / (ss / P) ** 1.5) / (6 * math.sqrt(P))
    t = sst.t.ppf(0.975, P - 1)
    want_lo = mu - stats.willink_G(t, beta) * se
    want_hi = mu - stats.willink_G(-t, beta) * se
    assert abs(lo - want_lo) < 1e-9 * se and abs(hi - want_hi) < 1e-9 * se
    # the von Neumann decision from its definition
    if m >= 2:
        C = 1.0 - (dn / (omega * (m - 1))) / (2.0 * ss / (P - 1))
        crit = sst.norm.ppf(0.8) / math.sqrt(omega * (m - 1))
        if abs(C - crit) > 1e-9:
            assert stats.von_neumann_passes(b) == (C <= crit)


def test_batch_statistics_degenerate():
    # all batch means equal: passes the randomness test, point interval
    b = np.full((10, 30), 5)
    assert stats.von_neumann_passes(b)
    assert stats.adjusted_ci(b, 9, 0.05) == (5 / 9, 5 / 9, 5 / 9)
    # one batch off: a proper interval around the mean
    b[3, 7] = 6
    mu, lo, hi = stats.adjusted_ci(b, 9, 0.05)
    assert lo < mu < hi and mu == (5 * 300 + 1) / (9 * 300)
    # alternating means within each chain: perfectly negatively correlated neighbours pass
    alt = np.tile([0, 4], (5, 60))
    assert stats.von_neumann_passes(alt)
    # a monotone ramp in every chain: strongly positively correlated, fails
    ramp = np.tile(np.arange(120) // 10, (5, 1))
    assert not stats.von_neumann_passes(ramp)


def test_skewness_exceeds_4_exactly():
    """The exact decision on 0-1 data agrees with the sample skewness of the
    data (scipy, population moments) away from the boundary, and with the
    boundary worked by hand: 20 q^2 - 20 q + 1 = 0 at q = 0.0528 and 0.9472."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        count = int(rng.integers(100, 3000))
        ones = int(rng.integers(1, count))
        x = np.zeros(count)
        x[:ones] = 1
        B = sst.skew(x)
        if abs(abs(B) - 4.0) > 1e-6:
            assert stats.skewness_exceeds_4(ones, count) == (abs(B) > 4.0), (ones, count)
    assert stats.skewness_exceeds_4(50, 1000) and not stats.skewness_exceeds_4(60, 1000)   # q = 0.05, 0.06
    assert stats.skewness_exceeds_4(950, 1000) and not stats.skewness_exceeds_4(940, 1000)
    assert stats.skewness_exceeds_4(0, 1280) and stats.skewness_exceeds_4(1280, 1280)
    assert not stats.skewness_exceeds_4(640, 1280)


class ScriptedChains:
    """Stand-in for oracle chains: position l holds ((l-1) div 2) mod 2."""

    def __init__(self, omega):
        self.omega = omega
        self.length = 0

    def extend_to(self, L):
        self.length = max(self.length, L)

    @property
    def bits(self):
        l = np.arange(1, self.length + 1)
        row = (((l - 1) // 2) % 2).astype(np.uint8)
        return np.tile(row, (1, self.omega, 1))


def test_parallel_two_state_hand_trace():
    g = _golden("parallel_two_state_hand_trace.txt")
    res = drivers.estimate_probability_in_parallel(ScriptedChains(2), 0, 4, 1.1, 1e-10, 0.01, 0.95, 1 << 20)
    for key in ("psi_gr", "psi", "n", "N", "M", "chain_len"):
        assert res[key] == int(g[key][0]), key
    assert res["prob"] == float(g["prob"][0])


class _Alternating:
    """A one-chain stand-in whose recorded indicator alternates 0, 1, 0, 1, ..."""
    omega = 1

    def __init__(self):
        self.length = 0
        self.bits = [np.zeros((1, 0), dtype=np.uint8)]

    def extend_to(self, l):
        self.length = max(self.length, l)
        self.bits = [(np.arange(self.length) % 2).astype(np.uint8)[None, :]]


def test_sequential_alternating_window():
    """Alg. 1 on a strictly alternating indicator: alpha = beta = 1, so the
    burn-in is 0 (|1 - alpha - beta| = 1) and the formula's sample size is 0,
    read as one position: the estimate is the last position of the initial
    trajectory of m0 + n0 = 20 positions (position 20: a one)."""
    r = drivers.estimate_probability(_Alternating(), 0, 4, 16, 1e-10, 0.01, 0.95, 1 << 20)
    assert (r["status"], r["M"], r["N"], r["chain_len"], r["prob"]) == (0, 0, 1, 20, 1.0)



class _Pattern:
    """A one-chain stand-in whose recorded indicator at 0-based position i is f(i)."""
    omega = 1

    def __init__(self, f):
        self.f = f
        self.length = 0
        self.bits = [np.zeros((1, 0), dtype=np.uint8)]

    def extend_to(self, l):
        self.length = max(self.length, l)
        self.bits = [np.array([self.f(i) for i in range(self.length)], dtype=np.uint8)[None, :]]


def test_sequential_skart_spacer_skips_warm_up():
    """Alg. 2 on the indicator 000111000111...: the adjacent batch means (kappa
    = 1: the skewness of a half-ones window is near 0) are strongly correlated,
    so the test fails without a spacer; with one spacer batch the tested means
    are x1, x3, x5, ... = 0,1,1,0,1,1,... (negatively correlated), which passes.
    The first zeta = 1 position is skipped and the estimate is the mean of
    positions 2..1280 (1-based): 213 whole periods of 6 minus the leading zero
    at position 1, i.e. 639 ones out of 1279."""
    r = drivers.estimate_ci(_Pattern(lambda i: (i // 3) % 2), 0, 0.1, 0.95, 1 << 20)
    assert (r["status"], r["kappa"], r["psi"], r["batches"], r["chain_len"]) == (0, 1, 1, 1279, 1280)
    assert r["prob"] == 639 / 1279
    assert r["ci_lo"] < r["prob"] < r["ci_hi"]


def test_sequential_skart_reduces_to_t_interval():
    """Alg. 2 on the alternating indicator 0101...: kappa = 1 (skewness 0), no
    spacer (lag-1 correlation -1 passes), lag-1 correlation <= 0 gives A = 1 and
    640 ones out of 1280 give zero skewness, so the CI is the textbook Student
    t interval on 1280 observations."""
    t = sst.t.ppf(0.975, 1279)
    half = t * math.sqrt((320.0 / 1279.0) / 1280.0)
    r = drivers.estimate_ci(_Pattern(lambda i: i % 2), 0, 0.1, 0.95, 1 << 20)
    assert (r["status"], r["kappa"], r["psi"], r["batches"], r["chain_len"]) == (0, 1, 0, 1280, 1280)
    assert r["prob"] == 0.5
    assert abs(r["ci_lo"] - (0.5 - half)) < 1e-12 and abs(r["ci_hi"] - (0.5 + half)) < 1e-12


def test_sequential_skart_batch_growth():
    """The same indicator with H* = 0.01: the t half-width above (about 0.0274)
    exceeds H*, so kappa grows to ceil((H/H*)^2) = 8; batches of 8 alternating
    positions all have mean 1/2, the CI collapses to a point and the procedure
    ends with 1280 batches of 8 (10240 positions)."""
    t = sst.t.ppf(0.975, 1279)
    H = t * math.sqrt((320.0 / 1279.0) / 1280.0)
    assert math.ceil((H / 0.01) ** 2) == 8
    r = drivers.estimate_ci(_Pattern(lambda i: i % 2), 0, 0.01, 0.95, 1 << 20)
    assert (r["status"], r["kappa"], r["psi"], r["batches"], r["chain_len"]) == (0, 8, 0, 1280, 10240)
    assert (r["prob"], r["ci_lo"], r["ci_hi"]) == (0.5, 0.5, 0.5)


def test_sequential_skart_constant_and_cap():
    """An indicator that is always 1 has unbounded skewness (kappa = 16) and
    equal batch means (the randomness test passes, the CI is a point at 1);
    with a cap below 16*1280 positions it does not converge."""
    r = drivers.estimate_ci(_Pattern(lambda i: 1), 0, 0.01, 0.95, 1 << 20)
    assert (r["status"], r["kappa"], r["psi"], r["batches"], r["chain_len"]) == (0, 16, 0, 1280, 20480)
    assert (r["prob"], r["ci_lo"], r["ci_hi"]) == (1.0, 1.0, 1.0)
    r = drivers.estimate_ci(_Pattern(lambda i: 1), 0, 0.01, 0.95, 20479)
    assert r["status"] == drivers.NOT_CONVERGED


class _TwoAlternating(_Pattern):
    """Two chains whose recorded indicators both alternate 0, 1, 0, 1, ..."""
    omega = 2

    def __init__(self):
        super().__init__(lambda i: i % 2)

    def extend_to(self, l):
        super().extend_to(l)
        self.bits = [np.repeat(self.bits[0], 2, axis=0)]


def test_skart_p_hand_worked():
    """Alg. 3 then Alg. 5 on two alternating chains, psi0 = 4.  The first window
    (positions 5..8) has equal chain means, so B = 0 and R = sqrt(1 - 1/psi) =
    sqrt(3)/2: converged at psi = 4.  Skart-P then reads 640 positions per chain
    from position 5 (1280 observations, zero skewness: kappa = 1); the adjacent
    batch means alternate (the randomness test passes, lag-1 correlation -1
    gives A = 1) and 640 ones of 1280 give zero skewness, so the CI is the
    Student t interval on 1280 values around 1/2.  With H* = 0.01 the half-width
    (about 0.0274) asks for kappa = ceil((H/H*)^2) = 8, where every batch mean is
    1/2: a point CI after 4 + 8 * 640 positions."""
    t = sst.t.ppf(0.975, 1279)
    half = t * math.sqrt((320.0 / 1279.0) / 1280.0)
    r = drivers.estimate_ci_in_parallel(_TwoAlternating(), 0, 4, 1.1, 0.1, 0.95, 1 << 20)
    assert (r["status"], r["psi_gr"], r["psi"], r["kappa"], r["batches"], r["n"], r["chain_len"]) == \
        (0, 4, 4, 1, 1280, 640, 644)
    assert abs(r["rhat"] - math.sqrt(3.0) / 2.0) < 1e-15
    assert r["prob"] == 0.5
    assert abs(r["ci_lo"] - (0.5 - half)) < 1e-12 and abs(r["ci_hi"] - (0.5 + half)) < 1e-12
    assert math.ceil((half / 0.01) ** 2) == 8
    r = drivers.estimate_ci_in_parallel(_TwoAlternating(), 0, 4, 1.1, 0.01, 0.95, 1 << 20)
    assert (r["status"], r["kappa"], r["batches"], r["n"], r["chain_len"]) == (0, 8, 1280, 5120, 5124)
    assert (r["prob"], r["ci_lo"], r["ci_hi"]) == (0.5, 0.5, 0.5)
