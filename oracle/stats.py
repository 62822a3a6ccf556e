"""The paper's statistics, written out plainly in FP64 (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Gelman-Rubin PSRF: Alg. 3 (Sec. 4.1), the per-chain means and standard
  deviations of the last psi values, B, W, sigma^2 and R.
* Two-state Markov chain sample sizes: Alg. 1, the M and N formulas of its
  burn-in / sample-size step (Sec. 3.1), with alpha and beta estimated from
  transition counts of the 0-1 process.
* Standard normal quantile: Wichura's AS 241 (PPND16), Applied Statistics 37
  (1988) 477-484.
* Student-t quantile: the Cornish-Fisher expansion in 1/nu (Abramowitz and
  Stegun 26.7.5), accurate to ~1e-12 for nu >= 1000 and ~1e-9 for nu >= 100.
* Skart-P pieces used by Alg. 5 (Sec. 4.3): the skewness decision on 0-1
  data, the von Neumann randomness statistic and the skewness- and
  autoregression-adjusted CI on batch means, each from exact integer sums of
  the batch sums (floating point only in the final ratios).
"""
from __future__ import annotations

import ctypes
import ctypes.util
import math
from typing import Sequence, Tuple

import numpy as np

_libm = ctypes.CDLL(ctypes.util.find_library("m") or "libm.so.6")
_libm.cbrt.restype = ctypes.c_double
_libm.cbrt.argtypes = [ctypes.c_double]


def cbrt(x: float) -> float:
    """Real cube root (C library cbrt)."""
    return float(_libm.cbrt(float(x)))


# ------------------------------------------------------------ quantiles

def normal_quantile(p: float) -> float:
    """Phi^{-1}(p) by AS 241 (PPND16)."""
    q = p - 0.5
    if abs(q) <= 0.425:
        r = 0.180625 - q * q
        num = (((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r
                    + 6.7265770927008700853e+4) * r + 4.5921953931549871457e+4) * r
                  + 1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r
                + 1.3314166789178437745e+2) * r + 3.3871328727963666080e0)
        den = (((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r
                    + 3.9307895800092710610e+4) * r + 2.1213794301586595867e+4) * r
                  + 5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r
                + 4.2313330701600911252e+1) * r + 1.0)
        return q * num / den
    r = p if q < 0.0 else 1.0 - p
    r = math.sqrt(-math.log(r))
    if r <= 5.0:
        r = r - 1.6
        num = (((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r
                    + 2.41780725177450611770e-1) * r + 1.27045825245236838258e0) * r
                  + 3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r
                + 4.63033784615654529590e0) * r + 1.42343711074968357734e0)
        den = (((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r
                    + 1.51986665636164571966e-2) * r + 1.48103976427480074590e-1) * r
                  + 6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r
                + 2.05319162663775882187e0) * r + 1.0)
    else:
        r = r - 5.0
        num = (((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r
                    + 1.24266094738807843860e-3) * r + 2.65321895265761230930e-2) * r
                  + 2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r
                + 5.46378491116411436990e0) * r + 6.65790464350110377720e0)
        den = (((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r
                    + 1.84631831751005468180e-5) * r + 7.86869131145613259100e-4) * r
                  + 1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r
                + 5.99832206555887937690e-1) * r + 1.0)
    val = num / den
    return -val if q < 0.0 else val


def z_of_confidence(s: float) -> float:
    """z = Phi^{-1}((1+s)/2) of Alg. 1's sample-size formula."""
    return normal_quantile(0.5 * (1.0 + s))


def t_quantile(p: float, nu: float) -> float:
    """Student-t quantile t_{p, nu}, Cornish-Fisher expansion (A&S 26.7.5)."""
    if nu < 100:
        raise ValueError("t_quantile: expansion used only for nu >= 100")
    z = normal_quantile(p)
    z2 = z * z
    g1 = (z2 + 1.0) * z / 4.0
    g2 = ((5.0 * z2 + 16.0) * z2 + 3.0) * z / 96.0
    g3 = (((3.0 * z2 + 19.0) * z2 + 17.0) * z2 - 15.0) * z / 384.0
    g4 = ((((79.0 * z2 + 776.0) * z2 + 1482.0) * z2 - 1920.0) * z2 - 945.0) * z / 92160.0
    return z + g1 / nu + g2 / (nu * nu) + g3 / (nu * nu * nu) + g4 / (nu * nu * nu * nu)


# ------------------------------------------------------- Gelman-Rubin

def psrf(window: np.ndarray) -> float:
    """R-hat of Alg. 3 for a [omega][psi] window of one scalar per position.

    mu_i and s_i are the mean and standard deviation (denominator psi-1) of
    chain i's window; B = psi/(omega-1) sum (mu_i-mu)^2; W = mean s_i^2;
    sigma^2 = (1-1/psi) W + B/psi; R = sqrt(sigma^2/W).  Returns +inf when
    W == 0 (the ratio is undefined: not converged)."""
    x = np.asarray(window, dtype=np.float64)
    omega, psi = x.shape
    mu_i = [float(np.sum(x[i])) / psi for i in range(omega)]
    s2_i = [float(np.sum((x[i] - mu_i[i]) ** 2)) / (psi - 1) for i in range(omega)]
    mu = sum(mu_i) / omega
    B = psi / (omega - 1) * sum((m - mu) ** 2 for m in mu_i)
    W = sum(s2_i) / omega
    if W == 0.0:
        return math.inf
    sigma2 = (1.0 - 1.0 / psi) * W + B / psi
    return math.sqrt(sigma2 / W)


# ------------------------------------------------ two-state Markov chain

def transition_counts(window: np.ndarray) -> Tuple[int, int, int, int]:
    """(n00, n01, n10, n11) over consecutive pairs inside each chain's window."""
    x = np.asarray(window, dtype=np.int64)
    a, b = x[:, :-1], x[:, 1:]
    n00 = int(np.sum((a == 0) & (b == 0)))
    n01 = int(np.sum((a == 0) & (b == 1)))
    n10 = int(np.sum((a == 1) & (b == 0)))
    n11 = int(np.sum((a == 1) & (b == 1)))
    return n00, n01, n10, n11


def alpha_beta(counts):
    """alpha = P(0->1), beta = P(1->0) estimated from pair counts; None if undefined."""
    n00, n01, n10, n11 = counts
    if n00 + n01 == 0 or n10 + n11 == 0:
        return None
    a = n01 / (n00 + n01)
    b = n10 / (n10 + n11)
    if a + b == 0.0:
        return None
    return a, b


def sample_size_N(a: float, b: float, z: float, r: float) -> float:
    """N of Alg. 1 (before the ceiling): ab(2-a-b)/(a+b)^3 * z^2/r^2."""
    x = (a * b * ((2.0 - a) - b)) / ((a + b) * (a + b) * (a + b))
    return x * ((z * z) / (r * r))


def burn_in_M(a: float, b: float, eps: float) -> int:
    """M of Alg. 1: ceil(log(eps (a+b)/max(a,b)) / log|1-a-b|); 0 when |1-a-b| is 0 or 1."""
    lam = abs((1.0 - a) - b)
    if lam == 0.0 or lam == 1.0:
        return 0
    return int(math.ceil(math.log(eps * (a + b) / max(a, b)) / math.log(lam)))


# ------------------------------------------------------------- Skart-P

def skewness(x: Sequence[float]) -> float:
    """Sample skewness m3 / m2^{3/2} (moments about the mean, denominator count)."""
    v = np.asarray(x, dtype=np.float64)
    m = float(np.sum(v)) / v.size
    m2 = float(np.sum((v - m) ** 2)) / v.size
    m3 = float(np.sum((v - m) ** 3)) / v.size
    if m2 == 0.0:
        return math.inf
    return m3 / m2 ** 1.5


def skewness_exceeds_4(ones: int, count: int) -> bool:
    """|sample skewness| > 4 for `count` 0-1 observations holding `ones` ones,
    decided exactly.  With q = ones/count the skewness of 0-1 data is
    (1-2q)/sqrt(q(1-q)), so |B| > 4 iff (count - 2 ones)^2 > 16 ones (count -
    ones); with no ones or no zeros the variance is 0 and the skewness is taken
    as unbounded (Skart's batch size 16 for a strongly skewed start)."""
    ones, count = int(ones), int(count)
    if ones == 0 or ones == count:
        return True
    return (count - 2 * ones) ** 2 > 16 * ones * (count - ones)


# Batch means Y = b / kappa of integer batch sums b[c][j] (chain c, batch j of
# kappa positions, P = omega m batches in all).  Every sum over the batches is
# taken exactly in integers; the moments about the grand mean follow from them
# by exact integer algebra, and floating point enters once per ratio:
#   S1 = sum b, S2 = sum b^2, S3 = sum b^3;
#   Q2 = P S2 - S1^2                      = kappa^2 P   sum (Y - mu)^2
#   Q3 = P^2 S3 - 3 P S1 S2 + 2 S1^3      = kappa^3 P^2 sum (Y - mu)^3
#   over the omega (m-1) within-chain pairs (b_j, b_{j+1}):
#   L = sum b_j b_{j+1}, E = sum (b_j + b_{j+1}), D2 = sum (b_{j+1} - b_j)^2;
#   QL = P^2 L - P S1 E + pairs S1^2      = kappa^2 P^2 sum (Y_{j+1} - mu)(Y_j - mu).
# The totals are limited to kappa P <= 2^40 observations so that a 128-bit
# integer holds each of these exactly (both sides stop there as not converged).
MAX_BATCH_OBS = 1 << 40


def batch_moments(bsum) -> dict:
    """The exact integer aggregates above for bsum[omega][m] (plain loops)."""
    rows = [[int(v) for v in row] for row in np.asarray(bsum).tolist()]
    omega, m = len(rows), len(rows[0])
    P = omega * m
    S1 = S2 = S3 = L = E = D2 = 0
    for row in rows:
        for j in range(m):
            v = row[j]
            S1 += v
            S2 += v * v
            S3 += v * v * v
            if j + 1 < m:
                w = row[j + 1]
                L += v * w
                E += v + w
                D2 += (w - v) * (w - v)
    pairs = omega * (m - 1)
    return dict(omega=omega, m=m, P=P, S1=S1, pairs=pairs, D2=D2,
                Q2=P * S2 - S1 * S1,
                Q3=P * P * S3 - 3 * P * S1 * S2 + 2 * S1 * S1 * S1,
                QL=P * P * L - P * S1 * E + pairs * S1 * S1)


def von_neumann_passes(bsum, level: float = 0.20) -> bool:
    """Randomness test over within-chain adjacent batch means (reading of Alg. 5):
    the von Neumann ratio C = 1 - (sum of squared successive differences / pairs)
    / (2 sum of squared deviations / (P-1)) against the one-sided normal
    critical value z_{1-level} / sqrt(pairs).  One batch per chain, or all batch
    means equal: passes.  From the exact aggregates C = 1 - D2 P (P-1) / (2 pairs
    Q2), the batch size cancelling."""
    g = batch_moments(bsum)
    if g["m"] < 2 or g["Q2"] == 0:
        return True
    P, pairs = g["P"], g["pairs"]
    C = 1.0 - float(g["D2"] * P * (P - 1)) / float(2 * pairs * g["Q2"])
    return C <= normal_quantile(1.0 - level) * math.sqrt(1.0 / pairs)


def adjusted_ci(bsum, kappa: int, alpha: float):
    """Skewness- and autoregression-adjusted CI on the batch means b/kappa
    (reading of Alg. 5): grand mean mu; sample variance S^2 (denominator P-1);
    lag-1 autocorrelation phi of within-chain adjacent means, A = (1+phi)/(1-phi)
    when phi > 0 else 1; skewness of the means, beta = skew/(6 sqrt(P)); Willink's
    map G of the t critical values; CI = [mu - G(t_{1-alpha/2}) se, mu -
    G(-t_{1-alpha/2}) se], se = sqrt(A S^2 / P).  Returns (mu, lo, hi).  From the
    exact aggregates: mu = S1/(kappa P), phi = QL/(pairs Q2), S^2/P = Q2/(kappa^2 P^2
    (P-1)), skew = Q3 / Q2^{3/2}; all batch means equal (Q2 = 0) gives the point
    interval at mu."""
    g = batch_moments(bsum)
    K, P = int(kappa), g["P"]
    mu = float(g["S1"]) / float(K * P)
    Q2 = g["Q2"]
    if Q2 == 0:
        return mu, mu, mu
    phi = float(g["QL"]) / float(g["pairs"] * Q2) if g["m"] >= 2 else 0.0
    A = (1.0 + phi) / (1.0 - phi) if phi > 0.0 else 1.0
    v = float(Q2) / float(K * K * P * P * (P - 1))
    q2 = float(Q2)
    skew = float(g["Q3"]) / (q2 * math.sqrt(q2))
    beta = skew / (6.0 * math.sqrt(float(P)))
    t_hi = t_quantile(1.0 - alpha / 2.0, float(P - 1))
    se = math.sqrt(A * v)
    lo = mu - willink_G(t_hi, beta) * se
    hi = mu - willink_G(-t_hi, beta) * se
    return mu, lo, hi


def willink_G(zeta: float, beta: float) -> float:
    """Skewness adjustment of a t critical value: ((1+6 beta (zeta-beta))^{1/3} - 1)/(2 beta).

    The cube root minus one is evaluated as expm1(log1p(x)/3) for |x| < 1/2 so
    that small skewness does not cancel catastrophically."""
    if beta == 0.0:
        return zeta
    x = 6.0 * beta * (zeta - beta)
    if abs(x) < 0.5:
        d = math.expm1(math.log1p(x) / 3.0)
    else:
        d = cbrt(1.0 + x) - 1.0
    return d / (2.0 * beta)
