"""The paper's parallel algorithms over oracle chains (plain Python control flow).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Positions are 1-based: position l of a chain is its l-th recorded state.  Each
property (state set) runs its own state machine on chains that depend only on
(network, seed, chain id), so a property's result does not depend on which other
properties share the chains; the oracle therefore solves each property alone.

Readings of the paper (where it is silent or garbled) that this file follows:
  * Alg. 3: the scalar monitored is the property's 0-1 indicator; s_i uses the
    denominator psi-1; the chains first reach 2*psi0 positions, and each check
    uses positions psi+1..2psi; "close to 1" means R < psrf_max; a check with
    W == 0 counts as not converged; the returned psi is the last one checked.
  * Alg. 4: the first pass estimates alpha, beta from the existing second halves
    (positions psi+1..2psi) without extending; the extension is
    ceil((N - omega*n)/omega) and the inner loop ends when it is <= 0; the
    estimate of alpha, beta uses all pairs of consecutive positions inside each
    chain's window (summed over chains); a re-run happens when M > psi and
    discards M - psi more positions from each chain's front (psi := M); if the
    window becomes empty it is refilled to the Gelman-Rubin psi; the estimate is
    the fraction of ones in the final window.  If alpha or beta is undefined the
    window is doubled.
  * Alg. 5 (Skart-P): eta0 = ceil(1280/omega)*omega initial observations from
    position psi+1; batch size 16 if the sample skewness exceeds 4 in absolute
    value, else 1; p batches of kappa positions, p/omega consecutive batches per
    chain (chain-major order); randomness test = von Neumann ratio over
    within-chain adjacent batch means at level 0.20, on failure kappa :=
    ceil(sqrt(2) kappa), p := ceil(0.9 p) rounded up to a multiple of omega (at
    most 10 times); CI = skewness- (Willink) and lag-1 autoregression-adjusted
    t interval on the batch means; if its half-width H exceeds H* the batch size
    grows to ceil(kappa (H/H*)^2).  The skewness decision on the 0-1 start and
    every moment of the batch means come from exact integer sums (see
    ``stats``), so no decision depends on a floating-point summation order; the
    batches stop, as not converged, beyond 2^40 observations.
  * Alg. 2 (Skart on one chain): an initial trajectory of eta = 1280 positions
    from position 1; the skewness of its last l = 1024 positions sets the batch
    size as in Alg. 5; p = 1280 batches of kappa positions from position 1; the
    randomness test (the von Neumann ratio above, one chain) runs on the spaced
    batch means, i.e. every (d+1)-th batch, each one preceded by d spacer
    batches, for d = 0, 1, ..., 10 on the same data, and passes at the first d
    that passes; when every spacer fails, kappa := ceil(sqrt(2) kappa), p :=
    ceil(0.9 p) and the spacers are tried again on the longer trajectory (at
    most 10 such increases; after the last one the spacer stays at 10).  The
    first zeta = d*kappa positions are then skipped and the CI of Alg. 5 is
    computed on the p' = p - d nonspaced batches after them; if H exceeds H*
    the batch size grows to ceil(kappa (H/H*)^2), p' stays, and the skipped
    part stays d batches long (zeta = d*kappa with the new kappa), so the
    trajectory has kappa (p' + d) positions.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

from . import Chains, Net
from . import stats

OK = 0
NOT_CONVERGED = 5


def _cdiv(a: int, b: int) -> int:
    return -((-a) // b)


class NotConverged(Exception):
    pass


def generate_converged_chains(ch: Chains, q: int, psi0: int, psrf_max: float, cap: int):
    """Alg. 3 for property q; returns (psi, R)."""
    psi = psi0
    while True:
        if 2 * psi > cap:
            raise NotConverged("psrf")
        ch.extend_to(2 * psi)
        R = stats.psrf(ch.bits[q][:, psi: 2 * psi])
        if R < psrf_max:
            return psi, R
        psi = 2 * psi


def estimate_probability_in_parallel(ch: Chains, q: int, psi0: int, psrf_max: float, eps: float,
                                     r: float, s: float, cap: int) -> Dict:
    """Alg. 4 for property q on chains ch."""
    omega = ch.omega
    z = stats.z_of_confidence(s)
    res = dict(status=OK, psi_gr=0, rhat=math.nan, psi=0, n=0, N=0, M=0, prob=math.nan,
               ci_lo=math.nan, ci_hi=math.nan, kappa=0, batches=0, chain_len=0)
    try:
        psi, R = generate_converged_chains(ch, q, psi0, psrf_max, cap)
    except NotConverged:
        res["status"] = NOT_CONVERGED
        res["chain_len"] = ch.length
        return res
    res["psi_gr"], res["rhat"] = psi, R
    psi_gr = psi
    n = psi
    N = 0
    while True:
        while True:
            if psi + n > cap:
                res.update(status=NOT_CONVERGED, psi=psi, n=n, chain_len=ch.length)
                return res
            ch.extend_to(psi + n)
            win = ch.bits[q][:, psi: psi + n]
            ab = stats.alpha_beta(stats.transition_counts(win))
            if ab is None:
                extend_by = n
            else:
                a, b = ab
                N = int(math.ceil(stats.sample_size_N(a, b, z, r)))
                extend_by = _cdiv(N - omega * n, omega)
                if extend_by <= 0:
                    break
            n += extend_by
        M = stats.burn_in_M(a, b, eps)
        if M > psi:
            n -= M - psi
            psi = M
            if n <= 0:
                n = psi_gr
            continue
        break
    win = ch.bits[q][:, psi: psi + n]
    res.update(psi=psi, n=n, N=N, M=M, prob=float(np.sum(win)) / (omega * n),
               chain_len=psi + n)
    return res


def _batch_sums(ch: Chains, q: int, base: int, kappa: int, p: int) -> np.ndarray:
    """Integer batch sums [omega][p/omega]: chain c's batch j holds positions
    base + j kappa + 1 .. base + (j+1) kappa (1-based)."""
    m = p // ch.omega
    ch.extend_to(base + kappa * m)
    x = ch.bits[q][:, base: base + kappa * m].astype(np.int64)
    return x.reshape(ch.omega, m, kappa).sum(axis=2)


def _batches_fit(base: int, kappa: int, p: int, omega: int, cap: int) -> bool:
    """p batches of kappa positions from base fit under the cap, and their
    kappa p observations within the exact-moment limit."""
    return base + kappa * (p // omega) <= cap and kappa * p <= stats.MAX_BATCH_OBS


def _grown_kappa(kappa: int, H: float, H_star: float) -> int:
    """Batch size after a CI wider than H*: ceil(kappa (H/H*)^2), evaluated in
    FP64 and saturated at 2^64 - 1."""
    ratio = H / H_star
    return min(int(math.ceil(kappa * (ratio * ratio))), (1 << 64) - 1)


def estimate_ci_in_parallel(ch: Chains, q: int, psi0: int, psrf_max: float, H_star: float,
                            s: float, cap: int) -> Dict:
    """Alg. 5 (Skart-P) for property q on chains ch."""
    omega = ch.omega
    alpha = 1.0 - s
    res = dict(status=OK, psi_gr=0, rhat=math.nan, psi=0, n=0, N=0, M=0, prob=math.nan,
               ci_lo=math.nan, ci_hi=math.nan, kappa=0, batches=0, chain_len=0)
    try:
        psi, R = generate_converged_chains(ch, q, psi0, psrf_max, cap)
    except NotConverged:
        res["status"] = NOT_CONVERGED
        res["chain_len"] = ch.length
        return res
    res.update(psi_gr=psi, rhat=R, psi=psi)
    base = psi
    eta0 = _cdiv(1280, omega) * omega
    m0 = eta0 // omega
    if base + m0 > cap:
        res.update(status=NOT_CONVERGED, chain_len=ch.length)
        return res
    ch.extend_to(base + m0)
    ones = int(np.sum(ch.bits[q][:, base: base + m0], dtype=np.int64))
    kappa = 16 if stats.skewness_exceeds_4(ones, eta0) else 1
    p = eta0
    if not _batches_fit(base, kappa, p, omega, cap):
        res.update(status=NOT_CONVERGED, chain_len=ch.length)
        return res
    b = _batch_sums(ch, q, base, kappa, p)
    tries = 0
    while not stats.von_neumann_passes(b) and tries < 10:
        kappa = int(math.ceil(math.sqrt(2.0) * kappa))
        p = max(omega, _cdiv(int(math.ceil(0.9 * p)), omega) * omega)
        tries += 1
        if not _batches_fit(base, kappa, p, omega, cap):
            res.update(status=NOT_CONVERGED, chain_len=ch.length)
            return res
        b = _batch_sums(ch, q, base, kappa, p)
    while True:
        if not _batches_fit(base, kappa, p, omega, cap):
            res.update(status=NOT_CONVERGED, chain_len=ch.length, kappa=kappa, batches=p)
            return res
        b = _batch_sums(ch, q, base, kappa, p)
        mu, lo, hi = stats.adjusted_ci(b, kappa, alpha)
        H = max(mu - lo, hi - mu)
        if H > H_star:
            kappa = _grown_kappa(kappa, H, H_star)
            continue
        break
    n = kappa * (p // omega)
    res.update(prob=mu, ci_lo=lo, ci_hi=hi, kappa=kappa, batches=p, n=n, chain_len=base + n)
    return res


DEFAULTS = dict(psi0=256, eps=1e-10, cap=1 << 26)


def estimate_probability(ch: Chains, q: int, m0: int, n0: int, eps: float, r: float, s: float,
                         cap: int) -> Dict:
    """Alg. 1 (the sequential two-state Markov chain approach, Sec. 3.1) for
    property q on the single chain of ch.  M := m0, N := n0 and a trajectory of
    length l := M + N; repeatedly extend the trajectory to length M + N (l := M +
    N), estimate alpha, beta from its last N positions and recompute M and N,
    until M + N <= l; the estimate is the fraction of ones in the last N
    positions.  Readings: when alpha or beta is undefined (a meta state never left
    or never reached in the window) N is doubled (and l grows to M + N if
    shorter); N is at least 1 (the formula gives 0 for a strictly alternating
    window, alpha = beta = 1)."""
    assert ch.omega == 1
    z = stats.z_of_confidence(s)
    res = dict(status=OK, psi_gr=0, rhat=math.nan, psi=0, n=0, N=0, M=0, prob=math.nan,
               ci_lo=math.nan, ci_hi=math.nan, kappa=0, batches=0, chain_len=0)
    M, N = m0, n0
    l = M + N
    while True:
        if l > cap:
            res.update(status=NOT_CONVERGED, psi=M, n=N, M=M, chain_len=ch.length)
            return res
        ch.extend_to(l)
        ab = stats.alpha_beta(stats.transition_counts(ch.bits[q][:, l - N: l]))
        if ab is None:
            N *= 2
            l = max(l, M + N)
            continue
        a, b = ab
        M = stats.burn_in_M(a, b, eps)
        # a sample of at least one position (N = 0 when alpha = beta = 1)
        N = max(1, int(math.ceil(stats.sample_size_N(a, b, z, r))))
        if M + N <= l:
            break
        l = M + N
    win = ch.bits[q][:, l - N: l]
    res.update(psi=M, n=N, N=N, M=M, prob=float(np.sum(win)) / N, chain_len=l)
    return res


def _spaced_passes(y: np.ndarray, d: int) -> bool:
    """Randomness test on the spaced batch sums of one chain: batches
    d, 2d+1, 3d+2, ... (0-based), each preceded by d spacer batches."""
    return stats.von_neumann_passes(y[d::d + 1].reshape(1, -1))


def estimate_ci(ch: Chains, q: int, H_star: float, s: float, cap: int) -> Dict:
    """Alg. 2 (the sequential Skart method, Sec. 3.2) for property q on the
    single chain of ch; the readings are listed in the module docstring."""
    assert ch.omega == 1
    alpha = 1.0 - s
    res = dict(status=OK, psi_gr=0, rhat=math.nan, psi=0, n=0, N=0, M=0, prob=math.nan,
               ci_lo=math.nan, ci_hi=math.nan, kappa=0, batches=0, chain_len=0)
    eta, l = 1280, 1024
    if eta > cap:
        res.update(status=NOT_CONVERGED, chain_len=ch.length)
        return res
    ch.extend_to(eta)
    ones = int(np.sum(ch.bits[q][0, eta - l: eta], dtype=np.int64))
    kappa = 16 if stats.skewness_exceeds_4(ones, l) else 1
    p = eta
    grows = 0
    while True:
        if kappa * p > cap:
            res.update(status=NOT_CONVERGED, chain_len=ch.length)
            return res
        y = _batch_sums(ch, q, 0, kappa, p)[0]
        d = next((d for d in range(11) if _spaced_passes(y, d)), None)
        if d is not None:
            break
        if grows == 10:
            d = 10
            break
        kappa = int(math.ceil(math.sqrt(2.0) * kappa))
        p = int(math.ceil(0.9 * p))
        grows += 1
    pp = p - d
    while True:
        zeta = d * kappa
        if zeta + kappa * pp > cap:
            res.update(status=NOT_CONVERGED, chain_len=ch.length)
            return res
        b = _batch_sums(ch, q, zeta, kappa, pp)
        mu, lo, hi = stats.adjusted_ci(b, kappa, alpha)
        H = max(mu - lo, hi - mu)
        if H > H_star:
            kappa = _grown_kappa(kappa, H, H_star)
            continue
        break
    n = kappa * pp
    res.update(prob=mu, ci_lo=lo, ci_hi=hi, kappa=kappa, batches=pp, psi=zeta, n=n, chain_len=zeta + n)
    return res


def solve(text: str, omega: int, seed: int, patterns, r: float, s: float, psrf_max: float,
          method: str = "two_state", psi0: int = 256, eps: float = 1e-10, cap: int = 1 << 26,
          threads: int | None = None, thin: int = 1) -> List[Dict]:
    """Solve every property alone (fresh chains, same seed); the per-property
    results equal those of a shared-chain run.  thin > 1: the procedures run on
    every thin-th state of the chains."""
    net = Net(text)
    out = []
    for q in range(len(patterns)):
        ch = Chains(net, omega, seed, [patterns[q]], threads=threads, thin=thin)
        if method == "two_state":
            out.append(estimate_probability_in_parallel(ch, 0, psi0, psrf_max, eps, r, s, cap))
        elif method == "skart":
            out.append(estimate_ci_in_parallel(ch, 0, psi0, psrf_max, r, s, cap))
        elif method == "sequential":
            out.append(estimate_probability(ch, 0, psi0, 4 * psi0, eps, r, s, cap))
        elif method == "sequential_skart":
            out.append(estimate_ci(ch, 0, r, s, cap))
        else:
            raise ValueError(method)
    return out
