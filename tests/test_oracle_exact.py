"""Pin the oracle's estimators to the exact stationary distribution (tiny network).

The tiny configuration (n = 10) has a 1024-state chain; its stationary
distribution is solved exactly in FP64 and P(node0 = 1 and node1 = 1) is
compared with the oracle's estimates over fixed seeds:
  * Alg. 4 (two-state, r = 0.01, s = 0.95): the estimate lands within r in at
    least 179 of 200 runs (179 is the 0.1% quantile of Binomial(200, 0.95));
  * Alg. 5 (Skart-P, H* = 0.01, 95%): the CI covers the exact value in at least
    88 of 100 runs (0.1% quantile of Binomial(100, 0.95)).
"""
import pbnsynth as ps
from oracle import drivers, exact


def _truth():
    j = ps.tiny()
    txt = ps.to_text(j.net)
    pi = exact.stationary(exact.transition_matrix(txt))
    return j, txt, exact.pattern_probability(pi, 10, j.patterns[0])


def test_two_state_within_r():
    j, txt, truth = _truth()
    hits = 0
    for k in range(200):
        r = drivers.solve(txt, j.chains, 1000 + k, j.patterns, 0.01, 0.95, 1.1, threads=1)[0]
        assert r["status"] == 0
        assert r["chain_len"] == r["psi"] + r["n"]
        assert r["N"] <= j.chains * r["n"]           # stop rule of Alg. 4
        assert r["M"] <= r["psi"]                     # burn-in check of Alg. 4
        hits += abs(r["prob"] - truth) < 0.01
    assert hits >= 179


def test_skart_covers():
    j, txt, truth = _truth()
    cover = 0
    for k in range(100):
        r = drivers.solve(txt, j.chains, 5000 + k, j.patterns, 0.01, 0.95, 1.1, method="skart", threads=1)[0]
        assert r["status"] == 0
        assert r["batches"] % j.chains == 0           # equal batches per chain (Fig. 2b)
        assert max(r["prob"] - r["ci_lo"], r["ci_hi"] - r["prob"]) <= 0.01
        cover += r["ci_lo"] <= truth <= r["ci_hi"]
    assert cover >= 88


def test_sequential_within_r():
    """Alg. 1 (one chain): within r of the exact pi at the binomial-bound rate,
    and its stop rule M + N <= l holds at the end."""
    j, txt, truth = _truth()
    hits = 0
    for k in range(200):
        r = drivers.solve(txt, 1, 3000 + k, j.patterns, 0.01, 0.95, 1.1, method="sequential", threads=1)[0]
        assert r["status"] == 0
        assert r["M"] + r["N"] <= r["chain_len"]
        assert r["n"] == r["N"] and r["psi"] == r["M"]
        hits += abs(r["prob"] - truth) < 0.01
    assert hits >= 179


def test_sequential_skart_covers():
    """Alg. 2 (one chain, H* = 0.01, 95%): the CI covers the exact value at the
    binomial-bound rate, its half-width meets H*, and the skipped warm-up is a
    whole number of batches."""
    j, txt, truth = _truth()
    cover = 0
    for k in range(100):
        r = drivers.solve(txt, 1, 7000 + k, j.patterns, 0.01, 0.95, 1.1, method="sequential_skart",
                          threads=1)[0]
        assert r["status"] == 0
        assert max(r["prob"] - r["ci_lo"], r["ci_hi"] - r["prob"]) <= 0.01
        assert r["psi"] % r["kappa"] == 0 and r["psi"] // r["kappa"] <= 10
        assert r["chain_len"] == r["psi"] + r["kappa"] * r["batches"]
        cover += r["ci_lo"] <= truth <= r["ci_hi"]
    assert cover >= 88
