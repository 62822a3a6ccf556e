"""Pins for the oracle's network parsing, step law and special cases.

* Thresholds: T_j = min(2^32-1, floor(2^32 C_j)) with C_j the left-to-right FP64
  sum, checked with exact rational arithmetic.
* One-step law (paper Sec. 2.2): empirical next-state frequencies out of a fixed
  state versus the exact row of the brute-force transition matrix, chi-square.
* Special case: with one predictor per node and no perturbation the step is the
  deterministic synchronous Boolean map; a perturbed step is s XOR gamma.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats as sst

import oracle
import pbnsynth as ps
from oracle import exact


def test_thresholds_exact():
    for seed in range(5):
        net = ps.small_network(seed, 8, l_max=4)
        o = oracle.Net(ps.to_text(net))
        assert o.p_thr == math.floor(Fraction(net.p) * 2 ** 32)
        for i, fs in enumerate(net.nodes):
            csum = 0.0
            want = []
            for f in fs:
                csum = csum + f.c
                want.append(min(2 ** 32 - 1, math.floor(Fraction(csum) * 2 ** 32)))
            assert o.thresholds(i) == want


@pytest.mark.parametrize("bad", [
    "PBN 2 0.5\nN 0 1\nF 1.0 1 0 2\nN 1 1\nF 0.9 1 0 1\n",          # sum != 1
    "PBN 2 0.5\nN 0 1\nF 1.0 2 1 1 6\nN 1 1\nF 1.0 1 0 1\n",        # duplicate parent
    "PBN 2 0.5\nN 0 1\nF 1.0 1 2 2\nN 1 1\nF 1.0 1 0 1\n",          # parent out of range
    "PBN 2 1.5\nN 0 1\nF 1.0 1 1 2\nN 1 1\nF 1.0 1 0 1\n",          # p out of (0,1)
    "PBN 2 0.5\nN 0 1\nF 1.0 1 1 1f\nN 1 1\nF 1.0 1 0 1\n",         # truth table too long
    "PBN 2 0.5\nN 1 1\nF 1.0 1 1 2\nN 0 1\nF 1.0 1 0 1\n",          # nodes out of order
])
def test_parse_rejects(bad):
    with pytest.raises(ValueError):
        oracle.Net(bad)


def _boolean_map(net, s):
    out = np.zeros(net.n, np.uint8)
    for i, fs in enumerate(net.nodes):
        f = fs[0]
        idx = sum(int(s[v]) << m for m, v in enumerate(f.parents))
        out[i] = (f.tt >> idx) & 1
    return out


def test_single_predictor_is_boolean_map():
    net = ps.small_network(3, 9, k_max=4, p=0.02, fixed_l=1)
    o = oracle.Net(ps.to_text(net))
    rng = np.random.default_rng(0)
    n_pert = 0
    for t in range(3000):
        s = rng.integers(0, 2, net.n).astype(np.uint8)
        nx, g = o.step_one(99, t, 5, s)
        if g.any():
            n_pert += 1
            assert np.array_equal(nx, s ^ g)
        else:
            assert np.array_equal(nx, _boolean_map(net, s))
    # fraction of perturbed steps ~ 1-(1-p)^n
    q = 1 - (1 - net.p) ** net.n
    assert abs(n_pert / 3000 - q) < 5 * math.sqrt(q * (1 - q) / 3000)


@pytest.mark.parametrize("p,seed,n", [(0.001, 1, 5), (0.05, 2, 6), (0.3, 3, 4), (0.3, 4, 6)])
def test_one_step_law_chi2(p, seed, n):
    net = ps.small_network(seed, n, l_max=3, k_max=3, p=p)
    text = ps.to_text(net)
    P = exact.transition_matrix(text)
    o = oracle.Net(text)
    rng = np.random.default_rng(seed)
    count = 200000
    for trial in range(2):
        s_idx = int(rng.integers(0, 1 << n))
        s = np.array([(s_idx >> i) & 1 for i in range(n)], np.uint8)
        nxt = o.sample_next(1234 + trial, 3, s, 0, count)
        obs = np.bincount(nxt.astype(np.int64), minlength=1 << n).astype(float)
        exp_ = P[s_idx] * count
        keep = exp_ >= 5
        # states the exact row says are impossible must never appear
        assert obs[P[s_idx] == 0].sum() == 0
        o_k = np.append(obs[keep], obs[~keep].sum())
        e_k = np.append(exp_[keep], exp_[~keep].sum())
        if e_k[-1] == 0:
            o_k, e_k = o_k[:-1], e_k[:-1]
        stat = ((o_k - e_k) ** 2 / e_k).sum()
        pval = sst.chi2.sf(stat, len(o_k) - 1)
        assert pval > 1e-4, (trial, pval)


def test_exact_matrix_invariants():
    j = ps.tiny()
    P = exact.transition_matrix(ps.to_text(j.net))
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    off = P[~np.eye(P.shape[0], dtype=bool)]
    assert off.min() > 0.0                       # perturbations connect every pair: ergodic
    pi = exact.stationary(P)
    assert abs(pi.sum() - 1.0) < 1e-12 and pi.min() > 0
    assert np.allclose(pi @ P, pi, atol=1e-14)
    # probabilities of a partition of the state space sum to one
    parts = [exact.pattern_probability(pi, 10, ((0, a), (1, b))) for a in (0, 1) for b in (0, 1)]
    assert abs(sum(parts) - 1.0) < 1e-12
