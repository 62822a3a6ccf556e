"""Brute-force transition matrix and stationary distribution of small PBNs.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For n <= 12 the DTMC of Sec. 2.1 is built explicitly over all 2^n states
(state index s = sum_i v_i 2^i) from the model of Sec. 2.2, with the quantised
probabilities the simulator realises: p~ = floor(p 2^32)/2^32 and
c~_j = (T_j - T_{j-1})/2^32 with T_j = min(2^32-1, floor(2^32 (c_1+..+c_j))),
and the last function taking the remaining mass.

Step law (perturbation read as: any perturbed node -> XOR with gamma, else the
synchronous function update):
    P(s, s') = (1-p~)^n prod_i [q_i(s) if s'_i = 1 else 1 - q_i(s)]
               + [s' != s] p~^h (1-p~)^(n-h),     h = Hamming(s, s'),
with q_i(s) = sum_j c~_j f_j^i(s).  The stationary distribution solves
pi P = pi, sum pi = 1 (ergodic for p > 0, Sec. 2.1).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

TWO32 = 4294967296.0


def parse(text: str):
    """Minimal parser of the canonical text: returns (n, p, nodes) with
    nodes[i] = [(c, parents, tt_int), ...]."""
    toks = [t for line in text.splitlines() if not line.lstrip().startswith("#")
            for t in line.split()]
    pos = 0

    def take():
        nonlocal pos
        pos += 1
        return toks[pos - 1]

    assert take() == "PBN"
    n = int(take())
    p = float(take())
    nodes = []
    for i in range(n):
        assert take() == "N" and int(take()) == i
        l = int(take())
        fs = []
        for _ in range(l):
            assert take() == "F"
            c = float(take())
            k = int(take())
            parents = tuple(int(take()) for _ in range(k))
            tt = int(take(), 16)
            fs.append((c, parents, tt))
        nodes.append(fs)
    return n, p, nodes


def quantised(p: float, cs: List[float]) -> Tuple[float, List[float]]:
    p_q = math.floor(p * TWO32) / TWO32
    out, prev, csum = [], 0, 0.0
    for j, c in enumerate(cs):
        csum = csum + c
        T = min(4294967295, int(math.floor(csum * TWO32)))
        if j == len(cs) - 1:
            out.append((TWO32 - prev) / TWO32)      # last function: remaining mass
        else:
            out.append((T - prev) / TWO32)
            prev = T
    return p_q, out


def transition_matrix(text: str) -> np.ndarray:
    n, p, nodes = parse(text)
    if n > 12:
        raise ValueError("exact matrix only for n <= 12")
    S = 1 << n
    states = np.arange(S, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)   # [S][n]
    p_q = math.floor(p * TWO32) / TWO32
    F = np.ones((S, S), dtype=np.float64)
    for i, fs in enumerate(nodes):
        _, cq = quantised(p, [f[0] for f in fs])
        qi = np.zeros(S, dtype=np.float64)
        for (c, parents, tt), cj in zip(fs, cq):
            idx = np.zeros(S, dtype=np.int64)
            for m, v in enumerate(parents):
                idx |= bits[:, v] << m
            qi += cj * ((tt >> idx) & 1).astype(np.float64)
        on = bits[:, i].astype(bool)                        # s'_i == 1, indexed by s'
        F *= np.where(on[None, :], qi[:, None], 1.0 - qi[:, None])
    x = states[:, None] ^ states[None, :]
    h = np.zeros_like(x)
    for i in range(n):
        h += (x >> i) & 1
    pert = np.where(h > 0, p_q ** h * (1.0 - p_q) ** (n - h), 0.0)
    return (1.0 - p_q) ** n * F + pert


def stationary(P: np.ndarray) -> np.ndarray:
    S = P.shape[0]
    A = P.T - np.eye(S)
    A[-1, :] = 1.0
    b = np.zeros(S)
    b[-1] = 1.0
    return np.linalg.solve(A, b)


def pattern_probability(pi: np.ndarray, n: int, pattern) -> float:
    states = np.arange(pi.size)
    ok = np.ones(pi.size, dtype=bool)
    for node, val in pattern:
        ok &= ((states >> node) & 1) == val
    return float(np.sum(pi[ok]))
