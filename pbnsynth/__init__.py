"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random network structures, state-set patterns and
arrival traces, and writes them in the canonical text format.  It contains
none of the steady-state method's arithmetic: no selection thresholds, no
simulation, no statistics.  Both the CPU oracle and the GPU library parse its
text output with parsers of their own.

Canonical text format (one token stream, '#' starts a comment line)::

    PBN <n> <p>
    N <i> <l>                       # node i (0-based) has l predictor functions
    F <c> <k> <par_1> .. <par_k> <tt>

``c`` is the selection probability (17 significant digits, so the FP64 value
round-trips), ``par_m`` are 0-based parent ids (distinct), and ``tt`` is the
truth table as a hexadecimal integer whose bit ``idx`` is the function value for
``idx = sum_m v(par_m) << (m-1)``: the first listed parent is the least
significant index bit.

Workload shapes follow the paper's random-network generator (five parameters:
node count, min/max predictors per node, min/max parents per predictor; Sec. 5.1)
and the sparse density class of its evaluation (density around 10; Sec. 5.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

STRUCT_SEED_BASE = 1508
SIM_SEED = 7828


@dataclass
class Function:
    c: float
    parents: Tuple[int, ...]
    tt: int                       # bit idx = value for parent index idx


@dataclass
class Network:
    n: int
    p: float
    nodes: List[List[Function]] = field(default_factory=list)

    def density(self) -> float:
        """Density of Sec. 2.2: total parent count over all predictors / n."""
        return sum(len(f.parents) for fs in self.nodes for f in fs) / self.n

    def n_functions(self) -> int:
        return sum(len(fs) for fs in self.nodes)


Pattern = Tuple[Tuple[int, int], ...]   # ((node, value), ...) conjunction


def _tt_hex(tt: int, k: int) -> str:
    digits = max(1, ((1 << k) + 3) // 4)
    return format(tt, "0{}x".format(digits))


def to_text(net: Network) -> str:
    out = ["PBN {} {!r}".format(net.n, float(net.p))]
    for i, fs in enumerate(net.nodes):
        out.append("N {} {}".format(i, len(fs)))
        for f in fs:
            out.append("F {!r} {} {} {}".format(
                float(f.c), len(f.parents), " ".join(str(v) for v in f.parents),
                _tt_hex(f.tt, len(f.parents))).replace("  ", " "))
    return "\n".join(out) + "\n"


def random_network(rng: np.random.Generator, n: int, l_range: Tuple[int, int],
                   k_range: Tuple[int, int], p: float, c_dist: str = "dirichlet",
                   fixed_l: int | None = None, fixed_k: int | None = None) -> Network:
    """Random PBN: l ~ U{l_range}, k ~ U{k_range}, parents drawn without
    replacement from all n nodes (self allowed), truth-table bits Bernoulli(1/2),
    selection probabilities Dirichlet(1) or U(0,1) normalised."""
    net = Network(n=n, p=p)
    for _ in range(n):
        l = fixed_l if fixed_l is not None else int(rng.integers(l_range[0], l_range[1] + 1))
        if c_dist == "dirichlet":
            cs = rng.dirichlet(np.ones(l))
        elif c_dist == "uniform":
            raw = rng.uniform(0.0, 1.0, size=l)
            cs = raw / raw.sum()
        else:
            raise ValueError(c_dist)
        fs = []
        for j in range(l):
            k = fixed_k if fixed_k is not None else int(rng.integers(k_range[0], k_range[1] + 1))
            k = min(k, n)
            parents = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
            bits = rng.integers(0, 2, size=1 << k)
            tt = 0
            for idx in range(1 << k):
                if bits[idx]:
                    tt |= 1 << idx
            fs.append(Function(c=float(cs[j]), parents=parents, tt=tt))
        net.nodes.append(fs)
    return net


def random_pattern(rng: np.random.Generator, n: int, size: int) -> Pattern:
    nodes = rng.choice(n, size=size, replace=False)
    vals = rng.integers(0, 2, size=size)
    return tuple((int(a), int(b)) for a, b in zip(nodes, vals))


# ---------------------------------------------------------------- workloads

@dataclass
class Job:
    """One steady-state query: a network, its chains and its state sets."""
    name: str
    net: Network
    chains: int
    seed: int
    patterns: List[Pattern]
    r: float
    confidence: float
    psrf_max: float
    method: str = "two_state"          # or "skart"
    arrival: float = 0.0               # seconds (serving trace only)
    text: str = ""                     # the network's canonical text, when drawn with it


def tiny() -> Job:
    rng = np.random.default_rng(STRUCT_SEED_BASE + 0)
    net = random_network(rng, 10, (2, 2), (3, 3), 0.001, c_dist="uniform")
    return Job("tiny", net, 8, SIM_SEED, [((0, 1), (1, 1))], 0.01, 0.95, 1.1)


def medium() -> Job:
    rng = np.random.default_rng(STRUCT_SEED_BASE + 1)
    net = random_network(rng, 100, (1, 3), (1, 5), 0.001)
    pat = random_pattern(rng, 100, 3)
    return Job("medium", net, 256, SIM_SEED, [pat], 0.01, 0.95, 1.1)


def large() -> Job:
    rng = np.random.default_rng(STRUCT_SEED_BASE + 2)
    net = random_network(rng, 2000, (1, 4), (1, 6), 0.0005)
    pats = [random_pattern(rng, 2000, 4) for _ in range(5)]
    return Job("large", net, 8192, SIM_SEED, pats, 0.005, 0.95, 1.05, method="skart")


def batched(count: int = 512) -> List[Job]:
    rng = np.random.default_rng(STRUCT_SEED_BASE + 3)
    jobs = []
    for b in range(count):
        n = int(round(math.exp(rng.uniform(math.log(20), math.log(2000)))))
        p = 1e-3 if rng.integers(0, 2) == 0 else 1e-4
        net = random_network(rng, n, (1, 3), (1, 5), p)
        chains = int(rng.integers(64, 1025))
        pat = random_pattern(rng, n, 2)
        jobs.append(Job("batched[{}]".format(b), net, chains, (SIM_SEED << 20) + b,
                        [pat], 0.01, 0.95, 1.1))
    return jobs


def _serving_request(args) -> Job:
    """Request b of the serving trace: its own generator, seeded by (trace seed,
    b), so that requests can be drawn in any order or in parallel."""
    b, t, chains = args
    rng = np.random.default_rng([STRUCT_SEED_BASE + 4, b])
    n = int(round(math.exp(rng.uniform(math.log(50), math.log(5000)))))
    net = random_network(rng, n, (1, 3), (1, 5), 0.001)
    r = 0.01 if rng.integers(0, 2) == 0 else 0.005
    pat = random_pattern(rng, n, int(rng.integers(1, 5)))
    return Job("serving[{}]".format(b), net, chains, (SIM_SEED << 24) + b, [pat], r, 0.95, 1.1, arrival=t,
               text=to_text(net))


def serving_request(b: int, chains: int = 256) -> Job:
    """Request b of the serving trace alone (its arrival time left at 0)."""
    return _serving_request((b, 0.0, chains))


def serving(duration_s: float = 60.0, rate: float = 200.0, chains: int = 256,
            limit: int | None = None, workers: int = 0) -> List[Job]:
    """Poisson arrivals at `rate` per second for duration_s (at most `limit`
    requests); each request's network, precision and state set are drawn from
    a generator of its own.  workers > 1 draws the requests in that many
    processes (the result does not depend on it)."""
    rng = np.random.default_rng(STRUCT_SEED_BASE + 4)
    times = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration_s or (limit is not None and len(times) >= limit):
            break
        times.append(t)
    args = [(b, tb, chains) for b, tb in enumerate(times)]
    if workers > 1 and len(args) > 64:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            return pool.map(_serving_request, args, chunksize=16)
    return [_serving_request(a) for a in args]


def multiprop(chains: int = 16384, r: float = 1e-4) -> Job:
    """Shape of the paper's multi-property experiment (Sec. 5.2, Table 2): a
    96-node network with 107 Boolean functions (11 nodes with two predictors,
    the others with one) and 7 state sets checked together: a target node's
    marginal and its joint values with each of three parents of one of its
    functions, in both parent values (the quantities of a long-term influence
    analysis).  The biological model itself is not available; structure,
    tables and selection probabilities are drawn as in random_network."""
    rng = np.random.default_rng(STRUCT_SEED_BASE + 5)
    n = 96
    net = random_network(rng, n, (1, 1), (1, 4), 0.001)
    for i in (int(v) for v in rng.choice(n, size=11, replace=False)):
        cs = rng.dirichlet(np.ones(2))
        k = int(rng.integers(1, 5))
        parents = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        bits = rng.integers(0, 2, size=1 << k)
        tt = sum(1 << idx for idx in range(1 << k) if bits[idx])
        first = net.nodes[i][0]
        net.nodes[i] = [Function(c=float(cs[0]), parents=first.parents, tt=first.tt),
                        Function(c=float(cs[1]), parents=parents, tt=tt)]
    # target: a node one of whose functions reads three other nodes
    target, par = None, None
    for i in (int(v) for v in rng.permutation(n)):
        for f in net.nodes[i]:
            others = [v for v in f.parents if v != i]
            if len(others) >= 3:
                target, par = i, others[:3]
                break
        if target is not None:
            break
    assert target is not None
    pats: List[Pattern] = [((target, 1),)]
    for v in par:
        pats.append(((target, 1), (v, 1)))
        pats.append(((target, 1), (v, 0)))
    return Job("multiprop", net, chains, SIM_SEED + 5, pats, r, 0.95, 1.1)


def small_network(seed: int, n: int, l_max: int = 3, k_max: int = 3, p: float = 0.01,
                  fixed_l: int | None = None) -> Network:
    """Small random networks for exhaustive tests (n <= 12)."""
    rng = np.random.default_rng(seed)
    return random_network(rng, n, (1, l_max), (1, min(k_max, n)), p, fixed_l=fixed_l)


def uniform_bytes(seed: int, count: int) -> np.ndarray:
    """Seeded uniform 32-bit words (for tests that need raw random inputs)."""
    return np.random.default_rng(seed).integers(0, 1 << 32, size=count, dtype=np.uint64).astype(np.uint32)


def pattern_text(p: Pattern) -> str:
    return " ".join("{}:{}".format(a, b) for a, b in p)


def all_configs() -> Sequence[str]:
    return ("tiny", "medium", "large", "batched", "serving")
