"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Bit-exact: initial states, chain states after every extension, recorded
indicator bits, window sums and pair counts, Skart batch sums, and every
integer decision of the procedures (psi, n, N, M, kappa, batches, chain
length, status).  Floating point (R, the estimates, the Skart CI): within
1e-12 relative, the tolerance stated for this path.
"""
import dataclasses
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1508_07828_amd as pkg
import pbnsynth as ps
from oracle import drivers, stats

pytestmark = pytest.mark.gpu

INT_KEYS = ("status", "psi_gr", "psi", "n", "N", "M", "kappa", "batches", "chain_len")
FP_KEYS = ("prob", "rhat", "ci_lo", "ci_hi")
CAP = 1 << 15
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def close(a, b, rel=1e-12):
    if np.isnan(a) and np.isnan(b):
        return True
    return abs(a - b) <= rel * max(1.0, abs(b))


def assert_same_result(got, want, tag=""):
    for k in INT_KEYS:
        assert got[k] == want[k], (tag, k, got[k], want[k])
    for k in FP_KEYS:
        assert close(got[k], want[k]), (tag, k, got[k], want[k])


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.lib()
    yield


def _ragged_net(n=37, p=0.05, seed=5, k_max=7):
    return ps.small_network(seed, n, l_max=4, k_max=k_max, p=p)


CASES = {
    "tiny": lambda: (ps.tiny().net, 8, ps.tiny().patterns),
    "medium": lambda: (ps.medium().net, 256, ps.medium().patterns),
    "ragged_k7_p05": lambda: (_ragged_net(), 100, [((0, 1), (5, 0)), ((36, 1),)]),
    "ragged_k6_p05": lambda: (_ragged_net(37, 0.05, 6, 6), 100, [((0, 1), (5, 0)), ((36, 1),), ((2, 0),)]),
    "high_p": lambda: (_ragged_net(20, 0.6, 9, 4), 70, [((3, 1),)]),
    "ragged_l6_k5": lambda: (ps.small_network(11, 45, l_max=6, k_max=5, p=0.02), 90, [((1, 1), (44, 0))]),
    "one_node": lambda: (ps.small_network(2, 1, l_max=2, k_max=1, p=0.3), 65, [((0, 1),)]),
    "n300_l4": lambda: (ps.random_network(np.random.default_rng(4), 300, (1, 4), (1, 6), 0.004), 130,
                        [((7, 1), (299, 0))]),
}

# (mode, waves): the lane-per-chain kernel and the bit-sliced kernel with 1 to 16 waves per block
KERNELS = [("lane", 0), ("bitsliced", 1), ("bitsliced", 2), ("bitsliced", 4), ("bitsliced", 5), ("bitsliced", 8),
           ("bitsliced", 12), ("bitsliced", 16)]


@pytest.fixture(params=KERNELS, ids=["lane", "bs1", "bs2", "bs4", "bs5", "bs8", "bs12", "bs16"])
def kernel(request):
    pkg.set_kernel(*request.param)
    yield request.param
    pkg.set_kernel("auto", 0)


@pytest.mark.parametrize("case", sorted(CASES))
def test_trajectories_bit_exact(case, kernel):
    net, omega, pats = CASES[case]()
    text = ps.to_text(net)
    say("trajectories {} n={} omega={} kernel={}".format(case, net.n, omega, kernel))
    sim = pkg.Simulation(pkg.Network(text), omega, 7828, max_props=len(pats), max_len=4096)
    sim.reset(pats)
    ch = oracle.Chains(oracle.Net(text), omega, 7828, pats)
    assert np.array_equal(sim.read_state(), ch.states)
    for steps in (37, 100, 63, 1):
        sim.run(steps)
        ch.extend(steps)
        assert np.array_equal(sim.read_state(), ch.states), steps
    L = ch.length
    for q in range(len(pats)):
        assert np.array_equal(sim.read_bits(q, 0, L), ch.bits[q]), q
    assert sim.position() == (L, L)


def test_degenerate_state_sets(kernel):
    """State sets with repeated and contradictory terms and with no terms: a
    node asked to be 1 and then 0 twice is the empty set, a repeated term is
    the term once, no terms is every state; both kernels record the oracle's
    indicators."""
    net, omega, _ = CASES["ragged_k6_p05"]()
    pats = [((0, 1), (0, 0), (0, 0)), ((1, 1), (1, 1)), ((4, 0), (4, 1), (4, 1), (2, 1)),
            ((3, 1), (35, 0), (3, 1)), ()]
    text = ps.to_text(net)
    say("degenerate state sets kernel={}".format(kernel))
    sim = pkg.Simulation(pkg.Network(text), omega, 5, max_props=len(pats), max_len=1024)
    sim.reset(pats)
    sim.run(200)
    ch = oracle.Chains(oracle.Net(text), omega, 5, pats)
    ch.extend(200)
    for q in range(len(pats)):
        assert np.array_equal(sim.read_bits(q, 0, 200), ch.bits[q]), q
    assert not ch.bits[0].any() and not ch.bits[2].any() and ch.bits[4].all()
    with pytest.raises(pkg.PbnError):
        sim.reset([((0, 2),)])


def test_burn_in_and_thinning(kernel):
    net, omega, pats = CASES["ragged_k6_p05"]()
    pats = pats[:2]
    text = ps.to_text(net)
    say("burn-in/thin kernel={}".format(kernel))
    sim = pkg.Simulation(pkg.Network(text), omega, 99, max_props=2, max_len=1024)
    sim.reset(pats)
    sim.run(50, burn_in=13, thin=3)
    ch = oracle.Chains(oracle.Net(text), omega, 99, pats)
    ch.extend(13 + 150)
    assert np.array_equal(sim.read_state(), ch.states)
    idx = 13 + 3 * np.arange(50) + 2
    for q in range(2):
        assert np.array_equal(sim.read_bits(q, 0, 50), ch.bits[q][:, idx])
    assert sim.position() == (50, 163)


# node-split form: a 64-chain group spread over P cooperating blocks
SPLIT_CASES = ["medium", "ragged_k6_p05", "ragged_l6_k5", "high_p", "n300_l4"]


@pytest.fixture(params=[2, 3, 5], ids=["split2", "split3", "split5"])
def split(request):
    pkg.set_split(request.param)
    yield request.param
    pkg.set_split(0)


@pytest.mark.parametrize("case", SPLIT_CASES)
def test_split_trajectories_bit_exact(case, split):
    net, omega, pats = CASES[case]()
    text = ps.to_text(net)
    say("split trajectories {} n={} omega={} parts={}".format(case, net.n, omega, split))
    sim = pkg.Simulation(pkg.Network(text), omega, 7828, max_props=len(pats), max_len=4096)
    sim.reset(pats)
    ch = oracle.Chains(oracle.Net(text), omega, 7828, pats)
    for steps in (37, 100, 63, 1):
        sim.run(steps)
        ch.extend(steps)
        assert np.array_equal(sim.read_state(), ch.states), steps
    L = ch.length
    for q in range(len(pats)):
        assert np.array_equal(sim.read_bits(q, 0, L), ch.bits[q]), q
    assert sim.position() == (L, L)


def test_split_burn_in_and_thinning(split):
    net, omega, pats = CASES["n300_l4"]()
    text = ps.to_text(net)
    say("split burn-in/thin parts={}".format(split))
    sim = pkg.Simulation(pkg.Network(text), omega, 99, max_props=1, max_len=1024)
    sim.reset(pats)
    sim.run(40, burn_in=11, thin=3)
    ch = oracle.Chains(oracle.Net(text), omega, 99, pats)
    ch.extend(11 + 120)
    assert np.array_equal(sim.read_state(), ch.states)
    idx = 11 + 3 * np.arange(40) + 2
    assert np.array_equal(sim.read_bits(0, 0, 40), ch.bits[0][:, idx])
    assert sim.position() == (40, 131)


def test_split_gives_up_cleanly():
    """With a one-poll limit a part that reaches a transition's barrier before
    its group gives up at once: the group ends early (no hang), leaves its
    state as the launch found it, and the call re-runs it in the one-block
    form, so it succeeds and the chains still equal the oracle's."""
    net, omega, pats = CASES["n300_l4"]()
    text = ps.to_text(net)
    say("split failure path: 5 parts, one poll")
    sim = pkg.Simulation(pkg.Network(text), omega, 7828, max_props=1, max_len=4096)
    ch = oracle.Chains(oracle.Net(text), omega, 7828, pats)
    pkg.set_split(5)
    pkg.set_split_polls(1)
    pkg.profile_reset()
    try:
        sim.reset(pats)
        for steps in (300, 45, 301):
            sim.run(steps)
            ch.extend(steps)
            assert np.array_equal(sim.read_state(), ch.states), steps
        fallbacks = pkg.profile_read()["split_fallbacks"]
    finally:
        pkg.set_split_polls(0)
        pkg.set_split(0)
    assert fallbacks > 0
    assert np.array_equal(sim.read_bits(0, 0, ch.length), ch.bits[0])


def test_split_give_up_in_estimates_and_server():
    """The same failure path inside rounds that reduce what they extended: a
    one-network estimate and a server round re-run the groups that gave up and
    repeat the round's reductions, and every result equals the oracle's."""
    job = ps.medium()
    text = ps.to_text(job.net)
    want = drivers.solve(text, job.chains, job.seed, job.patterns, job.r, job.confidence, job.psrf_max, cap=CAP)
    reqs = [(c, ps.to_text(CASES[c]()[0]), CASES[c]()[2][:1]) for c in ("n300_l4", "ragged_l6_k5", "medium")]
    pkg.set_split(3)
    pkg.set_split_polls(1)
    pkg.profile_reset()
    try:
        say("split give-up: estimate on medium, 3 parts, one poll")
        sim = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=1, max_len=CAP)
        got = sim.estimate(job.patterns, job.r, job.confidence, psrf_max=job.psrf_max)
        say("split give-up: server with three requests")
        srv = pkg.Server(256 << 20)
        ids = {c: srv.submit(pkg.Network(t), 64, 90 + i, p, 0.02, max_len=CAP, psrf_max=1.1)
               for i, (c, t, p) in enumerate(reqs)}
        rounds = 0
        while srv.step()[2] < len(reqs):
            rounds += 1
            assert rounds < 10000
        fallbacks = pkg.profile_read()["split_fallbacks"]
    finally:
        pkg.set_split_polls(0)
        pkg.set_split(0)
    assert fallbacks > 0
    assert_same_result(got[0], want[0], "medium estimate")
    for i, (c, t, p) in enumerate(reqs):
        w = drivers.solve(t, 64, 90 + i, p, 0.02, 0.95, 1.1, cap=CAP)[0]
        assert_same_result(srv.poll(ids[c])[0], w, c)


def test_server_bad_requests_refused_at_submit():
    """A state set naming a node beyond n, or more terms than the limit, is
    refused when submitted, so a server with good requests beside it runs on."""
    net, _, pats = CASES["ragged_k6_p05"]()
    text = ps.to_text(net)
    nw = pkg.Network(text)
    srv = pkg.Server(64 << 20)
    good = srv.submit(nw, 64, 3, pats[:1], 0.02, max_len=CAP, psrf_max=1.1)
    with pytest.raises(pkg.PbnError) as e:
        srv.submit(nw, 64, 4, [((net.n, 1),)], 0.02, max_len=CAP)
    assert e.value.code == pkg.PBN_EINVAL
    with pytest.raises(pkg.PbnError) as e:
        srv.submit(nw, 64, 5, [tuple((i % net.n, 1) for i in range(65))], 0.02, max_len=CAP)
    assert e.value.code == pkg.PBN_ELIMIT
    rounds = 0
    while srv.step()[2] < 1:
        rounds += 1
        assert rounds < 10000
    want = drivers.solve(text, 64, 3, pats[:1], 0.02, 0.95, 1.1, cap=CAP)[0]
    assert_same_result(srv.poll(good)[0], want, "good request")


def test_split_estimate_equals_oracle():
    job = ps.medium()
    text = ps.to_text(job.net)
    say("split estimate: medium two-state, 4 parts")
    pkg.set_split(4)
    try:
        sim = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=1, max_len=CAP)
        got = sim.estimate(job.patterns, job.r, job.confidence, psrf_max=job.psrf_max)
    finally:
        pkg.set_split(0)
    want = drivers.solve(text, job.chains, job.seed, job.patterns, job.r, job.confidence, job.psrf_max, cap=CAP)
    assert_same_result(got[0], want[0], "medium split")


@pytest.mark.parametrize("mode", [("lane", 0), ("auto", 0)], ids=["lane", "auto"])
def test_large_sampled_chains(mode):
    pkg.set_kernel(*mode)
    job = ps.large()
    text = ps.to_text(job.net)
    say("large: 8192 chains x 2000 nodes, 24 steps, sampled oracle chains, kernel {}".format(mode))
    sim = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=5, max_len=256)
    sim.reset(job.patterns)
    init = sim.read_state()
    sim.run(24)
    st = sim.read_state()
    bits = [sim.read_bits(q, 0, 24) for q in range(5)]
    onet = oracle.Net(text)
    for c0 in (0, 4031, 8128):
        ch = oracle.Chains(onet, 64, job.seed, job.patterns, chain0=c0)
        assert np.array_equal(init[c0:c0 + 64], ch.states)
        ch.extend(24)
        assert np.array_equal(st[c0:c0 + 64], ch.states), c0
        for q in range(5):
            assert np.array_equal(bits[q][c0:c0 + 64], ch.bits[q]), (c0, q)
    pkg.set_kernel("auto", 0)


def test_state_rows_beyond_lds():
    """n = 12000: neither the bit-sliced state (2n + sum(l-1) words) nor a chain's
    375-word rows fit in LDS, so the lane-per-chain kernel keeps its rows in
    device scratch; results stay bit-exact."""
    net = ps.random_network(np.random.default_rng(77), 12000, (1, 3), (1, 5), 0.001)
    text = ps.to_text(net)
    pats = [((0, 1), (11999, 0))]
    omega = 70
    say("state rows beyond LDS: n=12000, omega=70")
    sim = pkg.Simulation(pkg.Network(text), omega, 4242, max_props=1, max_len=256)
    sim.reset(pats)
    ch = oracle.Chains(oracle.Net(text), omega, 4242, pats)
    for steps in (5, 3):
        sim.run(steps)
        ch.extend(steps)
        assert np.array_equal(sim.read_state(), ch.states), steps
    assert np.array_equal(sim.read_bits(0, 0, 8), ch.bits[0])


def test_window_counts_batch_sums_psrf():
    job = ps.medium()
    text = ps.to_text(job.net)
    pats = job.patterns + [((0, 1),)]
    say("window counts / batch sums / psrf on medium")
    sim = pkg.Simulation(pkg.Network(text), 256, 31, max_props=2, max_len=2048)
    sim.reset(pats)
    sim.run(700)
    ch = oracle.Chains(oracle.Net(text), 256, 31, pats)
    ch.extend(700)
    for q in range(2):
        x = ch.bits[q].astype(np.int64)
        for lo, hi in ((0, 700), (5, 6), (31, 33), (64, 128), (100, 613), (699, 700)):
            got = sim.window_counts(q, lo, hi)
            S = x[:, lo:hi].sum(axis=1)
            n00, n01, n10, n11 = stats.transition_counts(x[:, lo:hi])
            want = dict(T1=int(S.sum()), T2=int((S * S).sum()), n00=n00, n01=n01, n10=n10, n11=n11)
            assert got == want, (q, lo, hi)
        for base, kappa, m in ((0, 1, 700), (17, 16, 5), (256, 33, 13)):
            got = sim.batch_sums(q, base, kappa, m)
            want = x[:, base: base + kappa * m].reshape(256, m, kappa).sum(axis=2)
            assert np.array_equal(got, want)
        for psi in (2, 64, 350):
            assert close(sim.psrf(q, psi), stats.psrf(x[:, 700 - psi:]))


@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_estimate_two_state(name):
    job = getattr(ps, name)()
    text = ps.to_text(job.net)
    say("estimate two-state " + name)
    sim = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=1, max_len=CAP)
    got = sim.estimate(job.patterns, job.r, job.confidence, psrf_max=job.psrf_max)
    want = drivers.solve(text, job.chains, job.seed, job.patterns, job.r, job.confidence, job.psrf_max, cap=CAP)
    assert_same_result(got[0], want[0], name)


@pytest.mark.parametrize("case", ["tiny", "medium", "ragged_k6_p05", "ragged_k7_p05", "n300_l4"])
def test_sequential_equals_oracle(case):
    """Alg. 1 (the sequential two-state method on one chain) against the oracle."""
    net, _, pats = CASES[case]()
    text = ps.to_text(net)
    say("sequential two-state " + case)
    sim = pkg.Simulation(pkg.Network(text), 1, 2024, max_props=1, max_len=CAP)
    got = sim.estimate(pats[:1], 0.02, 0.95, method="sequential")
    want = drivers.solve(text, 1, 2024, pats[:1], 0.02, 0.95, 1.1, method="sequential", cap=CAP)
    assert_same_result(got[0], want[0], case)


@pytest.mark.parametrize("case", ["tiny", "medium", "ragged_k6_p05", "ragged_k7_p05", "n300_l4"])
def test_sequential_skart_equals_oracle(case):
    """Alg. 2 (the sequential Skart method on one chain) against the oracle on
    three seeds: spacers from 0 to 8 batches, batch sizes from 2 to 16, and one
    run whose batches grow after every spacer failed (ragged_k6_p05, seed 7)."""
    net, _, pats = CASES[case]()
    text = ps.to_text(net)
    nw = pkg.Network(text)
    for seed in (2024, 7, 99):
        say("sequential skart {} seed {}".format(case, seed))
        sim = pkg.Simulation(nw, 1, seed, max_props=1, max_len=CAP)
        got = sim.estimate(pats[:1], 0.02, 0.95, method="sequential_skart")
        want = drivers.solve(text, 1, seed, pats[:1], 0.02, 0.95, 1.1, method="sequential_skart", cap=CAP)
        assert got[0]["status"] == 0
        assert_same_result(got[0], want[0], (case, seed))


@pytest.mark.parametrize("case,cap", [("medium", 16000), ("tiny", 2000)])
def test_sequential_skart_cap(case, cap):
    """A cap on the positions ends Alg. 2 as not converged, in the randomness
    stage (medium: 16 x 1280 positions) and in the CI stage (tiny: the batch
    size grows past the cap), with the same report as the oracle's."""
    job = getattr(ps, case)()
    text = ps.to_text(job.net)
    say("sequential skart cap {} {}".format(case, cap))
    sim = pkg.Simulation(pkg.Network(text), 1, 7, max_props=1, max_len=CAP)
    got = sim.estimate(job.patterns[:1], 0.02, 0.95, method="sequential_skart", max_len=cap)
    want = drivers.solve(text, 1, 7, job.patterns[:1], 0.02, 0.95, 1.1, method="sequential_skart", cap=cap)
    assert got[0]["status"] == pkg.PBN_ENOTCONV
    assert_same_result(got[0], want[0], case)


def test_sequential_batched_equals_oracle():
    """Several one-chain simulations in one batched call, for each sequential
    method: every result equals the oracle's solo run."""
    names = ["tiny", "ragged_k7_p05", "n300_l4", "ragged_k6_p05"]
    nets = [CASES[c]() for c in names]
    texts = [ps.to_text(net) for net, _, _ in nets]
    for method in ("sequential", "sequential_skart"):
        say("batched " + method)
        sims = [pkg.Simulation(pkg.Network(t), 1, 40 + i, max_props=1, max_len=CAP) for i, t in enumerate(texts)]
        got = pkg.batch_estimate(sims, [p[:1] for _, _, p in nets], [0.02] * len(sims), [0.95] * len(sims),
                                 method=method)
        for i, (t, (_, _, p)) in enumerate(zip(texts, nets)):
            want = drivers.solve(t, 1, 40 + i, p[:1], 0.02, 0.95, 1.1, method=method, cap=CAP)
            assert_same_result(got[i][0], want[0], (method, names[i]))


def test_threads_use_the_library_at_once():
    """Two host threads on their own simulations at the same time, one through
    the batched lanes and one through one-network estimates (which fork over
    the shared stream pool), both recording profile marks: every result
    equals the oracle's.  The node-split form is off here, since its parts
    need the device to themselves."""
    import threading
    names = [["tiny", "ragged_k7_p05"], ["ragged_k6_p05", "n300_l4"]]
    want, got, errors = {}, {}, []
    for t, group in enumerate(names):
        for c in group:
            net, omega, pats = CASES[c]()
            want[c] = drivers.solve(ps.to_text(net), omega, 60 + t, pats[:1], 0.02, 0.95, 1.1, cap=CAP)[0]

    def work(t, group):
        try:
            cases = [CASES[c]() for c in group]
            sims = [pkg.Simulation(pkg.Network(ps.to_text(net)), omega, 60 + t, max_props=1, max_len=CAP)
                    for net, omega, _ in cases]
            for rep in range(3):
                if t == 0:
                    res = [r[0] for r in pkg.batch_estimate(sims, [p[:1] for _, _, p in cases], [0.02] * 2,
                                                            [0.95] * 2, psrf_max=1.1)]
                else:
                    res = [sm.estimate(p[:1], 0.02, 0.95, psrf_max=1.1)[0] for sm, (_, _, p) in zip(sims, cases)]
                for c, r in zip(group, res):
                    got[(c, rep)] = r
        except Exception as e:                 # reported by the main thread
            errors.append(e)

    pkg.set_split(1)
    pkg.profile_enable(True)
    try:
        say("two threads: batched lanes and one-network estimates")
        th = [threading.Thread(target=work, args=(t, g)) for t, g in enumerate(names)]
        for x in th:
            x.start()
        for x in th:
            x.join(timeout=100)
        assert not any(x.is_alive() for x in th)
    finally:
        pkg.profile_enable(False)
        pkg.set_split(0)
    assert not errors, errors
    for (c, rep), r in got.items():
        assert_same_result(r, want[c], (c, rep))
    assert len(got) == 12


def test_server_rejects_sequential_methods():
    job = ps.tiny()
    net = pkg.Network(ps.to_text(job.net))
    srv = pkg.Server(64 << 20)
    for method in ("sequential", "sequential_skart"):
        with pytest.raises(pkg.PbnError):
            srv.submit(net, 8, 1, job.patterns, 0.02, method=method)


def test_estimate_two_state_seeds_and_reruns():
    # several seeds and a small psi0 so that Alg. 4's burn-in re-run (M > psi) occurs
    job = ps.tiny()
    text = ps.to_text(job.net)
    net = pkg.Network(text)
    reruns = 0
    for seed in range(20):
        say("tiny seed {}".format(seed))
        sim = pkg.Simulation(net, 8, seed, max_props=1, max_len=CAP)
        got = sim.estimate(job.patterns, 0.02, 0.95, psi0=4, psrf_max=1.1)[0]
        want = drivers.solve(text, 8, seed, job.patterns, 0.02, 0.95, 1.1, psi0=4, cap=CAP)[0]
        assert_same_result(got, want, seed)
        reruns += got["psi"] != got["psi_gr"]
    assert reruns > 0


def test_estimate_skart():
    job = ps.medium()
    text = ps.to_text(job.net)
    say("estimate skart on medium network, 64 chains")
    pats = job.patterns + [((1, 1), (2, 0))]
    sim = pkg.Simulation(pkg.Network(text), 64, 5, max_props=2, max_len=CAP)
    got = sim.estimate(pats, 0.01, 0.95, method="skart", psrf_max=1.1)
    want = drivers.solve(text, 64, 5, pats, 0.01, 0.95, 1.1, method="skart", cap=CAP)
    for q in range(2):
        assert_same_result(got[q], want[q], q)


def test_multi_property_equals_solo():
    job = ps.medium()
    text = ps.to_text(job.net)
    rng = np.random.default_rng(8)
    pats = [ps.random_pattern(rng, 100, k) for k in (1, 2, 3, 1)]
    say("multi-property")
    sim = pkg.Simulation(pkg.Network(text), 128, 77, max_props=4, max_len=CAP)
    got = sim.estimate(pats, 0.01, 0.95, psrf_max=1.1)
    want = drivers.solve(text, 128, 77, pats, 0.01, 0.95, 1.1, cap=CAP)
    for q in range(4):
        assert_same_result(got[q], want[q], q)
    # the shared chains are as long as the longest requirement
    assert sim.position()[0] == max(w["chain_len"] for w in want)


def test_multiprop_equals_oracle_and_solo():
    """The multi-property shape (96 nodes, 7 state sets): the simultaneous GPU
    estimate equals the oracle's, and each property equals its solo GPU run."""
    job = ps.multiprop(chains=256, r=1e-2)
    text = ps.to_text(job.net)
    say("multiprop: 96 nodes, 7 state sets, 256 chains")
    sim = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=7, max_len=CAP)
    got = sim.estimate(job.patterns, job.r, job.confidence, psrf_max=job.psrf_max)
    want = drivers.solve(text, job.chains, job.seed, job.patterns, job.r, job.confidence, job.psrf_max, cap=CAP)
    for q in range(7):
        assert_same_result(got[q], want[q], q)
    for q in (0, 4):
        solo = pkg.Simulation(pkg.Network(text), job.chains, job.seed, max_props=1, max_len=CAP)
        one = solo.estimate([job.patterns[q]], job.r, job.confidence, psrf_max=job.psrf_max)
        assert_same_result(one[0], got[q], ("solo", q))


def test_batched_equals_oracle():
    jobs = sorted(ps.batched(), key=lambda j: j.net.n * j.chains)[:10]
    say("batched estimate of {} networks".format(len(jobs)))
    nets = [pkg.Network(ps.to_text(j.net)) for j in jobs]
    sims = [pkg.Simulation(nt, j.chains, j.seed, max_props=1, max_len=CAP) for nt, j in zip(nets, jobs)]
    got = pkg.batch_estimate(sims, [j.patterns for j in jobs], [j.r for j in jobs],
                             [j.confidence for j in jobs], psrf_max=1.1)
    for j, g in zip(jobs, got):
        want = drivers.solve(ps.to_text(j.net), j.chains, j.seed, j.patterns, j.r, j.confidence, 1.1, cap=CAP)
        assert_same_result(g[0], want[0], j.name)


def test_batched_lanes_equal_oracle():
    # many small networks: every lane's rounds, lanes rebalanced
    jobs = sorted(ps.batched(), key=lambda j: j.net.n * j.chains)[:24]
    say("laned batched estimate of {} networks".format(len(jobs)))
    nets = [pkg.Network(ps.to_text(j.net)) for j in jobs]
    sims = [pkg.Simulation(nt, j.chains, j.seed, max_props=1, max_len=CAP) for nt, j in zip(nets, jobs)]
    got = pkg.batch_estimate(sims, [j.patterns for j in jobs], [j.r for j in jobs],
                             [j.confidence for j in jobs], psrf_max=1.1)
    for j, g in zip(jobs, got):
        want = drivers.solve(ps.to_text(j.net), j.chains, j.seed, j.patterns, j.r, j.confidence, 1.1, cap=CAP)
        assert_same_result(g[0], want[0], j.name)
    # a second batch on the same simulations restarts them and gives the same results
    again = pkg.batch_estimate(sims, [j.patterns for j in jobs], [j.r for j in jobs],
                               [j.confidence for j in jobs], psrf_max=1.1)
    for a, b in zip(got, again):
        assert_same_result(b[0], a[0], "rerun")


def test_sliced_rounds_equal_oracle():
    # the largest networks take several time slices per extension (16-wave
    # lane), beside small ones in the other lanes
    big = sorted(ps.batched(), key=lambda j: -j.net.n)[:3]
    small = sorted(ps.batched(), key=lambda j: j.net.n)[:3]
    jobs = [dataclasses.replace(j, chains=96) for j in big] + small
    say("sliced rounds: n = {}".format([j.net.n for j in jobs]))
    nets = [pkg.Network(ps.to_text(j.net)) for j in jobs]
    sims = [pkg.Simulation(nt, j.chains, j.seed, max_props=1, max_len=CAP) for nt, j in zip(nets, jobs)]
    got = pkg.batch_estimate(sims, [j.patterns for j in jobs], [j.r for j in jobs],
                             [j.confidence for j in jobs], psrf_max=1.1)
    for j, g in zip(jobs, got):
        want = drivers.solve(ps.to_text(j.net), j.chains, j.seed, j.patterns, j.r, j.confidence, 1.1, cap=CAP)
        assert_same_result(g[0], want[0], j.name)


def test_autotune_keeps_results():
    # the measured kernel shapes change launches, never results
    jobs = sorted(ps.batched(), key=lambda j: j.net.n * j.chains)[:6] + sorted(ps.batched(), key=lambda j: -j.net.n)[:2]
    jobs = [dataclasses.replace(j, chains=min(j.chains, 128)) for j in jobs]
    nets = [pkg.Network(ps.to_text(j.net)) for j in jobs]

    def solve():
        sims = [pkg.Simulation(nt, j.chains, j.seed, max_props=1, max_len=CAP) for nt, j in zip(nets, jobs)]
        return pkg.batch_estimate(sims, [j.patterns for j in jobs], [j.r for j in jobs],
                                  [j.confidence for j in jobs], psrf_max=1.1)

    before = solve()
    say("autotune")
    rows = pkg.autotune()
    try:
        assert len(rows) == 8
        for r in rows:
            assert r["waves_throughput"] in (1, 2, 4, 5, 8, 12, 16) and r["waves_latency"] in (1, 2, 4, 5, 8, 12, 16)
            assert r["node_updates_per_s"] > 0 and r["transition_us"] > 0
        after = solve()
    finally:
        pkg.autotune_reset()
    for a, b, j in zip(after, before, jobs):
        assert_same_result(a[0], b[0], j.name)


def test_server_isolation():
    jobs = sorted(ps.serving(limit=40), key=lambda j: j.net.n)[:8]
    say("server with {} requests".format(len(jobs)))
    nets = [pkg.Network(ps.to_text(j.net)) for j in jobs]
    need = [nt.sim_bytes(64, 1, CAP) for nt in nets]
    arena = sum(sorted(need)[-3:]) + (1 << 16)       # room for about three at a time
    srv = pkg.Server(arena)
    ids = [srv.submit(nt, 64, j.seed, j.patterns, j.r, j.confidence, max_len=CAP, psrf_max=1.1)
           for nt, j in zip(nets, jobs)]
    rounds = 0
    while True:
        active, waiting, done = srv.step()
        rounds += 1
        assert srv.memory()[0] <= arena
        if done == len(jobs):
            break
        assert rounds < 10000
    assert srv.memory()[1] <= arena
    for rid, j in zip(ids, jobs):
        got = srv.poll(rid)
        want = drivers.solve(ps.to_text(j.net), 64, j.seed, j.patterns, j.r, j.confidence, 1.1, cap=CAP)
        assert_same_result(got[0], want[0], j.name)


def test_server_admissions_with_several_state_sets():
    """Requests with two state sets each, two-state and Skart alternating,
    arriving in two waves (the second while the first is on the device): the
    batched admission resets each simulation with its own sets, and every
    result equals the oracle's solo run."""
    cases = ["ragged_k7_p05", "ragged_k6_p05", "n300_l4", "medium", "ragged_l6_k5", "high_p"]
    reqs = []
    for i, c in enumerate(cases):
        net, _, pats = CASES[c]()
        pats = (pats + [((0, 0),)])[:2]
        reqs.append((c, ps.to_text(net), pats, "two_state" if i % 2 == 0 else "skart", 70 + i))
    srv = pkg.Server(256 << 20)
    ids = {}
    say("server: two waves of requests with two state sets")
    for c, text, pats, method, seed in reqs[:3]:
        ids[c] = srv.submit(pkg.Network(text), 64, seed, pats, 0.02, max_len=CAP, psrf_max=1.1, method=method)
    srv.step()
    for c, text, pats, method, seed in reqs[3:]:
        ids[c] = srv.submit(pkg.Network(text), 64, seed, pats, 0.02, max_len=CAP, psrf_max=1.1, method=method)
    rounds = 0
    while srv.step()[2] < len(reqs):
        rounds += 1
        assert rounds < 10000
    for c, text, pats, method, seed in reqs:
        got = srv.poll(ids[c])
        want = drivers.solve(text, 64, seed, pats, 0.02, 0.95, 1.1, method=method, cap=CAP)
        for q in range(2):
            assert_same_result(got[q], want[q], (c, method, q))


def test_rejects_bad_arguments():
    net = pkg.Network(ps.to_text(ps.tiny().net))
    sim = pkg.Simulation(net, 1, 1, max_props=1, max_len=64)
    with pytest.raises(pkg.PbnError):
        sim.estimate([((0, 1),)], 0.01, 0.95)          # Gelman-Rubin needs two chains
    sim2 = pkg.Simulation(net, 4, 1, max_props=1, max_len=64)
    sim2.reset([((0, 1),)])
    with pytest.raises(pkg.PbnError):
        sim2.run(100)                                  # beyond the bit-stream capacity
    with pytest.raises(pkg.PbnError):
        sim2.window_counts(0, 0, 10)                   # nothing recorded yet
    res = sim2.estimate([((0, 1),)], 1e-4, 0.95, psrf_max=1.1)[0]
    assert res["status"] == pkg.PBN_ENOTCONV           # cap reached before N
    # sizes whose sums or products wrap around 2^64 are refused on the host
    big = (1 << 64) - 1
    for call in (lambda: sim2.run(big, burn_in=1), lambda: sim2.run(2, thin=(1 << 32) - 1),
                 lambda: pkg.batch_run([sim2], [big]), lambda: sim2.batch_sums(0, 0, 1 << 63, 2),
                 lambda: sim2.read_bits(0, big, 2),
                 # one simulation twice in a batched call
                 lambda: pkg.batch_run([sim2, sim2], [1, 1]),
                 lambda: pkg.batch_estimate([sim2, sim2], [[((0, 1),)]] * 2, [0.02] * 2, [0.95] * 2)):
        with pytest.raises(pkg.PbnError):
            call()
    with pytest.raises(pkg.PbnError) as e:
        pkg.Simulation(net, 4, 1, max_props=1, max_len=1 << 32)
    assert e.value.code == pkg.PBN_ELIMIT
    with pytest.raises(pkg.PbnError) as e:
        pkg.Server(64 << 20).submit(net, (1 << 24) + 1, 1, [((0, 1),)], 0.02)
    assert e.value.code == pkg.PBN_ELIMIT


@pytest.mark.parametrize("method", ["two_state", "skart"])
def test_estimate_with_thinning(method):
    """pbn_opts.thin = 3: the procedures run on every third state of the
    chains; every result equals the oracle's on its thinned chains, and the
    sample size is omega n."""
    net, omega, pats = CASES["ragged_k6_p05"]()
    text = ps.to_text(net)
    say("estimate with thin 3, " + method)
    sim = pkg.Simulation(pkg.Network(text), omega, 313, max_props=2, max_len=CAP)
    got = sim.estimate(pats[:2], 0.02, 0.95, method=method, psrf_max=1.1, thin=3)
    want = drivers.solve(text, omega, 313, pats[:2], 0.02, 0.95, 1.1, method=method, cap=CAP, thin=3)
    for q in range(2):
        assert_same_result(got[q], want[q], (method, q))
        assert got[q]["sample_size"] == omega * want[q]["n"] and got[q]["rounds"] >= 2
    # the chains made three transitions per recorded position
    L, T = sim.position()
    assert T == 3 * L


def test_kernel_choice_per_simulation():
    """Per-simulation kernel and node-split choices override the process-wide
    ones for that simulation only; results equal the oracle's either way."""
    net, omega, pats = CASES["n300_l4"]()
    text = ps.to_text(net)
    nw = pkg.Network(text)
    a = pkg.Simulation(nw, omega, 21, max_props=1, max_len=4096)
    b = pkg.Simulation(nw, omega, 21, max_props=1, max_len=4096)
    a.set_kernel("lane")
    b.set_split(3)
    pkg.set_kernel("bitsliced", 2)
    pkg.profile_reset()
    pkg.profile_enable(True)
    try:
        say("per-simulation kernel choice: lane-per-chain beside 3 parts")
        for s in (a, b):
            s.reset(pats)
            s.run(150)
        prof = pkg.profile_read()
    finally:
        pkg.profile_enable(False)
        pkg.set_kernel("auto", 0)
    ch = oracle.Chains(oracle.Net(text), omega, 21, pats)
    ch.extend(150)
    for s in (a, b):
        assert np.array_equal(s.read_state(), ch.states)
        assert np.array_equal(s.read_bits(0, 0, 150), ch.bits[0])
    assert prof["split_launches"] >= 1
    a.set_kernel("global")
    b.set_split(-1)
    with pytest.raises(pkg.PbnError):
        a.set_kernel("bitsliced", 17)


def test_split_workspace_grows():
    """Launches whose node-split groups outnumber the previous launch's make
    the workspace grow its group tables; later launches still run and every
    chain equals the oracle's (a regression test: the growth once freed one
    buffer twice, and the next launch failed)."""
    cases = ["n300_l4", "ragged_l6_k5", "medium"]
    nets = [CASES[c]() for c in cases]
    texts = [ps.to_text(n) for n, _, _ in nets]
    sims = [pkg.Simulation(pkg.Network(t), 64, 500 + i, max_props=1, max_len=1024) for i, t in enumerate(texts)]
    for s, (_, _, p) in zip(sims, nets):
        s.reset(p[:1])
    pkg.set_split(2)
    try:
        say("split workspace growth: 1 group, then 3, then 3 again")
        pkg.batch_run(sims[:1], [40])
        pkg.batch_run(sims, [40, 80, 80])
        pkg.batch_run(sims, [20, 20, 20])
    finally:
        pkg.set_split(0)
    for i, (s, t, (_, _, p)) in enumerate(zip(sims, texts, nets)):
        ch = oracle.Chains(oracle.Net(t), 64, 500 + i, p[:1])
        ch.extend(s.position()[0])
        assert np.array_equal(s.read_state(), ch.states), cases[i]
        assert np.array_equal(s.read_bits(0, 0, ch.length), ch.bits[0]), cases[i]


def test_library_loaded_before_torch():
    """A process that loads the library before it touches torch (a network
    compiled first) still runs on the one HIP runtime torch uses: a regression
    test, since the library once bound to a second runtime there and its first
    device call failed."""
    import subprocess
    script = (
        "import sys; sys.path.insert(0, {root!r})\n"
        "import numpy as np\n"
        "import paper_1508_07828_amd as pkg, pbnsynth as ps\n"
        "net = pkg.Network(ps.to_text(ps.medium().net))\n"
        "srv = pkg.Server(64 << 20)\n"
        "rid = srv.submit(net, 64, 3, ps.medium().patterns, 0.02, max_len=1 << 15, psrf_max=1.1)\n"
        "while srv.step()[2] < 1: pass\n"
        "print('status', srv.poll(rid)[0]['status'])\n").format(root=ROOT)
    say("library loaded before torch, in a child process")
    out = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "status 0" in out.stdout, out.stdout


# requests of the serving trace with n >= 2000 at r = 0.005 (trace index: chain
# length, n): 1262: 512, 2109; 484: 512, 3056; 441: 682, 2013; 1307: 684, 2613;
# 1285: 923, 2016; 588: 795, 3149; 356: 1715, 2172
SERVE_BIG = (1262, 484, 441, 1307, 1285, 588, 356)


def test_server_large_requests_and_long_lane():
    """The top of the serving trace (n >= 2000, r = 0.005) in one server with
    smaller requests, node-split parts planned per round: with a low threshold
    the longer ones move to the long-request lane (a CU-masked stream of its
    own, slices collected asynchronously) while the others keep to the
    remaining CUs.  Every result equals the oracle's solo run."""
    jobs = [ps.serving_request(i) for i in SERVE_BIG] + sorted(ps.serving(limit=60), key=lambda j: j.net.n)[:6]
    srv = pkg.Server(2 << 30)
    srv.configure(long_lane_us=2000.0, long_slice_us=3000.0, ahead_us=500.0)
    say("server: {} requests, n = {}".format(len(jobs), [j.net.n for j in jobs]))
    ids = [srv.submit(pkg.Network(ps.to_text(j.net)), j.chains, j.seed, j.patterns, j.r, j.confidence,
                      max_len=CAP, psrf_max=j.psrf_max) for j in jobs]
    pkg.profile_reset()
    pkg.profile_enable(True)
    rounds = 0
    try:
        while srv.step()[2] < len(jobs):
            rounds += 1
            assert rounds < 100000
        prof = pkg.profile_read()
    finally:
        pkg.profile_enable(False)
    assert prof["split_launches"] > 0
    moved, long_rounds = srv.lane_stats()
    say("long lane: {} requests, {} rounds".format(moved, long_rounds))
    assert moved >= 2 and long_rounds >= 2
    for rid, j in zip(ids, jobs):
        say("oracle: trace request n={} r={}".format(j.net.n, j.r))
        want = drivers.solve(ps.to_text(j.net), j.chains, j.seed, j.patterns, j.r, j.confidence, j.psrf_max,
                             cap=CAP)
        assert_same_result(srv.poll(rid)[0], want[0], j.name)
