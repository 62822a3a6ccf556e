/*
 * pbnssa — steady-state analysis of probabilistic Boolean networks on MI355X.
 *
 * C ABI of the GPU library (libpbnssa.so).  Plain C types only: host pointers,
 * device pointers passed as void*, sizes.  No exceptions cross this boundary.
 *
 * Model (Mizera, Pang, Yuan, "Parallel approximate steady-state analysis of
 * large probabilistic Boolean networks", Sec. 2.2): n binary nodes; node i has
 * l(i) predictor functions, one chosen per step with probabilities c_j^(i)
 * (instantaneously random PBN); a perturbation vector gamma(t) with
 * gamma_i ~ Bernoulli(p); if gamma(t) = 0 the state is updated synchronously by
 * the selected functions, otherwise s(t+1) = s(t) XOR gamma(t).
 *
 * Method (Sec. 3-4): omega chains run in parallel; Gelman & Rubin's potential
 * scale reduction factor (Alg. 3) certifies convergence; then either the
 * two-state Markov chain approach (Alg. 4, sample size N and burn-in M of
 * Alg. 1) or a parallel Skart batch-means procedure (Alg. 5) decides how long
 * the chains must run to estimate the steady-state probability of a set of
 * states within precision r at confidence s.
 *
 * Random stream (the paper leaves it open; fixed here so results are
 * reproducible and independent of launch shapes): Philox4x32-10 with key =
 * (seed low 32, seed high 32); for transition t (0-based) of chain c, the
 * perturbation and selection uniforms of node i are 32-bit values
 * (byte << 24) | low24 where byte is byte (i mod 16) of Philox((t, c, i/16, tag))
 * and low24 the low 24 bits of word (i mod 4) of Philox((t, c, i/4, tag+1)),
 * tag 0 (perturbation) or 2 (selection).  gamma_i = (u < floor(p 2^32)); the
 * selected function is the first j with u < T_j, T_j = min(2^32-1,
 * floor(2^32 (c_1+..+c_j))), else the last one.  Initial states: bit i of chain
 * c is bit (i mod 32) of word (w mod 4) of Philox((0, c, w/4, 4)), w = i/32.
 *
 * Status codes: every int-returning call returns one of PBN_* below; details
 * of the last error on the calling thread come from pbn_last_error().
 *
 * Threads: a handle (network, simulation, server) is used by one thread at a
 * time; different handles may be used from different threads at once.  The
 * batched calls share one set of lane streams, so concurrent batched solves
 * run one after the other.  The node-split form needs the device to itself;
 * under concurrent calls its parts can give up (then re-run in the one-block
 * form, about a second later, with the same results), so callers on several
 * threads turn it off with pbn_set_split(1).
 */
#ifndef PBNSSA_H
#define PBNSSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PBN_OK = 0,
    PBN_EINVAL = 1,     /* bad argument (omega < 2, r <= 0, s not in (0,1), ...)      */
    PBN_EFORMAT = 2,    /* malformed network text                                     */
    PBN_ENOMEM = 3,     /* device buffer too small / server budget exhausted          */
    PBN_EDEVICE = 4,    /* a HIP call failed (message in pbn_last_error)              */
    PBN_ENOTCONV = 5,   /* result status: a chain-length cap was hit before the stop  */
    PBN_ELIMIT = 6      /* a structural limit was exceeded (see the limits below)     */
};

enum { PBN_TWO_STATE = 0, PBN_SKART = 1, PBN_SEQ_TWO_STATE = 2, PBN_SEQ_SKART = 3 };

/* Limits: n <= 65535 nodes, l(i) <= 64 functions per node, k <= 16 parents per
 * function, at most PBN_MAX_PROPS state sets per simulation and
 * PBN_MAX_TERMS (node, value) terms over all of them, at most PBN_MAX_CHAINS
 * chains per simulation, transitions per chain below 2^32 and recorded
 * positions per chain (max_len) at most PBN_MAX_LEN.  Every n is simulated: networks whose bit-sliced state does not
 * fit in LDS run the lane-per-chain kernel, whose per-chain state rows move
 * from LDS to library-owned device scratch beyond n = 10240. */
#define PBN_MAX_PROPS 8
#define PBN_MAX_TERMS 64
#define PBN_MAX_CHAINS (1u << 24)
#define PBN_MAX_LEN 0xFFFFFFFFull

typedef struct pbn_net pbn_net;      /* parsed + compiled network (host memory, library-owned) */
typedef struct pbn_sim pbn_sim;      /* omega chains of one network on one device buffer      */
typedef struct pbn_server pbn_server;

/* A set of states of interest (Sec. 3.1: meta state 1): the conjunction
 * node[m] == val[m] over nterms terms (0-based node ids, val 0 or 1; any other
 * value is PBN_EINVAL).  No terms: every state; a node asked to be both 0 and
 * 1: no state.  Caller-owned; copied by the call that takes it. */
typedef struct {
    uint32_t nterms;
    const uint32_t *node;
    const uint8_t *val;
} pbn_pattern;

typedef struct {
    int method;                   /* PBN_TWO_STATE (Alg. 4), PBN_SKART (Alg. 5),
                                     PBN_SEQ_TWO_STATE (Alg. 1: the sequential two-state
                                     method on a single chain, omega = 1; initial burn-in
                                     m0 = psi0 and sample n0 = 4 psi0, no Gelman-Rubin), or
                                     PBN_SEQ_SKART (Alg. 2: the sequential Skart method on
                                     a single chain, omega = 1: 1280 initial positions,
                                     spaced randomness test with up to 10 spacer batches,
                                     the spacer batches skipped as warm-up, no
                                     Gelman-Rubin; psi0 and psrf_max are unused)          */
    uint64_t psi0;                /* initial Gelman-Rubin psi (Alg. 3); 0 -> 256          */
    double psrf_max;              /* "close to 1": converged when R < psrf_max; 0 -> 1.1  */
    double eps;                   /* Alg. 1's epsilon for M; 0 -> 1e-10                   */
    uint64_t max_len;             /* cap on recorded positions per chain; 0 -> buffer cap;
                                     the Skart methods stop below 2^31 positions (32-bit
                                     batch sums), and Gelman-Rubin where omega psi^2 would
                                     exceed its exact 63-bit sum of squares            */
    uint32_t thin;                /* transitions per recorded position; 0 or 1 -> every
                                     state (the paper's methods); k > 1 records every k-th
                                     state, so the procedures run on the thinned chains  */
    uint32_t reserved;
} pbn_opts;

/* Result per state set.  prob is the estimate (two-state: ones in the final
 * window / (omega n); Skart: grand batch mean).  ci_lo/ci_hi only for Skart.
 * psi_gr: psi returned by Alg. 3; psi: final window start (after Alg. 4's
 * burn-in re-runs); n: window length per chain; N, M: Alg. 1's sample size and
 * burn-in of the last pass; kappa, batches: Skart batch size and count;
 * chain_len: positions this state set needed (recorded positions: thin transitions
 * each); status: PBN_OK or PBN_ENOTCONV
 * (prob then holds NaN or the last estimate), or for a server request that
 * could not run, the error that ended it (prob NaN). */
typedef struct {
    double prob, ci_lo, ci_hi, rhat;
    uint64_t psi_gr, psi, n, N, M, kappa, batches, chain_len;
    int status;
    int reserved;
    uint64_t sample_size;         /* observations behind prob: omega n (two-state, Skart),
                                     N (Alg. 1), kappa p' (Alg. 2); 0 when not converged */
    uint64_t rounds;              /* window or batch results this state set consumed    */
} pbn_result;

typedef struct {
    uint32_t n, W, nfun, p_thr;   /* W = ceil(n/32) state words per chain                 */
    uint32_t max_k, max_l;
    uint64_t blob_bytes;          /* compiled network size on the device                  */
    double density;               /* Sec. 2.2: total parents of all predictors / n        */
} pbn_net_info;

/* Window aggregates of one state set over positions [lo, hi) (0-based) of all
 * chains: T1 = sum_c S_c, T2 = sum_c S_c^2 (S_c = ones of chain c in the
 * window) and the counts of consecutive pairs (x_l, x_{l+1}) inside the window. */
typedef struct {
    int64_t T1, T2, n00, n01, n10, n11;
} pbn_counts;

/* ---------------------------------------------------------------- networks */

/* Parse and compile a network given as canonical text (see pbnsynth):
 *   "PBN n p" then per node "N i l" and l lines "F c k par_1..par_k tt_hex".
 * Checks: n <= 65535, p in (0,1), c_j in [0,1] summing to 1 within 1e-12,
 * 1 <= k <= 16, parents distinct and < n, truth table fits 2^k bits.
 * Host only (no device call).  On success *out owns the network. */
int pbn_load(const char *text, size_t len, pbn_net **out);
/* The same from a file holding the canonical text.  Errors as pbn_load, and
 * PBN_EINVAL when the file cannot be read. */
int pbn_load_file(const char *path, pbn_net **out);
void pbn_free(pbn_net *net);
int pbn_net_get_info(const pbn_net *net, pbn_net_info *out);
/* Thresholds T_1..T_l of node i (for tests); returns l or -1. */
int pbn_net_thresholds(const pbn_net *net, uint32_t node, uint32_t *out, uint32_t cap);

/* ------------------------------------------------------------ simulations */

/* Device bytes needed for omega chains, up to max_props state sets and
 * max_len recorded positions per chain (bit-streams, one bit per position);
 * 0 when omega, max_props or max_len is beyond the limits above. */
size_t pbn_sim_bytes(const pbn_net *net, uint32_t omega, uint32_t max_props, uint64_t max_len);

/* Create a simulation in a caller-owned device buffer (e.g. a torch tensor)
 * of at least pbn_sim_bytes(...) bytes, on the given HIP stream (NULL = the
 * default stream).  Uploads the compiled network and initialises the chains
 * (transition counter 0, no recorded positions, no state sets).  The buffer
 * must outlive the simulation.  Errors: PBN_EINVAL (omega < 1), PBN_ELIMIT
 * (omega, max_props or max_len beyond the limits), PBN_ENOMEM (buffer too
 * small), PBN_EDEVICE. */
int pbn_sim_create(const pbn_net *net, uint32_t omega, uint64_t seed, uint32_t max_props,
                   uint64_t max_len, void *dev_buf, size_t dev_bytes, void *hip_stream,
                   pbn_sim **out);
void pbn_sim_free(pbn_sim *sim);

/* Restart the chains from s(0) (transition counter 0) and record the given
 * state sets from now on (nprops <= max_props).  Asynchronous on the stream. */
int pbn_sim_reset(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops);

/* Advance every chain: burn_in transitions unrecorded, then `steps` recorded
 * positions, each taken after `thin` transitions (Sec. 4: the chains are
 * extended in parallel).  Asynchronous on the stream.  Errors: PBN_ELIMIT if
 * the bit-stream capacity or the 2^32 transition limit would be exceeded. */
int run_chains(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): run_chains with the same
 * arguments, results and errors, making no allocation of any kind.  Its launch
 * table (one entry per 64-chain group) lives in a fixed device array of the
 * library (PBN_NOALLOC_MAX_CHAINS / 64 entries, 384 KiB per device, held until
 * the process ends) and is written on the device, so no host-to-device copy is
 * made either.  Asynchronous on the simulation's stream; the simulation's
 * device must be current.  Limits: at most PBN_NOALLOC_MAX_CHAINS chains
 * (PBN_ELIMIT beyond); networks whose lane-per-chain rows exceed LDS (more
 * than 10240 nodes with a predictor of more than 6 parents) are PBN_ELIMIT;
 * the node-split form is not used.  Every call on one device shares that
 * device's array: calls that overlap on one device (other streams or threads)
 * race, so the caller serialises them. */
#define PBN_NOALLOC_MAX_CHAINS (1u << 18)
int run_chains_noalloc(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin);

/* Gelman-Rubin R (Alg. 3) of state set `prop` over the last psi recorded
 * positions of every chain (positions len-psi+1..len).  Synchronises.
 * *rhat = +inf when the within-chain variance W is 0. */
int psrf(pbn_sim *sim, uint32_t prop, uint64_t psi, double *rhat);

/* Window aggregates over positions [lo, hi) of state set prop.  Synchronises. */
int pbn_window_counts(pbn_sim *sim, uint32_t prop, uint64_t lo, uint64_t hi, pbn_counts *out);

/* Batch sums for Skart: for each chain c and batch b < m, the ones in
 * positions [base + b kappa, base + (b+1) kappa); out[c*m + b].  Synchronises. */
int pbn_batch_sums(pbn_sim *sim, uint32_t prop, uint64_t base, uint64_t kappa, uint64_t m,
                   int32_t *out);

/* Current chain states, packed: out[c*W + w] bit b = node 32w+b.  Synchronises. */
int pbn_sim_read_state(pbn_sim *sim, uint32_t *out);
/* Recorded indicators of prop for positions [pos0, pos0+npos): out[c*npos + k]. */
int pbn_sim_read_bits(pbn_sim *sim, uint32_t prop, uint64_t pos0, uint64_t npos, uint8_t *out);
/* Recorded positions per chain and transitions done so far. */
int pbn_sim_position(const pbn_sim *sim, uint64_t *len, uint64_t *transitions);
int pbn_sim_sync(pbn_sim *sim);

/* Full estimate (Alg. 3 then Alg. 4 or Alg. 5) for nprops state sets sharing
 * the chains (Sec. 4.2, multiple properties): the chains restart from s(0);
 * each set runs its own procedure; the chains are extended to the smallest
 * pending requirement.  confidence is s (two-state) or 1 - alpha (Skart); for
 * Skart r is H*.  out[nprops].  Returns PBN_OK even when a set ends with
 * status PBN_ENOTCONV. */
int estimate_prob(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops, double r,
                  double confidence, const pbn_opts *opts, pbn_result *out);

/* ---------------------------------------------------------------- batched */

/* Advance `count` simulations by steps[i] recorded positions each (thin 1,
 * no burn-in) in one launch on `hip_stream`. */
int pbn_batch_run(pbn_sim *const *sims, uint32_t count, const uint64_t *steps, void *hip_stream);

/* Estimate for `count` simulations at once: each simulation i has nprops[i]
 * state sets starting at props[prop_off[i]], precision r[i] and confidence
 * conf[i]; every round extends all pending simulations in one launch and
 * reduces all pending windows in one launch.  out[prop_off[i] + q].
 * Each result equals that of estimate_prob on the simulation alone. */
int pbn_batch_estimate(pbn_sim *const *sims, uint32_t count, const pbn_pattern *props,
                       const uint32_t *nprops, const uint32_t *prop_off, const double *r,
                       const double *conf, const pbn_opts *opts, void *hip_stream,
                       pbn_result *out);

/* ---------------------------------------------------------------- serving */

/* A server owns a caller-provided device arena of arena_bytes and streams of
 * its own (non-blocking; the work queued on hip_stream before the call, e.g.
 * the arena's allocation, comes first).  Requests are
 * admitted when their footprint (pbn_sim_bytes) fits in the free arena; their
 * chains stay on the device across extension rounds; each call to
 * pbn_server_step runs one round for every active request (one batched
 * extension launch, one batched reduction launch) and admits waiting requests
 * into freed space at the round boundary (continuous batching; the requests
 * admitted at one boundary are initialised together). */
int pbn_server_create(void *dev_arena, size_t arena_bytes, void *hip_stream, pbn_server **out);
void pbn_server_free(pbn_server *srv);
/* Queue a request (the network is copied).  *id receives its handle.
 * omega >= 2 chains (at most PBN_MAX_CHAINS), max_len <= PBN_MAX_LEN, and a
 * parallel method (PBN_TWO_STATE or PBN_SKART; opts NULL means two-state).
 * The state sets are checked here: every node below n, at most PBN_MAX_TERMS
 * terms in all.  Errors: PBN_EINVAL (bad arguments, a node out of range or a
 * sequential method), PBN_ELIMIT (beyond the limits), PBN_ENOMEM (footprint
 * larger than the whole arena). */
int pbn_server_submit(pbn_server *srv, const pbn_net *net, uint32_t omega, uint64_t seed,
                      const pbn_pattern *props, uint32_t nprops, double r, double confidence,
                      const pbn_opts *opts, uint64_t max_len, uint64_t *id);
/* How a server schedules its rounds (all times are kernel time in
 * microseconds, as predicted by the library's per-transition model).
 *   slice_us      extension per request and round (0: 1500); a round lasts
 *                 about its longest slice, so short requests see rounds of
 *                 about this length
 *   ahead_us      behind each round, one more slice of this length for the
 *                 requests still more than 3000 us short of their requirement,
 *                 so that the device works while the host takes the round's
 *                 decisions (0: none, the default)
 *   long_lane_us  a request whose pending extension exceeds this moves to a
 *                 lane of its own: a stream restricted to long_quarters
 *                 quarters of every XCD's CUs (0: 3), whose rounds extend its
 *                 requests in slices of long_slice_us (0: 20000) and are
 *                 collected at later steps without holding the other rounds;
 *                 while it has requests, the other rounds keep to the other
 *                 CUs (0: no long lane, the default)
 * Results do not depend on any of these.  The CU share is fixed once the
 * server has stepped; the lane cannot be turned off while it has requests;
 * negative values are PBN_EINVAL.  On the serving workload (Poisson 200/s,
 * n up to 5000) neither ahead slices nor the long lane shortened the tail:
 * both are off by default. */
typedef struct {
    double slice_us, ahead_us, long_lane_us, long_slice_us;
    uint32_t long_quarters;
    uint32_t reserved;
} pbn_server_opts;
int pbn_server_configure(pbn_server *srv, const pbn_server_opts *opts);
/* Requests moved to the long lane so far, and the rounds that lane began. */
int pbn_server_lane_stats(const pbn_server *srv, uint64_t *long_requests, uint64_t *long_rounds);
/* One round.  *active / *waiting / *done receive the counts after the round.
 * A request that cannot be admitted (its device set-up fails) ends at once,
 * and a failed round ends every request that was in it: such a request is
 * done, with the error code as the status of each of its results, and its
 * arena slot is free again; the step returns the first such error (details in
 * pbn_last_error) and the server goes on with the other requests at the next
 * step. */
int pbn_server_step(pbn_server *srv, uint32_t *active, uint32_t *waiting, uint32_t *done);
/* Results of a finished request: returns PBN_OK and fills out[nprops] once
 * done (each status PBN_OK, PBN_ENOTCONV, or the error that ended the
 * request); returns PBN_EINVAL for unknown ids, and sets *ready = 0 while the
 * request is still queued or running. */
int pbn_server_poll(pbn_server *srv, uint64_t id, int *ready, pbn_result *out);
/* Bytes of the arena currently in use and the peak so far. */
int pbn_server_memory(const pbn_server *srv, size_t *in_use, size_t *peak);

/* ---------------------------------------------------------------- profiling */

/* Per-launch timing of the trajectory kernel.  While enabled, every step
 * launch is bracketed by HIP events recorded on the stream it runs on; the
 * read call waits for the recorded events and returns the totals since the
 * last reset.  alg_ops counts the algorithmic 32-bit integer operations of the
 * launched chain-steps (Philox4x32-10 evaluations at 100 operations each, one
 * comparison per uniform draw, and for function updates the selection
 * comparisons, two operations per parent bit gathered and one per truth-table
 * lookup), taken as expectations over the network's structure and p. */
typedef struct {
    uint64_t launches;
    double kernel_ms;            /* sum of event-timed launch durations      */
    double chain_steps;          /* transitions x chains                     */
    double node_updates;         /* chain_steps x n                          */
    double alg_ops;              /* see above                                */
    double philox_evals;         /* expected Philox4x32-10 evaluations       */
    uint64_t split_launches;     /* launches of the node-split form (k_step_split) among them */
    uint64_t split_fallbacks;    /* node-split groups that gave up waiting and were re-run in
                                    the one-block form (counted whether or not timing is on) */
} pbn_profile;

int pbn_profile_enable(int on);
/* The kernel and node-split choices of one simulation's launches, instead of
 * the process-wide ones below (so that threads with their own simulations
 * need not share them): mode and waves as in pbn_set_kernel, parts as in
 * pbn_set_split; mode -1 or parts -1 return to the process-wide setting.
 * Results do not depend on the choice. */
int pbn_sim_set_kernel(pbn_sim *sim, int mode, uint32_t waves);
int pbn_sim_set_split(pbn_sim *sim, int parts);

/* Trajectory-kernel selection for subsequent launches: mode 0 = automatic
 * (bit-sliced kernel when every predictor has at most 6 parents and the
 * bit-sliced state fits in LDS, else lane-per-chain), 1 = lane-per-chain only,
 * 2 = bit-sliced where possible; waves = waves sharing one 64-chain block in
 * the bit-sliced kernel (0 = chosen from n and from whether the launch has the
 * CUs to itself, else 1..16; multiples of 4 keep a CU's four SIMDs even).
 * Results do not depend on the choice.  Returns PBN_EINVAL for waves > 16. */
int pbn_set_kernel(int mode, uint32_t waves);
/* Node-split form of the bit-sliced trajectory step (a latency-bound 64-chain
 * group spread over several CUs: each block owns a contiguous range of nodes,
 * and the blocks of a group exchange their nodes' next-state words through
 * device memory once per transition, behind a bounded arrival counter).  It
 * is used only by calls that own the device while they run: run_chains,
 * pbn_batch_run, estimate_prob, a single-network pbn_batch_estimate and the
 * server rounds.  parts: 0 = automatic (while a launch has fewer 64-chain
 * groups than the device has CUs, the spare CUs go one at a time to the group
 * with the most remaining work per part, each group taking at most 16 parts
 * of at least 8 16-node blocks), 1 = never, P >= 2 = P parts for every
 * bit-sliced group whose network has at least P 16-node blocks (fewer
 * otherwise) while the launch stays within one block per CU.  Results do not
 * depend on the choice.  A group whose blocks are not all resident together
 * (another process or stream holding CUs) gives up after about a second,
 * leaving its chains as the launch found them; the call then re-runs that
 * group in the one-block form (and repeats the round's reductions), so it
 * still succeeds with the same results, about a second later. */
int pbn_set_split(uint32_t parts);
/* Polls of its group's arrival counter that a node-split block makes before it
 * gives up (0 = the default, 2^20, about a second).  For tests of the failure
 * path: with a tiny value a group whose parts do not arrive together ends
 * early and is re-run in the one-block form (pbn_profile.split_fallbacks). */
int pbn_set_split_polls(uint32_t polls);
int pbn_profile_read(pbn_profile *out);
int pbn_profile_reset(void);

/* ---------------------------------------------------------------- autotuning */

/* One row of the kernel-shape table: for networks of about n nodes, the waves
 * per 64-chain block of the bit-sliced kernel that gave the highest node-update
 * rate with the chip full of blocks (throughput) and the shortest transition
 * of one block alone (latency), with the measured figures. */
typedef struct {
    uint32_t n;
    uint32_t waves_throughput;
    uint32_t waves_latency;
    uint32_t reserved;
    double node_updates_per_s;   /* at waves_throughput, 131072 chains        */
    double transition_us;        /* at waves_latency, 64 chains               */
} pbn_tune_row;

/* Measures the bit-sliced kernel's shapes (1, 2, 4, 5, 8, 12, 16 waves per
 * block) on synthetic networks of 24..3072 nodes drawn like the paper's random
 * networks (Sec. 5.1: 1-3 predictors per node, 1-5 parents, p = 1e-3), with
 * short event-timed launches on hip_stream (about a second of GPU time), one
 * network alone on the chip, and uses the result for every later latency and
 * one-network launch in this process instead of the built-in rule (the batched
 * lanes, whose launches share the CUs, keep their built-in shapes).  Results
 * of the method do not depend on the shapes.  Fills
 * rows[0 .. min(cap, *count)) and sets *count to the number of rows (8).
 * The library allocates and frees its own device memory for the runs.
 * Errors: PBN_ENOMEM, PBN_EDEVICE (message in pbn_last_error). */
int pbn_autotune(void *hip_stream, pbn_tune_row *rows, uint32_t cap, uint32_t *count);
/* Back to the built-in shape rule. */
int pbn_autotune_reset(void);

/* ---------------------------------------------------------------- Skart statistics */

/* Limit on the observations (batch size x batch count) that one Skart CI or
 * randomness test takes: every moment of the batch means is then computed
 * exactly in 128-bit integers.  The Skart methods end as not converged beyond
 * it. */
#define PBN_SKART_MAX_OBS (1ull << 40)

/* Statistics of one set of Skart batch sums (Sec. 4.3, the parallel Skart
 * procedure, and Sec. 3.2): the grand mean, the skewness- and lag-1
 * autoregression-adjusted confidence interval and its half-width
 * H = max(mu - ci_lo, ci_hi - mu), and the von Neumann randomness test over
 * within-chain adjacent batch means at level 0.2 (statistic vn_C against the
 * limit vn_limit; both NaN, and the test passed, with one batch per chain or
 * all batch means equal). */
typedef struct {
    double mu, ci_lo, ci_hi, H;
    double vn_C, vn_limit;
    int vn_passes;
    int reserved;
} pbn_skart_stats;

/* The statistics estimate_prob's Skart method takes on its batches, for batch
 * sums computed elsewhere (e.g. by pbn_batch_sums): bsum[c*m + j] is the count
 * of ones in batch j (of kappa positions) of chain c, omega chains, m batches
 * each.  Every sum over the batches is exact; floating point enters only in
 * the final ratios, so equal inputs give bit-equal outputs.  Host only (no
 * device call).  Errors: PBN_EINVAL (null pointers, omega, m or kappa zero,
 * confidence not in (0,1), fewer than 101 batches in all, a sum outside
 * [0, kappa]), PBN_ELIMIT (kappa omega m > PBN_SKART_MAX_OBS). */
int pbn_skart_batch_stats(const int32_t *bsum, uint32_t omega, uint64_t m, uint64_t kappa,
                          double confidence, pbn_skart_stats *out);

/* ---------------------------------------------------------------- misc */

/* Phi^{-1}(p) (AS 241) and the Student-t quantile used by the statistics. */
double pbn_normal_quantile(double p);
double pbn_t_quantile(double p, double nu);
const char *pbn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
