// Host control of the method: one state machine per state set (property),
// and the round loop that serves many simulations with one extension launch
// and one reduction launch per round.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pbn_internal.h"

struct pbn_net {
    pbn::Net net;
};

namespace pbn {

// Device + pinned host scratch for one round's tables and results.
struct Workspace {
    StepItem *d_items = nullptr, *h_items = nullptr;
    Query *d_queries = nullptr, *h_queries = nullptr;
    WindowResult *d_win = nullptr, *h_win = nullptr;
    int32_t *d_bsum = nullptr, *h_bsum = nullptr;
    DevSim *d_stage = nullptr, *h_stage = nullptr;
    DevSim **d_dst = nullptr, **h_dst = nullptr;
    size_t cap_items = 0, cap_q = 0, cap_bsum = 0, cap_stage = 0;
    // the last copies out of h_items / h_queries: the host waits for them
    // before rewriting those pinned tables
    hipEvent_t ev_items = nullptr, ev_queries = nullptr;
    bool items_in_flight = false, queries_in_flight = false;
    int ensure(size_t items, size_t queries, size_t bsum, std::string &err);
    // wait for the previous copy out of a pinned table, record the next one
    int before_write(hipEvent_t &ev, bool &in_flight, std::string &err);
    int after_copy(hipEvent_t &ev, bool &in_flight, hipStream_t stream, std::string &err);
    int ensure_stage(size_t count, std::string &err);
    // node-split form: group descriptors (pinned staging, device), exchange
    // area (the last launch's first xch_used words), and a status word per
    // group (the last launch's copied to h_stat)
    SplitGroup *d_grp = nullptr, *h_grp = nullptr;
    uint64_t *d_xch = nullptr;
    uint32_t *d_stat = nullptr, *h_stat = nullptr;
    size_t cap_grp = 0, cap_xch = 0, xch_used = 0;
    // the last launch's node-split groups as whole 64-chain items (one-block
    // shapes) and its stream, for the re-run of a group that gave up; the
    // reduction that followed it in the same round (queries, batch sums)
    std::vector<StepItem> split_items;
    hipStream_t split_stream = nullptr;
    size_t redo_queries = 0, redo_bsum = 0;
    // lane-per-chain state rows of networks too large for LDS
    uint32_t *d_rows = nullptr;
    size_t cap_rows = 0;
    int ensure_rows(size_t words, std::string &err);
    size_t split_used = 0;        // node-split groups in the last launch
    int ensure_split(size_t groups, size_t xch_words, std::string &err);
    // After the stream reached the last launch: every node-split group that
    // gave up waiting (its state unchanged) is re-run in the one-block form on
    // the same stream, then the round's reduction is repeated, and the stream
    // is synchronised again.
    int check_split(std::string &err);
    void release();
    ~Workspace() { release(); }
};

// What a state machine needs next: a window or batch query on its property,
// served once the chains hold need_len positions.
struct Request {
    uint32_t kind;              // kQueryWindow / kQueryBatch
    uint64_t lo, hi, kappa, m;  // window [lo, hi) or m batches of kappa from lo
    uint64_t need_len;
};

struct MachineParams {
    int method;
    uint32_t omega;
    uint64_t psi0, cap;
    double psrf_max, eps, r, conf;
};

class Machine {
public:
    Machine(const MachineParams &p, uint32_t prop);
    bool done() const { return done_; }
    const Request &request() const { return req_; }
    uint32_t prop() const { return prop_; }
    void feed_window(const WindowResult &w, uint64_t chain_len);
    void feed_batch(const int32_t *bsum, uint64_t chain_len);
    const pbn_result &result() const { return res_; }

private:
    enum State {
        kGR, kTwoState, kSkartSkew, kSkartRandomness, kSkartCI,
        kSeqTwoState, kSeqFinal, kSeqSkartSkew, kSeqSkartRandomness
    };
    // Alg. 2: initial trajectory, skewness tail, largest spacer (in batches)
    static constexpr uint64_t kSeqSkartEta = 1280, kSeqSkartTail = 1024, kSeqSkartMaxSpacer = 10;
    void ask_window(uint64_t lo, uint64_t hi);
    bool gr_window_fits(uint64_t psi) const;
    void ask_batch();
    bool batches_fit() const;
    void not_converged(uint64_t chain_len);
    void finish_two_state(int64_t T1);
    void skart_ci(const int32_t *bsum, uint64_t chain_len);

    MachineParams P_;
    uint32_t prop_;
    State st_ = kGR;
    bool done_ = false;
    Request req_{};
    pbn_result res_{};
    double z_ = 0.0;
    uint64_t psi_ = 0, psi_gr_ = 0, n_ = 0, N_ = 0;
    double a_ = 0.0, b_ = 0.0;
    // Skart-P and Alg. 2: first batch position, batch size, batch count
    uint64_t base_ = 0, kappa_ = 0, p_ = 0;
    int tries_ = 0;
    // Alg. 1 (one chain): burn-in M, trajectory length l
    uint64_t M_ = 0, l_ = 0;
    // Alg. 2 (one chain): spacer batches skipped before the CI batches
    uint64_t d_ = 0;
    void seq_next(uint64_t chain_len);
};

}  // namespace pbn

struct pbn_sim {
    ~pbn_sim();
    pbn::Net net;
    uint32_t omega = 0, max_props = 0, nprops = 0;
    uint64_t seed = 0, max_len = 0, words_cap = 0;
    uint8_t *dbuf = nullptr;
    size_t dbytes = 0;
    hipStream_t stream = nullptr;
    int device = -1;              // the device current when the simulation was created
    // kernel and node-split choice of this simulation's launches (-1: the
    // process-wide setting), and the transitions per recorded position of its
    // estimates
    int kmode = -1, split = -1;
    uint32_t kwaves = 0, thin = 1;
    pbn::DevSim desc{};
    pbn::DevSim *d_desc = nullptr;
    uint64_t len = 0, t_done = 0;
    pbn::Workspace ws;
    // node-split tables uploaded so far, by part count
    struct SplitTab {
        uint32_t P = 0, groups = 0, n_own = 0, m_own = 0;
        uint32_t *d_tab = nullptr;
    };
    std::vector<SplitTab> split_tabs;
};

namespace pbn {

size_t sim_bytes(const Net &net, uint32_t omega, uint32_t max_props, uint64_t max_len);
// Lay out a simulation in dev_buf and upload the network; with reset, also
// write its descriptor and initial states (else the caller resets it, e.g. in
// a batch with sims_reset_batch).
int sim_setup(pbn_sim *sim, const Net &net, uint32_t omega, uint64_t seed, uint32_t max_props,
              uint64_t max_len, void *dev_buf, size_t dev_bytes, hipStream_t stream, std::string &err,
              bool reset = true);
int sim_prepare_reset(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops, std::string &err);
int sim_reset(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops, hipStream_t stream, std::string &err);
// Reset many simulations with one descriptor upload and one setup launch on stream.
int sims_reset_batch(pbn_sim *const *sims, uint32_t count, const pbn_pattern *props, const uint32_t *nprops,
                     const uint32_t *prop_off, Workspace &ws, hipStream_t stream, std::string &err);
// Kernel shape (waves per 64-chain block) of a launch:
//   kShapeShared  throughput for launches of many networks of mixed sizes, or
//                 that share the CUs with other concurrent launches (batched
//                 class lanes, server rounds): few block shapes, each leaving
//                 room for the others;
//   kShapeLatency the shortest transition (the chip holds every block at once);
//   kShapeAlone   throughput for one network's launch with the CUs to itself
//                 (plain runs): more waves per block for larger networks.
// A bool converts to the first two (false: shared, true: latency).
enum Shape : int { kShapeShared = 0, kShapeLatency = 1, kShapeAlone = 2 };
// Append the step items that extend sim by `steps` recorded positions, in
// the given kernel shape.
void sim_extend_items(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin,
                      std::vector<StepItem> &items, int shape);
// Latency shapes are picked while every 64-chain block of the unfinished work,
// in its latency shape, fits on the chip at once (waves of 256 CUs at six
// waves per SIMD).
constexpr uint64_t kLatencyWaves = 256 * 24;
// Waves that the blocks of sim need in latency shapes.
uint64_t latency_waves(const pbn_sim *sim);
// Kernel time (us) of extending sim by `positions` recorded positions in its
// latency shape, its 64-chain groups in `parts` node-split parts each (a
// model fitted to single-group timings).
double extension_us(const pbn_sim *sim, uint64_t positions, uint32_t parts);
// Kernel time per extension slice of a time-sliced round (microseconds).
constexpr double kTickUs = 5000.0;
// Server rounds: shorter slices, since a request's result waits for the end of
// the round it finishes in (continuous batching admits and answers at round
// boundaries); measured on the serving stream, 1.5 ms balanced the median
// against the latency of the largest requests.
constexpr double kServeTickUs = 1500.0;
// The express lane of a batch takes its latency shape once its unfinished work
// is at most this many waves (a few CUs' worth beside the bulk).
constexpr uint64_t kExpressLatencyWaves = 512;
// XCDs of the chip: block i of a launch runs on XCD i mod kXcds.
constexpr size_t kXcds = 8;

// A simulation together with the machines of its state sets.
struct SimRun {
    pbn_sim *sim = nullptr;
    std::vector<Machine> machines;
    bool finished() const;
};

MachineParams make_params(const pbn_sim *sim, const pbn_opts *opts, double r, double conf);

// Streams for concurrent launch groups (default priority, non-blocking),
// restricted to the CUs of cu_mask when it is set (hipExtStreamCreateWithCUMask
// words); one caller at a time.
struct StreamPool {
    static constexpr int kN = 4;
    hipStream_t s[kN] = {};
    hipEvent_t fork = nullptr, join[kN] = {};
    bool ready = false;
    std::mutex mu;
    std::vector<uint32_t> cu_mask;
    int init(std::string &err);
    void release();
    ~StreamPool() { release(); }
};

// How a round's step launches run: fork spreads its kernel groups over a
// stream pool (pool, or the library's shared one); split allows node-split
// parts, which needs the launch to own `cus` CUs while it runs (nothing else
// on them).
struct LaunchCfg {
    bool fork = true, split = true;
    // the launch shares the CUs with other lanes' launches: throughput
    // shapes are kShapeShared even for one network
    bool shared = false;
    uint32_t cus = 256;
    StreamPool *pool = nullptr;
};

// One round over all runs: extension launch for the runs that wait for
// positions, reduction launch for every ready request, one synchronisation.
// round_begin enqueues a round and records ctx.done; round_end feeds the
// results to the machines once ctx.done has completed.
struct RoundCtx {
    struct Owner { SimRun *run; size_t mi; uint64_t off; };
    std::vector<Owner> owners;
    std::vector<uint32_t> kinds;
    hipEvent_t done = nullptr;
    bool pending = false;
};
// tick_us > 0 limits each extension to a slice of about that much kernel time;
// latency 1/0 forces the kernel shapes, -1 decides from the runs' chain groups.
int round_begin(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, RoundCtx &ctx, std::string &err,
                const LaunchCfg &cfg = LaunchCfg{}, double tick_us = 0.0, int latency = -1);
void round_end(Workspace &ws, RoundCtx &ctx);
// Queue, behind a round, one more slice of about tick_us of kernel time for
// every run whose pending requirement is still more than min_left_us of
// kernel time away (its next round would extend it anyway): the device works
// through the host's decisions for the round.  Only while those runs' groups
// fit on the chip in latency shapes.  *launched tells whether anything was
// queued (ws.check_split then applies once the stream has passed it).
int ahead_begin(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, const LaunchCfg &cfg,
                double tick_us, double min_left_us, bool *launched, std::string &err);
// One synchronous round; tick_us > 0 time-slices its extensions.
int run_round(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, std::string &err,
              double tick_us = 0.0, const LaunchCfg &cfg = LaunchCfg{});
// Many simulations: lanes by step-kernel class, each with its own stream and
// asynchronous, time-sliced round loop (run_to_completion for one simulation).
int run_lanes(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, std::string &err);
// Rounds until every run is finished.
int run_to_completion(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, std::string &err);

// Profiling of step launches (HIP events on the launch stream).
struct ProfileMark {
    hipEvent_t start = nullptr, stop = nullptr;
    double chain_steps = 0, node_updates = 0, ops = 0, philox = 0;
    bool split = false;
};
bool profiling();
void profile_begin(ProfileMark &m, hipStream_t stream);
void profile_end(ProfileMark &m, hipStream_t stream);
int profile_collect(pbn_profile *out, std::string &err);
void profile_set(bool on);
void profile_clear();

// Kernel selection for a step item of sim (see pbn_driver.cpp): the
// simulation's own setting, else the process-wide one.
void choose_kernel(const pbn_sim *sim, StepItem &it, int shape);
// Autotuner (pbn_tune.cpp): measured shapes per size bucket, if measured.
bool tuned_waves(uint32_t n, int shape, uint32_t *G);
int autotune(hipStream_t stream, pbn_tune_row *rows, uint32_t cap, uint32_t *count, std::string &err);
void autotune_reset();
uint32_t waves_for(uint32_t n, int shape);
void set_kernel_mode(int mode, uint32_t waves);
// Node-split form: 0 = automatic, 1 = never, P >= 2 = P parts wherever the
// network has P node blocks (launches that allow it).
void set_split_mode(uint32_t parts);
// Polls a node-split part makes before it gives up (0 = the default).
void set_split_spins(uint32_t polls);
// Node-split groups re-run in the one-block form after a give-up (process-wide).
uint64_t split_fallbacks();

// run_chains without allocation (pbn_noalloc.hip): the launch table lives in
// a fixed device array; at most PBN_NOALLOC_MAX_CHAINS chains, no node-split
// form, no device scratch rows.
int run_chains_noalloc_impl(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin, std::string &err);

// Launch step items for several sims (sorted by cost) on stream.  allow_split:
// the launch owns the device (nothing else runs beside it that could hold the
// CUs its node-split groups wait for), so latency-bound 64-chain groups may
// be spread over several CUs; ws.check_split then tells whether they finished.
int launch_items(std::vector<StepItem> &items, Workspace &ws, hipStream_t stream, std::string &err,
                 bool allow_fork = true, bool allow_split = false, uint32_t cus = 256, StreamPool *pool = nullptr);

}  // namespace pbn
