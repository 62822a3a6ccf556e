// C ABI of libpbnssa: networks, simulations, the plain and batched estimate
// entry points and the serving loop.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "pbn_driver.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int sync(hipStream_t s)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(PBN_EDEVICE, std::string("sync: ") + hipGetErrorString(e));
    return PBN_OK;
}

// Window aggregates of one sim, synchronously, through its own workspace.
int window_query(pbn_sim *sim, uint32_t prop, uint64_t lo, uint64_t hi, pbn::WindowResult *out)
{
    std::string err;
    if (prop >= sim->nprops) return fail(PBN_EINVAL, "state set index out of range");
    if (!(lo < hi) || hi > sim->len) return fail(PBN_EINVAL, "window outside the recorded positions");
    int rc = sim->ws.ensure(0, 1, 0, err);
    if (rc) return fail(rc, err);
    pbn::Query q{};
    q.sim = sim->d_desc;
    q.prop = prop;
    q.kind = pbn::kQueryWindow;
    q.lo = lo;
    q.hi = hi;
    *sim->ws.h_queries = q;
    if (hipMemcpyAsync(sim->ws.d_queries, sim->ws.h_queries, sizeof q, hipMemcpyHostToDevice, sim->stream) != hipSuccess)
        return fail(PBN_EDEVICE, "query upload");
    if ((rc = pbn::launch_reduce(sim->ws.d_queries, 1, sim->ws.d_win, sim->ws.d_bsum, sim->stream, err)))
        return fail(rc, err);
    if (hipMemcpyAsync(sim->ws.h_win, sim->ws.d_win, sizeof(pbn::WindowResult), hipMemcpyDeviceToHost,
                       sim->stream) != hipSuccess)
        return fail(PBN_EDEVICE, "result download");
    if ((rc = sync(sim->stream))) return rc;
    *out = *sim->ws.h_win;
    return PBN_OK;
}

// base + count * size <= limit, decided without wrapping around 2^64.
bool fits(uint64_t base, uint64_t count, uint64_t size, uint64_t limit)
{
    if (base > limit) return false;
    return size == 0 || count <= (limit - base) / size;
}

// Transition indices of a chain stay below 2^32 (the counter of the random stream).
constexpr uint64_t kMaxTransition = (1ull << 32) - 1;

// Recorded positions a simulation can still hold.
uint64_t position_cap(const pbn_sim *sim) { return sim->words_cap * 32 - 32; }

// Each simulation at most once in a batched call (two runs on one simulation
// would extend the same chains).
bool distinct(pbn_sim *const *sims, uint32_t count)
{
    std::vector<const pbn_sim *> v(sims, sims + count);
    std::sort(v.begin(), v.end());
    return std::adjacent_find(v.begin(), v.end()) == v.end();
}

bool valid_patterns(const pbn_pattern *props, uint32_t nprops)
{
    if (nprops && !props) return false;
    for (uint32_t q = 0; q < nprops; ++q) {
        if (props[q].nterms && (!props[q].node || !props[q].val)) return false;
        for (uint32_t m = 0; m < props[q].nterms; ++m)
            if (props[q].val[m] > 1) return false;
    }
    return true;
}

}  // namespace

extern "C" {

const char *pbn_last_error(void) { return g_last_error.c_str(); }

int pbn_load(const char *text, size_t len, pbn_net **out)
{
    if (!text || !out) return fail(PBN_EINVAL, "null argument");
    std::unique_ptr<pbn_net> net(new pbn_net());
    std::string err;
    int rc = pbn::parse_and_compile(text, len, net->net, err);
    if (rc) return fail(rc, err);
    *out = net.release();
    return PBN_OK;
}

int pbn_load_file(const char *path, pbn_net **out)
{
    if (!path || !out) return fail(PBN_EINVAL, "null argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(PBN_EINVAL, std::string("cannot open ") + path);
    std::string text;
    char buf[1 << 16];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    const bool bad = std::ferror(f) != 0;
    std::fclose(f);
    if (bad) return fail(PBN_EINVAL, std::string("cannot read ") + path);
    return pbn_load(text.data(), text.size(), out);
}

void pbn_free(pbn_net *net) { delete net; }

int pbn_net_get_info(const pbn_net *net, pbn_net_info *out)
{
    if (!net || !out) return fail(PBN_EINVAL, "null argument");
    const pbn::Net &n = net->net;
    out->n = n.n;
    out->W = n.W;
    out->nfun = n.F;
    out->p_thr = n.p_thr;
    out->max_k = n.max_k;
    out->max_l = n.max_l;
    out->blob_bytes = n.blob_bytes;
    out->density = n.density;
    return PBN_OK;
}

int pbn_net_thresholds(const pbn_net *net, uint32_t node, uint32_t *out, uint32_t cap)
{
    if (!net || node >= net->net.n) return -1;
    const uint32_t a = net->net.nd_first[node], b = net->net.nd_first[node + 1];
    for (uint32_t j = a; j < b && j - a < cap; ++j) out[j - a] = net->net.fn_thr[j];
    return (int)(b - a);
}

size_t pbn_sim_bytes(const pbn_net *net, uint32_t omega, uint32_t max_props, uint64_t max_len)
{
    if (!net) return 0;
    return pbn::sim_bytes(net->net, omega, max_props, max_len);
}

int pbn_sim_create(const pbn_net *net, uint32_t omega, uint64_t seed, uint32_t max_props, uint64_t max_len,
                   void *dev_buf, size_t dev_bytes, void *hip_stream, pbn_sim **out)
{
    if (!net || !out) return fail(PBN_EINVAL, "null argument");
    std::unique_ptr<pbn_sim> sim(new pbn_sim());
    std::string err;
    int rc = pbn::sim_setup(sim.get(), net->net, omega, seed, max_props, max_len, dev_buf, dev_bytes,
                            (hipStream_t)hip_stream, err);
    if (rc) return fail(rc, err);
    *out = sim.release();
    return PBN_OK;
}

void pbn_sim_free(pbn_sim *sim)
{
    if (!sim) return;
    (void)hipStreamSynchronize(sim->stream);
    delete sim;
}

int pbn_sim_reset(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops)
{
    if (!sim || !valid_patterns(props, nprops)) return fail(PBN_EINVAL, "bad argument");
    std::string err;
    int rc = pbn::sim_reset(sim, props, nprops, sim->stream, err);
    return rc ? fail(rc, err) : PBN_OK;
}

int run_chains(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin)
{
    if (!sim || thin < 1) return fail(PBN_EINVAL, "bad argument");
    if (!fits(sim->len, steps, 1, position_cap(sim))) return fail(PBN_ELIMIT, "bit-stream capacity exceeded");
    if (!fits(sim->t_done, burn_in, 1, kMaxTransition) || !fits(sim->t_done + burn_in, steps, thin, kMaxTransition))
        return fail(PBN_ELIMIT, "transition index limit (2^32)");
    std::vector<pbn::StepItem> items;
    pbn::sim_extend_items(sim, burn_in, steps, thin, items,
                          pbn::latency_waves(sim) <= pbn::kLatencyWaves ? pbn::kShapeLatency : pbn::kShapeAlone);
    std::string err;
    int rc = pbn::launch_items(items, sim->ws, sim->stream, err, true, true);
    if (!rc && sim->ws.split_used) {
        // a node-split launch is checked before the call returns
        if (hipStreamSynchronize(sim->stream) != hipSuccess) return fail(PBN_EDEVICE, "stream synchronize");
        rc = sim->ws.check_split(err);
    }
    return rc ? fail(rc, err) : PBN_OK;
}

int run_chains_noalloc(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin)
{
    if (!sim || thin < 1) return fail(PBN_EINVAL, "bad argument");
    if (!fits(sim->len, steps, 1, position_cap(sim))) return fail(PBN_ELIMIT, "bit-stream capacity exceeded");
    if (!fits(sim->t_done, burn_in, 1, kMaxTransition) || !fits(sim->t_done + burn_in, steps, thin, kMaxTransition))
        return fail(PBN_ELIMIT, "transition index limit (2^32)");
    std::string err;
    const int rc = pbn::run_chains_noalloc_impl(sim, burn_in, steps, thin, err);
    return rc ? fail(rc, err) : PBN_OK;
}

int psrf(pbn_sim *sim, uint32_t prop, uint64_t psi, double *rhat)
{
    if (!sim || !rhat || psi < 2 || psi > sim->len || sim->omega < 2) return fail(PBN_EINVAL, "bad argument");
    pbn::WindowResult w;
    int rc = window_query(sim, prop, sim->len - psi, sim->len, &w);
    if (rc) return rc;
    bool defined;
    *rhat = pbn::rhat_from_sums(w.T1, w.T2, sim->omega, psi, &defined);
    return PBN_OK;
}

int pbn_window_counts(pbn_sim *sim, uint32_t prop, uint64_t lo, uint64_t hi, pbn_counts *out)
{
    if (!sim || !out) return fail(PBN_EINVAL, "null argument");
    pbn::WindowResult w;
    int rc = window_query(sim, prop, lo, hi, &w);
    if (rc) return rc;
    out->T1 = w.T1; out->T2 = w.T2; out->n00 = w.n00; out->n01 = w.n01; out->n10 = w.n10; out->n11 = w.n11;
    return PBN_OK;
}

int pbn_batch_sums(pbn_sim *sim, uint32_t prop, uint64_t base, uint64_t kappa, uint64_t m, int32_t *out)
{
    if (!sim || !out || kappa < 1 || m < 1) return fail(PBN_EINVAL, "bad argument");
    if (prop >= sim->nprops || !fits(base, kappa, m, sim->len))
        return fail(PBN_EINVAL, "batches outside the recorded positions");
    if (kappa > INT32_MAX) return fail(PBN_EINVAL, "batch sums are 32-bit: kappa < 2^31");
    std::string err;
    const uint64_t total = (uint64_t)sim->omega * m;
    int rc = sim->ws.ensure(0, 1, total, err);
    if (rc) return fail(rc, err);
    pbn::Query q{};
    q.sim = sim->d_desc;
    q.prop = prop;
    q.kind = pbn::kQueryBatch;
    q.lo = base;
    q.hi = base + kappa * m;
    q.kappa = kappa;
    q.m = m;
    *sim->ws.h_queries = q;
    if (hipMemcpyAsync(sim->ws.d_queries, sim->ws.h_queries, sizeof q, hipMemcpyHostToDevice, sim->stream) != hipSuccess)
        return fail(PBN_EDEVICE, "query upload");
    if ((rc = pbn::launch_reduce(sim->ws.d_queries, 1, sim->ws.d_win, sim->ws.d_bsum, sim->stream, err)))
        return fail(rc, err);
    if (hipMemcpyAsync(sim->ws.h_bsum, sim->ws.d_bsum, total * 4, hipMemcpyDeviceToHost, sim->stream) != hipSuccess)
        return fail(PBN_EDEVICE, "download");
    if ((rc = sync(sim->stream))) return rc;
    std::memcpy(out, sim->ws.h_bsum, total * 4);
    return PBN_OK;
}

int pbn_sim_read_state(pbn_sim *sim, uint32_t *out)
{
    if (!sim || !out) return fail(PBN_EINVAL, "null argument");
    const size_t words = (size_t)sim->net.W * sim->omega;
    std::vector<uint32_t> tmp(words);
    if (hipMemcpyAsync(tmp.data(), sim->desc.state, words * 4, hipMemcpyDeviceToHost, sim->stream) != hipSuccess)
        return fail(PBN_EDEVICE, "download");
    int rc = sync(sim->stream);
    if (rc) return rc;
    for (uint32_t c = 0; c < sim->omega; ++c)
        for (uint32_t w = 0; w < sim->net.W; ++w) out[(size_t)c * sim->net.W + w] = tmp[(size_t)w * sim->omega + c];
    return PBN_OK;
}

int pbn_sim_read_bits(pbn_sim *sim, uint32_t prop, uint64_t pos0, uint64_t npos, uint8_t *out)
{
    if (!sim || !out || prop >= sim->nprops || !fits(pos0, npos, 1, sim->len)) return fail(PBN_EINVAL, "bad argument");
    if (npos == 0) return PBN_OK;
    const uint64_t w0 = pos0 / 32, w1 = (pos0 + npos + 31) / 32;
    const size_t words = (size_t)(w1 - w0) * sim->omega;
    std::vector<uint32_t> tmp(words);
    const uint32_t *src = sim->desc.bits + ((size_t)prop * sim->words_cap + w0) * sim->omega;
    if (hipMemcpyAsync(tmp.data(), src, words * 4, hipMemcpyDeviceToHost, sim->stream) != hipSuccess)
        return fail(PBN_EDEVICE, "download");
    int rc = sync(sim->stream);
    if (rc) return rc;
    for (uint32_t c = 0; c < sim->omega; ++c)
        for (uint64_t k = 0; k < npos; ++k) {
            const uint64_t pos = pos0 + k;
            out[(size_t)c * npos + k] = (tmp[(size_t)(pos / 32 - w0) * sim->omega + c] >> (pos % 32)) & 1u;
        }
    return PBN_OK;
}

int pbn_sim_position(const pbn_sim *sim, uint64_t *len, uint64_t *transitions)
{
    if (!sim) return fail(PBN_EINVAL, "null argument");
    if (len) *len = sim->len;
    if (transitions) *transitions = sim->t_done;
    return PBN_OK;
}

int pbn_sim_sync(pbn_sim *sim)
{
    if (!sim) return fail(PBN_EINVAL, "null argument");
    return sync(sim->stream);
}

int estimate_prob(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops, double r, double confidence,
                  const pbn_opts *opts, pbn_result *out)
{
    uint32_t off = 0;
    return pbn_batch_estimate(&sim, 1, props, &nprops, &off, &r, &confidence, opts, sim ? sim->stream : nullptr,
                              out);
}

int pbn_batch_run(pbn_sim *const *sims, uint32_t count, const uint64_t *steps, void *hip_stream)
{
    if (!sims || !steps) return fail(PBN_EINVAL, "null argument");
    if (!distinct(sims, count)) return fail(PBN_EINVAL, "a simulation appears twice");
    std::vector<pbn::StepItem> items;
    for (uint32_t i = 0; i < count; ++i) {
        pbn_sim *s = sims[i];
        if (!s) return fail(PBN_EINVAL, "null simulation");
        if (!fits(s->len, steps[i], 1, position_cap(s))) return fail(PBN_ELIMIT, "bit-stream capacity exceeded");
        if (!fits(s->t_done, steps[i], 1, kMaxTransition)) return fail(PBN_ELIMIT, "transition index limit (2^32)");
    }
    uint64_t waves = 0;
    for (uint32_t i = 0; i < count; ++i)
        if (steps[i]) waves += pbn::latency_waves(sims[i]);
    const bool latency = waves <= pbn::kLatencyWaves;
    uint32_t extended = 0;
    for (uint32_t i = 0; i < count; ++i) extended += steps[i] != 0;
    const int shape = latency ? pbn::kShapeLatency : extended > 1 ? pbn::kShapeShared : pbn::kShapeAlone;
    for (uint32_t i = 0; i < count; ++i)
        if (steps[i]) pbn::sim_extend_items(sims[i], 0, steps[i], 1, items, shape);
    static thread_local pbn::Workspace ws;
    std::string err;
    int rc = pbn::launch_items(items, ws, (hipStream_t)hip_stream, err, true, true);
    if (rc) return fail(rc, err);
    if ((rc = sync((hipStream_t)hip_stream))) return rc;
    if ((rc = ws.check_split(err))) return fail(rc, err);
    return PBN_OK;
}

int pbn_batch_estimate(pbn_sim *const *sims, uint32_t count, const pbn_pattern *props, const uint32_t *nprops,
                       const uint32_t *prop_off, const double *r, const double *conf, const pbn_opts *opts,
                       void *hip_stream, pbn_result *out)
{
    if (!sims || !nprops || !prop_off || !r || !conf || !out) return fail(PBN_EINVAL, "null argument");
    if (!distinct(sims, count)) return fail(PBN_EINVAL, "a simulation appears twice");
    std::vector<pbn::SimRun> runs(count);
    std::string err;
    hipStream_t stream = (hipStream_t)hip_stream;
    for (uint32_t i = 0; i < count; ++i) {
        pbn_sim *s = sims[i];
        if (!s) return fail(PBN_EINVAL, "null simulation");
        if (opts && (opts->method < PBN_TWO_STATE || opts->method > PBN_SEQ_SKART))
            return fail(PBN_EINVAL, "unknown method");
        const bool seq = opts && (opts->method == PBN_SEQ_TWO_STATE || opts->method == PBN_SEQ_SKART);
        if (seq && s->omega != 1)
            return fail(PBN_EINVAL, "the sequential methods (Alg. 1, Alg. 2) run one chain: omega = 1");
        if (!seq && s->omega < 2) return fail(PBN_EINVAL, "Gelman-Rubin needs omega >= 2 chains");
        if (!(r[i] > 0.0) || !(conf[i] > 0.0 && conf[i] < 1.0)) return fail(PBN_EINVAL, "r must be > 0 and s in (0,1)");
        if (nprops[i] < 1 || !valid_patterns(props + prop_off[i], nprops[i])) return fail(PBN_EINVAL, "bad state sets");
        // work already queued on a simulation's own stream finishes first
        if (s->stream != stream) {
            int rc = sync(s->stream);
            if (rc) return rc;
        }
    }
    static thread_local pbn::Workspace ws;
    pbn::Workspace &w = count == 1 ? sims[0]->ws : ws;
    int rc0 = count == 1 ? pbn::sim_reset(sims[0], props + prop_off[0], nprops[0], stream, err)
                         : pbn::sims_reset_batch(sims, count, props, nprops, prop_off, w, stream, err);
    if (rc0) return fail(rc0, err);
    for (uint32_t i = 0; i < count; ++i) {
        runs[i].sim = sims[i];
        sims[i]->thin = opts && opts->thin > 1 ? opts->thin : 1;
        const pbn::MachineParams P = pbn::make_params(sims[i], opts, r[i], conf[i]);
        for (uint32_t q = 0; q < nprops[i]; ++q) runs[i].machines.emplace_back(P, q);
    }
    std::vector<pbn::SimRun *> ptrs;
    for (auto &x : runs) ptrs.push_back(&x);
    int rc = pbn::run_lanes(ptrs, w, stream, err);
    if (!rc) rc = sync(stream);
    if (rc) return fail(rc, err);
    for (uint32_t i = 0; i < count; ++i)
        for (uint32_t q = 0; q < nprops[i]; ++q) out[prop_off[i] + q] = runs[i].machines[q].result();
    return PBN_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ serving

namespace {

// First-fit arena over the caller's device buffer (256-byte granules).
struct Arena {
    size_t size = 0, in_use = 0, peak = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t bytes) { size = bytes & ~size_t(255); free_.clear(); free_[0] = size; in_use = peak = 0; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t noff = it->first + bytes;
            free_.erase(it);
            if (rest) free_[noff] = rest;
            in_use += bytes;
            peak = std::max(peak, in_use);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~size_t(255);
        in_use -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct ServeReq {
    uint64_t id = 0;
    pbn::Net net;
    uint32_t omega = 0;
    uint64_t seed = 0, max_len = 0;
    std::vector<std::vector<uint32_t>> nodes;
    std::vector<std::vector<uint8_t>> vals;
    double r = 0, conf = 0;
    pbn_opts opts{};
    size_t bytes = 0, off = 0;
    int state = 0;   // 0 queued, 1 active, 2 done
    std::unique_ptr<pbn_sim> sim;
    pbn::SimRun run;
    std::vector<pbn_result> results;
};

}  // namespace

// Long-request lane of the server.  A request whose pending extension would
// take more than kLongUs of kernel time moves to a lane of its own: a stream
// restricted to a share of the CUs (kLongQuarters quarters of every XCD's),
// whose rounds run in slices of kLongTickUs beside the short requests' rounds
// and are collected when they complete, without holding those rounds.  While
// it has requests, the short requests' launches keep to the other CUs (a
// masked stream pool), so each lane's node-split groups have their CUs to
// themselves.  The long requests are few but carry most of the work (on the
// serving trace 7% of the requests, 74% of the node-updates), hence three
// quarters of the CUs by default.
constexpr double kLongTickUs = 20000.0;
constexpr uint32_t kLongQuarters = 3;
// Ahead slices (off by default): behind each round, the requests still more
// than kAheadLeftUs of kernel time short of their requirement get one more
// slice.
constexpr double kAheadLeftUs = 3000.0;

struct pbn_server {
    uint8_t *arena_base = nullptr;
    Arena arena;
    // the server's own non-blocking stream (ordered after the caller's stream
    // at creation): work on the legacy default stream would wait for the
    // long lane's slices, which run on blocking (CU-masked) streams
    hipStream_t stream = nullptr;
    pbn::Workspace ws;
    uint64_t next_id = 1;
    std::deque<ServeReq *> queue;
    std::vector<ServeReq *> active;          // the short requests' lane
    std::map<uint64_t, std::unique_ptr<ServeReq>> all;
    uint32_t done = 0;
    // long lane (lanes: 0 not yet set up, 1 ready, -1 unavailable or off)
    int lanes = 0;
    double long_us = INFINITY, long_tick_us = kLongTickUs;
    uint32_t long_quarters = kLongQuarters;
    double slice_us = pbn::kServeTickUs, ahead_us = 0.0;
    pbn::Workspace ahead_ws;
    hipEvent_t ahead_ev = nullptr;
    bool ahead_pending = false;
    uint64_t long_moved = 0, long_rounds = 0;
    uint32_t cus = 0, long_cus = 0;
    hipStream_t long_stream = nullptr, main_masked = nullptr;
    hipEvent_t admit_ev = nullptr;
    pbn::StreamPool main_pool;
    pbn::Workspace long_ws;
    pbn::RoundCtx long_ctx;
    std::vector<ServeReq *> long_active;
    ~pbn_server()
    {
        if (stream) {
            (void)hipStreamSynchronize(stream);
            (void)hipStreamDestroy(stream);
        }
        if (long_stream) {
            (void)hipStreamSynchronize(long_stream);
            (void)hipStreamDestroy(long_stream);
        }
        if (main_masked) {
            (void)hipStreamSynchronize(main_masked);
            (void)hipStreamDestroy(main_masked);
        }
        if (admit_ev) (void)hipEventDestroy(admit_ev);
        if (ahead_ev) (void)hipEventDestroy(ahead_ev);
        if (long_ctx.done) (void)hipEventDestroy(long_ctx.done);
    }
};

namespace {

// CU masks of the two lanes: CU bit i goes to the long lane when (i / 8) % 4 <
// long_quarters, the same share of every XCD's CUs whether the mask's bits run
// XCD by XCD or interleave the XCDs.
int setup_lanes(pbn_server *srv, std::string &err)
{
    if (srv->lanes) return srv->lanes > 0 ? PBN_OK : PBN_OK;
    srv->lanes = -1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        err = "device attributes";
        return PBN_EDEVICE;
    }
    if (cus < 128) return PBN_OK;                 // too few CUs to give a lane its own
    std::vector<uint32_t> lm((cus + 31) / 32, 0u), mm((cus + 31) / 32, 0u);
    uint32_t nl = 0;
    for (int i = 0; i < cus; ++i) {
        const bool lng = (uint32_t)(i / 8) % 4 < srv->long_quarters;
        (lng ? lm : mm)[i / 32] |= 1u << (i % 32);
        nl += lng;
    }
    if (hipExtStreamCreateWithCUMask(&srv->long_stream, (uint32_t)lm.size(), lm.data()) != hipSuccess ||
        hipExtStreamCreateWithCUMask(&srv->main_masked, (uint32_t)mm.size(), mm.data()) != hipSuccess ||
        hipEventCreateWithFlags(&srv->admit_ev, hipEventDisableTiming) != hipSuccess) {
        err = "CU-masked server streams";
        return PBN_EDEVICE;
    }
    srv->main_pool.cu_mask = mm;
    srv->cus = (uint32_t)cus;
    srv->long_cus = nl;
    srv->lanes = 1;
    return PBN_OK;
}

}  // namespace

extern "C" {

int pbn_server_create(void *dev_arena, size_t arena_bytes, void *hip_stream, pbn_server **out)
{
    if (!dev_arena || !out) return fail(PBN_EINVAL, "null argument");
    std::unique_ptr<pbn_server> s(new pbn_server());
    s->arena_base = (uint8_t *)dev_arena;
    s->arena.init(arena_bytes);
    hipEvent_t ready = nullptr;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ready, (hipStream_t)hip_stream) != hipSuccess ||
        hipStreamWaitEvent(s->stream, ready, 0) != hipSuccess) {
        if (ready) (void)hipEventDestroy(ready);
        return fail(PBN_EDEVICE, "server stream");
    }
    (void)hipEventDestroy(ready);
    *out = s.release();
    return PBN_OK;
}

void pbn_server_free(pbn_server *srv)
{
    if (!srv) return;
    (void)hipStreamSynchronize(srv->stream);
    delete srv;
}

int pbn_server_submit(pbn_server *srv, const pbn_net *net, uint32_t omega, uint64_t seed, const pbn_pattern *props,
                      uint32_t nprops, double r, double confidence, const pbn_opts *opts, uint64_t max_len,
                      uint64_t *id)
{
    if (!srv || !net || !id || nprops < 1 || nprops > PBN_MAX_PROPS || !valid_patterns(props, nprops))
        return fail(PBN_EINVAL, "bad argument");
    if (omega < 2 || !(r > 0.0) || !(confidence > 0.0 && confidence < 1.0)) return fail(PBN_EINVAL, "bad parameters");
    if (opts && opts->method != PBN_TWO_STATE && opts->method != PBN_SKART)
        return fail(PBN_EINVAL, "the server runs the parallel methods (Alg. 4, Alg. 5)");
    if (omega > PBN_MAX_CHAINS || max_len > PBN_MAX_LEN) return fail(PBN_ELIMIT, "omega or max_len beyond the limits");
    // the state sets are checked here, so that admission cannot fail on them
    uint64_t terms = 0;
    for (uint32_t q = 0; q < nprops; ++q) {
        for (uint32_t m = 0; m < props[q].nterms; ++m)
            if (props[q].node[m] >= net->net.n) return fail(PBN_EINVAL, "state-set node out of range");
        terms += props[q].nterms;
    }
    if (terms > PBN_MAX_TERMS) return fail(PBN_ELIMIT, "too many state-set terms");
    auto rq = std::make_unique<ServeReq>();
    rq->id = srv->next_id++;
    rq->net = net->net;
    rq->omega = omega;
    rq->seed = seed;
    rq->max_len = max_len;
    rq->r = r;
    rq->conf = confidence;
    if (opts) rq->opts = *opts;
    for (uint32_t q = 0; q < nprops; ++q) {
        rq->nodes.emplace_back(props[q].node, props[q].node + props[q].nterms);
        rq->vals.emplace_back(props[q].val, props[q].val + props[q].nterms);
    }
    rq->bytes = pbn::sim_bytes(rq->net, omega, nprops, max_len);
    if (rq->bytes > srv->arena.size) return fail(PBN_ENOMEM, "request larger than the whole arena");
    *id = rq->id;
    srv->queue.push_back(rq.get());
    srv->all[rq->id] = std::move(rq);
    return PBN_OK;
}

int pbn_server_step(pbn_server *srv, uint32_t *active, uint32_t *waiting, uint32_t *done)
{
    if (!srv) return fail(PBN_EINVAL, "null argument");
    std::string err;
    // a request that cannot run ends with its error code as every state set's
    // status, and its arena slot is freed; the other requests go on
    auto retire = [&](ServeReq *rq, int status) {
        pbn_result bad{};
        bad.prob = bad.ci_lo = bad.ci_hi = bad.rhat = NAN;
        bad.status = status;
        rq->results.assign(rq->nodes.size(), bad);
        rq->run.machines.clear();
        rq->run.sim = nullptr;
        rq->sim.reset();
        srv->arena.release(rq->off, rq->bytes);
        rq->state = 2;
        ++srv->done;
    };
    // admission at the round boundary: first fit, in arrival order; the
    // admitted simulations are laid out one by one and reset in one batch
    // (one descriptor upload, one set-up launch, no synchronisation)
    std::vector<ServeReq *> admitted;
    std::deque<ServeReq *> still;
    int first_rc = PBN_OK;
    std::string first_err;
    auto note = [&](int rc) {
        if (!first_rc) {
            first_rc = rc;
            first_err = err;
        }
    };
    for (ServeReq *rq : srv->queue) {
        size_t off;
        if (!srv->arena.alloc(rq->bytes, &off)) { still.push_back(rq); continue; }
        rq->off = off;
        rq->sim.reset(new pbn_sim());
        int rc = pbn::sim_setup(rq->sim.get(), rq->net, rq->omega, rq->seed, (uint32_t)rq->nodes.size(), rq->max_len,
                                srv->arena_base + off, rq->bytes, srv->stream, err, false);
        if (!rc) {
            std::vector<pbn_pattern> pats;
            for (size_t q = 0; q < rq->nodes.size(); ++q)
                pats.push_back({(uint32_t)rq->nodes[q].size(), rq->nodes[q].data(), rq->vals[q].data()});
            rc = pbn::sim_prepare_reset(rq->sim.get(), pats.data(), (uint32_t)pats.size(), err);
        }
        if (rc) {
            (void)hipStreamSynchronize(srv->stream);      // its uploads are done before the slot is reused
            note(rc);
            retire(rq, rc);
            continue;
        }
        rq->sim->thin = rq->opts.thin > 1 ? rq->opts.thin : 1;
        admitted.push_back(rq);
    }
    srv->queue.swap(still);
    if (!admitted.empty()) {
        std::vector<pbn_sim *> sims;
        std::vector<pbn_pattern> pats;
        std::vector<uint32_t> nprops, prop_off;
        for (ServeReq *rq : admitted) {
            sims.push_back(rq->sim.get());
            prop_off.push_back((uint32_t)pats.size());
            nprops.push_back((uint32_t)rq->nodes.size());
            for (size_t q = 0; q < rq->nodes.size(); ++q)
                pats.push_back({(uint32_t)rq->nodes[q].size(), rq->nodes[q].data(), rq->vals[q].data()});
        }
        int rc = pbn::sims_reset_batch(sims.data(), (uint32_t)sims.size(), pats.data(), nprops.data(),
                                       prop_off.data(), srv->ws, srv->stream, err);
        if (rc) {
            (void)hipStreamSynchronize(srv->stream);
            note(rc);
            for (ServeReq *rq : admitted) retire(rq, rc);
            admitted.clear();
        }
        for (ServeReq *rq : admitted) {
            rq->run.sim = rq->sim.get();
            const pbn::MachineParams P = pbn::make_params(rq->sim.get(), &rq->opts, rq->r, rq->conf);
            for (uint32_t q = 0; q < rq->nodes.size(); ++q) rq->run.machines.emplace_back(P, q);
            rq->state = 1;
            srv->active.push_back(rq);
        }
    }
    // retire finished requests and free their memory for the next admission
    auto retire_finished = [&](std::vector<ServeReq *> &lane) {
        bool waited = false;
        for (auto it = lane.begin(); it != lane.end();) {
            ServeReq *rq = *it;
            if (!rq->run.finished()) { ++it; continue; }
            // an ahead slice queued behind the round may still extend it: its
            // memory is freed once that slice has run
            if (!waited && srv->ahead_pending) {
                (void)hipEventSynchronize(srv->ahead_ev);
                waited = true;
            }
            for (auto &m : rq->run.machines) rq->results.push_back(m.result());
            rq->run.machines.clear();
            rq->sim.reset();
            srv->arena.release(rq->off, rq->bytes);
            rq->state = 2;
            ++srv->done;
            it = lane.erase(it);
        }
    };
    auto fail_lane = [&](std::vector<ServeReq *> &lane, hipStream_t s, int rc) {
        // the lane's chains are in an unknown state: every request in it ends
        // with the error, and the queued ones are admitted later
        (void)hipStreamSynchronize(s);
        note(rc);
        for (ServeReq *rq : lane) retire(rq, rc);
        lane.clear();
    };
    // the long lane's round, once it has completed
    if (srv->long_ctx.pending) {
        const hipError_t e = hipEventQuery(srv->long_ctx.done);
        if (e == hipSuccess) {
            int rc = srv->long_ws.check_split(err);
            if (rc) {
                srv->long_ctx.pending = false;
                fail_lane(srv->long_active, srv->long_stream, rc);
            } else {
                pbn::round_end(srv->long_ws, srv->long_ctx);
                retire_finished(srv->long_active);
            }
        } else if (e != hipErrorNotReady) {
            err = std::string("long lane: ") + hipGetErrorString(e);
            srv->long_ctx.pending = false;
            fail_lane(srv->long_active, srv->long_stream, PBN_EDEVICE);
        }
    }
    const bool long_busy = !srv->long_active.empty();
    std::vector<pbn::SimRun *> runs;
    for (ServeReq *rq : srv->active) runs.push_back(&rq->run);
    if (!runs.empty()) {
        // time-sliced: a request that needs a long extension does not hold the
        // others (or the next admissions) for its whole length.  Beside a busy
        // long lane the round keeps to the other CUs, after the admissions'
        // set-up on the server's stream.
        hipStream_t ms = srv->stream;
        pbn::LaunchCfg cfg;
        int rc = PBN_OK;
        if (long_busy) {
            ms = srv->main_masked;
            cfg.cus = srv->cus - srv->long_cus;
            cfg.pool = &srv->main_pool;
            if (hipEventRecord(srv->admit_ev, srv->stream) != hipSuccess ||
                hipStreamWaitEvent(ms, srv->admit_ev, 0) != hipSuccess) {
                err = "lane event";
                rc = PBN_EDEVICE;
            }
        }
        // the previous step's ahead slice has run (it was queued behind that
        // step's round); a node-split group of it that gave up is re-run first
        if (!rc && srv->ahead_pending) {
            srv->ahead_pending = false;
            if (hipEventSynchronize(srv->ahead_ev) != hipSuccess) {
                err = "ahead slice";
                rc = PBN_EDEVICE;
            } else {
                rc = srv->ahead_ws.check_split(err);
            }
        }
        pbn::RoundCtx ctx;
        if (!rc) rc = pbn::round_begin(runs, srv->ws, ms, ctx, err, cfg, srv->slice_us);
        if (!rc && srv->ahead_us > 0.0) {
            bool launched = false;
            rc = pbn::ahead_begin(runs, srv->ahead_ws, ms, cfg, srv->ahead_us, kAheadLeftUs, &launched, err);
            if (!rc && launched) {
                if ((!srv->ahead_ev && hipEventCreateWithFlags(&srv->ahead_ev, hipEventDisableTiming) != hipSuccess) ||
                    hipEventRecord(srv->ahead_ev, ms) != hipSuccess) {
                    err = "ahead event";
                    rc = PBN_EDEVICE;
                } else {
                    srv->ahead_pending = true;
                }
            }
        }
        if (!rc && ctx.pending) {
            const hipError_t e = hipEventSynchronize(ctx.done);
            if (e != hipSuccess) {
                err = std::string("round sync: ") + hipGetErrorString(e);
                rc = PBN_EDEVICE;
            } else if (!(rc = srv->ws.check_split(err))) {
                pbn::round_end(srv->ws, ctx);
            }
        }
        if (ctx.done) (void)hipEventDestroy(ctx.done);
        // the next admission rewrites the pinned descriptor staging: this
        // round's copy of it has completed once the stream is idle
        if (!admitted.empty() && hipStreamSynchronize(srv->stream) != hipSuccess && !rc) {
            err = "stream synchronize";
            rc = PBN_EDEVICE;
        }
        if (rc) {
            srv->ahead_pending = false;
            fail_lane(srv->active, ms, rc);
        }
    }
    retire_finished(srv->active);
    // requests whose pending extension is long move to the long lane
    if (srv->lanes == 0) {
        int rc = setup_lanes(srv, err);
        if (rc) note(rc);
    }
    if (srv->lanes > 0) {
        for (auto it = srv->active.begin(); it != srv->active.end();) {
            ServeReq *rq = *it;
            uint64_t need = UINT64_MAX;
            for (auto &m : rq->run.machines)
                if (!m.done()) need = std::min(need, m.request().need_len);
            const pbn_sim *sim = rq->sim.get();
            const uint32_t groups = (sim->omega + 63) / 64;
            const uint32_t parts = std::max<uint32_t>(1, std::min<uint32_t>(16, srv->long_cus / groups));
            if (need != UINT64_MAX && need > sim->len && groups <= srv->long_cus &&
                pbn::extension_us(sim, need - sim->len, parts) > srv->long_us) {
                srv->long_active.push_back(rq);
                ++srv->long_moved;
                it = srv->active.erase(it);
            } else {
                ++it;
            }
        }
        if (!srv->long_ctx.pending && !srv->long_active.empty()) {
            // the long lane's next slice, after everything queued on the
            // server's stream (the moved requests' earlier rounds)
            std::vector<pbn::SimRun *> lr;
            for (ServeReq *rq : srv->long_active) lr.push_back(&rq->run);
            const pbn::LaunchCfg lcfg{false, true, false, srv->long_cus, nullptr};
            int rc = PBN_OK;
            if (hipEventRecord(srv->admit_ev, srv->stream) != hipSuccess ||
                hipStreamWaitEvent(srv->long_stream, srv->admit_ev, 0) != hipSuccess) {
                err = "lane event";
                rc = PBN_EDEVICE;
            }
            if (!rc)
                rc = pbn::round_begin(lr, srv->long_ws, srv->long_stream, srv->long_ctx, err, lcfg, srv->long_tick_us, 1);
            if (!rc) ++srv->long_rounds;
            if (rc) {
                srv->long_ctx.pending = false;
                fail_lane(srv->long_active, srv->long_stream, rc);
            }
        }
    }
    if (active) *active = (uint32_t)(srv->active.size() + srv->long_active.size());
    if (waiting) *waiting = (uint32_t)srv->queue.size();
    if (done) *done = srv->done;
    if (first_rc) {
        err = first_err;
        return fail(first_rc, err);
    }
    return PBN_OK;
}

int pbn_server_configure(pbn_server *srv, const pbn_server_opts *o)
{
    if (!srv || !o || o->long_quarters > 3) return fail(PBN_EINVAL, "bad argument");
    if (!(o->slice_us >= 0.0) || !(o->long_slice_us >= 0.0) || !(o->ahead_us >= 0.0) || !(o->long_lane_us >= 0.0))
        return fail(PBN_EINVAL, "bad argument");
    const uint32_t q = o->long_quarters ? o->long_quarters : kLongQuarters;
    if (q != srv->long_quarters && srv->lanes != 0)
        return fail(PBN_EINVAL, "the lanes' CU shares are fixed once the server has stepped");
    const double long_us = o->long_lane_us > 0.0 ? o->long_lane_us : INFINITY;
    if (std::isinf(long_us) && !srv->long_active.empty()) return fail(PBN_EINVAL, "the long lane has requests");
    srv->long_quarters = q;
    srv->long_us = long_us;
    srv->long_tick_us = o->long_slice_us > 0.0 ? o->long_slice_us : kLongTickUs;
    srv->slice_us = o->slice_us > 0.0 ? o->slice_us : pbn::kServeTickUs;
    srv->ahead_us = o->ahead_us > 0.0 ? o->ahead_us : 0.0;
    return PBN_OK;
}

int pbn_server_lane_stats(const pbn_server *srv, uint64_t *long_requests, uint64_t *long_rounds)
{
    if (!srv) return fail(PBN_EINVAL, "null argument");
    if (long_requests) *long_requests = srv->long_moved;
    if (long_rounds) *long_rounds = srv->long_rounds;
    return PBN_OK;
}

int pbn_server_poll(pbn_server *srv, uint64_t id, int *ready, pbn_result *out)
{
    if (!srv || !ready) return fail(PBN_EINVAL, "null argument");
    auto it = srv->all.find(id);
    if (it == srv->all.end()) return fail(PBN_EINVAL, "unknown request");
    ServeReq *rq = it->second.get();
    *ready = rq->state == 2;
    if (*ready && out) std::copy(rq->results.begin(), rq->results.end(), out);
    return PBN_OK;
}

int pbn_set_kernel(int mode, uint32_t waves)
{
    if (mode < 0 || mode > 2 || waves > 16)
        return fail(PBN_EINVAL, "mode must be 0..2 and waves 0..16");
    pbn::set_kernel_mode(mode, waves);
    return PBN_OK;
}

int pbn_set_split(uint32_t parts)
{
    pbn::set_split_mode(parts);
    return PBN_OK;
}

int pbn_sim_set_kernel(pbn_sim *sim, int mode, uint32_t waves)
{
    if (!sim || mode < -1 || mode > 2 ||
        waves > 16)
        return fail(PBN_EINVAL, "mode must be -1..2 and waves 0..16");
    sim->kmode = mode;
    sim->kwaves = mode < 0 ? 0 : waves;
    return PBN_OK;
}

int pbn_sim_set_split(pbn_sim *sim, int parts)
{
    if (!sim || parts < -1) return fail(PBN_EINVAL, "parts must be -1 or more");
    sim->split = parts;
    return PBN_OK;
}

int pbn_set_split_polls(uint32_t polls)
{
    pbn::set_split_spins(polls);
    return PBN_OK;
}

int pbn_autotune(void *hip_stream, pbn_tune_row *rows, uint32_t cap, uint32_t *count)
{
    std::string err;
    int rc = pbn::autotune((hipStream_t)hip_stream, rows, cap, count, err);
    return rc ? fail(rc, err) : PBN_OK;
}

int pbn_autotune_reset(void)
{
    pbn::autotune_reset();
    return PBN_OK;
}

int pbn_profile_enable(int on)
{
    pbn::profile_set(on != 0);
    return PBN_OK;
}

int pbn_profile_read(pbn_profile *out)
{
    if (!out) return fail(PBN_EINVAL, "null argument");
    std::string err;
    int rc = pbn::profile_collect(out, err);
    return rc ? fail(rc, err) : PBN_OK;
}

int pbn_profile_reset(void)
{
    pbn::profile_clear();
    return PBN_OK;
}

int pbn_server_memory(const pbn_server *srv, size_t *in_use, size_t *peak)
{
    if (!srv) return fail(PBN_EINVAL, "null argument");
    if (in_use) *in_use = srv->arena.in_use;
    if (peak) *peak = srv->arena.peak;
    return PBN_OK;
}

}  // extern "C"
