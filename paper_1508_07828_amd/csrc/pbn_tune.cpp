// Autotuner of the bit-sliced kernel's shape: waves per 64-chain block, per
// network-size bucket, for throughput (one network's blocks filling the chip)
// and for latency (one block alone), from short event-timed launches on synthetic
// networks drawn like the workloads' (1-3 predictors per node, 1-5 parents,
// random truth tables, p = 1e-3; the paper's random-network recipe of Sec. 5.1).
// The measured table replaces the built-in latency and one-network rules for
// the rest of the process; the batched lanes keep their built-in shapes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "pbn_driver.h"

namespace pbn {
namespace {

struct TuneRow {
    uint32_t n, g_thr, g_lat;
    double nu_per_s, lat_us;
};

std::mutex g_tune_mu;
std::vector<TuneRow> g_tune;             // sorted by n; empty = built-in rule

uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

std::string synth_network(uint32_t n, uint64_t seed)
{
    uint64_t s = seed;
    std::string out = "PBN " + std::to_string(n) + " 0.001\n";
    char buf[64];
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t l = 1 + (uint32_t)(splitmix(s) % 3);
        out += "N " + std::to_string(i) + " " + std::to_string(l) + "\n";
        double c[3], sum = 0.0;
        for (uint32_t j = 0; j < l; ++j) {
            c[j] = 0.05 + (double)(splitmix(s) >> 11) * 0x1.0p-53;
            sum += c[j];
        }
        for (uint32_t j = 0; j < l; ++j) {
            const uint32_t k = 1 + (uint32_t)(splitmix(s) % std::min<uint32_t>(5, n));
            std::snprintf(buf, sizeof buf, "F %.17g %u", c[j] / sum, k);
            out += buf;
            std::vector<uint32_t> par;
            while (par.size() < k) {
                const uint32_t v = (uint32_t)(splitmix(s) % n);
                bool dup = false;
                for (uint32_t u : par) dup |= u == v;
                if (!dup) par.push_back(v);
            }
            for (uint32_t v : par) out += " " + std::to_string(v);
            const uint32_t bits = 1u << k;
            const uint64_t tt = splitmix(s) & (bits >= 64 ? ~0ull : ((1ull << bits) - 1));
            std::snprintf(buf, sizeof buf, " %llx\n", (unsigned long long)tt);
            out += buf;
        }
    }
    return out;
}

// Event-timed launch of `steps` transitions of every chain of sim with G waves.
int timed_run(pbn_sim *sim, uint32_t G, uint64_t steps, Workspace &ws, hipStream_t stream, hipEvent_t e0,
              hipEvent_t e1, double *ms, std::string &err)
{
    std::vector<StepItem> items;
    sim_extend_items(sim, 0, steps, 1, items, false);
    for (StepItem &it : items) {
        it.kernel = G;
        it.lds = (uint32_t)bs_lds_bytes(sim->net.n, sim->net.msel_total, G);
        it.small = sim->net.nblk <= G && sim->net.F_pad <= 64 * G;
    }
    if (hipEventRecord(e0, stream) != hipSuccess) { err = "event"; return PBN_EDEVICE; }
    int rc = launch_items(items, ws, stream, err, false);
    if (rc) return rc;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        err = "tuning launch";
        return PBN_EDEVICE;
    }
    float t = 0.0f;
    (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t;
    return PBN_OK;
}

int measure(uint32_t n, hipStream_t stream, TuneRow &row, std::string &err)
{
    Net net;
    const std::string text = synth_network(n, 0x1508078280ull + n);
    int rc = parse_and_compile(text.c_str(), text.size(), net, err);
    if (rc) return rc;
    if (!net.bitsliced) { err = "synthetic network not bit-sliced"; return PBN_ELIMIT; }
    const uint32_t big = 64u * 2048u;
    const uint64_t thr_steps = std::max<uint64_t>(4, (uint64_t)(2e9 / ((double)big * n)));
    const uint64_t lat_steps = 64;
    const uint64_t max_len = std::max(thr_steps, lat_steps) * 2 + 64;
    const size_t bytes = sim_bytes(net, big, 1, max_len);
    void *buf = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) { err = "tuning buffer"; return PBN_ENOMEM; }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    Workspace ws;
    const uint32_t node0 = 0;
    const uint8_t val1 = 1;
    const pbn_pattern pat{1, &node0, &val1};
    row = TuneRow{n, 0, 0, 0.0, 1e300};
    for (uint32_t omega : {big, 64u}) {
        pbn_sim sim;
        rc = sim_setup(&sim, net, omega, 7828, 1, max_len, buf, bytes, stream, err);
        if (rc) break;
        const uint64_t steps = omega == big ? thr_steps : lat_steps;
        for (uint32_t G : {1u, 2u, 4u, 5u, 8u, 12u, 16u}) {
            if (bs_lds_bytes(net.n, net.msel_total, G) > 160 * 1024) continue;
            double ms = 0.0, warm = 0.0;
            if ((rc = sim_reset(&sim, &pat, 1, stream, err))) break;
            if ((rc = timed_run(&sim, G, 2, ws, stream, e0, e1, &warm, err))) break;
            if ((rc = timed_run(&sim, G, steps, ws, stream, e0, e1, &ms, err))) break;
            if (omega == big) {
                const double nu = (double)omega * n * steps / (ms * 1e-3);
                if (nu > row.nu_per_s) row.nu_per_s = nu, row.g_thr = G;
            } else {
                const double us = ms * 1e3 / steps;
                if (us < row.lat_us) row.lat_us = us, row.g_lat = G;
            }
        }
        if (rc) break;
    }
    (void)hipStreamSynchronize(stream);
    ws.release();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (!rc && (row.g_thr == 0 || row.g_lat == 0)) { err = "no kernel shape fits"; rc = PBN_ELIMIT; }
    return rc;
}

}  // namespace

bool tuned_waves(uint32_t n, int shape, uint32_t *G)
{
    // the table times one network alone on the chip: it stands for the latency
    // and one-network shapes, not for the batched lanes' shared one
    if (shape == kShapeShared) return false;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (g_tune.empty()) return false;
    const TuneRow *best = &g_tune[0];
    double dbest = 1e300;
    for (const TuneRow &r : g_tune) {
        const double d = std::fabs(std::log2((double)n) - std::log2((double)r.n));
        if (d < dbest) dbest = d, best = &r;
    }
    *G = shape == kShapeLatency ? best->g_lat : best->g_thr;
    return true;
}

int autotune(hipStream_t stream, pbn_tune_row *rows, uint32_t cap, uint32_t *count, std::string &err)
{
    static const uint32_t sizes[] = {24, 48, 96, 192, 384, 768, 1536, 3072};
    std::vector<TuneRow> table;
    for (uint32_t n : sizes) {
        TuneRow r{};
        int rc = measure(n, stream, r, err);
        if (rc) return rc;
        table.push_back(r);
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune = table;
    }
    uint32_t k = 0;
    for (const TuneRow &r : table) {
        if (rows && k < cap) {
            rows[k] = pbn_tune_row{r.n, r.g_thr, r.g_lat, 0u, r.nu_per_s, r.lat_us};
        }
        ++k;
    }
    if (count) *count = k;
    return PBN_OK;
}

void autotune_reset()
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
}

}  // namespace pbn
