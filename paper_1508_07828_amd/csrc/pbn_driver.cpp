// Host control of the method (Alg. 3, Alg. 4, Alg. 5 and the multi-property
// scheme of Sec. 4.2) over device-resident chains.
//
// Readings of the paper that this file implements (it is silent or garbled on
// them):
//   Alg. 3  the monitored scalar is the state set's 0-1 indicator; s_i uses the
//           denominator psi-1; the chains reach 2*psi0 positions first and each
//           check uses positions psi+1..2psi; converged when R < psrf_max; a
//           check with W = 0 is "not converged"; the returned psi is the last
//           one checked.
//   Alg. 4  the first pass uses the existing second halves without extending;
//           the extension is ceil((N - omega n)/omega) and the pass loop ends
//           when it is <= 0; alpha and beta come from all consecutive pairs
//           inside each chain's window; if either is undefined the window
//           doubles; a re-run happens when M > psi and moves the window start
//           to M (psi := M), refilling it to the Gelman-Rubin psi if it
//           became empty; the estimate is the fraction of ones in the window.
//   Alg. 5  (Skart-P) eta0 = ceil(1280/omega) omega first observations;
//           batch size 16 if |skewness| > 4 else 1; p/omega consecutive
//           batches per chain; von Neumann randomness test on within-chain
//           adjacent batch means at level 0.2, on failure kappa :=
//           ceil(sqrt 2 kappa) and p := ceil(0.9 p) rounded up to a multiple of
//           omega (at most 10 times); CI skewness- (Willink) and lag-1
//           autoregression-adjusted; if the half-width H > H* the batch size
//           grows to ceil(kappa (H/H*)^2).
//   Sec. 4.2  every state set runs its own machine on the shared chains;
//           the chains grow to the smallest pending requirement.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <queue>
#include <thread>

#include "pbn_driver.h"

namespace pbn {

// ------------------------------------------------------------ workspace

int Workspace::ensure(size_t items, size_t queries, size_t bsum, std::string &err)
{
    auto grow = [&](auto *&d, auto *&h, size_t &cap, size_t need, size_t elem) -> int {
        if (need <= cap) return PBN_OK;
        size_t nc = std::max<size_t>(need, 2 * cap);
        if (d) (void)hipFree(d);
        if (h) (void)hipHostFree(h);
        d = nullptr; h = nullptr; cap = 0;
        if (hipMalloc((void **)&d, nc * elem) != hipSuccess) { err = "workspace hipMalloc"; return PBN_ENOMEM; }
        if (hipHostMalloc((void **)&h, nc * elem, hipHostMallocDefault) != hipSuccess) {
            err = "workspace hipHostMalloc";
            return PBN_ENOMEM;
        }
        cap = nc;
        return PBN_OK;
    };
    int rc;
    if ((rc = grow(d_items, h_items, cap_items, std::max<size_t>(items, 1), sizeof(StepItem)))) return rc;
    size_t qcap = cap_q;
    if ((rc = grow(d_queries, h_queries, cap_q, std::max<size_t>(queries, 1), sizeof(Query)))) return rc;
    if (cap_q != qcap || !d_win) {
        if (d_win) (void)hipFree(d_win);
        if (h_win) (void)hipHostFree(h_win);
        d_win = nullptr; h_win = nullptr;
        if (hipMalloc((void **)&d_win, cap_q * sizeof(WindowResult)) != hipSuccess ||
            hipHostMalloc((void **)&h_win, cap_q * sizeof(WindowResult), hipHostMallocDefault) != hipSuccess) {
            err = "workspace results";
            return PBN_ENOMEM;
        }
    }
    if ((rc = grow(d_bsum, h_bsum, cap_bsum, std::max<size_t>(bsum, 1), sizeof(int32_t)))) return rc;
    return PBN_OK;
}

int Workspace::before_write(hipEvent_t &ev, bool &in_flight, std::string &err)
{
    if (!in_flight) return PBN_OK;
    if (hipEventSynchronize(ev) != hipSuccess) { err = "table copy"; return PBN_EDEVICE; }
    in_flight = false;
    return PBN_OK;
}

int Workspace::after_copy(hipEvent_t &ev, bool &in_flight, hipStream_t stream, std::string &err)
{
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { err = "event"; return PBN_EDEVICE; }
    if (hipEventRecord(ev, stream) != hipSuccess) { err = "event"; return PBN_EDEVICE; }
    in_flight = true;
    return PBN_OK;
}

int Workspace::ensure_stage(size_t count, std::string &err)
{
    if (count <= cap_stage) return PBN_OK;
    const size_t nc = std::max<size_t>(count, 2 * cap_stage);
    if (d_stage) (void)hipFree(d_stage);
    if (h_stage) (void)hipHostFree(h_stage);
    if (d_dst) (void)hipFree(d_dst);
    if (h_dst) (void)hipHostFree(h_dst);
    d_stage = h_stage = nullptr;
    d_dst = h_dst = nullptr;
    cap_stage = 0;
    if (hipMalloc((void **)&d_stage, nc * sizeof(DevSim)) != hipSuccess ||
        hipHostMalloc((void **)&h_stage, nc * sizeof(DevSim), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&d_dst, nc * sizeof(DevSim *)) != hipSuccess ||
        hipHostMalloc((void **)&h_dst, nc * sizeof(DevSim *), hipHostMallocDefault) != hipSuccess) {
        err = "staging allocation";
        return PBN_ENOMEM;
    }
    cap_stage = nc;
    return PBN_OK;
}

int Workspace::ensure_split(size_t groups, size_t xch_words, std::string &err)
{
    if (groups > cap_grp) {
        const size_t nc = std::max(groups, 2 * cap_grp);
        if (d_grp) (void)hipFree(d_grp);
        if (h_grp) (void)hipHostFree(h_grp);
        if (d_stat) (void)hipFree(d_stat);
        if (h_stat) (void)hipHostFree(h_stat);
        d_grp = h_grp = nullptr;
        d_stat = h_stat = nullptr;
        cap_grp = 0;
        // one status word per group (one clear and one download per launch)
        if (hipMalloc((void **)&d_grp, nc * sizeof(SplitGroup)) != hipSuccess ||
            hipHostMalloc((void **)&h_grp, nc * sizeof(SplitGroup), hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&d_stat, nc * sizeof(uint32_t)) != hipSuccess ||
            hipHostMalloc((void **)&h_stat, nc * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
            err = "workspace split groups";
            return PBN_ENOMEM;
        }
        cap_grp = nc;
    }
    if (xch_words > cap_xch) {
        const size_t nc = std::max(xch_words, 2 * cap_xch);
        if (d_xch) (void)hipFree(d_xch);
        d_xch = nullptr;
        cap_xch = 0;
        if (hipMalloc((void **)&d_xch, nc * sizeof(uint64_t)) != hipSuccess) {
            err = "workspace split exchange";
            return PBN_ENOMEM;
        }
        cap_xch = nc;
    }
    return PBN_OK;
}

int Workspace::ensure_rows(size_t words, std::string &err)
{
    if (words <= cap_rows) return PBN_OK;
    const size_t nc = std::max(words, 2 * cap_rows);
    if (d_rows) (void)hipFree(d_rows);
    d_rows = nullptr;
    cap_rows = 0;
    if (hipMalloc((void **)&d_rows, nc * sizeof(uint32_t)) != hipSuccess) {
        err = "workspace state rows";
        return PBN_ENOMEM;
    }
    cap_rows = nc;
    return PBN_OK;
}

namespace {
std::atomic<uint64_t> g_split_fallbacks{0};
}  // namespace

uint64_t split_fallbacks() { return g_split_fallbacks.load(); }

int Workspace::check_split(std::string &err)
{
    if (!split_used) return PBN_OK;
    const size_t ng = split_used;
    split_used = 0;
    std::vector<StepItem> redo;
    for (size_t q = 0; q < ng && q < split_items.size(); ++q)
        if (h_stat[q] == 1u) redo.push_back(split_items[q]);
    const size_t nq = redo_queries, nb = redo_bsum;
    redo_queries = redo_bsum = 0;
    if (redo.empty()) return PBN_OK;
    // the groups that gave up left their state as the launch found it and
    // wrote only indicator words that the re-run writes again unchanged
    g_split_fallbacks += redo.size();
    hipStream_t stream = split_stream;
    int rc = launch_items(redo, *this, stream, err, false, false);
    if (rc) return rc;
    if (nq) {
        if ((rc = launch_reduce(d_queries, (uint32_t)nq, d_win, d_bsum, stream, err))) return rc;
        if (hipMemcpyAsync(h_win, d_win, nq * sizeof(WindowResult), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            (nb && hipMemcpyAsync(h_bsum, d_bsum, nb * sizeof(int32_t), hipMemcpyDeviceToHost, stream) !=
                       hipSuccess)) {
            err = "result download";
            return PBN_EDEVICE;
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess) {
        err = "node-split re-run";
        return PBN_EDEVICE;
    }
    return PBN_OK;
}

void Workspace::release()
{
    if (d_rows) (void)hipFree(d_rows);
    d_rows = nullptr;
    cap_rows = 0;
    if (d_grp) (void)hipFree(d_grp);
    if (h_grp) (void)hipHostFree(h_grp);
    if (d_stat) (void)hipFree(d_stat);
    if (d_xch) (void)hipFree(d_xch);
    if (h_stat) (void)hipHostFree(h_stat);
    d_grp = h_grp = nullptr;
    d_xch = nullptr;
    d_stat = h_stat = nullptr;
    cap_grp = cap_xch = 0;
    split_used = 0;
    split_items.clear();
    if (ev_items) (void)hipEventSynchronize(ev_items), (void)hipEventDestroy(ev_items);
    if (ev_queries) (void)hipEventSynchronize(ev_queries), (void)hipEventDestroy(ev_queries);
    ev_items = ev_queries = nullptr;
    items_in_flight = queries_in_flight = false;
    if (d_stage) (void)hipFree(d_stage);
    if (h_stage) (void)hipHostFree(h_stage);
    if (d_dst) (void)hipFree(d_dst);
    if (h_dst) (void)hipHostFree(h_dst);
    d_stage = h_stage = nullptr;
    d_dst = h_dst = nullptr;
    cap_stage = 0;
    if (d_items) (void)hipFree(d_items);
    if (h_items) (void)hipHostFree(h_items);
    if (d_queries) (void)hipFree(d_queries);
    if (h_queries) (void)hipHostFree(h_queries);
    if (d_win) (void)hipFree(d_win);
    if (h_win) (void)hipHostFree(h_win);
    if (d_bsum) (void)hipFree(d_bsum);
    if (h_bsum) (void)hipHostFree(h_bsum);
    d_items = h_items = nullptr;
    d_queries = h_queries = nullptr;
    d_win = h_win = nullptr;
    d_bsum = h_bsum = nullptr;
    cap_items = cap_q = cap_bsum = 0;
}

// ------------------------------------------------------------ formulas

namespace {

int64_t cdiv(int64_t a, int64_t b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }

// Alg. 1's N (before the ceiling): ab(2-a-b)/(a+b)^3 * z^2/r^2.
double formula_N(double a, double b, double z, double r)
{
    double x = (a * b * ((2.0 - a) - b)) / ((a + b) * (a + b) * (a + b));
    return x * ((z * z) / (r * r));
}

// Alg. 1's M: ceil(log(eps (a+b)/max(a,b)) / log|1-a-b|), 0 when |1-a-b| is 0 or 1.
uint64_t formula_M(double a, double b, double eps)
{
    double lam = std::fabs((1.0 - a) - b);
    if (lam == 0.0 || lam == 1.0) return 0;
    double v = std::ceil(std::log(eps * (a + b) / std::max(a, b)) / std::log(lam));
    return v <= 0.0 ? 0 : (uint64_t)v;
}

// Alg. 2's randomness test on one chain's spaced batch sums: batches d, 2d+1,
// 3d+2, ... (0-based), each one preceded by d spacer batches.
bool spaced_randomness_passes(const int32_t *bsum, uint64_t p, uint64_t d)
{
    std::vector<int32_t> sel;
    for (uint64_t b = d; b < p; b += d + 1) sel.push_back(bsum[b]);
    return randomness_passes(batch_moments(sel.data(), 1, sel.size()));
}

// Batch size after a CI wider than H*: ceil(kappa (H/H*)^2) in FP64, saturated
// at 2^64 - 1.
uint64_t grown_kappa(uint64_t kappa, double H, double H_star)
{
    const double ratio = H / H_star;
    const double k = std::ceil((double)kappa * (ratio * ratio));
    return k >= 18446744073709551616.0 ? UINT64_MAX : (uint64_t)k;
}

}  // namespace

// ------------------------------------------------------------ machine

Machine::Machine(const MachineParams &p, uint32_t prop) : P_(p), prop_(prop)
{
    res_.prob = res_.ci_lo = res_.ci_hi = res_.rhat = NAN;
    res_.status = PBN_OK;
    z_ = normal_quantile(0.5 * (1.0 + P_.conf));
    psi_ = P_.psi0;
    if (P_.method == PBN_SEQ_TWO_STATE) {
        // Alg. 1: M := m0, N := n0, l := M + N, a trajectory of length l
        st_ = kSeqTwoState;
        M_ = P_.psi0;
        N_ = 4 * P_.psi0;
        l_ = M_ + N_;
        seq_next(0);
        return;
    }
    if (P_.method == PBN_SEQ_SKART) {
        // Alg. 2: an initial trajectory of eta = 1280 positions; the skewness
        // of its last l = 1024 sets the batch size
        st_ = kSeqSkartSkew;
        psi_ = 0;
        if (kSeqSkartEta > P_.cap) not_converged(0);
        else ask_window(kSeqSkartEta - kSeqSkartTail, kSeqSkartEta);
        return;
    }
    if (!gr_window_fits(psi_)) not_converged(0);
    else ask_window(psi_, 2 * psi_);
}

// Alg. 1: the next window is the last N positions of the trajectory of length
// l (extended to l first when it is shorter).
void Machine::seq_next(uint64_t chain_len)
{
    if (l_ > P_.cap) {
        res_.status = PBN_ENOTCONV;
        res_.psi = M_;
        res_.n = N_;
        res_.M = M_;
        res_.chain_len = chain_len;
        done_ = true;
        return;
    }
    ask_window(l_ - N_, l_);
}

// The Gelman-Rubin window [psi, 2 psi) fits under the cap, and its exact sum
// of squares (omega chains, each at most psi ones) fits in 63 bits.
bool Machine::gr_window_fits(uint64_t psi) const
{
    return 2 * psi <= P_.cap && (double)P_.omega * (double)psi * (double)psi < 9.0e18;
}

void Machine::ask_window(uint64_t lo, uint64_t hi)
{
    req_ = Request{kQueryWindow, lo, hi, 0, 0, hi};
}

void Machine::ask_batch()
{
    const uint64_t m = p_ / P_.omega;
    req_ = Request{kQueryBatch, base_, base_ + kappa_ * m, kappa_, m, base_ + kappa_ * m};
}

void Machine::not_converged(uint64_t chain_len)
{
    res_.status = PBN_ENOTCONV;
    res_.psi = psi_;
    res_.n = n_;
    res_.chain_len = chain_len;
    done_ = true;
}

void Machine::feed_window(const WindowResult &w, uint64_t chain_len)
{
    const uint32_t omega = P_.omega;
    ++res_.rounds;
    switch (st_) {
    case kGR: {
        bool defined;
        double R = rhat_from_sums(w.T1, w.T2, omega, psi_, &defined);
        if (defined && R < P_.psrf_max) {
            res_.psi_gr = psi_;
            res_.rhat = R;
            psi_gr_ = psi_;
            if (P_.method == PBN_TWO_STATE) {
                n_ = psi_;
                st_ = kTwoState;
                if (psi_ + n_ > P_.cap) return not_converged(chain_len);
                ask_window(psi_, psi_ + n_);
            } else {
                res_.psi = psi_;
                base_ = psi_;
                const uint64_t eta0 = (uint64_t)cdiv(1280, omega) * omega;
                st_ = kSkartSkew;
                if (base_ + eta0 / omega > P_.cap) return not_converged(chain_len);
                ask_window(base_, base_ + eta0 / omega);
            }
        } else {
            psi_ *= 2;
            if (!gr_window_fits(psi_)) return not_converged(chain_len);
            ask_window(psi_, 2 * psi_);
        }
        return;
    }
    case kTwoState: {
        int64_t extend_by;
        const bool undefined = (w.n00 + w.n01 == 0) || (w.n10 + w.n11 == 0);
        double a = 0.0, b = 0.0;
        if (!undefined) {
            a = (double)w.n01 / (double)(w.n00 + w.n01);
            b = (double)w.n10 / (double)(w.n10 + w.n11);
        }
        if (undefined || a + b == 0.0) {
            extend_by = (int64_t)n_;
        } else {
            a_ = a;
            b_ = b;
            const double Nf = std::ceil(formula_N(a, b, z_, P_.r));
            if (!(Nf < 9.0e15)) return not_converged(chain_len);
            N_ = (uint64_t)Nf;
            extend_by = cdiv((int64_t)N_ - (int64_t)omega * (int64_t)n_, omega);
            if (extend_by <= 0) {
                const uint64_t M = formula_M(a_, b_, P_.eps);
                res_.M = M;
                if (M > psi_) {
                    int64_t n = (int64_t)n_ - (int64_t)(M - psi_);
                    psi_ = M;
                    n_ = n <= 0 ? psi_gr_ : (uint64_t)n;
                    if (psi_ + n_ > P_.cap) return not_converged(chain_len);
                    ask_window(psi_, psi_ + n_);
                    return;
                }
                return finish_two_state(w.T1);
            }
        }
        n_ += (uint64_t)extend_by;
        if (psi_ + n_ > P_.cap) return not_converged(chain_len);
        ask_window(psi_, psi_ + n_);
        return;
    }
    case kSkartSkew: {
        const uint64_t eta0 = (uint64_t)cdiv(1280, omega) * omega;
        kappa_ = skewness_exceeds_4((uint64_t)w.T1, eta0) ? 16 : 1;
        p_ = eta0;
        tries_ = 0;
        st_ = kSkartRandomness;
        if (!batches_fit()) return not_converged(chain_len);
        ask_batch();
        return;
    }
    case kSeqSkartSkew: {
        kappa_ = skewness_exceeds_4((uint64_t)w.T1, kSeqSkartTail) ? 16 : 1;
        p_ = kSeqSkartEta;
        base_ = 0;
        tries_ = 0;
        st_ = kSeqSkartRandomness;
        if (kappa_ * p_ > P_.cap) return not_converged(chain_len);
        ask_batch();
        return;
    }
    case kSeqTwoState: {
        // alpha, beta from the last N positions; undefined (a meta state never
        // left, or never seen): the sample is doubled
        const bool undefined = (w.n00 + w.n01 == 0) || (w.n10 + w.n11 == 0);
        double a = 0.0, b = 0.0;
        if (!undefined) {
            a = (double)w.n01 / (double)(w.n00 + w.n01);
            b = (double)w.n10 / (double)(w.n10 + w.n11);
        }
        if (undefined || a + b == 0.0) {
            N_ *= 2;
            l_ = std::max(l_, M_ + N_);
            return seq_next(chain_len);
        }
        a_ = a;
        b_ = b;
        const double Nf = std::ceil(formula_N(a, b, z_, P_.r));
        if (!(Nf < 9.0e15)) return not_converged(chain_len);
        M_ = formula_M(a, b, P_.eps);
        N_ = std::max<uint64_t>(1, (uint64_t)Nf);     // at least one position (alpha = beta = 1 gives 0)
        if (M_ + N_ <= l_) {
            // until M + N <= l: the estimate comes from the last N positions
            st_ = kSeqFinal;
            ask_window(l_ - N_, l_);
            return;
        }
        l_ = M_ + N_;
        return seq_next(chain_len);
    }
    case kSeqFinal:
        res_.psi = M_;
        res_.M = M_;
        res_.n = N_;
        res_.N = N_;
        res_.sample_size = N_;
        res_.prob = (double)w.T1 / (double)N_;
        res_.chain_len = l_;
        done_ = true;
        return;
    default:
        return;
    }
}

void Machine::feed_batch(const int32_t *bsum, uint64_t chain_len)
{
    const uint32_t omega = P_.omega;
    ++res_.rounds;
    const uint64_t m = p_ / omega;
    if (st_ == kSkartRandomness) {
        if (randomness_passes(batch_moments(bsum, omega, m)) || tries_ >= 10) {
            st_ = kSkartCI;
            return skart_ci(bsum, chain_len);
        }
        kappa_ = (uint64_t)std::ceil(std::sqrt(2.0) * (double)kappa_);
        const uint64_t p09 = (uint64_t)std::ceil(0.9 * (double)p_);
        p_ = std::max<uint64_t>(omega, (uint64_t)cdiv((int64_t)p09, omega) * omega);
        ++tries_;
        if (!batches_fit()) return not_converged(chain_len);
        ask_batch();
        return;
    }
    if (st_ == kSeqSkartRandomness) {
        // spacers d = 0..10 on the same batch means; when all fail, longer
        // batches (at most 10 times, then the spacer stays at 10)
        uint64_t d = 0;
        while (d <= kSeqSkartMaxSpacer && !spaced_randomness_passes(bsum, p_, d)) ++d;
        if (d > kSeqSkartMaxSpacer && tries_ >= 10) d = kSeqSkartMaxSpacer;
        if (d <= kSeqSkartMaxSpacer) {
            // skip zeta = d kappa positions: the CI uses the p' = p - d batches after them
            d_ = d;
            base_ = d_ * kappa_;
            p_ -= d_;
            st_ = kSkartCI;
            return skart_ci(bsum + d_, chain_len);
        }
        kappa_ = (uint64_t)std::ceil(std::sqrt(2.0) * (double)kappa_);
        p_ = (uint64_t)std::ceil(0.9 * (double)p_);
        ++tries_;
        if (kappa_ * p_ > P_.cap) return not_converged(chain_len);
        ask_batch();
        return;
    }
    if (st_ == kSkartCI) skart_ci(bsum, chain_len);
}

void Machine::skart_ci(const int32_t *bsum, uint64_t chain_len)
{
    const uint32_t omega = P_.omega;
    const uint64_t m = p_ / omega;
    double mu, lo, hi;
    adjusted_ci(batch_moments(bsum, omega, m), kappa_, P_.conf, &mu, &lo, &hi);
    const double H = std::max(mu - lo, hi - mu);
    if (H > P_.r) {
        kappa_ = grown_kappa(kappa_, H, P_.r);
        if (P_.method == PBN_SEQ_SKART) {
            // the skipped part stays d batches
            if (kappa_ > P_.cap) return not_converged(chain_len);
            base_ = d_ * kappa_;
        }
        if (!batches_fit()) {
            not_converged(chain_len);
            if (P_.method == PBN_SKART) {
                res_.kappa = kappa_;
                res_.batches = p_;
            }
            return;
        }
        ask_batch();
        return;
    }
    res_.prob = mu;
    res_.ci_lo = lo;
    res_.ci_hi = hi;
    res_.kappa = kappa_;
    res_.batches = p_;
    res_.n = kappa_ * m;
    res_.sample_size = kappa_ * p_;
    res_.chain_len = base_ + res_.n;
    res_.psi = base_;
    done_ = true;
}

// p batches of kappa positions from base fit under the cap, and their
// kappa p observations within the exact-moment limit.
bool Machine::batches_fit() const
{
    const uint64_t m = p_ / P_.omega;
    if (kappa_ > P_.cap || m > P_.cap) return false;
    return base_ + kappa_ * m <= P_.cap && (double)kappa_ * (double)p_ <= (double)PBN_SKART_MAX_OBS;
}

void Machine::finish_two_state(int64_t T1)
{
    res_.psi = psi_;
    res_.n = n_;
    res_.N = N_;
    res_.sample_size = (uint64_t)P_.omega * n_;
    res_.prob = (double)T1 / (double)((uint64_t)P_.omega * n_);
    res_.chain_len = psi_ + n_;
    done_ = true;
}

// ------------------------------------------------------------ simulations

namespace {
size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

size_t sim_bytes(const Net &net, uint32_t omega, uint32_t max_props, uint64_t max_len)
{
    // within these limits the products below stay far from 2^64
    if (omega > PBN_MAX_CHAINS || max_props > kMaxProps || max_len > PBN_MAX_LEN) return 0;
    const uint64_t words_cap = (max_len + 31) / 32 + 1;
    return a256(sizeof(DevSim)) + a256(net.blob_bytes) + a256((size_t)net.W * omega * 4) +
           a256((size_t)std::max<uint32_t>(max_props, 1) * words_cap * omega * 4);
}

int sim_setup(pbn_sim *sim, const Net &net, uint32_t omega, uint64_t seed, uint32_t max_props,
              uint64_t max_len, void *dev_buf, size_t dev_bytes, hipStream_t stream, std::string &err, bool reset)
{
    if (omega < 1) { err = "omega must be >= 1"; return PBN_EINVAL; }
    if (max_props > kMaxProps) { err = "too many state sets"; return PBN_ELIMIT; }
    if (omega > PBN_MAX_CHAINS) { err = "too many chains"; return PBN_ELIMIT; }
    if (max_len > PBN_MAX_LEN) { err = "max_len beyond 2^32 - 1 positions"; return PBN_ELIMIT; }
    const size_t need = sim_bytes(net, omega, max_props, max_len);
    if (!dev_buf || dev_bytes < need) { err = "device buffer too small"; return PBN_ENOMEM; }
    sim->net = net;
    sim->omega = omega;
    sim->max_props = max_props;
    sim->seed = seed;
    sim->max_len = max_len;
    sim->words_cap = (max_len + 31) / 32 + 1;
    sim->dbuf = (uint8_t *)dev_buf;
    sim->dbytes = dev_bytes;
    sim->stream = stream;
    if (hipGetDevice(&sim->device) != hipSuccess) { err = "hipGetDevice"; return PBN_EDEVICE; }
    uint8_t *p = sim->dbuf;
    sim->d_desc = (DevSim *)p;
    p += a256(sizeof(DevSim));
    uint8_t *blob = p;
    p += a256(net.blob_bytes);
    uint32_t *state = (uint32_t *)p;
    p += a256((size_t)net.W * omega * 4);
    uint32_t *bits = (uint32_t *)p;
    DevSim &d = sim->desc;
    std::memset(&d, 0, sizeof d);
    d.nd_first = (const uint32_t *)(blob + net.off_nd_first);
    d.fn_thr = (const uint32_t *)(blob + net.off_fn_thr);
    d.fn_desc = (const uint32_t *)(blob + net.off_fn_desc);
    d.fn_tt = (const uint32_t *)(blob + net.off_fn_tt);
    d.tt_ext = (const uint32_t *)(blob + net.off_tt_ext);
    d.par = (const uint16_t *)(blob + net.off_par);
    d.state = state;
    d.bits = bits;
    d.words_cap = sim->words_cap;
    d.n = net.n;
    d.W = net.W;
    d.p_thr = net.p_thr;
    d.omega = omega;
    d.key0 = (uint32_t)seed;
    d.key1 = (uint32_t)(seed >> 32);
    d.nprops = 0;
    d.nd_info = (const uint32_t *)(blob + net.off_nd_info);
    d.blk_sel = (const uint32_t *)(blob + net.off_blk_sel);
    d.fs_rec = (const uint32_t *)(blob + net.off_fs_rec);
    d.fg_K = (const uint32_t *)(blob + net.off_fg_K);
    d.F_pad = net.F_pad;
    d.msel_total = net.msel_total;
    d.nblk = net.nblk;
    if (hipMemcpyAsync(blob, net.blob.data(), net.blob_bytes, hipMemcpyHostToDevice, stream) != hipSuccess) {
        err = "blob upload";
        return PBN_EDEVICE;
    }
    return reset ? sim_reset(sim, nullptr, 0, stream, err) : PBN_OK;
}

int sim_prepare_reset(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops, std::string &err)
{
    if (nprops > sim->max_props) { err = "more state sets than max_props"; return PBN_EINVAL; }
    DevSim &d = sim->desc;
    uint32_t nt = 0;
    d.prop_off[0] = 0;
    for (uint32_t q = 0; q < nprops; ++q) {
        // group the terms of a conjunction by state word: (s[word] & mask) == value
        struct WordTerm { uint32_t word, mask, val; bool empty; };
        std::vector<WordTerm> words;
        for (uint32_t m = 0; m < props[q].nterms; ++m) {
            const uint32_t v = props[q].node[m];
            if (v >= sim->net.n) { err = "state-set node out of range"; return PBN_EINVAL; }
            const uint32_t w = v >> 5, bit = 1u << (v & 31);
            auto it = std::find_if(words.begin(), words.end(), [&](const WordTerm &e) { return e.word == w; });
            if (it == words.end()) { words.push_back({w, 0u, 0u, false}); it = words.end() - 1; }
            const uint32_t want = props[q].val[m] ? bit : 0u;
            // a node asked to be both 0 and 1 makes the set empty, whatever follows
            if ((it->mask & bit) && ((it->val & bit) != want)) it->empty = true;
            it->mask |= bit;
            it->val |= want & it->mask;
        }
        for (auto &e : words) {
            if (nt >= kMaxTerms) { err = "too many state-set terms"; return PBN_ELIMIT; }
            d.term_word[nt] = e.word;
            // an empty set: a value bit outside the mask never matches
            d.term_mask[nt] = e.empty ? 0u : e.mask;
            d.term_val[nt] = e.empty ? 1u : e.val;
            ++nt;
        }
        d.prop_off[q + 1] = nt;
    }
    // the same sets as (node, value) terms for the bit-sliced kernel
    uint32_t nn = 0;
    d.pn_off[0] = 0;
    for (uint32_t q = 0; q < nprops; ++q) {
        for (uint32_t m = 0; m < props[q].nterms; ++m) {
            if (nn >= kMaxTerms) { err = "too many state-set terms"; return PBN_ELIMIT; }
            d.pn_node[nn] = props[q].node[m];
            d.pn_val[nn] = props[q].val[m] ? 1u : 0u;
            ++nn;
        }
        d.pn_off[q + 1] = nn;
    }
    d.nprops = nprops;
    d.nterms = nt;
    sim->nprops = nprops;
    sim->len = 0;
    sim->t_done = 0;
    return PBN_OK;
}

int sim_reset(pbn_sim *sim, const pbn_pattern *props, uint32_t nprops, hipStream_t stream, std::string &err)
{
    int rc = sim_prepare_reset(sim, props, nprops, err);
    if (rc) return rc;
    if (hipMemcpyAsync(sim->d_desc, &sim->desc, sizeof(DevSim), hipMemcpyHostToDevice, stream) != hipSuccess) {
        err = "descriptor upload";
        return PBN_EDEVICE;
    }
    // the copy reads pageable memory that the next reset rewrites
    if (hipStreamSynchronize(stream) != hipSuccess) { err = "sync"; return PBN_EDEVICE; }
    return launch_init(sim->d_desc, sim->omega, sim->net.W, stream, err);
}

int sims_reset_batch(pbn_sim *const *sims, uint32_t count, const pbn_pattern *props, const uint32_t *nprops,
                     const uint32_t *prop_off, Workspace &ws, hipStream_t stream, std::string &err)
{
    int rc = ws.ensure_stage(count, err);
    if (rc) return rc;
    for (uint32_t i = 0; i < count; ++i) {
        if ((rc = sim_prepare_reset(sims[i], props + prop_off[i], nprops[i], err))) return rc;
        ws.h_stage[i] = sims[i]->desc;
        ws.h_dst[i] = sims[i]->d_desc;
    }
    // h_stage is pinned and rewritten only by the next batch, after its predecessor synchronised
    if (hipMemcpyAsync(ws.d_stage, ws.h_stage, count * sizeof(DevSim), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(ws.d_dst, ws.h_dst, count * sizeof(DevSim *), hipMemcpyHostToDevice, stream) != hipSuccess) {
        err = "descriptor upload";
        return PBN_EDEVICE;
    }
    return launch_setup(ws.d_stage, ws.d_dst, count, stream, err);
}


void sim_extend_items(pbn_sim *sim, uint64_t burn_in, uint64_t steps, uint32_t thin,
                      std::vector<StepItem> &items, int shape)
{
    for (uint32_t c0 = 0; c0 < sim->omega; c0 += 64) {
        StepItem it{};
        it.sim = sim->d_desc;
        it.chain0 = c0;
        it.nchains = std::min<uint32_t>(64, sim->omega - c0);
        it.t0 = (uint32_t)sim->t_done;
        it.nburn = (uint32_t)burn_in;
        it.nrec = (uint32_t)steps;
        it.thin = thin;
        it.pos0 = sim->len;
        it.nodes = sim->net.n;
        it.ops_per_step = (float)sim->net.ops_per_step;
        it.philox_per_step = (float)sim->net.philox_per_step;
        it.owner = sim;
        choose_kernel(sim, it, shape);
        items.push_back(it);
    }
    sim->t_done += burn_in + steps * thin;
    sim->len += steps;
}

// Kernel choice per item: the bit-sliced kernel when every predictor has
// k <= 6 and its LDS fits, else the lane-per-chain kernel.  The waves per
// 64-chain block follow measured kernel times on the device (65536 chains, one
// network alone, and the batched solve):
//   latency (the chip holds every block of the work at once): 2 waves below 40
//     nodes, 8 below 150, else 16, which shortens each transition's critical
//     path;
//   alone (throughput, one network's launch with the CUs to itself): 2 below
//     40 nodes, 4 below 400, 8 below 1000, else 12.  Waves are spread over a
//     CU's four SIMDs in turn, so multiples of four keep the SIMDs even; more
//     waves per block give a CU more waves in all within its LDS (8 waves at
//     n = 803: 32 waves per CU against 16, 13% faster; 12 at n = 1500-2000:
//     24 against 16, 12-17%);
//   shared (throughput, many networks of mixed sizes: the batched lanes and
//     server rounds): 2 below 40 nodes, 4 below 900, else 8.  There the alone
//     shapes are slower (61 -> 64-74 ms per 512-network solve): more block
//     shapes mean more launches per round, and wider blocks leave less room
//     for the others'.
// kernel_mode forces one kernel or wave count (testing and tuning).
// Process-wide settings, read by launches on any thread.
namespace {
std::atomic<int> g_kernel_mode{0};     // 0 auto, 1 lane-per-chain, 2 bit-sliced
std::atomic<uint32_t> g_waves_override{0};
}  // namespace

void set_kernel_mode(int mode, uint32_t waves)
{
    g_kernel_mode = mode;
    g_waves_override = waves;
}

namespace {
std::atomic<uint32_t> g_split_mode{0};
std::atomic<uint32_t> g_split_spins{kSplitSpins};
}  // namespace

void set_split_mode(uint32_t parts) { g_split_mode = parts; }
void set_split_spins(uint32_t polls) { g_split_spins = polls ? polls : kSplitSpins; }

uint64_t latency_waves(const pbn_sim *sim)
{
    StepItem probe{};
    choose_kernel(sim, probe, kShapeLatency);
    return (uint64_t)((sim->omega + 63) / 64) * (probe.kernel ? probe.kernel : 1);
}

uint32_t waves_for(uint32_t n, int shape)
{
    uint32_t G = 0;
    if (tuned_waves(n, shape, &G)) return G;
    if (shape == kShapeLatency) return n < 40 ? 2 : n < 150 ? 8 : 16;
    if (shape == kShapeAlone) return n < 40 ? 2 : n < 400 ? 4 : n < 1000 ? 8 : 12;
    return n < 40 ? 2 : n < 900 ? 4 : 8;
}

int kernel_mode_of(const pbn_sim *sim) { return sim && sim->kmode >= 0 ? sim->kmode : g_kernel_mode.load(); }
uint32_t waves_override_of(const pbn_sim *sim) { return sim && sim->kmode >= 0 ? sim->kwaves : g_waves_override.load(); }
uint32_t split_mode_of(const pbn_sim *sim) { return sim && sim->split >= 0 ? (uint32_t)sim->split : g_split_mode.load(); }

void choose_kernel(const pbn_sim *sim, StepItem &it, int shape)
{
    const Net &net = sim->net;
    it.kernel = 0;
    it.lds = 0;
    it.small = 0;
    if (kernel_mode_of(sim) == 1 || !net.bitsliced) return;
    const uint32_t forced = waves_override_of(sim);
    uint32_t G = forced ? forced : waves_for(net.n, shape);
    size_t lds = bs_lds_bytes(net.n, net.msel_total, G);
    // a shape whose LDS does not fit falls back to fewer waves (12 to 8, then halves)
    while (lds > 160 * 1024 && G > 1 && !forced) {
        G = G > 8 ? 8 : G / 2;
        lds = bs_lds_bytes(net.n, net.msel_total, G);
    }
    if (lds > 160 * 1024) return;
    it.kernel = G;
    it.lds = (uint32_t)lds;
    it.small = net.nblk <= G && net.F_pad <= 64 * G;
}

namespace {

// The process-wide pools live until the process ends and are never destroyed:
// a static destructor would call the HIP runtime (stream and event
// destruction) while the process shuts down, when the runtime or a tool
// attached to it may already be gone; the driver reclaims them at exit.
StreamPool &stream_pool()
{
    static StreamPool *p = new StreamPool;
    return *p;
}
}  // namespace

int StreamPool::init(std::string &err)
{
    if (ready) return PBN_OK;
    for (int i = 0; i < kN; ++i) {
        const hipError_t e = cu_mask.empty()
                                 ? hipStreamCreateWithFlags(&s[i], hipStreamNonBlocking)
                                 : hipExtStreamCreateWithCUMask(&s[i], (uint32_t)cu_mask.size(), cu_mask.data());
        if (e != hipSuccess || hipEventCreateWithFlags(&join[i], hipEventDisableTiming) != hipSuccess) {
            err = "stream pool";
            return PBN_EDEVICE;
        }
    }
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) { err = "stream pool"; return PBN_EDEVICE; }
    ready = true;
    return PBN_OK;
}

void StreamPool::release()
{
    if (!ready) return;
    for (int i = 0; i < kN; ++i) {
        (void)hipStreamSynchronize(s[i]);
        (void)hipStreamDestroy(s[i]);
        (void)hipEventDestroy(join[i]);
    }
    (void)hipEventDestroy(fork);
    ready = false;
}

namespace {



// Node-split tables of sim for P parts, built and uploaded on first use.
int split_table(pbn_sim *sim, uint32_t P, pbn_sim::SplitTab &out, std::string &err)
{
    for (const pbn_sim::SplitTab &t : sim->split_tabs)
        if (t.P == P) {
            out = t;
            return PBN_OK;
        }
    const Net &net = sim->net;
    std::vector<uint32_t> tab;
    build_split_tables(net, P, tab);
    pbn_sim::SplitTab t;
    t.P = P;
    t.groups = tab[2 * P + 1];
    for (uint32_t r = 0; r < P; ++r) {
        const uint32_t i_lo = 16 * tab[r], i_hi = std::min(net.n, 16 * tab[r + 1]);
        const uint32_t m_lo = net.nd_meta[i_lo] >> 8, m_hi = i_hi < net.n ? net.nd_meta[i_hi] >> 8 : net.msel_total;
        t.n_own = std::max(t.n_own, i_hi - i_lo);
        t.m_own = std::max(t.m_own, m_hi - m_lo);
    }
    if (hipMalloc((void **)&t.d_tab, tab.size() * sizeof(uint32_t)) != hipSuccess) {
        err = "node-split tables";
        return PBN_ENOMEM;
    }
    if (hipMemcpy(t.d_tab, tab.data(), tab.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(t.d_tab);
        err = "node-split table upload";
        return PBN_EDEVICE;
    }
    sim->split_tabs.push_back(t);
    out = t;
    return PBN_OK;
}

// Spread latency-bound 64-chain groups over several CUs.  Automatic: while
// the launch has fewer blocks than the chip has CUs, the spare CUs go, one
// part at a time, to the group with the largest remaining work per part
// (node count x transitions / parts), each group taking at most 16 parts of
// at least 8 node blocks; every block of the launch then has a CU of its own,
// so a group's parts are resident together.  Forced: P parts for every
// bit-sliced group (at most one per node block).  The parts of a node-split
// group are marked small = 2.
int split_expand(std::vector<StepItem> &items, Workspace &ws, std::string &err, size_t &ngroups, size_t kCus)
{
    ngroups = 0;
    std::vector<uint32_t> parts(items.size(), 1);
    {
        std::vector<size_t> cand;
        // forced: every group that still keeps the launch within one block
        // per CU (the parts of a group must all be resident at once)
        size_t blocks = items.size();
        for (size_t i = 0; i < items.size(); ++i) {
            const StepItem &it = items[i];
            if (it.kernel == 0 || !it.owner || it.nchains == 0) continue;
            const pbn_sim *owner = (const pbn_sim *)it.owner;
            const uint32_t nblk = owner->net.nblk, mode = split_mode_of(owner);
            if (mode == 1) continue;
            if (mode >= 2) {
                const uint32_t P = std::min(std::min(mode, kSplitMaxParts), nblk);
                if (P >= 2 && blocks + P - 1 <= kCus) {
                    parts[i] = P;
                    blocks += P - 1;
                }
            } else {
                cand.push_back(i);
            }
        }
        bool hinted = false;
        for (size_t i : cand)
            if (items[i].parts_hint >= 2) {
                parts[i] = std::min(items[i].parts_hint, kSplitMaxParts);
                hinted = true;
            }
        if (!hinted && items.size() < kCus && !cand.empty()) {
            auto work = [&](size_t i) {
                const StepItem &it = items[i];
                return (double)it.nodes * (double)(it.nburn + (uint64_t)it.nrec * it.thin) / (double)parts[i];
            };
            auto cap = [&](size_t i) {
                return std::min<uint32_t>(kSplitMaxParts, ((const pbn_sim *)items[i].owner)->net.nblk / 8);
            };
            auto lower = [&](size_t a, size_t b) { return work(a) < work(b); };
            std::priority_queue<size_t, std::vector<size_t>, decltype(lower)> pq(lower);
            for (size_t i : cand)
                if (cap(i) >= 2) pq.push(i);
            size_t spare = kCus - items.size();
            while (spare > 0 && !pq.empty()) {
                const size_t i = pq.top();
                pq.pop();
                ++parts[i];
                --spare;
                if (parts[i] < cap(i)) pq.push(i);
            }
        }
    }
    struct Plan {
        size_t idx;
        uint32_t P, G, lds;
        pbn_sim::SplitTab tab;
    };
    std::vector<Plan> plan;
    size_t xwords = 0, extra = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        const uint32_t P = parts[i];
        if (P < 2) continue;
        pbn_sim *sim = (pbn_sim *)items[i].owner;
        const uint32_t nblk = sim->net.nblk;
        const uint32_t per = (nblk + P - 1) / P;
        uint32_t G = 16;
        while (G > 1 && G > per) G /= 2;
        const uint32_t forced = waves_override_of(sim);
        if (forced) G = forced;
        pbn_sim::SplitTab tab;
        int rc = split_table(sim, P, tab, err);
        if (rc) return rc;
        size_t lds = split_lds_bytes(sim->net.n, tab.n_own, tab.m_own, G);
        while (lds > 160 * 1024 && G > 1 && !forced) {
            G /= 2;
            lds = split_lds_bytes(sim->net.n, tab.n_own, tab.m_own, G);
        }
        if (lds > 160 * 1024) continue;
        plan.push_back(Plan{i, P, G, (uint32_t)lds, tab});
        xwords += split_xch_words(sim->net.n, P);
        extra += P - 1;
    }
    if (plan.empty()) return PBN_OK;
    int rc = ws.ensure_split(plan.size(), xwords, err);
    if (rc) return rc;
    ws.split_items.clear();
    std::vector<StepItem> out;
    out.reserve(items.size() + extra);
    std::vector<int> which(items.size(), -1);
    for (size_t q = 0; q < plan.size(); ++q) which[plan[q].idx] = (int)q;
    size_t xoff = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        if (which[i] < 0) {
            out.push_back(items[i]);
            continue;
        }
        const size_t q = (size_t)which[i];
        const Plan &p = plan[q];
        const pbn_sim *sim = (const pbn_sim *)items[i].owner;
        SplitGroup &g = ws.h_grp[q];
        g.tab = p.tab.d_tab;
        g.xch = ws.d_xch + xoff;
        g.stat = ws.d_stat + q;
        g.nparts = p.P;
        g.groups = p.tab.groups;
        g.spins = g_split_spins;
        g.pad_ = 0;
        xoff += split_xch_words(sim->net.n, p.P);
        // the whole group in its one-block latency shape, should it give up
        StepItem whole = items[i];
        choose_kernel(sim, whole, true);
        whole.part = 0;
        whole.grp = nullptr;
        whole.parts_hint = 0;
        ws.split_items.push_back(whole);
        for (uint32_t r = 0; r < p.P; ++r) {
            StepItem s = items[i];
            s.part = r;
            s.grp = ws.d_grp + q;
            s.kernel = p.G;
            s.lds = p.lds;
            s.small = 2;
            out.push_back(s);
        }
    }
    items.swap(out);
    ngroups = plan.size();
    ws.xch_used = xoff;
    return PBN_OK;
}

}  // namespace

int launch_items(std::vector<StepItem> &items, Workspace &ws, hipStream_t stream, std::string &err,
                 bool allow_fork, bool allow_split, uint32_t cus, StreamPool *pool)
{
    if (items.empty()) return PBN_OK;
    int rc = ws.before_write(ws.ev_items, ws.items_in_flight, err);
    if (rc) return rc;
    size_t nsplit = 0;
    if (allow_split && (rc = split_expand(items, ws, err, nsplit, cus))) return rc;
    // groups of equal kernel form; inside a group the longest
    // items first, since the hardware dispatches blocks roughly in order
    struct Key { uint32_t kernel, cls; double cost; size_t idx; };
    std::vector<Key> keys(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
        const StepItem &it = items[i];
        // one launch per kernel form: separate launches of one lane run one
        // after the other, and each one's tail costs more than the residency a
        // smaller LDS size would gain
        keys[i] = Key{it.kernel, it.kernel ? (it.small << 16) : 0u,
                      (double)(it.nburn + (uint64_t)it.nrec * it.thin) * (double)it.nodes, i};
    }
    std::stable_sort(keys.begin(), keys.end(), [](const Key &a, const Key &b) {
        if (a.kernel != b.kernel) return a.kernel < b.kernel;
        if (a.cls != b.cls) return a.cls < b.cls;
        return a.cost > b.cost;
    });
    struct Group { size_t first, count; uint32_t kernel, cls, lds, maxW; double cost; };
    std::vector<Group> groups;
    std::vector<StepItem> laid;
    laid.reserve(items.size() + 64);
    for (size_t a = 0; a < keys.size();) {
        size_t b = a;
        while (b < keys.size() && keys[b].kernel == keys[a].kernel && keys[b].cls == keys[a].cls) ++b;
        Group g{laid.size(), 0, keys[a].kernel, keys[a].cls, 0, 1, 0.0};
        for (size_t i = a; i < b; ++i) {
            const StepItem &it = items[keys[i].idx];
            g.lds = std::max(g.lds, it.lds);
            g.maxW = std::max(g.maxW, (it.nodes + 31) / 32);
            g.cost += keys[i].cost * it.nchains;
        }
        // (not for node-split parts: in launch order, block i on XCD i mod 8,
        // a launch of at most 256 blocks has a CU for every part at once)
        if (g.kernel != 0 && (g.cls >> 16) != 2 && b - a >= 2 * kXcds) {
            // XCD-aware placement: block i of a launch runs on XCD i mod 8, so
            // all blocks of one network go to one XCD (its records then live in
            // one L2), networks spread over the XCDs by cost; short lists are
            // padded with empty items, which exit at once
            std::vector<std::vector<size_t>> per_sim;
            std::vector<double> sim_cost;
            std::vector<const DevSim *> sim_of;
            for (size_t i = a; i < b; ++i) {
                const DevSim *sp = items[keys[i].idx].sim;
                size_t s_idx = 0;
                while (s_idx < sim_of.size() && sim_of[s_idx] != sp) ++s_idx;
                if (s_idx == sim_of.size()) {
                    sim_of.push_back(sp);
                    per_sim.emplace_back();
                    sim_cost.push_back(0.0);
                }
                per_sim[s_idx].push_back(keys[i].idx);
                sim_cost[s_idx] += keys[i].cost * items[keys[i].idx].nchains;
            }
            std::vector<size_t> sord(per_sim.size());
            for (size_t i = 0; i < sord.size(); ++i) sord[i] = i;
            std::stable_sort(sord.begin(), sord.end(), [&](size_t x, size_t y) { return sim_cost[x] > sim_cost[y]; });
            // a network stays on one XCD while that XCD is under its share of
            // the group's cost; a network larger than a share spills its
            // remaining blocks onto the least loaded XCDs
            std::vector<std::vector<size_t>> xl(kXcds);
            std::vector<double> load(kXcds, 0.0);
            double total = 0.0;
            for (double c : sim_cost) total += c;
            const double share = total / (double)kXcds;
            for (size_t si : sord) {
                size_t x = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
                for (size_t idx : per_sim[si]) {
                    const double c = (double)(items[idx].nburn + (uint64_t)items[idx].nrec * items[idx].thin) *
                                     items[idx].nodes * items[idx].nchains;
                    if (load[x] > 0.0 && load[x] + c > share * 1.0001)
                        x = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
                    xl[x].push_back(idx);
                    load[x] += c;
                }
            }
            size_t rows = 0;
            for (auto &l : xl) {
                std::stable_sort(l.begin(), l.end(), [&](size_t x, size_t y) {
                    return (double)(items[x].nburn + (uint64_t)items[x].nrec * items[x].thin) * items[x].nodes >
                           (double)(items[y].nburn + (uint64_t)items[y].nrec * items[y].thin) * items[y].nodes;
                });
                rows = std::max(rows, l.size());
            }
            StepItem empty = items[keys[a].idx];
            empty.nchains = 0;
            empty.nburn = empty.nrec = 0;
            for (size_t r = 0; r < rows; ++r)
                for (size_t x = 0; x < kXcds; ++x) laid.push_back(r < xl[x].size() ? items[xl[x][r]] : empty);
        } else {
            for (size_t i = a; i < b; ++i) laid.push_back(items[keys[i].idx]);
        }
        g.count = laid.size() - g.first;
        groups.push_back(g);
        a = b;
    }
    if ((rc = ws.ensure(laid.size(), 0, 0, err))) return rc;
    for (const Group &g : groups)
        if (g.kernel == 0 && (rc = ws.ensure_rows(step_rows_words((uint32_t)g.count, g.maxW), err))) return rc;
    std::memcpy(ws.h_items, laid.data(), laid.size() * sizeof(StepItem));
    if (hipMemcpyAsync(ws.d_items, ws.h_items, laid.size() * sizeof(StepItem), hipMemcpyHostToDevice,
                       stream) != hipSuccess) {
        err = "item upload";
        return PBN_EDEVICE;
    }
    if (nsplit) {
        if (hipMemcpyAsync(ws.d_grp, ws.h_grp, nsplit * sizeof(SplitGroup), hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            hipMemsetAsync(ws.d_stat, 0, nsplit * sizeof(uint32_t), stream) != hipSuccess ||
            hipMemsetAsync(ws.d_xch, 0, ws.xch_used * sizeof(uint64_t), stream) != hipSuccess) {
            err = "node-split group upload";
            return PBN_EDEVICE;
        }
    }
    if ((rc = ws.after_copy(ws.ev_items, ws.items_in_flight, stream, err))) return rc;
    // one profiling mark per kernel dispatch, on the stream it runs on
    const bool prof_on = profiling();
    auto launch_group = [&](const Group &g, hipStream_t s) -> int {
        const StepItem *d = ws.d_items + g.first;
        ProfileMark mark;
        if (prof_on) {
            for (size_t i = g.first; i < g.first + g.count; ++i) {
                const StepItem &it = ws.h_items[i];
                if (it.small == 2 && it.part != 0) continue;     // a node-split group counts once
                const double cs = (double)(it.nburn + (uint64_t)it.nrec * it.thin) * it.nchains;
                mark.chain_steps += cs;
                mark.node_updates += cs * it.nodes;
                mark.ops += cs * it.ops_per_step;
                mark.philox += cs * it.philox_per_step;
            }
            mark.split = (g.cls >> 16) == 2;
            profile_begin(mark, s);
        }
        const int r = g.kernel == 0           ? launch_step(d, (uint32_t)g.count, g.maxW, ws.d_rows, s, err)
                      : (g.cls >> 16) == 2 ? launch_step_split(d, (uint32_t)g.count, g.kernel, g.lds, s, err)
                                           : launch_step_bs(d, (uint32_t)g.count, g.kernel, (g.cls >> 16) != 0, g.lds, s, err);
        if (prof_on) profile_end(mark, s);
        return r;
    };
    if (groups.size() == 1 || !allow_fork) {
        for (size_t g = 0; g < groups.size() && !rc; ++g) rc = launch_group(groups[g], stream);
    } else {
        // largest groups first, spread over the pool's streams, joined back
        std::sort(groups.begin(), groups.end(), [](const Group &a, const Group &b) { return a.cost > b.cost; });
        StreamPool &P = pool ? *pool : stream_pool();
        std::lock_guard<std::mutex> hold(P.mu);
        if ((rc = P.init(err))) return rc;
        if (hipEventRecord(P.fork, stream) != hipSuccess) { err = "fork event"; return PBN_EDEVICE; }
        const int used = std::min<int>(StreamPool::kN, (int)groups.size());
        for (int k = 0; k < used; ++k)
            if (hipStreamWaitEvent(P.s[k], P.fork, 0) != hipSuccess) { err = "fork wait"; return PBN_EDEVICE; }
        for (size_t g = 0; g < groups.size() && !rc; ++g) rc = launch_group(groups[g], P.s[g % StreamPool::kN]);
        for (int k = 0; k < used; ++k) {
            if (hipEventRecord(P.join[k], P.s[k]) != hipSuccess ||
                hipStreamWaitEvent(stream, P.join[k], 0) != hipSuccess) {
                err = "join";
                return PBN_EDEVICE;
            }
        }
    }
    if (!rc && nsplit) {
        if (hipMemcpyAsync(ws.h_stat, ws.d_stat, nsplit * sizeof(uint32_t), hipMemcpyDeviceToHost, stream) !=
            hipSuccess) {
            err = "node-split status download";
            return PBN_EDEVICE;
        }
        ws.split_used = nsplit;
        ws.split_stream = stream;
        ws.redo_queries = ws.redo_bsum = 0;
    }
    return rc;
}

// ------------------------------------------------------------ profiling

namespace {
struct ProfState {
    uint64_t fallback_base = 0;       // node-split re-runs before the last reset
    std::mutex mu;                    // launches on several threads record marks
    std::atomic<bool> on{false};
    std::vector<ProfileMark> pending;
    std::vector<hipEvent_t> pool;
    pbn_profile acc{};
};
ProfState &prof()
{
    static ProfState p;
    return p;
}
hipEvent_t get_event()
{
    ProfState &p = prof();
    std::lock_guard<std::mutex> hold(p.mu);
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
}  // namespace

bool profiling() { return prof().on; }

void profile_begin(ProfileMark &m, hipStream_t stream)
{
    m.start = get_event();
    m.stop = get_event();
    (void)hipEventRecord(m.start, stream);
}

void profile_end(ProfileMark &m, hipStream_t stream)
{
    (void)hipEventRecord(m.stop, stream);
    ProfState &p = prof();
    std::lock_guard<std::mutex> hold(p.mu);
    p.pending.push_back(m);
}

int profile_collect(pbn_profile *out, std::string &err)
{
    ProfState &p = prof();
    std::lock_guard<std::mutex> hold(p.mu);
    for (ProfileMark &m : p.pending) {
        if (hipEventSynchronize(m.stop) != hipSuccess) { err = "profile event"; return PBN_EDEVICE; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, m.start, m.stop);
        p.acc.launches += 1;
        p.acc.kernel_ms += ms;
        p.acc.chain_steps += m.chain_steps;
        p.acc.node_updates += m.node_updates;
        p.acc.alg_ops += m.ops;
        p.acc.philox_evals += m.philox;
        p.acc.split_launches += m.split ? 1 : 0;
        p.pool.push_back(m.start);
        p.pool.push_back(m.stop);
    }
    p.pending.clear();
    if (out) {
        *out = p.acc;
        out->split_fallbacks = split_fallbacks() - p.fallback_base;
    }
    return PBN_OK;
}

void profile_set(bool on) { prof().on = on; }

void profile_clear()
{
    std::string err;
    profile_collect(nullptr, err);
    ProfState &p = prof();
    std::lock_guard<std::mutex> hold(p.mu);
    p.acc = pbn_profile{};
    p.fallback_base = split_fallbacks();
}

// ------------------------------------------------------------ rounds

bool SimRun::finished() const
{
    for (auto &m : machines)
        if (!m.done()) return false;
    return true;
}

MachineParams make_params(const pbn_sim *sim, const pbn_opts *opts, double r, double conf)
{
    MachineParams p{};
    p.method = opts ? opts->method : PBN_TWO_STATE;
    p.omega = sim->omega;
    p.psi0 = (opts && opts->psi0) ? opts->psi0 : 256;
    p.psrf_max = (opts && opts->psrf_max > 0.0) ? opts->psrf_max : 1.1;
    p.eps = (opts && opts->eps > 0.0) ? opts->eps : 1e-10;
    uint64_t cap = sim->max_len;
    if (opts && opts->max_len && opts->max_len < cap) cap = opts->max_len;
    // Skart batch sums are 32-bit: a batch (at most the whole chain) stays below 2^31 positions
    if (p.method == PBN_SKART || p.method == PBN_SEQ_SKART) cap = std::min<uint64_t>(cap, INT32_MAX);
    p.cap = cap;
    p.r = r;
    p.conf = conf;
    return p;
}

// Transitions of one slice: about tick_us of the step kernel for this network,
// from a model of the per-transition latency of one 64-chain block (the
// per-node work divided over the block's waves), in multiples of 32.
// Per-transition latency of one 64-chain block of this network, fitted to
// single-block timings: about 2.5 us plus 0.17 us per node and wave (0.25 us
// with 16 waves, whose barriers cost more); about 1 us per node for the
// lane-per-chain kernel.
double step_latency_us(const pbn_sim *sim, int shape)
{
    StepItem probe{};
    choose_kernel(sim, probe, shape);
    const double n = sim->net.n;
    const double per = probe.kernel == 16 ? 0.25 : 0.17;
    return probe.kernel ? 2.5 + per * n / probe.kernel : 1.0 + 1.0 * n;
}

// Node-split parts per simulation of one launch: the CUs beyond the launch's
// 64-chain groups go, a part at a time, to the simulation with the most work
// per part (n x transitions / parts); one more part costs one CU per 64-chain
// group of that simulation.  At most kSplitMaxParts parts of at least 8 node
// blocks, bit-sliced networks only.
static void plan_parts(const std::vector<std::pair<pbn_sim *, uint64_t>> &ext, std::vector<uint32_t> &parts,
                       uint64_t kCus)
{
    uint64_t used = 0;
    for (const auto &e : ext) used += (e.first->omega + 63) / 64;
    if (used >= kCus) return;
    uint64_t spare = kCus - used;
    auto cap = [&](size_t k) {
        const Net &net = ext[k].first->net;
        if (split_mode_of(ext[k].first) != 0) return 1u;
        return net.bitsliced ? std::min<uint32_t>(kSplitMaxParts, net.nblk / 8) : 1u;
    };
    auto work = [&](size_t k) { return (double)ext[k].first->net.n * (double)ext[k].second / parts[k]; };
    auto lower = [&](size_t a, size_t b) { return work(a) < work(b); };
    std::priority_queue<size_t, std::vector<size_t>, decltype(lower)> pq(lower);
    for (size_t k = 0; k < ext.size(); ++k)
        if (cap(k) >= 2) pq.push(k);
    while (!pq.empty()) {
        const size_t k = pq.top();
        pq.pop();
        const uint64_t groups = (ext[k].first->omega + 63) / 64;
        if (groups > spare) continue;
        ++parts[k];
        spare -= groups;
        if (parts[k] < cap(k)) pq.push(k);
    }
}

double extension_us(const pbn_sim *sim, uint64_t positions, uint32_t parts)
{
    double us = step_latency_us(sim, kShapeLatency);
    if (parts >= 2 && sim->net.bitsliced && split_mode_of(sim) != 1) us = std::min(us, 6.0 + us / parts);
    return us * (double)sim->thin * (double)positions;
}

// parts: the network's 64-chain groups are spread over that many CUs in the
// node-split form (forced part counts included); a transition then costs
// about 6 us of exchange plus the one-block time over the parts.
uint64_t slice_len(const pbn_sim *sim, double tick_us, int shape, uint32_t parts)
{
    const bool latency = shape == kShapeLatency;
    double us = step_latency_us(sim, shape);
    const uint32_t mode = split_mode_of(sim);
    if (mode >= 2) parts = std::min(std::min(mode, kSplitMaxParts), sim->net.nblk);
    if (latency && parts >= 2 && mode != 1 && sim->net.bitsliced) us = std::min(us, 6.0 + us / parts);
    us *= sim->thin;                  // a slice counts recorded positions, each thin transitions long
    const double q = std::floor(tick_us / us / 32.0) * 32.0;
    return (uint64_t)std::max(32.0, q);
}

int round_begin(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, RoundCtx &ctx, std::string &err,
                const LaunchCfg &cfg, double tick_us, int latency)
{
    ctx.owners.clear();
    ctx.kinds.clear();
    ctx.pending = false;
    if (latency < 0) {
        uint64_t waves = 0;
        for (SimRun *run : runs)
            if (!run->finished()) waves += latency_waves(run->sim);
        latency = waves <= kLatencyWaves;
    }
    // 1. extensions for runs with no request ready at their current length
    std::vector<StepItem> items;
    std::vector<std::pair<pbn_sim *, uint64_t>> ext;
    for (SimRun *run : runs) {
        if (run->finished()) continue;
        pbn_sim *sim = run->sim;
        bool ready = false;
        uint64_t target = UINT64_MAX;
        for (auto &m : run->machines) {
            if (m.done()) continue;
            if (m.request().need_len <= sim->len) ready = true;
            target = std::min(target, m.request().need_len);
        }
        if (!ready) {
            if (target > sim->max_len) { err = "request beyond the bit-stream capacity"; return PBN_ELIMIT; }
            if (target - sim->len > ((1ull << 32) - 1 - sim->t_done) / sim->thin) {
                err = "transition index limit";
                return PBN_ELIMIT;
            }
            ext.push_back({sim, target - sim->len});
        }
    }
    // node-split parts per simulation (time-sliced rounds that own the device),
    // decided before slicing so that each slice is about tick_us long
    std::vector<uint32_t> parts(ext.size(), 1);
    if (tick_us > 0.0 && cfg.split && latency) plan_parts(ext, parts, cfg.cus);
    // one network alone on the device takes its own best shape; several share
    const int shape = latency ? kShapeLatency : cfg.shared || ext.size() > 1 ? kShapeShared : kShapeAlone;
    for (size_t k = 0; k < ext.size(); ++k) {
        pbn_sim *sim = ext[k].first;
        uint64_t e = ext[k].second;
        if (tick_us > 0.0) e = std::min(e, slice_len(sim, tick_us, shape, cfg.split ? parts[k] : 1));
        const size_t first = items.size();
        sim_extend_items(sim, 0, e, sim->thin, items, shape);
        for (size_t i = first; i < items.size(); ++i) items[i].parts_hint = parts[k];
    }
    int rc = launch_items(items, ws, stream, err, cfg.fork, cfg.split, cfg.cus, cfg.pool);
    if (rc) return rc;
    // 2. queries for every ready request
    std::vector<Query> qs;
    uint64_t bsum_total = 0;
    for (SimRun *run : runs) {
        for (size_t mi = 0; mi < run->machines.size(); ++mi) {
            Machine &m = run->machines[mi];
            if (m.done() || m.request().need_len > run->sim->len) continue;
            const Request &rq = m.request();
            Query q{};
            q.sim = run->sim->d_desc;
            q.prop = m.prop();
            q.kind = rq.kind;
            q.lo = rq.lo;
            q.hi = rq.hi;
            q.kappa = rq.kappa;
            q.m = rq.m;
            q.out_off = bsum_total;
            if (rq.kind == kQueryBatch) bsum_total += (uint64_t)run->sim->omega * rq.m;
            ctx.owners.push_back({run, mi, q.out_off});
            ctx.kinds.push_back(rq.kind);
            qs.push_back(q);
        }
    }
    if (qs.empty() && items.empty()) return PBN_OK;
    if (qs.empty()) {
        // extension only: the round still completes on an event, since the
        // next round rewrites the pinned item table this one copies from
        if (!ctx.done && hipEventCreateWithFlags(&ctx.done, hipEventDisableTiming) != hipSuccess) {
            err = "round event";
            return PBN_EDEVICE;
        }
        if (hipEventRecord(ctx.done, stream) != hipSuccess) { err = "round event"; return PBN_EDEVICE; }
        ctx.pending = true;
        return PBN_OK;
    }
    if ((rc = ws.before_write(ws.ev_queries, ws.queries_in_flight, err))) return rc;
    if ((rc = ws.ensure(0, qs.size(), bsum_total, err))) return rc;
    std::memcpy(ws.h_queries, qs.data(), qs.size() * sizeof(Query));
    if (hipMemcpyAsync(ws.d_queries, ws.h_queries, qs.size() * sizeof(Query), hipMemcpyHostToDevice, stream) !=
        hipSuccess) { err = "query upload"; return PBN_EDEVICE; }
    if ((rc = ws.after_copy(ws.ev_queries, ws.queries_in_flight, stream, err))) return rc;
    if ((rc = launch_reduce(ws.d_queries, (uint32_t)qs.size(), ws.d_win, ws.d_bsum, stream, err))) return rc;
    if (ws.split_used) {
        // a node-split group re-run after a give-up repeats this reduction
        ws.redo_queries = qs.size();
        ws.redo_bsum = bsum_total;
    }
    if (hipMemcpyAsync(ws.h_win, ws.d_win, qs.size() * sizeof(WindowResult), hipMemcpyDeviceToHost, stream) !=
        hipSuccess) { err = "result download"; return PBN_EDEVICE; }
    if (bsum_total && hipMemcpyAsync(ws.h_bsum, ws.d_bsum, bsum_total * sizeof(int32_t), hipMemcpyDeviceToHost,
                                     stream) != hipSuccess) { err = "batch download"; return PBN_EDEVICE; }
    if (!ctx.done && hipEventCreateWithFlags(&ctx.done, hipEventDisableTiming) != hipSuccess) {
        err = "round event";
        return PBN_EDEVICE;
    }
    if (hipEventRecord(ctx.done, stream) != hipSuccess) { err = "round event"; return PBN_EDEVICE; }
    ctx.pending = true;
    return PBN_OK;
}

int ahead_begin(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, const LaunchCfg &cfg,
                double tick_us, double min_left_us, bool *launched, std::string &err)
{
    *launched = false;
    // runs still short of their pending requirement by more than min_left_us
    // of kernel time, after the round queued before
    std::vector<std::pair<pbn_sim *, uint64_t>> ext;
    uint64_t waves = 0;
    for (SimRun *run : runs) {
        if (run->finished()) continue;
        pbn_sim *sim = run->sim;
        uint64_t target = UINT64_MAX;
        for (auto &m : run->machines)
            if (!m.done()) target = std::min(target, m.request().need_len);
        if (target == UINT64_MAX || target <= sim->len || target > sim->max_len) continue;
        if (target - sim->len > ((1ull << 32) - 1 - sim->t_done) / sim->thin) continue;
        if (extension_us(sim, target - sim->len, kSplitMaxParts) < min_left_us) continue;
        ext.push_back({sim, target - sim->len});
        waves += latency_waves(sim);
    }
    if (ext.empty() || waves > kLatencyWaves) return PBN_OK;
    std::vector<uint32_t> parts(ext.size(), 1);
    if (cfg.split) plan_parts(ext, parts, cfg.cus);
    std::vector<StepItem> items;
    for (size_t k = 0; k < ext.size(); ++k) {
        pbn_sim *sim = ext[k].first;
        const uint64_t e = std::min(ext[k].second, slice_len(sim, tick_us, kShapeLatency, cfg.split ? parts[k] : 1));
        const size_t first = items.size();
        sim_extend_items(sim, 0, e, sim->thin, items, kShapeLatency);
        for (size_t i = first; i < items.size(); ++i) items[i].parts_hint = parts[k];
    }
    const int rc = launch_items(items, ws, stream, err, cfg.fork, cfg.split, cfg.cus, cfg.pool);
    if (!rc) *launched = true;
    return rc;
}

void round_end(Workspace &ws, RoundCtx &ctx)
{
    for (size_t i = 0; i < ctx.owners.size(); ++i) {
        Machine &m = ctx.owners[i].run->machines[ctx.owners[i].mi];
        const uint64_t L = ctx.owners[i].run->sim->len;
        if (ctx.kinds[i] == kQueryWindow) m.feed_window(ws.h_win[i], L);
        else m.feed_batch(ws.h_bsum + ctx.owners[i].off, L);
    }
    ctx.owners.clear();
    ctx.kinds.clear();
    ctx.pending = false;
}

int run_round(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, std::string &err, double tick_us,
              const LaunchCfg &cfg)
{
    RoundCtx ctx;
    int rc = round_begin(runs, ws, stream, ctx, err, cfg, tick_us);
    if (!rc && ctx.pending) {
        hipError_t e = hipEventSynchronize(ctx.done);
        if (e != hipSuccess) { err = std::string("round sync: ") + hipGetErrorString(e); rc = PBN_EDEVICE; }
        else if (!(rc = ws.check_split(err))) round_end(ws, ctx);
    }
    if (ctx.done) (void)hipEventDestroy(ctx.done);
    return rc;
}

int run_to_completion(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, std::string &err)
{
    for (;;) {
        bool all = true;
        for (SimRun *r : runs)
            if (!r->finished()) { all = false; break; }
        if (all) return PBN_OK;
        int rc = run_round(runs, ws, stream, err);
        if (rc) return rc;
    }
}

// Lanes: one stream each, every lane with its own asynchronous round loop.
//   - express lane (the caller's stream): the few networks whose first round
//     alone is a large share of the whole batch's expected time (the longest
//     serial paths), unsliced, so their decisions and continuations overlap
//     the bulk instead of following it;
//   - three class lanes (own streams: the hardware queues left beside the
//     caller's): the rest by step-kernel class (8 waves, 4 waves, the others,
//     for throughput), so one launch serves one class; an empty lane takes
//     half of the busiest one.  Their rounds are time-sliced: an extension
//     advances at most about kTickUs of kernel time per round, so a network
//     that needs a long extension never holds back the decisions of the
//     others in its lane, and every round returns the results of the networks
//     whose extension completed in it.
namespace {
struct Lane {
    std::vector<SimRun *> runs;
    hipStream_t stream = nullptr;
    Workspace ws;
    RoundCtx ctx;
    bool finished() const
    {
        for (SimRun *r : runs)
            if (!r->finished()) return false;
        return true;
    }
};
// One batched solve at a time: its lanes and events are shared.
struct LanePool {
    static constexpr int kN = 3;
    std::mutex mu;
    hipEvent_t ev[kN] = {};
    std::vector<std::unique_ptr<Lane>> lane;
    Lane express;                     // runs on the caller's stream
    bool ready = false;
    int init(std::string &err)
    {
        if (ready) return PBN_OK;
        for (int i = 0; i < kN; ++i) {
            lane.emplace_back(new Lane());
            if (hipStreamCreateWithFlags(&lane.back()->stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
                err = "lane streams";
                return PBN_EDEVICE;
            }
        }
        ready = true;
        return PBN_OK;
    }
};
LanePool &lane_pool()
{
    static LanePool *p = new LanePool;    // never destroyed, as the stream pool
    return *p;
}
}  // namespace

int run_lanes(std::vector<SimRun *> &runs, Workspace &ws, hipStream_t stream, std::string &err)
{
    if (runs.size() < 2) return run_to_completion(runs, ws, stream, err);
    LanePool &P = lane_pool();
    std::lock_guard<std::mutex> hold(P.mu);
    int rc = P.init(err);
    if (rc) return rc;
    const int nl = LanePool::kN;
    for (int k = 0; k < nl; ++k) P.lane[k]->runs.clear();
    P.express.runs.clear();
    P.express.stream = stream;
    std::vector<SimRun *> order(runs);
    std::stable_sort(order.begin(), order.end(),
                     [](const SimRun *a, const SimRun *b) { return a->sim->net.n < b->sim->net.n; });
    // express: first-round serial time above a quarter of the batch's expected
    // time at about 8e11 node-updates/s, at most 8 networks, only with a bulk
    // of at least 8 others beside them
    {
        std::vector<std::pair<double, SimRun *>> crit;
        double bulk_us = 0.0;
        for (SimRun *r : order) {
            const uint64_t first = r->machines.empty() ? 0 : r->machines[0].request().need_len;
            bulk_us += (double)r->sim->net.n * r->sim->omega * (double)first / 8e5;
        }
        for (SimRun *r : order) {
            const uint64_t first = r->machines.empty() ? 0 : r->machines[0].request().need_len;
            const double serial = (double)first * step_latency_us(r->sim, kShapeShared);
            if (serial > 0.25 * bulk_us) crit.push_back({serial, r});
        }
        std::stable_sort(crit.begin(), crit.end(),
                         [](const std::pair<double, SimRun *> &a, const std::pair<double, SimRun *> &b) {
                             return a.first > b.first;
                         });
        if (crit.size() > 8) crit.resize(8);
        if (order.size() >= crit.size() + 8) {
            for (auto &c : crit) P.express.runs.push_back(c.second);
            std::vector<SimRun *> rest;
            for (SimRun *r : order)
                if (std::find(P.express.runs.begin(), P.express.runs.end(), r) == P.express.runs.end())
                    rest.push_back(r);
            order.swap(rest);
        }
    }
    for (SimRun *r : order) {
        StepItem probe{};
        choose_kernel(r->sim, probe, kShapeShared);
        const int k = probe.kernel >= 8 ? 0 : probe.kernel >= 4 ? 1 : 2;
        P.lane[k]->runs.push_back(r);
    }
    auto work = [](const Lane &L) {
        double w = 0.0;
        for (const SimRun *r : L.runs) w += (double)r->sim->net.n * r->sim->omega;
        return w;
    };
    for (int k = 0; k < nl; ++k) {
        if (!P.lane[k]->runs.empty()) continue;
        int big = 0;
        for (int j = 1; j < nl; ++j)
            if (work(*P.lane[j]) > work(*P.lane[big])) big = j;
        std::vector<SimRun *> &from = P.lane[big]->runs;
        if (from.size() < 2) continue;
        std::vector<SimRun *> keep;
        for (size_t i = 0; i < from.size(); ++i) (i % 2 ? P.lane[k]->runs : keep).push_back(from[i]);
        from.swap(keep);
    }
    // lane streams start after everything queued so far on the caller's stream
    hipEvent_t start;
    if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess) { err = "event"; return PBN_EDEVICE; }
    (void)hipEventRecord(start, stream);
    for (int k = 0; k < nl; ++k) (void)hipStreamWaitEvent(P.lane[k]->stream, start, 0);
    for (;;) {
        bool any_pending = false, all_done = true;
        // latency mode once the unfinished work fits on the chip at once
        uint64_t waves = 0;
        for (SimRun *r : runs)
            if (!r->finished()) waves += latency_waves(r->sim);
        const int latency = waves <= kLatencyWaves;
        // a small express remainder runs in its latency shape beside the bulk
        uint64_t xwaves = 0;
        for (SimRun *r : P.express.runs)
            if (!r->finished()) xwaves += latency_waves(r->sim);
        const int xlatency = latency || xwaves <= kExpressLatencyWaves;
        for (int k = 0; k <= nl; ++k) {
            Lane &L = k < nl ? *P.lane[k] : P.express;
            if (L.ctx.pending) { any_pending = true; all_done = false; continue; }
            if (L.finished()) continue;
            all_done = false;
            // the express lane takes whole extensions
            const double tick = k < nl ? kTickUs : 0.0;
            const LaunchCfg lane_cfg{false, false, true, 256, nullptr};
            if ((rc = round_begin(L.runs, L.ws, L.stream, L.ctx, err, lane_cfg, tick, k < nl ? latency : xlatency)))
                break;
            if (L.ctx.pending) any_pending = true;
        }
        if (rc || all_done) break;
        if (!any_pending) continue;
        // wait for the first lane whose round completes
        bool progressed = false;
        while (!progressed) {
            for (int k = 0; k <= nl; ++k) {
                Lane &L = k < nl ? *P.lane[k] : P.express;
                if (!L.ctx.pending) continue;
                hipError_t e = hipEventQuery(L.ctx.done);
                if (e == hipSuccess) {
                    round_end(L.ws, L.ctx);
                    progressed = true;
                } else if (e != hipErrorNotReady) {
                    err = std::string("lane round: ") + hipGetErrorString(e);
                    rc = PBN_EDEVICE;
                    progressed = true;
                    break;
                }
            }
            if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        if (rc) break;
    }
    // drain and join back into the caller's stream
    for (int k = 0; k <= nl; ++k) {
        Lane &L = k < nl ? *P.lane[k] : P.express;
        if (L.ctx.pending) {
            (void)hipEventSynchronize(L.ctx.done);
            L.ctx.pending = false;
        }
        if (k < nl) {
            (void)hipEventRecord(P.ev[k], L.stream);
            (void)hipStreamWaitEvent(stream, P.ev[k], 0);
        }
        L.runs.clear();
    }
    (void)hipEventDestroy(start);
    return rc;
}

}  // namespace pbn

pbn_sim::~pbn_sim()
{
    if (!split_tabs.empty()) (void)hipDeviceSynchronize();
    for (SplitTab &t : split_tabs)
        if (t.d_tab) (void)hipFree(t.d_tab);
}
