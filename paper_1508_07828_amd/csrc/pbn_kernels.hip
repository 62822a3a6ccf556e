// Device kernels of libpbnssa for gfx950 (CDNA4, wave64), besides the
// bit-sliced trajectory kernel:
//
//   k_init     s(0) of every chain from the Philox stream (tag 4)
//   k_step     trajectories, one lane per chain, state rows in LDS: the
//              general kernel (any parent count up to 16)
//   k_reduce   window aggregates (popcount sums, sums of squares, pair counts)
//              and Skart batch sums over the recorded indicator bit-streams
//
// Everything on the device is integer arithmetic; FP64 only happens on the
// host from the exact aggregates.
#include "pbn_device.h"

#include <mutex>
#include <utility>

namespace pbn {

// Any byte of x strictly below m (1 <= m <= 128): classic SWAR test.
__device__ __forceinline__ bool has_byte_below(uint32_t x, uint32_t m)
{
    return ((x - 0x01010101u * m) & ~x & 0x80808080u) != 0;
}

// ------------------------------------------------------------------ init
__global__ void k_init(const DevSim *__restrict__ sim)
{
    const View v = load_view(sim);
    const uint32_t omega = v.omega, W = v.W, n = v.n;
    const uint32_t quads = (W + 3) / 4;
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= omega * quads) return;
    const uint32_t c = gid % omega, q = gid / omega;
    uint32_t w4[4];
    philox4(0u, c, q, kTagInit, v.key, w4);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t w = 4 * q + j;
        if (w < W) {
            uint32_t val = w4[j];
            const uint32_t nb = n - 32 * w;
            if (nb < 32) val &= (1u << nb) - 1u;
            v.state[(size_t)w * omega + c] = val;
        }
    }
}

// Many simulations at once: block b copies descriptor b from a staging array
// to its simulation's buffer and writes that simulation's initial states.
__global__ void __launch_bounds__(256) k_setup(const DevSim *__restrict__ staging, DevSim *const *__restrict__ dst)
{
    const DevSim *src = staging + blockIdx.x;
    DevSim *d = ((DevSim *const PBN_CAS *)dst)[blockIdx.x];
    const PBN_CAS uint32_t *from = (const PBN_CAS uint32_t *)src;
    PBN_GAS uint32_t *to = (PBN_GAS uint32_t *)d;
    for (uint32_t w = threadIdx.x; w < sizeof(DevSim) / 4; w += blockDim.x) to[w] = from[w];
    const View v = load_view(src);
    const uint32_t omega = v.omega, W = v.W, n = v.n, quads = (W + 3) / 4;
    for (uint32_t g = threadIdx.x; g < omega * quads; g += blockDim.x) {
        const uint32_t c = g % omega, q = g / omega;
        uint32_t w4[4];
        philox4(0u, c, q, kTagInit, v.key, w4);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t w = 4 * q + j;
            if (w < W) {
                uint32_t val = w4[j];
                const uint32_t nb = n - 32 * w;
                if (nb < 32) val &= (1u << nb) - 1u;
                v.state[(size_t)w * omega + c] = val;
            }
        }
    }
}

// ------------------------------------------------------------------ step

// Perturbation pass over all nodes of one chain at transition t.  With
// APPLY = false it counts perturbed nodes and remembers the first four; with
// APPLY = true it XORs every perturbed node into the state row.
struct Flips {
    uint32_t nf, s0, s1, s2, s3;
};

template <bool APPLY>
__device__ __forceinline__ Flips perturb_scan(const View &v, uint32_t t, uint32_t c, uint32_t *row)
{
    const uint32_t n = v.n, p_thr = v.p_thr;
    const uint32_t thr8 = p_thr >> 24;
    const bool swar = thr8 < 127u;
    uint32_t nf = 0, s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    const uint32_t nblk = (n + 15) >> 4;
    for (uint32_t b = 0; b < nblk; ++b) {
        uint32_t w[4];
        philox4(t, c, b, kTagPert, v.key, w);
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t node0 = b * 16 + q * 4;
            if (node0 < n) {
                const uint32_t nvalid = min(4u, n - node0);
                uint32_t x = w[q];
                if (nvalid < 4) x |= 0xFFFFFFFFu << (8 * nvalid);
                if (!swar || has_byte_below(x, thr8 + 1)) {
                    for (uint32_t bb = 0; bb < nvalid; ++bb) {
                        const uint32_t byte = (x >> (8 * bb)) & 0xFFu;
                        const uint32_t i = node0 + bb;
                        bool g;
                        if (byte != thr8) g = byte < thr8;
                        else g = ((byte << 24) | refine24(v.key, t, c, i, kTagPert)) < p_thr;
                        if (g) {
                            if (APPLY) {
                                row[i >> 5] ^= 1u << (i & 31);
                            } else {
                                if (nf == 0) s0 = i;
                                else if (nf == 1) s1 = i;
                                else if (nf == 2) s2 = i;
                                else if (nf == 3) s3 = i;
                            }
                            ++nf;
                        }
                    }
                }
            }
        }
    }
    return Flips{nf, s0, s1, s2, s3};
}

// Synchronous update with one predictor drawn per node: reads cur, writes nxt.
__device__ __forceinline__ void function_update(const View &v, uint32_t t, uint32_t c, const uint32_t *cur,
                                                uint32_t *nxt)
{
    const uint32_t n = v.n;
    uint32_t sw[4] = {0, 0, 0, 0};
    uint32_t have_blk = 0xFFFFFFFFu;
    uint32_t acc = 0;
    uint32_t first = v.nd_first[0];
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t next_first = v.nd_first[i + 1];
        const uint32_t l = next_first - first;
        uint32_t j = l - 1;
        if (l > 1) {
            const uint32_t blk = i >> 4;
            if (blk != have_blk) {
                philox4(t, c, blk, kTagSel, v.key, sw);
                have_blk = blk;
            }
            const uint32_t byte = (pick4(sw, (i >> 2) & 3) >> (8 * (i & 3))) & 0xFFu;
            uint32_t u = 0;
            bool have_u = false;
            for (uint32_t jj = 0; jj + 1 < l; ++jj) {
                const uint32_t T = v.fn_thr[first + jj];
                const uint32_t tb = T >> 24;
                bool lt;
                if (byte != tb) {
                    lt = byte < tb;
                } else {
                    if (!have_u) {
                        u = (byte << 24) | refine24(v.key, t, c, i, kTagSel);
                        have_u = true;
                    }
                    lt = u < T;
                }
                if (lt) { j = jj; break; }
            }
        }
        const uint32_t f = first + j;
        const uint32_t desc = v.fn_desc[f];
        const uint32_t k = desc & 31u, po = desc >> 5;
        uint32_t idx = 0;
        for (uint32_t m = 0; m < k; ++m) {
            const uint32_t par = v.par[po + m];
            idx |= ((cur[par >> 5] >> (par & 31)) & 1u) << m;
        }
        uint32_t bit;
        if (k <= 5) bit = (v.fn_tt[f] >> idx) & 1u;
        else bit = (v.tt_ext[v.fn_tt[f] + (idx >> 5)] >> (idx & 31)) & 1u;
        acc |= bit << (i & 31);
        if ((i & 31) == 31 || i + 1 == n) {
            nxt[i >> 5] = acc;
            acc = 0;
        }
        first = next_first;
    }
}

__device__ __forceinline__ uint32_t prop_value(const View &v, uint32_t q, const uint32_t *row)
{
    uint32_t ok = 1;
    for (uint32_t m = v.d->prop_off[q]; m < v.d->prop_off[q + 1]; ++m)
        ok &= ((row[v.d->term_word[m]] & v.d->term_mask[m]) == v.d->term_val[m]) ? 1u : 0u;
    return ok;
}

extern __shared__ uint32_t lds_rows[];

// One 64-lane block per work item; lane = chain.  Two LDS rows per lane
// (current and next state) of stride S words (S odd: conflict-free rows).
// GLOBAL: the two state rows of each chain live in a device scratch area
// (rows[(block * 64 + lane) * 2 * S ...]) instead of LDS, for networks whose
// rows do not fit in LDS (more than 320 words, n > 10240); same arithmetic.
template <bool GLOBAL>
__global__ void __launch_bounds__(64) k_step(const StepItem *__restrict__ items, uint32_t S, uint32_t *rows)
{
    const StepItem it = load_item(items, blockIdx.x);
    const View v = load_view(it.sim);
    const uint32_t lane = threadIdx.x;
    if (lane >= it.nchains) return;
    const uint32_t c = it.chain0 + lane;
    const uint32_t W = v.W, omega = v.omega, nprops = v.nprops;
    uint32_t *cur, *nxt;
    if (GLOBAL) {
        cur = rows + ((size_t)blockIdx.x * 64 + lane) * 2 * S;
        nxt = cur + S;
    } else {
        cur = lds_rows + lane * S;
        nxt = lds_rows + (64 + lane) * S;
    }
    for (uint32_t w = 0; w < W; ++w) cur[w] = v.state[(size_t)w * omega + c];

    uint32_t acc[kMaxProps];
    uint64_t pos = it.pos0;
#pragma unroll
    for (uint32_t q = 0; q < kMaxProps; ++q) {
        acc[q] = 0;
        if (q < nprops && it.nrec > 0 && (pos & 31)) {
            const uint32_t old = v.bits[((size_t)q * v.words_cap + (pos >> 5)) * omega + c];
            acc[q] = old & ((1u << (pos & 31)) - 1u);
        }
    }

    const uint32_t total = it.nburn + it.nrec * it.thin;
    uint32_t since = 0;
    for (uint32_t s = 0; s < total; ++s) {
        const uint32_t t = it.t0 + s;
        const Flips fl = perturb_scan<false>(v, t, c, cur);
        const uint32_t nf = fl.nf;
        if (nf > 0) {
            if (nf <= 4) {
                cur[fl.s0 >> 5] ^= 1u << (fl.s0 & 31);
                if (nf > 1) cur[fl.s1 >> 5] ^= 1u << (fl.s1 & 31);
                if (nf > 2) cur[fl.s2 >> 5] ^= 1u << (fl.s2 & 31);
                if (nf > 3) cur[fl.s3 >> 5] ^= 1u << (fl.s3 & 31);
            } else {
                perturb_scan<true>(v, t, c, cur);
            }
        } else {
            function_update(v, t, c, cur, nxt);
            uint32_t *tmp = cur; cur = nxt; nxt = tmp;
        }
        if (s >= it.nburn && ++since == it.thin) {
            since = 0;
            const uint32_t b = (uint32_t)(pos & 31);
#pragma unroll
            for (uint32_t q = 0; q < kMaxProps; ++q)
                if (q < nprops) acc[q] |= prop_value(v, q, cur) << b;
            if (b == 31) {
#pragma unroll
                for (uint32_t q = 0; q < kMaxProps; ++q)
                    if (q < nprops) {
                        v.bits[((size_t)q * v.words_cap + (pos >> 5)) * omega + c] = acc[q];
                        acc[q] = 0;
                    }
            }
            ++pos;
        }
    }
    if (it.nrec > 0 && (pos & 31)) {
#pragma unroll
        for (uint32_t q = 0; q < kMaxProps; ++q)
            if (q < nprops) v.bits[((size_t)q * v.words_cap + (pos >> 5)) * omega + c] = acc[q];
    }
    for (uint32_t w = 0; w < W; ++w) v.state[(size_t)w * omega + c] = cur[w];
}

// ------------------------------------------------------------------ reduce

// Bits [lo, hi) of a word starting at position 32*wi, as a mask.
__device__ __forceinline__ uint32_t range_mask(uint64_t wi, uint64_t lo, uint64_t hi)
{
    const uint64_t base = wi * 32;
    if (hi <= base) return 0;
    const uint64_t a = lo > base ? lo - base : 0;
    const uint64_t b = hi - base >= 32 ? 32 : hi - base;
    if (b <= a) return 0;
    const uint32_t upto = b == 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
    return upto & ~((1u << a) - 1u);
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *part)
{
    // wave64 reduction then across the waves of the block
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    int64_t tot = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
    __syncthreads();
    return tot;
}

// One 256-thread block per query.
__global__ void __launch_bounds__(256) k_reduce(const Query *__restrict__ qs, WindowResult *__restrict__ win,
                                                int32_t *__restrict__ bsum)
{
    __shared__ int64_t part[8];
    const Query qy = load_query(qs, blockIdx.x);
    const View v = load_view(qy.sim);
    const uint32_t omega = v.omega;
    const PBN_GAS uint32_t *bits = v.bits + (size_t)qy.prop * v.words_cap * omega;
    if (qy.kind == kQueryWindow) {
        int64_t T1 = 0, T2 = 0, n01 = 0, n10 = 0, n11 = 0;
        const uint64_t lo = qy.lo, hi = qy.hi;
        const uint64_t w0 = lo >> 5, w1 = (hi + 31) >> 5;
        const uint64_t pair_hi = hi - 1 > lo ? hi - 1 : lo;     // pairs (l, l+1) with l in [lo, hi-1)
        for (uint32_t c = threadIdx.x; c < omega; c += blockDim.x) {
            int64_t S = 0;
            uint32_t x = w0 < w1 ? bits[w0 * omega + c] : 0u;
            for (uint64_t wi = w0; wi < w1; ++wi) {
                const uint32_t nx = (wi + 1 < w1) ? bits[(wi + 1) * omega + c] : 0u;
                S += __popc(x & range_mask(wi, lo, hi));
                const uint32_t pm = range_mask(wi, lo, pair_hi);
                const uint32_t y = (x >> 1) | (nx << 31);
                n11 += __popc(x & y & pm);
                n10 += __popc(x & ~y & pm);
                n01 += __popc(~x & y & pm);
                x = nx;
            }
            T1 += S;
            T2 += S * S;
        }
        T1 = block_sum(T1, part);
        T2 = block_sum(T2, part);
        n01 = block_sum(n01, part);
        n10 = block_sum(n10, part);
        n11 = block_sum(n11, part);
        if (threadIdx.x == 0) {
            const int64_t pairs = hi > lo ? (int64_t)(hi - lo - 1) * omega : 0;
            WindowResult r;
            r.T1 = T1; r.T2 = T2; r.n01 = n01; r.n10 = n10; r.n11 = n11;
            r.n00 = pairs - n01 - n10 - n11;
            r.pad0 = r.pad1 = 0;
            win[blockIdx.x] = r;
        }
    } else {
        const uint64_t m = qy.m, kappa = qy.kappa;
        const uint64_t total = (uint64_t)omega * m;
        for (uint64_t e = threadIdx.x; e < total; e += blockDim.x) {
            const uint32_t c = (uint32_t)(e / m);
            const uint64_t b = e % m;
            const uint64_t lo = qy.lo + b * kappa, hi = lo + kappa;
            int32_t S = 0;
            for (uint64_t wi = lo >> 5; wi < ((hi + 31) >> 5); ++wi)
                S += __popc(bits[wi * omega + c] & range_mask(wi, lo, hi));
            bsum[qy.out_off + e] = S;
        }
    }
}

// ------------------------------------------------------------------ launches

static int check(hipError_t e, const char *what, std::string &err)
{
    if (e == hipSuccess) return PBN_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return PBN_EDEVICE;
}

int launch_init(const DevSim *dsim, uint32_t omega, uint32_t W, void *stream, std::string &err)
{
    const uint32_t total = omega * ((W + 3) / 4);
    hipLaunchKernelGGL(k_init, dim3((total + 255) / 256), dim3(256), 0, (hipStream_t)stream, dsim);
    return check(hipGetLastError(), "k_init launch", err);
}

int launch_setup(const DevSim *d_staging, DevSim *const *d_dst, uint32_t count, void *stream, std::string &err)
{
    if (count == 0) return PBN_OK;
    hipLaunchKernelGGL(k_setup, dim3(count), dim3(256), 0, (hipStream_t)stream, d_staging, d_dst);
    return check(hipGetLastError(), "k_setup launch", err);
}

// Raise a kernel's dynamic-LDS limit to the full 160 KB once per device and
// kernel.  Setting the attribute can wait for running launches of the same
// kernel, so it must not sit on the launch path.
int allow_full_lds(const void *fn, std::string &err)
{
    // (kernel, device) pairs already raised, in a fixed table: no allocation
    // here, so that launch paths which must not allocate can use it
    constexpr int kSlots = 256;
    static std::mutex mu;
    static std::pair<const void *, int> done[kSlots];
    static int used = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        err = "hipGetDevice";
        return PBN_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; ++i)
        if (done[i].first == fn && done[i].second == dev) return PBN_OK;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return check(e, "LDS attribute", err);
    if (used < kSlots) done[used++] = {fn, dev};
    return PBN_OK;
}

size_t step_rows_words(uint32_t nitems, uint32_t max_W)
{
    const size_t S = max_W | 1u;
    return 2 * 64 * S * 4 <= 160 * 1024 ? 0 : (size_t)nitems * 64 * 2 * S;
}

int launch_step(const StepItem *d_items, uint32_t nitems, uint32_t max_W, uint32_t *rows, void *stream,
                std::string &err)
{
    if (nitems == 0) return PBN_OK;
    const uint32_t S = max_W | 1u;
    const size_t lds = (size_t)2 * 64 * S * 4;
    if (lds > 160 * 1024) {
        if (!rows) {
            err = "state rows exceed LDS and no row scratch was given";
            return PBN_ELIMIT;
        }
        hipLaunchKernelGGL(k_step<true>, dim3(nitems), dim3(64), 0, (hipStream_t)stream, d_items, S, rows);
        return check(hipGetLastError(), "k_step launch", err);
    }
    if (lds > 64 * 1024) {
        int rc = allow_full_lds((const void *)k_step<false>, err);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_step<false>, dim3(nitems), dim3(64), lds, (hipStream_t)stream, d_items, S, rows);
    return check(hipGetLastError(), "k_step launch", err);
}

int launch_reduce(const Query *d_queries, uint32_t nq, WindowResult *d_win, int32_t *d_bsum, void *stream,
                  std::string &err)
{
    if (nq == 0) return PBN_OK;
    hipLaunchKernelGGL(k_reduce, dim3(nq), dim3(256), 0, (hipStream_t)stream, d_queries, d_win, d_bsum);
    return check(hipGetLastError(), "k_reduce launch", err);
}

}  // namespace pbn
