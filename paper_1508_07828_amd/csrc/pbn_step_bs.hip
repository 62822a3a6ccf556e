// Bit-sliced trajectory kernel (gfx950, wave64).
//
// One block of G waves advances 64 chains.  State is bit-sliced in LDS: S[i]
// holds node i of all 64 chains (bit = lane = chain).  Per transition:
//   A  lane = chain: the waves share the 16-node blocks; each lane draws its
//      chain's perturbation and selection bytes; wave ballots turn the byte
//      comparisons into 64-chain masks (perturbation flips into Gm[i],
//      selection masks m_j = [u < T_j] into M); byte ties that need the
//      24-bit refinement are queued per wave and resolved 64 at a time
//   B  lane = node: Gm[i] := P & (S[i] ^ gamma_i), P = perturbed chains
//   C  lane = predictor slot (sorted by parent count): K-input multiplexer
//      tree over the parents' masks, restricted to the chains that selected
//      this predictor and were not perturbed, OR-ed into Gm[node]
//   D  record the state-set indicators; clear S (next step's gamma) and M;
//      swap S and Gm
// LDS (u64 words): S[n], Gm[n], M[msel_total], Pw[G], then the u32 queues.
// Lanes beyond the item's chain count run along on their own bit positions and
// are never stored.
#include "pbn_device.h"

namespace pbn {

// What the bit-sliced kernel reads, with as few live pointers as possible.
struct BsView {
    const PBN_CAS DevSim *d;
    cu32 nd_info, blk_sel, fs_rec, fg_K, fn_thr, nd_first;
    Key key;
    uint32_t n, W, p_thr, omega, nprops, F_pad, msel_total, nblk;
};

__device__ __forceinline__ BsView load_bs_view(const DevSim *p)
{
    const PBN_CAS DevSim *d = (const PBN_CAS DevSim *)p;
    BsView v;
    v.d = d;
    v.nd_info = (cu32)d->nd_info;
    v.blk_sel = (cu32)d->blk_sel;
    v.fs_rec = (cu32)d->fs_rec;
    v.fg_K = (cu32)d->fg_K;
    v.fn_thr = (cu32)d->fn_thr;
    v.nd_first = (cu32)d->nd_first;
    v.key = Key{d->key0, d->key1};
    v.n = d->n;
    v.W = d->W;
    v.p_thr = d->p_thr;
    v.omega = d->omega;
    v.nprops = d->nprops;
    v.F_pad = d->F_pad;
    v.msel_total = d->msel_total;
    v.nblk = d->nblk;
    return v;
}

__device__ __forceinline__ uint64_t bsel(uint64_t m, uint64_t a, uint64_t b)
{
    return (m & a) | (~m & b);          // a where m is set, else b
}

template <int K>
__device__ __forceinline__ uint64_t mux_tree(uint32_t lo, uint32_t hi, const uint64_t *x)
{
    constexpr int L = 1 << K;
    uint64_t r[L / 2];
#pragma unroll
    for (int m = 0; m < L / 2; ++m) {
        const int e0 = 2 * m, e1 = 2 * m + 1;
        const uint32_t w0 = e0 < 32 ? lo : hi, w1 = e1 < 32 ? lo : hi;
        const uint64_t A = 0ull - (uint64_t)((w0 >> (e0 & 31)) & 1u);
        const uint64_t B = 0ull - (uint64_t)((w1 >> (e1 & 31)) & 1u);
        r[m] = bsel(x[0], B, A);
    }
#pragma unroll
    for (int lev = 1; lev < K; ++lev) {
#pragma unroll
        for (int m = 0; m < (L >> (lev + 1)); ++m) r[m] = bsel(x[lev], r[2 * m + 1], r[2 * m]);
    }
    return r[0];
}

__device__ __forceinline__ uint64_t eval_slot(uint32_t K, uint32_t lo, uint32_t hi, const uint64_t *x)
{
    switch (K) {
    case 1: return mux_tree<1>(lo, hi, x);
    case 2: return mux_tree<2>(lo, hi, x);
    case 3: return mux_tree<3>(lo, hi, x);
    case 4: return mux_tree<4>(lo, hi, x);
    case 5: return mux_tree<5>(lo, hi, x);
    default: return mux_tree<6>(lo, hi, x);
    }
}

__device__ __forceinline__ void lds_or(uint64_t *p, uint64_t v)
{
    atomicOr((unsigned long long *)p, (unsigned long long)v);
}

// Queue entry: node (16 bits) | j (6) << 16 | kind (1) << 22 | lane (6) << 23.
__device__ __forceinline__ void resolve_queue(const BsView &v, uint32_t t, uint32_t chain0, uint32_t *Q, uint32_t qlen,
                                              uint64_t *Gm, uint64_t *M, uint64_t *Pw_mine, uint32_t lane)
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (uint32_t e = lane; e < qlen; e += 64) {
        const uint32_t ent = Q[e];
        const uint32_t node = ent & 0xFFFFu, j = (ent >> 16) & 63u, kind = (ent >> 22) & 1u, cl = ent >> 23;
        const uint64_t bit = 1ull << cl;
        const uint32_t r24 = refine24(v.key, t, chain0 + cl, node, kind ? kTagSel : kTagPert);
        if (kind == 0) {
            if (r24 < (v.p_thr & 0xFFFFFFu)) {
                lds_or(&Gm[node], bit);
                lds_or(Pw_mine, bit);
            }
        } else {
            const uint32_t T = v.fn_thr[v.nd_first[node] + j];
            if (r24 < (T & 0xFFFFFFu)) lds_or(&M[(v.nd_info[2 * node] >> 8) + j], bit);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ void enqueue(uint64_t tie, uint32_t payload, uint32_t lane, uint32_t *Q, uint32_t &qlen,
                                        const BsView &v, uint32_t t, uint32_t chain0, uint64_t *Gm, uint64_t *M,
                                        uint64_t *Pw_mine)
{
    const uint32_t cnt = (uint32_t)__popcll(tie);
    if (qlen + cnt > kQCap) {
        resolve_queue(v, t, chain0, Q, qlen, Gm, M, Pw_mine, lane);
        qlen = 0;
    }
    if ((tie >> lane) & 1ull) {
        const uint32_t pos = qlen + (uint32_t)__popcll(tie & ((1ull << lane) - 1ull));
        Q[pos] = payload | (lane << 23);
    }
    qlen += cnt;
}

// Put the 64-bit uniform value m into lane k of (lo, hi).
__device__ __forceinline__ void put_lane(uint32_t &lo, uint32_t &hi, uint64_t m, uint32_t k, uint32_t lane)
{
    const bool mine = lane == k;
    lo = mine ? (uint32_t)m : lo;
    hi = mine ? (uint32_t)(m >> 32) : hi;
}

extern __shared__ uint64_t lds_bs[];

template <int G>
__global__ void __launch_bounds__(64 * G) k_step_bs(const StepItem *__restrict__ items)
{
    const StepItem it = load_item(items, blockIdx.x);
    const BsView v = load_bs_view(it.sim);
    const uint32_t n = v.n, W = v.W, omega = v.omega;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t chain0 = it.chain0;
    const uint32_t c = chain0 + lane;
    const bool active = lane < it.nchains;
    uint64_t *S = lds_bs;
    uint64_t *Gm = lds_bs + n;
    uint64_t *M = lds_bs + 2 * n;
    uint64_t *Pw = M + v.msel_total;
    uint32_t *Q = (uint32_t *)(Pw + G) + wave * kQCap;
    const uint64_t words_cap = v.d->words_cap;

    // transpose the chains' packed words into node masks
    {
        gu32 state = (gu32)v.d->state;
        for (uint32_t w = wave; w < W; w += G) {
            const uint32_t word = active ? state[(size_t)w * omega + c] : 0u;
            const uint32_t nb = min(32u, n - 32 * w);
            for (uint32_t b = 0; b < nb; ++b) {
                const uint64_t m = __ballot((word >> b) & 1u);
                if (lane == 0) S[32 * w + b] = m;
            }
        }
    }
    for (uint32_t i = threadIdx.x; i < n; i += 64 * G) Gm[i] = 0ull;
    for (uint32_t i = threadIdx.x; i < v.msel_total; i += 64 * G) M[i] = 0ull;
    if (threadIdx.x < G) Pw[threadIdx.x] = 0ull;

    uint32_t acc[kMaxProps];
    uint64_t pos = it.pos0;
    const uint32_t nprops = v.nprops;
#pragma unroll
    for (uint32_t q = 0; q < kMaxProps; ++q) {
        acc[q] = 0;
        if (wave == 0 && active && q < nprops && it.nrec > 0 && (pos & 31)) {
            gu32 bits = (gu32)v.d->bits;
            const uint32_t old = bits[((size_t)q * words_cap + (pos >> 5)) * omega + c];
            acc[q] = old & ((1u << (pos & 31)) - 1u);
        }
    }
    __syncthreads();

    const uint32_t p_thr = v.p_thr, thr8 = p_thr >> 24;
    const uint32_t nblk = v.nblk, F_pad = v.F_pad;
    const uint32_t total = it.nburn + it.nrec * it.thin;
    uint32_t since = 0;
    for (uint32_t s = 0; s < total; ++s) {
        const uint32_t t = it.t0 + s;
        // ---- A: draws, lane = chain
        uint64_t P_acc = 0;
        uint32_t qlen = 0;
        for (uint32_t b = wave; b < nblk; b += G) {
            const uint32_t i0 = 16 * b, ib = min(16u, n - i0);
            const uint32_t has_sel = v.blk_sel[b];
            // node metadata of the block, one node per lane, fetched ahead of the draws
            uint32_t my_meta = 0, my_tb = 0;
            if (lane < ib) {
                my_meta = v.nd_info[2 * (i0 + lane)];
                my_tb = v.nd_info[2 * (i0 + lane) + 1];
            }
            uint32_t wp[4];
            philox4(t, c, b, kTagPert, v.key, wp);
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) {
                if (4 * q < ib) {
                    uint32_t x = wp[q];
                    if (ib - 4 * q < 4) x |= 0xFFFFFFFFu << (8 * (ib - 4 * q));   // no such nodes
                    // byte == thr8 needs the refinement, byte < thr8 perturbs outright
                    bool any = true;
                    if (thr8 == 0) any = __ballot(((x - 0x01010101u) & ~x & 0x80808080u) != 0) != 0;
                    if (any) {
#pragma unroll
                        for (uint32_t bb = 0; bb < 4; ++bb) {
                            const uint32_t k = 4 * q + bb;
                            if (k < ib) {
                                const uint32_t byte = (x >> (8 * bb)) & 0xFFu;
                                if (thr8 > 0) {
                                    const uint64_t d1 = __ballot(byte < thr8);
                                    if (d1) {
                                        if (lane == 0) lds_or(&Gm[i0 + k], d1);
                                        P_acc |= d1;
                                    }
                                }
                                const uint64_t tie = __ballot(byte == thr8);
                                if (tie) enqueue(tie, i0 + k, lane, Q, qlen, v, t, chain0, Gm, M, &Pw[wave]);
                            }
                        }
                    }
                }
            }
            if (has_sel) {
                uint32_t ws[4];
                philox4(t, c, b, kTagSel, v.key, ws);
                // masks of thresholds 1..3 of node k collect in lane k
                uint32_t m0l = 0, m0h = 0, m1l = 0, m1h = 0, m2l = 0, m2h = 0;
#pragma unroll
                for (uint32_t k = 0; k < 16; ++k) {
                    if (k < ib) {
                        const uint32_t meta = __builtin_amdgcn_readlane(my_meta, k);
                        const uint32_t l = meta & 0xFFu;
                        if (l >= 2) {
                            const uint32_t i = i0 + k;
                            const uint32_t tbs = __builtin_amdgcn_readlane(my_tb, k);
                            const uint32_t byte = (ws[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                            {
                                const uint32_t tb = tbs & 0xFFu;
                                put_lane(m0l, m0h, __ballot(byte < tb), k, lane);
                                const uint64_t eq = __ballot(byte == tb);
                                if (eq) enqueue(eq, i | (1u << 22), lane, Q, qlen, v, t, chain0, Gm, M, &Pw[wave]);
                            }
                            if (l >= 3) {
                                const uint32_t tb = (tbs >> 8) & 0xFFu;
                                put_lane(m1l, m1h, __ballot(byte < tb), k, lane);
                                const uint64_t eq = __ballot(byte == tb);
                                if (eq) enqueue(eq, i | (1u << 16) | (1u << 22), lane, Q, qlen, v, t, chain0, Gm, M, &Pw[wave]);
                            }
                            if (l >= 4) {
                                const uint32_t tb = (tbs >> 16) & 0xFFu;
                                put_lane(m2l, m2h, __ballot(byte < tb), k, lane);
                                const uint64_t eq = __ballot(byte == tb);
                                if (eq) enqueue(eq, i | (2u << 16) | (1u << 22), lane, Q, qlen, v, t, chain0, Gm, M, &Pw[wave]);
                            }
                            // more than four predictors: thresholds 4.. straight from fn_thr
                            for (uint32_t j = 3; j + 1 < l; ++j) {
                                const uint32_t tb = v.fn_thr[v.nd_first[i] + j] >> 24;
                                const uint64_t lt = __ballot(byte < tb);
                                if (lane == 0) lds_or(&M[(meta >> 8) + j], lt);
                                const uint64_t eq = __ballot(byte == tb);
                                if (eq) enqueue(eq, i | (j << 16) | (1u << 22), lane, Q, qlen, v, t, chain0, Gm, M, &Pw[wave]);
                            }
                        }
                    }
                }
                if (lane < ib) {
                    const uint32_t l = my_meta & 0xFFu, moff = my_meta >> 8;
                    if (l >= 2) lds_or(&M[moff], ((uint64_t)m0h << 32) | m0l);
                    if (l >= 3) lds_or(&M[moff + 1], ((uint64_t)m1h << 32) | m1l);
                    if (l >= 4) lds_or(&M[moff + 2], ((uint64_t)m2h << 32) | m2l);
                }
            }
        }
        if (qlen) resolve_queue(v, t, chain0, Q, qlen, Gm, M, &Pw[wave], lane);
        if (P_acc && lane == 0) lds_or(&Pw[wave], P_acc);
        __syncthreads();

        // ---- B: S' := P & (S ^ gamma), lane = node
        uint64_t P = 0;
#pragma unroll
        for (int w = 0; w < G; ++w) P |= Pw[w];
        for (uint32_t i = threadIdx.x; i < n; i += 64 * G) Gm[i] = P & (S[i] ^ Gm[i]);
        __syncthreads();

        // ---- C: predictor slots, lane = slot
        const uint64_t nP = ~P;
        for (uint32_t s0 = 64 * wave; s0 < F_pad; s0 += 64 * G) {
            const uint32_t slot = s0 + lane;
            const uint32_t K = v.fg_K[s0 >> 6];
            const cu32 rec = v.fs_rec + 8 * (size_t)slot;
            const uint32_t node = rec[0], tlo = rec[1], thi = rec[2], mlo = rec[3], mhi = rec[4];
            const uint32_t p01 = rec[5], p23 = rec[6], p45 = rec[7];
            uint64_t x[6];
            x[0] = S[p01 & 0xFFFFu];
            x[1] = K > 1 ? S[p01 >> 16] : 0ull;
            x[2] = K > 2 ? S[p23 & 0xFFFFu] : 0ull;
            x[3] = K > 3 ? S[p23 >> 16] : 0ull;
            x[4] = K > 4 ? S[p45 & 0xFFFFu] : 0ull;
            x[5] = K > 5 ? S[p45 >> 16] : 0ull;
            const uint64_t f = eval_slot(K, tlo, thi, x);
            const uint64_t below = mlo == kNoMask ? 0ull : M[mlo];
            const uint64_t upto = mhi == kNoMask ? ~0ull : M[mhi];
            if (node != kNoNode) {
                const uint64_t val = f & upto & ~below & nP;
                if (val) lds_or(&Gm[node], val);
            }
        }
        __syncthreads();

        // ---- D: record, clear, swap (Pw and M were last read before C's barrier)
        if (s >= it.nburn && ++since == it.thin) {
            since = 0;
            if (wave == 0) {
                const uint32_t bpos = (uint32_t)(pos & 31);
#pragma unroll
                for (uint32_t q = 0; q < kMaxProps; ++q) {
                    if (q < nprops) {
                        uint64_t xm = ~0ull;
                        for (uint32_t m = v.d->pn_off[q]; m < v.d->pn_off[q + 1]; ++m) {
                            const uint64_t g = Gm[v.d->pn_node[m]];
                            xm &= v.d->pn_val[m] ? g : ~g;
                        }
                        acc[q] |= (uint32_t)((xm >> lane) & 1ull) << bpos;
                    }
                }
                if (bpos == 31 && active) {
                    gu32 bits = (gu32)v.d->bits;
#pragma unroll
                    for (uint32_t q = 0; q < kMaxProps; ++q) {
                        if (q < nprops) {
                            bits[((size_t)q * words_cap + (pos >> 5)) * omega + c] = acc[q];
                            acc[q] = 0;
                        }
                    }
                }
            }
            ++pos;
        }
        for (uint32_t i = threadIdx.x; i < n; i += 64 * G) S[i] = 0ull;
        for (uint32_t i = threadIdx.x; i < v.msel_total; i += 64 * G) M[i] = 0ull;
        if (threadIdx.x < G) Pw[threadIdx.x] = 0ull;
        uint64_t *tmp = S; S = Gm; Gm = tmp;
        __syncthreads();
    }

    if (wave == 0 && active && it.nrec > 0 && (pos & 31)) {
        gu32 bits = (gu32)v.d->bits;
#pragma unroll
        for (uint32_t q = 0; q < kMaxProps; ++q)
            if (q < nprops) bits[((size_t)q * words_cap + (pos >> 5)) * omega + c] = acc[q];
    }
    // transpose back
    gu32 state = (gu32)v.d->state;
    for (uint32_t w = wave; w < W; w += G) {
        uint32_t word = 0;
        const uint32_t nb = min(32u, n - 32 * w);
        for (uint32_t b = 0; b < nb; ++b) word |= (uint32_t)((S[32 * w + b] >> lane) & 1ull) << b;
        if (active) state[(size_t)w * omega + c] = word;
    }
}

static int check_bs(hipError_t e, const char *what, std::string &err)
{
    if (e == hipSuccess) return PBN_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return PBN_EDEVICE;
}

size_t bs_lds_bytes(uint32_t n, uint32_t msel_total, uint32_t G)
{
    return (size_t)8 * (2 * (size_t)n + msel_total + G) + (size_t)4 * kQCap * G;
}

template <int G>
static int launch_bs_g(const StepItem *d_items, uint32_t nitems, size_t lds, hipStream_t s, std::string &err)
{
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_step_bs<G>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return check_bs(e, "k_step_bs LDS attribute", err);
    }
    hipLaunchKernelGGL(k_step_bs<G>, dim3(nitems), dim3(64 * G), lds, s, d_items);
    return check_bs(hipGetLastError(), "k_step_bs launch", err);
}

int launch_step_bs(const StepItem *d_items, uint32_t nitems, uint32_t G, size_t lds, void *stream, std::string &err)
{
    if (nitems == 0) return PBN_OK;
    if (lds > 160 * 1024) {
        err = "bit-sliced state exceeds LDS";
        return PBN_ELIMIT;
    }
    hipStream_t s = (hipStream_t)stream;
    switch (G) {
    case 1: return launch_bs_g<1>(d_items, nitems, lds, s, err);
    case 2: return launch_bs_g<2>(d_items, nitems, lds, s, err);
    case 4: return launch_bs_g<4>(d_items, nitems, lds, s, err);
    case 8: return launch_bs_g<8>(d_items, nitems, lds, s, err);
    default: return launch_bs_g<16>(d_items, nitems, lds, s, err);
    }
}

}  // namespace pbn
