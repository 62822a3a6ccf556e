// Device kernels of libpbnssa for gfx950 (CDNA4, wave64).
//
//   k_init     s(0) of every chain from the Philox stream (tag 4)
//   k_step     trajectories: each lane advances one chain; one 64-lane block
//              per (simulation, 64-chain slice) work item, so one launch serves
//              any number of simulations of different sizes (batched form)
//   k_reduce   window aggregates (popcount sums, sums of squares, pair counts)
//              and Skart batch sums over the recorded indicator bit-streams
//
// Everything on the device is integer arithmetic; FP64 only happens on the
// host from the exact aggregates.
#include <hip/hip_runtime.h>

#include "pbn_internal.h"

namespace pbn {

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products,
// key bumped by the Weyl constants between rounds.
struct Key {
    uint32_t k0, k1;
};

__device__ __forceinline__ void philox4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        Key key, uint32_t out[4])
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// w[j] for a per-lane j in 0..3, as two levels of selects (kept in registers).
__device__ __forceinline__ uint32_t pick4(const uint32_t w[4], uint32_t j)
{
    const bool odd = (j & 1u) != 0, high = (j & 2u) != 0;
    const uint32_t a = odd ? w[1] : w[0];
    const uint32_t b = odd ? w[3] : w[2];
    return high ? b : a;
}

// Low 24 bits of the refinement word of node i (tag + 1).
__device__ __forceinline__ uint32_t refine24(Key key, uint32_t t, uint32_t c, uint32_t i, uint32_t tag)
{
    uint32_t w[4];
    philox4(t, c, i >> 2, tag + 1, key, w);
    return pick4(w, i & 3) & 0xFFFFFFu;
}

// Any byte of x strictly below m (1 <= m <= 128): classic SWAR test.
__device__ __forceinline__ bool has_byte_below(uint32_t x, uint32_t m)
{
    return ((x - 0x01010101u * m) & ~x & 0x80808080u) != 0;
}

// ------------------------------------------------------------------ init
__global__ void k_init(const DevSim *__restrict__ sim)
{
    const uint32_t omega = sim->omega, W = sim->W, n = sim->n;
    const uint32_t quads = (W + 3) / 4;
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= omega * quads) return;
    const uint32_t c = gid % omega, q = gid / omega;
    uint32_t w4[4];
    philox4(0u, c, q, kTagInit, Key{sim->key0, sim->key1}, w4);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        uint32_t w = 4 * q + j;
        if (w >= W) break;
        uint32_t v = w4[j];
        uint32_t nb = n - 32 * w;
        if (nb < 32) v &= (1u << nb) - 1u;
        sim->state[(size_t)w * omega + c] = v;
    }
}

// ------------------------------------------------------------------ step

// Perturbation pass over all nodes of one chain at transition t.  With
// APPLY = false it counts perturbed nodes and remembers the first four; with
// APPLY = true it XORs every perturbed node into the state row.
template <bool APPLY>
__device__ __forceinline__ uint32_t perturb_scan(const DevSim &sm, Key key, uint32_t t, uint32_t c,
                                                 uint32_t *row, uint32_t slot[4])
{
    const uint32_t n = sm.n, p_thr = sm.p_thr;
    const uint32_t thr8 = p_thr >> 24;
    const bool swar = thr8 < 127u;
    uint32_t nf = 0;
    const uint32_t nblk = (n + 15) >> 4;
    for (uint32_t b = 0; b < nblk; ++b) {
        uint32_t w[4];
        philox4(t, c, b, kTagPert, key, w);
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t node0 = b * 16 + q * 4;
            if (node0 >= n) break;
            const uint32_t nvalid = min(4u, n - node0);
            uint32_t x = w[q];
            if (nvalid < 4) x |= 0xFFFFFFFFu << (8 * nvalid);
            if (swar && !has_byte_below(x, thr8 + 1)) continue;
            for (uint32_t bb = 0; bb < nvalid; ++bb) {
                const uint32_t byte = (x >> (8 * bb)) & 0xFFu;
                bool g;
                if (byte != thr8) {
                    g = byte < thr8;
                } else {
                    const uint32_t i = node0 + bb;
                    g = ((byte << 24) | refine24(key, t, c, i, kTagPert)) < p_thr;
                }
                if (g) {
                    const uint32_t i = node0 + bb;
                    if (APPLY) {
                        row[i >> 5] ^= 1u << (i & 31);
                    } else {
                        if (nf == 0) slot[0] = i;
                        else if (nf == 1) slot[1] = i;
                        else if (nf == 2) slot[2] = i;
                        else if (nf == 3) slot[3] = i;
                    }
                    ++nf;
                }
            }
        }
    }
    return nf;
}

// Synchronous update with one predictor drawn per node: reads cur, writes nxt.
__device__ __forceinline__ void function_update(const DevSim &sm, Key key, uint32_t t, uint32_t c,
                                                const uint32_t *cur, uint32_t *nxt)
{
    const uint32_t n = sm.n;
    const uint32_t *__restrict__ nd_first = sm.nd_first;
    const uint32_t *__restrict__ fn_thr = sm.fn_thr;
    const uint32_t *__restrict__ fn_desc = sm.fn_desc;
    const uint32_t *__restrict__ fn_tt = sm.fn_tt;
    const uint32_t *__restrict__ tt_ext = sm.tt_ext;
    const uint16_t *__restrict__ par = sm.par;
    uint32_t sw[4] = {0, 0, 0, 0};
    uint32_t have_blk = 0xFFFFFFFFu;
    uint32_t acc = 0;
    uint32_t first = nd_first[0];
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t next_first = nd_first[i + 1];
        const uint32_t l = next_first - first;
        uint32_t j = l - 1;
        if (l > 1) {
            const uint32_t blk = i >> 4;
            if (blk != have_blk) {
                philox4(t, c, blk, kTagSel, key, sw);
                have_blk = blk;
            }
            const uint32_t byte = (pick4(sw, (i >> 2) & 3) >> (8 * (i & 3))) & 0xFFu;
            uint32_t u = 0;
            bool have_u = false;
            for (uint32_t jj = 0; jj + 1 < l; ++jj) {
                const uint32_t T = fn_thr[first + jj];
                const uint32_t tb = T >> 24;
                bool lt;
                if (byte != tb) {
                    lt = byte < tb;
                } else {
                    if (!have_u) {
                        u = (byte << 24) | refine24(key, t, c, i, kTagSel);
                        have_u = true;
                    }
                    lt = u < T;
                }
                if (lt) { j = jj; break; }
            }
        }
        const uint32_t f = first + j;
        const uint32_t desc = fn_desc[f];
        const uint32_t k = desc & 31u, po = desc >> 5;
        uint32_t idx = 0;
        for (uint32_t m = 0; m < k; ++m) {
            const uint32_t v = par[po + m];
            idx |= ((cur[v >> 5] >> (v & 31)) & 1u) << m;
        }
        uint32_t bit;
        if (k <= 5) bit = (fn_tt[f] >> idx) & 1u;
        else bit = (tt_ext[fn_tt[f] + (idx >> 5)] >> (idx & 31)) & 1u;
        acc |= bit << (i & 31);
        if ((i & 31) == 31 || i + 1 == n) {
            nxt[i >> 5] = acc;
            acc = 0;
        }
        first = next_first;
    }
}

__device__ __forceinline__ uint32_t prop_value(const DevSim &sm, uint32_t q, const uint32_t *row)
{
    uint32_t ok = 1;
    for (uint32_t m = sm.prop_off[q]; m < sm.prop_off[q + 1]; ++m)
        ok &= ((row[sm.term_word[m]] & sm.term_mask[m]) == sm.term_val[m]) ? 1u : 0u;
    return ok;
}

extern __shared__ uint32_t lds_rows[];

// One 64-lane block per work item; lane = chain.  Two LDS rows per lane
// (current and next state) of stride S words (S odd: conflict-free rows).
__global__ void __launch_bounds__(64) k_step(const StepItem *__restrict__ items, uint32_t S)
{
    const StepItem it = items[blockIdx.x];
    const DevSim &sm = *it.sim;
    const uint32_t lane = threadIdx.x;
    if (lane >= it.nchains) return;
    const uint32_t c = it.chain0 + lane;
    const uint32_t W = sm.W, omega = sm.omega, nprops = sm.nprops;
    const Key key{sm.key0, sm.key1};
    uint32_t *cur = lds_rows + lane * S;
    uint32_t *nxt = lds_rows + (64 + lane) * S;
    for (uint32_t w = 0; w < W; ++w) cur[w] = sm.state[(size_t)w * omega + c];

    uint32_t acc[kMaxProps];
    uint64_t pos = it.pos0;
#pragma unroll
    for (uint32_t q = 0; q < kMaxProps; ++q) {
        acc[q] = 0;
        if (q < nprops && it.nrec > 0 && (pos & 31)) {
            const uint32_t old = sm.bits[((size_t)q * sm.words_cap + (pos >> 5)) * omega + c];
            acc[q] = old & ((1u << (pos & 31)) - 1u);
        }
    }

    const uint32_t total = it.nburn + it.nrec * it.thin;
    uint32_t since = 0;
    for (uint32_t s = 0; s < total; ++s) {
        const uint32_t t = it.t0 + s;
        uint32_t slot[4];
        const uint32_t nf = perturb_scan<false>(sm, key, t, c, cur, slot);
        if (nf > 0) {
            if (nf <= 4) {
                cur[slot[0] >> 5] ^= 1u << (slot[0] & 31);
                if (nf > 1) cur[slot[1] >> 5] ^= 1u << (slot[1] & 31);
                if (nf > 2) cur[slot[2] >> 5] ^= 1u << (slot[2] & 31);
                if (nf > 3) cur[slot[3] >> 5] ^= 1u << (slot[3] & 31);
            } else {
                perturb_scan<true>(sm, key, t, c, cur, slot);
            }
        } else {
            function_update(sm, key, t, c, cur, nxt);
            uint32_t *tmp = cur; cur = nxt; nxt = tmp;
        }
        if (s >= it.nburn && ++since == it.thin) {
            since = 0;
            const uint32_t b = (uint32_t)(pos & 31);
#pragma unroll
            for (uint32_t q = 0; q < kMaxProps; ++q)
                if (q < nprops) acc[q] |= prop_value(sm, q, cur) << b;
            if (b == 31) {
#pragma unroll
                for (uint32_t q = 0; q < kMaxProps; ++q)
                    if (q < nprops) {
                        sm.bits[((size_t)q * sm.words_cap + (pos >> 5)) * omega + c] = acc[q];
                        acc[q] = 0;
                    }
            }
            ++pos;
        }
    }
    if (it.nrec > 0 && (pos & 31)) {
#pragma unroll
        for (uint32_t q = 0; q < kMaxProps; ++q)
            if (q < nprops) sm.bits[((size_t)q * sm.words_cap + (pos >> 5)) * omega + c] = acc[q];
    }
    for (uint32_t w = 0; w < W; ++w) sm.state[(size_t)w * omega + c] = cur[w];
}

// ------------------------------------------------------------ bit-sliced step
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
//   D  record the state-set indicators; clear S (next step's gamma); swap
// LDS (u64 words): S[n], Gm[n], M[msel_total], Pw[G], then the u32 queues.

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

// Queue entry: node (16 bits) | j (6) << 16 | kind (1) << 22 | lane (6) << 23.
__device__ __forceinline__ void resolve_queue(const DevSim &sm, Key key, uint32_t t, uint32_t chain0,
                                              uint32_t *Q, uint32_t qlen, uint64_t *Gm, uint64_t *M,
                                              uint64_t *Pw_mine, uint32_t lane)
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (uint32_t e = lane; e < qlen; e += 64) {
        const uint32_t ent = Q[e];
        const uint32_t node = ent & 0xFFFFu, j = (ent >> 16) & 63u, kind = (ent >> 22) & 1u, cl = ent >> 23;
        const uint64_t bit = 1ull << cl;
        const uint32_t r24 = refine24(key, t, chain0 + cl, node, kind ? kTagSel : kTagPert);
        if (kind == 0) {
            if (r24 < (sm.p_thr & 0xFFFFFFu)) {
                atomicOr((unsigned long long *)&Gm[node], (unsigned long long)bit);
                atomicOr((unsigned long long *)Pw_mine, (unsigned long long)bit);
            }
        } else {
            const uint32_t T = sm.fn_thr[sm.nd_first[node] + j];
            if (r24 < (T & 0xFFFFFFu))
                atomicOr((unsigned long long *)&M[(sm.nd_meta[node] >> 8) + j], (unsigned long long)bit);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ void enqueue(uint64_t tie, uint32_t payload, uint32_t lane, uint32_t *Q, uint32_t &qlen,
                                        const DevSim &sm, Key key, uint32_t t, uint32_t chain0, uint64_t *Gm,
                                        uint64_t *M, uint64_t *Pw_mine)
{
    const uint32_t cnt = (uint32_t)__popcll(tie);
    if (qlen + cnt > kQCap) {
        resolve_queue(sm, key, t, chain0, Q, qlen, Gm, M, Pw_mine, lane);
        qlen = 0;
    }
    if ((tie >> lane) & 1ull) {
        const uint32_t pos = qlen + (uint32_t)__popcll(tie & ((1ull << lane) - 1ull));
        Q[pos] = payload | (lane << 23);
    }
    qlen += cnt;
}

extern __shared__ uint64_t lds_bs[];

template <int G>
__global__ void __launch_bounds__(64 * G) k_step_bs(const StepItem *__restrict__ items)
{
    const StepItem it = items[blockIdx.x];
    const DevSim &sm = *it.sim;
    const uint32_t n = sm.n, W = sm.W, omega = sm.omega;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t chain0 = it.chain0;
    const uint32_t c = chain0 + lane;
    const bool active = lane < it.nchains;
    const uint64_t amask = it.nchains >= 64 ? ~0ull : ((1ull << it.nchains) - 1ull);
    const Key key{sm.key0, sm.key1};
    uint64_t *S = lds_bs;
    uint64_t *Gm = lds_bs + n;
    uint64_t *M = lds_bs + 2 * n;
    uint64_t *Pw = M + sm.msel_total;
    uint32_t *Q = (uint32_t *)(Pw + G) + wave * kQCap;

    // transpose the chains' packed words into node masks
    for (uint32_t w = wave; w < W; w += G) {
        const uint32_t word = active ? sm.state[(size_t)w * omega + c] : 0u;
        const uint32_t nb = min(32u, n - 32 * w);
        for (uint32_t b = 0; b < nb; ++b) {
            const uint64_t m = __ballot((word >> b) & 1u);
            if (lane == 0) S[32 * w + b] = m;
        }
    }
    for (uint32_t i = threadIdx.x; i < n; i += 64 * G) Gm[i] = 0ull;
    if (threadIdx.x < G) Pw[threadIdx.x] = 0ull;

    uint32_t acc[kMaxProps];
    uint64_t pos = it.pos0;
    const uint32_t nprops = sm.nprops;
#pragma unroll
    for (uint32_t q = 0; q < kMaxProps; ++q) {
        acc[q] = 0;
        if (wave == 0 && active && q < nprops && it.nrec > 0 && (pos & 31)) {
            const uint32_t old = sm.bits[((size_t)q * sm.words_cap + (pos >> 5)) * omega + c];
            acc[q] = old & ((1u << (pos & 31)) - 1u);
        }
    }
    __syncthreads();

    const uint32_t p_thr = sm.p_thr, thr8 = p_thr >> 24;
    const uint32_t nblk = sm.nblk, F_pad = sm.F_pad;
    const uint32_t total = it.nburn + it.nrec * it.thin;
    uint32_t since = 0;
    for (uint32_t s = 0; s < total; ++s) {
        const uint32_t t = it.t0 + s;
        // ---- A: draws, lane = chain
        uint64_t P_acc = 0;
        uint32_t qlen = 0;
        for (uint32_t b = wave; b < nblk; b += G) {
            const uint32_t i0 = 16 * b, ib = min(16u, n - i0);
            uint32_t wp[4];
            philox4(t, c, b, kTagPert, key, wp);
#pragma unroll
            for (uint32_t k = 0; k < 16; ++k) {
                if (k >= ib) break;
                const uint32_t byte = (wp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                if (thr8 > 0) {
                    const uint64_t d1 = __ballot(byte < thr8) & amask;
                    if (d1) {
                        if (lane == 0) atomicOr((unsigned long long *)&Gm[i0 + k], (unsigned long long)d1);
                        P_acc |= d1;
                    }
                }
                const uint64_t tie = __ballot(byte == thr8) & amask;
                if (tie) enqueue(tie, i0 + k, lane, Q, qlen, sm, key, t, chain0, Gm, M, &Pw[wave]);
            }
            if (sm.blk_sel[b]) {
                uint32_t ws[4];
                philox4(t, c, b, kTagSel, key, ws);
#pragma unroll
                for (uint32_t k = 0; k < 16; ++k) {
                    if (k >= ib) break;
                    const uint32_t i = i0 + k;
                    const uint32_t meta = sm.nd_meta[i];
                    const uint32_t l = meta & 0xFFu;
                    if (l < 2) continue;
                    const uint32_t moff = meta >> 8;
                    const uint32_t byte = (ws[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                    const uint32_t tbs = sm.nd_tb[i];
                    for (uint32_t j = 0; j + 1 < l; ++j) {
                        const uint32_t tb = j < 3 ? (tbs >> (8 * j)) & 0xFFu : sm.fn_thr[sm.nd_first[i] + j] >> 24;
                        const uint64_t lt = __ballot(byte < tb) & amask;
                        if (lane == 0) M[moff + j] = lt;
                        const uint64_t eq = __ballot(byte == tb) & amask;
                        if (eq) enqueue(eq, i | (j << 16) | (1u << 22), lane, Q, qlen, sm, key, t, chain0, Gm, M, &Pw[wave]);
                    }
                }
            }
        }
        if (qlen) resolve_queue(sm, key, t, chain0, Q, qlen, Gm, M, &Pw[wave], lane);
        if (P_acc && lane == 0) atomicOr((unsigned long long *)&Pw[wave], (unsigned long long)P_acc);
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
            const uint32_t K = sm.fg_K[s0 >> 6];
            const uint32_t node = sm.fs_node[slot];
            uint64_t x[6];
#pragma unroll
            for (uint32_t m = 0; m < 6; ++m) x[m] = (m < K) ? S[sm.fs_par[(size_t)m * F_pad + slot]] : 0ull;
            const uint64_t f = eval_slot(K, sm.fs_tt_lo[slot], sm.fs_tt_hi[slot], x);
            const uint32_t mlo = sm.fs_mlo[slot], mhi = sm.fs_mhi[slot];
            const uint64_t below = mlo == kNoMask ? 0ull : M[mlo];
            const uint64_t upto = mhi == kNoMask ? ~0ull : M[mhi];
            if (node != kNoNode) {
                const uint64_t v = f & upto & ~below & nP;
                if (v) atomicOr((unsigned long long *)&Gm[node], (unsigned long long)v);
            }
        }
        __syncthreads();

        // ---- D: record, clear, swap (Pw was last read in B, before C's barrier)
        if (s >= it.nburn && ++since == it.thin) {
            since = 0;
            if (wave == 0) {
                const uint32_t bpos = (uint32_t)(pos & 31);
#pragma unroll
                for (uint32_t q = 0; q < kMaxProps; ++q) {
                    if (q < nprops) {
                        uint64_t xm = ~0ull;
                        for (uint32_t m = sm.pn_off[q]; m < sm.pn_off[q + 1]; ++m) {
                            const uint64_t v = Gm[sm.pn_node[m]];
                            xm &= sm.pn_val[m] ? v : ~v;
                        }
                        acc[q] |= (uint32_t)((xm >> lane) & 1ull) << bpos;
                    }
                }
                if (bpos == 31 && active) {
#pragma unroll
                    for (uint32_t q = 0; q < kMaxProps; ++q) {
                        if (q < nprops) {
                            sm.bits[((size_t)q * sm.words_cap + (pos >> 5)) * omega + c] = acc[q];
                            acc[q] = 0;
                        }
                    }
                }
            }
            ++pos;
        }
        for (uint32_t i = threadIdx.x; i < n; i += 64 * G) S[i] = 0ull;
        if (threadIdx.x < G) Pw[threadIdx.x] = 0ull;
        uint64_t *tmp = S; S = Gm; Gm = tmp;
        __syncthreads();
    }

    if (wave == 0 && active && it.nrec > 0 && (pos & 31)) {
#pragma unroll
        for (uint32_t q = 0; q < kMaxProps; ++q)
            if (q < nprops) sm.bits[((size_t)q * sm.words_cap + (pos >> 5)) * omega + c] = acc[q];
    }
    // transpose back
    for (uint32_t w = wave; w < W; w += G) {
        uint32_t word = 0;
        const uint32_t nb = min(32u, n - 32 * w);
        for (uint32_t b = 0; b < nb; ++b) word |= (uint32_t)((S[32 * w + b] >> lane) & 1ull) << b;
        if (active) sm.state[(size_t)w * omega + c] = word;
    }
}

// ------------------------------------------------------------------ reduce

// Bits [lo, hi) of a word starting at position 32*wi, as a mask.
__device__ __forceinline__ uint32_t range_mask(uint64_t wi, uint64_t lo, uint64_t hi)
{
    const uint64_t base = wi * 32;
    const uint64_t a = lo > base ? lo - base : 0;
    const uint64_t b = hi - base >= 32 ? 32 : hi - base;
    if (b <= a) return 0;
    const uint32_t upto = b == 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
    return upto & ~((1u << a) - 1u);
}

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *scratch)
{
    // wave64 reduction then across the 4 waves of a 256-thread block
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    int64_t tot = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += scratch[w];
    __syncthreads();
    return tot;
}

// One 256-thread block per query.
__global__ void __launch_bounds__(256) k_reduce(const Query *__restrict__ qs, WindowResult *__restrict__ win,
                                                int32_t *__restrict__ bsum)
{
    __shared__ int64_t scratch[8];
    const Query qy = qs[blockIdx.x];
    const DevSim &sm = *qy.sim;
    const uint32_t omega = sm.omega;
    const uint32_t *bits = sm.bits + (size_t)qy.prop * sm.words_cap * omega;
    if (qy.kind == kQueryWindow) {
        int64_t T1 = 0, T2 = 0, n01 = 0, n10 = 0, n11 = 0;
        const uint64_t lo = qy.lo, hi = qy.hi;
        const uint64_t w0 = lo >> 5, w1 = (hi + 31) >> 5;
        for (uint32_t c = threadIdx.x; c < omega; c += blockDim.x) {
            int64_t S = 0;
            uint32_t x = w0 < w1 ? bits[w0 * omega + c] : 0u;
            for (uint64_t wi = w0; wi < w1; ++wi) {
                const uint32_t nx = (wi + 1 < w1) ? bits[(wi + 1) * omega + c] : 0u;
                const uint32_t m = range_mask(wi, lo, hi);
                S += __popc(x & m);
                // pair (l, l+1) counted at l when both lie in [lo, hi)
                const uint32_t pm = range_mask(wi, lo, hi - 1 > lo ? hi - 1 : lo);
                const uint32_t y = (x >> 1) | (nx << 31);
                n11 += __popc(x & y & pm);
                n10 += __popc(x & ~y & pm);
                n01 += __popc(~x & y & pm);
                x = nx;
            }
            T1 += S;
            T2 += S * S;
        }
        T1 = block_sum(T1, scratch);
        T2 = block_sum(T2, scratch);
        n01 = block_sum(n01, scratch);
        n10 = block_sum(n10, scratch);
        n11 = block_sum(n11, scratch);
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

int launch_step(const StepItem *d_items, uint32_t nitems, uint32_t max_W, void *stream, std::string &err)
{
    if (nitems == 0) return PBN_OK;
    const uint32_t S = max_W | 1u;
    const size_t lds = (size_t)2 * 64 * S * 4;
    if (lds > 160 * 1024) {
        err = "state rows exceed LDS";
        return PBN_ELIMIT;
    }
    hipLaunchKernelGGL(k_step, dim3(nitems), dim3(64), lds, (hipStream_t)stream, d_items, S);
    return check(hipGetLastError(), "k_step launch", err);
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
        if (e != hipSuccess) return check(e, "k_step_bs LDS attribute", err);
    }
    hipLaunchKernelGGL(k_step_bs<G>, dim3(nitems), dim3(64 * G), lds, s, d_items);
    return check(hipGetLastError(), "k_step_bs launch", err);
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
    default: return launch_bs_g<4>(d_items, nitems, lds, s, err);
    }
}

int launch_reduce(const Query *d_queries, uint32_t nq, WindowResult *d_win, int32_t *d_bsum, void *stream,
                  std::string &err)
{
    if (nq == 0) return PBN_OK;
    hipLaunchKernelGGL(k_reduce, dim3(nq), dim3(256), 0, (hipStream_t)stream, d_queries, d_win, d_bsum);
    return check(hipGetLastError(), "k_reduce launch", err);
}

}  // namespace pbn
