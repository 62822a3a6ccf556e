// Bit-sliced trajectory kernel (gfx950, wave64).
//
// One block of G waves (G = blockDim.x / 64, 1..16) advances 64 chains.  State
// is bit-sliced in LDS: S[i] holds node i of all 64 chains (bit = lane =
// chain).  Wave w owns the 16-node blocks b = w, w + G, ...  Per transition:
//   A  lane = chain, own blocks: each lane draws its chain's perturbation and
//      selection bytes for the block (one Philox evaluation each).  Selection
//      masks m_j = [u < T_j] come from one ballot per (node, threshold) and are
//      written whole into M.  Perturbations are rare: bytes below the primary
//      threshold flip at once (only when p >= 2^-8), bytes equal to it are
//      ties.  Ties of either kind are queued per lane and block as bit flags
//      and resolved with the 24-bit refinement words, 64 queue entries per
//      pass.  Flips go into Gm[i] (the next state, zero so far), the chains
//      with any flip into this wave's word of P.
//   -- barrier (P complete, every M written)
//   C  lane = predictor slot (sorted by parent count): K-input multiplexer
//      tree over the parents' masks, restricted to the chains that selected
//      this predictor and were not perturbed, OR-ed into Gm[node]; before
//      that, wave w records the indicators of state sets w, w + G, ... for the
//      state reached by the previous transition
//   -- barrier (every slot done)
//   D  own nodes: Gm[i] ^= P & S[i] (perturbed chains: S XOR gamma, the
//      others keep the functions' values), S[i] := 0 (the next transition's
//      Gm); swap S and Gm.  The next A touches only the same wave's nodes, so
//      no barrier follows D; P is double-buffered by transition parity.
// LDS (u64 words): S[n], Gm[n], M[msel_total], Pw[2][G], then per wave a queue
// of kQCap entries (three u32 arrays: header, flags low, flags high), then the
// indicator words under construction (u32, [state set][lane]).
// Lanes beyond the item's chain count run along on their own bit positions and
// are never stored.
#include "pbn_device.h"

#include <algorithm>

namespace pbn {

// v_writelane: lane `lane` of `old` takes the wave-uniform value `src`.
__device__ uint32_t amdgcn_writelane(uint32_t src, uint32_t lane, uint32_t old) __asm("llvm.amdgcn.writelane.i32");

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

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

// Bit e of w as an all-zeros or all-ones word (one signed bit-field extract).
__device__ __forceinline__ uint32_t bit_mask(uint32_t w, int e)
{
    return (uint32_t)(((int32_t)(w << (31 - e))) >> 31);
}

// Multiplexer tree, evaluated depth first so that at most one partial result
// per level is live: node (LEV, BASE) selects between the subtrees of table
// indices BASE.. and BASE + 2^LEV.. with parent mask x[LEV]; level 0 picks
// table bit BASE or BASE + 1 with x[0].
template <int LEV, int BASE>
struct Mux {
    static __device__ __forceinline__ uint64_t eval(uint32_t lo, uint32_t hi, const uint64_t *x)
    {
        const uint64_t a = Mux<LEV - 1, BASE>::eval(lo, hi, x);
        const uint64_t b = Mux<LEV - 1, BASE + (1 << LEV)>::eval(lo, hi, x);
        return bsel(x[LEV], b, a);
    }
};

template <int BASE>
struct Mux<0, BASE> {
    static __device__ __forceinline__ uint64_t eval(uint32_t lo, uint32_t hi, const uint64_t *x)
    {
        constexpr int e0 = BASE, e1 = BASE + 1;
        const uint32_t w0 = e0 < 32 ? lo : hi, w1 = e1 < 32 ? lo : hi;
        // table bits e0 / e1 broadcast to whole words, selected by x0
        const uint32_t A = bit_mask(w0, e0 & 31), B = bit_mask(w1, e1 & 31);
        const uint32_t x0l = (uint32_t)x[0], x0h = (uint32_t)(x[0] >> 32);
        const uint32_t rl = (x0l & B) | (~x0l & A), rh = (x0h & B) | (~x0h & A);
        return ((uint64_t)rh << 32) | rl;
    }
};

template <int K>
__device__ __forceinline__ uint64_t mux_tree(uint32_t lo, uint32_t hi, const uint64_t *x)
{
    return Mux<K - 1, 0>::eval(lo, hi, x);
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

// Bit 7 of byte j of the result is set iff byte j of x equals the byte m
// (m4 = m * 0x01010101).  No carry crosses a byte, so every byte is exact.
__device__ __forceinline__ uint32_t bytes_eq(uint32_t x, uint32_t m4)
{
    const uint32_t y = x ^ m4;
    return ~(((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y | 0x7F7F7F7Fu);
}

// Queue entry: header and a 64-bit flag word (lo, hi).
//   kind 0, perturbation ties of chain lane: header 0 | lane << 1 | block << 7,
//     flag 8 bb + q = node 16 b + 4 q + bb
//   kind 1, selection ties of threshold j of node k (of block b):
//     header 1 | k << 1 | j << 5 | block << 7, flag x = chain x
__device__ __forceinline__ void push(bool mine, uint32_t hdr, uint32_t flo, uint32_t fhi, uint32_t *Q,
                                     uint32_t &qlen)
{
    const uint64_t who = __ballot(mine);
    if (who) {
        if (mine) {
            const uint32_t pos = qlen + __builtin_amdgcn_mbcnt_hi((uint32_t)(who >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)who, 0u));
            Q[pos] = hdr;
            Q[kQCap + pos] = flo;
            Q[2 * kQCap + pos] = fhi;
        }
        qlen += (uint32_t)__popcll(who);
    }
}

// Resolve queued ties with the refinement words (stream tag + 1), lane = entry.
// Both kinds run one code path: a selection entry's node, threshold and mask
// index are fixed per entry (loaded before its flags are walked), a
// perturbation entry's chain is; each flag then names the other coordinate,
// and a refined draw below the threshold sets one bit of an LDS word (the mask
// M for a selection, the next state Gm for a perturbation).
__device__ __forceinline__ void resolve(const BsView &v, uint32_t t, uint32_t chain0, const uint32_t *Q,
                                        uint32_t qlen, uint64_t *Gm, uint32_t i_lo, uint64_t *M, uint32_t m_lo,
                                        uint64_t *Pw_mine, uint32_t lane)
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint32_t pthr24 = v.p_thr & 0xFFFFFFu;
    for (uint32_t e = lane; e < qlen; e += 64) {
        const uint32_t hdr = Q[e];
        const bool sel = (hdr & 1u) != 0;
        const uint32_t b = hdr >> 7;
        uint64_t f = (uint64_t)Q[kQCap + e] | ((uint64_t)Q[2 * kQCap + e] << 32);
        const uint32_t tag = (sel ? kTagSel : kTagPert) + 1;
        // per entry: a selection's node i_s, threshold (low 24 bits) and mask word;
        // a perturbation's chain
        const uint32_t i_s = 16 * b + ((hdr >> 1) & 15u), j_s = (hdr >> 5) & 3u;
        uint32_t thr = pthr24, midx = 0;
        if (sel) {
            thr = v.fn_thr[v.nd_first[i_s] + j_s] & 0xFFFFFFu;
            midx = (v.nd_info[2 * i_s] >> 8) + j_s - m_lo;
        }
        const uint32_t cl_p = (hdr >> 1) & 63u;
        uint32_t rq = 0xFFFFFFFFu, r[4] = {0u, 0u, 0u, 0u};
        bool flipped = false;
        while (f) {
            const uint32_t x = (uint32_t)__builtin_ctzll(f);
            f &= f - 1;
            const uint32_t cl = sel ? x : cl_p;
            const uint32_t i = sel ? i_s : 16 * b + 4 * (x & 7u) + (x >> 3);
            const uint32_t key = (cl << 24) | (i >> 2);
            if (key != rq) {
                rq = key;
                philox4(t, chain0 + cl, i >> 2, tag, v.key, r);
            }
            const uint32_t r24 = pick4(r, i & 3u) & 0xFFFFFFu;
            if (r24 < thr) {
                lds_or(sel ? &M[midx] : &Gm[i - i_lo], 1ull << cl);
                flipped |= !sel;
            }
        }
        if (flipped) lds_or(Pw_mine, 1ull << cl_p);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// A register with no defined contents and no instruction to produce it, for
// accumulators whose lanes are read only after being written.
__device__ __forceinline__ uint32_t unspecified()
{
    uint32_t x;
    asm volatile("" : "=v"(x));
    return x;
}

// A-phase work of one 16-node block b, lane = chain: the perturbation draws
// (flips into Gm, chains with a flip into P_acc, ties queued) and, when some
// node of the block has two or more predictors (lmax >= 2), the selection
// draws (masks into M, ties queued).  Gm is indexed from node i_lo, M from
// mask m_lo.
__device__ __forceinline__ void draw_block(const BsView &v, uint32_t t, uint32_t c, uint32_t lane, uint32_t b,
                                           uint32_t lmax, uint32_t thr8, uint32_t thr8x4, uint64_t *Gm,
                                           uint32_t i_lo, uint64_t *M, uint32_t m_lo, uint32_t *Q, uint32_t &qlen,
                                           uint64_t &P_acc)
{
    const uint32_t n = v.n, i0 = 16 * b, ib = min(16u, n - i0);
    uint32_t wp[4];
    philox4(t, c, b, kTagPert, v.key, wp);
    // tie flags: bit 8 bb + q <-> node 4 q + bb (byte bb of word q)
    uint32_t tie = (bytes_eq(wp[0], thr8x4) >> 7) | (bytes_eq(wp[1], thr8x4) >> 6) |
                   (bytes_eq(wp[2], thr8x4) >> 5) | (bytes_eq(wp[3], thr8x4) >> 4);
    if (ib < 16) {
        uint32_t valid = 0;
        for (uint32_t bb = 0; bb < 4; ++bb) {
            const uint32_t cnt = ib > bb ? (ib - bb + 3) >> 2 : 0u;   // words q with 4 q + bb < ib
            valid |= ((1u << cnt) - 1u) << (8 * bb);
        }
        tie &= valid;
    }
    if (thr8 > 0) {
        // bytes below the primary threshold flip at once
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) {
            if (k < ib) {
                const uint32_t byte = (wp[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                const uint64_t d1 = __ballot(byte < thr8);
                if (d1) {
                    if (lane == 0) lds_or(&Gm[i0 + k - i_lo], d1);
                    P_acc |= d1;
                }
            }
        }
    }
    push(tie != 0, (lane << 1) | (b << 7), tie, 0u, Q, qlen);
    if (lmax >= 2) {
        uint32_t ws[4];
        philox4(t, c, b, kTagSel, v.key, ws);
        // one ballot per (node k, threshold j < 3) against the top byte of
        // T_j (uniform, from scalar loads); lane k of a[j] gathers node k's
        // mask, and each (node, threshold) with equal bytes is queued with
        // its chain flags
        const PBN_CAS uint32_t *info = v.nd_info + 32 * (size_t)b;
        const PBN_CAS u32x8 *quads = (const PBN_CAS u32x8 *)info;
        // lanes of al, ah (masks) and eh, el, eu (queued ties) are read only
        // where they were written, so they start unspecified (no register
        // copies to clear them); mv must start at 0 (l = 0: no masks)
        uint32_t al[3] = {unspecified(), unspecified(), unspecified()};
        uint32_t ah[3] = {unspecified(), unspecified(), unspecified()};
        uint32_t eh = unspecified(), el = unspecified(), eu = unspecified(), ne = 0;
        uint32_t mv = 0;                  // lane k: node k's record (l | mask offset << 8)
        // node records four at a time (one scalar load each), the next
        // quad's load issued before the current quad's compares
        u32x8 rq = quads[0], rn = rq;
#pragma unroll
        for (uint32_t k = 0; k < 16; ++k) {
            if ((k & 3u) == 0) {
                rq = rn;
                if (k < 12) rn = quads[(k >> 2) + 1];
            }
            const uint32_t tbs = rq[2 * (k & 3u) + 1];
            const uint32_t l = tbs >> 24;     // 0 for nodes past n
            if (l < 2) continue;
            mv = amdgcn_writelane(rq[2 * (k & 3u)], k, mv);
            const uint32_t byte = (ws[k >> 2] >> (8 * (k & 3))) & 0xFFu;
#pragma unroll
            for (uint32_t j = 0; j < 3; ++j) {
                if (j + 2 > l) break;
                const uint32_t tb = (tbs >> (8 * j)) & 0xFFu;
                const uint64_t lt = __ballot(byte < tb);
                const uint64_t eq = __ballot(byte == tb);
                al[j] = amdgcn_writelane((uint32_t)lt, k, al[j]);
                ah[j] = amdgcn_writelane((uint32_t)(lt >> 32), k, ah[j]);
                if (eq) {
                    eh = amdgcn_writelane(1u | (k << 1) | (j << 5) | (b << 7), ne, eh);
                    el = amdgcn_writelane((uint32_t)eq, ne, el);
                    eu = amdgcn_writelane((uint32_t)(eq >> 32), ne, eu);
                    ++ne;
                }
            }
        }
        {
            const uint32_t l = mv & 0xFFu, moff = mv >> 8;
#pragma unroll
            for (uint32_t j = 0; j < 3; ++j)
                if (j + 2 <= l) M[moff + j - m_lo] = ((uint64_t)ah[j] << 32) | al[j];
        }
        if (ne) {
            if (lane < ne) {
                Q[qlen + lane] = eh;
                Q[kQCap + qlen + lane] = el;
                Q[2 * kQCap + qlen + lane] = eu;
            }
            qlen += ne;
        }
        if (lmax >= 5) {
            // thresholds 4.. of nodes with more than four predictors,
            // straight from fn_thr with their ties refined in place
            for (uint32_t k = 0; k < ib; ++k) {
                const uint32_t meta = info[2 * k];
                const uint32_t l = meta & 0xFFu;
                if (l < 5) continue;
                const uint32_t i = i0 + k;
                const uint32_t byte = (pick4(ws, k >> 2) >> (8 * (k & 3))) & 0xFFu;
                for (uint32_t j = 3; j + 1 < l; ++j) {
                    const uint32_t T = v.fn_thr[v.nd_first[i] + j];
                    const uint32_t tb = T >> 24;
                    bool below = byte < tb;
                    const bool eq = byte == tb;
                    if (__ballot(eq)) {
                        if (eq) below = refine24(v.key, t, c, i, kTagSel) < (T & 0xFFFFFFu);
                    }
                    const uint64_t lt = __ballot(below);
                    if (lane == 0) M[(meta >> 8) + j - m_lo] = lt;
                }
            }
        }
    }
}

extern __shared__ uint64_t lds_bs[];

// SMALL: every wave owns at most one 16-node block and one 64-slot group (the
// host launches it only then), whose metadata stay in registers; the general
// form reloads them per transition and spends no registers on them.
template <bool SMALL>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) k_step_bs(const StepItem *__restrict__ items)
{
    const StepItem it = load_item(items, blockIdx.x);
    if (it.nchains == 0) return;         // padding of an XCD-aware launch
    const BsView v = load_bs_view(it.sim);
    const uint32_t n = v.n, W = v.W, omega = v.omega;
    const uint32_t G = blockDim.x >> 6;
    const uint32_t lane = threadIdx.x & 63u;
    // wave index as a scalar: block and slot loops branch on the scalar unit
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t chain0 = it.chain0;
    const uint32_t c = chain0 + lane;
    const bool active = lane < it.nchains;
    uint64_t *S = lds_bs;
    uint64_t *Gm = lds_bs + n;
    uint64_t *M = lds_bs + 2 * n;
    uint64_t *Pw = M + v.msel_total;
    uint32_t *Q = (uint32_t *)(Pw + 2 * G) + wave * 3 * kQCap;
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
    if (threadIdx.x < 2 * G) Pw[threadIdx.x] = 0ull;

    // indicator words under construction, one per state set and chain, in LDS
    // (state set q is recorded by wave q mod G)
    uint32_t *acc = (uint32_t *)(Pw + 2 * G) + G * 3 * kQCap + lane;
    uint64_t pos = it.pos0;
    const uint32_t nprops = v.nprops;
    if (wave == 0) {
        for (uint32_t q = 0; q < nprops; ++q) {
            uint32_t a = 0;
            if (active && it.nrec > 0 && (pos & 31)) {
                gu32 bits = (gu32)v.d->bits;
                const uint32_t old = bits[((size_t)q * words_cap + (pos >> 5)) * omega + c];
                a = old & ((1u << (pos & 31)) - 1u);
            }
            acc[64 * q] = a;
        }
    }
    __syncthreads();

    const uint32_t p_thr = v.p_thr, thr8 = p_thr >> 24, thr8x4 = thr8 * 0x01010101u;
    const uint32_t nblk = v.nblk, F_pad = v.F_pad;
    // Small networks: at most one node block and one slot group per wave, whose
    // metadata then stay in registers for the whole launch.
    // (the small form keeps them register-resident; the flags stay run-time so
    // the compiler does not trade registers for the single-iteration loops)
    const bool res_a = SMALL && nblk <= G, res_c = SMALL && F_pad <= 64 * G;
    uint32_t ra_lmax = 0;
    if (res_a && wave < nblk) ra_lmax = v.blk_sel[wave];
    uint32_t rc_K = 1;
    u32x4 rc0 = {0u, 0u, 0u, 0u}, rc1 = {0u, 0u, 0u, 0u};
    if (res_c && 64 * wave < F_pad) {
        rc_K = v.fg_K[wave];
        const PBN_CAS u32x4 *rec = (const PBN_CAS u32x4 *)(v.fs_rec + 8 * (size_t)(64 * wave + lane));
        rc0 = rec[0];
        rc1 = rec[1];
    }
    const uint32_t total = it.nburn + it.nrec * it.thin;
    uint32_t since = 0;
    bool pending = false;             // the state in S awaits recording
    // the indicators of the current state S, at position pos (this wave's state sets)
    auto record = [&]() {
        const uint32_t bpos = (uint32_t)(pos & 31);
        for (uint32_t q = wave; q < nprops; q += G) {
            uint64_t xm = ~0ull;
            for (uint32_t m = v.d->pn_off[q]; m < v.d->pn_off[q + 1]; ++m) {
                const uint64_t sv = S[v.d->pn_node[m]];
                xm &= v.d->pn_val[m] ? sv : ~sv;
            }
            const uint32_t a = acc[64 * q] | ((uint32_t)((xm >> lane) & 1ull) << bpos);
            if (bpos == 31) {
                if (active) ((gu32)v.d->bits)[((size_t)q * words_cap + (pos >> 5)) * omega + c] = a;
                acc[64 * q] = 0;
            } else {
                acc[64 * q] = a;
            }
        }
    };
    for (uint32_t s = 0; s < total; ++s) {
        const uint32_t t = it.t0 + s;
        uint64_t *Pt = Pw + (s & 1) * G;  // this transition's perturbed-chain words
        // ---- A: draws, lane = chain
        uint64_t P_acc = 0;
        uint32_t qlen = 0;
        if (lane == 0) Pt[wave] = 0ull;   // last read two transitions ago
        for (uint32_t b = wave;; b += G) {
            const bool last = b >= nblk;
            // a block queues at most 128 entries: resolve before the queue could overflow
            if (qlen != 0 && (last || qlen + 128 > kQCap)) {
                resolve(v, t, chain0, Q, qlen, Gm, 0u, M, 0u, &Pt[wave], lane);
                qlen = 0;
            }
            if (last) break;
            draw_block(v, t, c, lane, b, res_a ? ra_lmax : v.blk_sel[b], thr8, thr8x4, Gm, 0u, M, 0u, Q, qlen, P_acc);
        }
        if (P_acc && lane == 0) lds_or(&Pt[wave], P_acc);
        __syncthreads();

        // ---- C: predictor slots, lane = slot
        if (pending) {
            record();
            ++pos;
        }
        pending = false;
        uint64_t P = 0;
        for (uint32_t w = 0; w < G; ++w) P |= Pt[w];
        const uint64_t nP = ~P;
        for (uint32_t s0 = 64 * wave; s0 < F_pad; s0 += 64 * G) {
            const uint32_t slot = s0 + lane;
            uint32_t K = rc_K;
            u32x4 r0 = rc0, r1 = rc1;
            if (!res_c) {
                K = v.fg_K[s0 >> 6];
                const PBN_CAS u32x4 *rec = (const PBN_CAS u32x4 *)(v.fs_rec + 8 * (size_t)slot);
                r0 = rec[0];
                r1 = rec[1];
            }
            const uint32_t node = r0.x, tlo = r0.y, thi = r0.z, mlo = r0.w, mhi = r1.x;
            const uint32_t p01 = r1.y, p23 = r1.z, p45 = r1.w;
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

        // ---- D: own nodes, lane = (block, node); blocks w + G m, four per pass
        for (uint32_t m0 = 0;; m0 += 4) {
            const uint32_t b0 = wave + G * m0;
            if (b0 >= nblk) break;
            const uint32_t b = wave + G * (m0 + (lane >> 4)), i = 16 * b + (lane & 15u);
            if (b < nblk && i < n) {
                Gm[i] ^= P & S[i];
                S[i] = 0ull;
            }
        }
        if (s >= it.nburn && ++since == it.thin) {
            since = 0;
            pending = true;
        }
        uint64_t *tmp = S; S = Gm; Gm = tmp;
    }
    __syncthreads();
    if (pending) {
        record();
        ++pos;
    }

    if (active && it.nrec > 0 && (pos & 31)) {
        gu32 bits = (gu32)v.d->bits;
        for (uint32_t q = wave; q < nprops; q += G)
            bits[((size_t)q * words_cap + (pos >> 5)) * omega + c] = acc[64 * q];
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

// Node-split form.  P blocks (on P CUs) share one 64-chain group: block r of
// the group owns the 16-node blocks [tab[r], tab[r + 1]) and the predictor
// slot groups [tab[P + 1 + r], tab[P + 2 + r]) of those nodes.  Each keeps the
// whole state S in LDS (every slot may read any parent) but only its own
// nodes' next-state words, function values and selection masks.  Per
// transition s (A of the first transition runs before the loop):
//   C  own slots: the K-input multiplexers, restricted to the chains that
//      selected the predictor, OR-ed into Fm[node] (the function values)
//   -- barrier
//   X1 with Pr the chains this block perturbed, publish for every own node
//      h_i = Pr & (S_i ^ flips_i) | ~Pr & f_i and the word Pr to the group's
//      exchange area, each 64-bit word a 32-bit half tagged with the
//      transition (h_i kept in Fm, the flips cleared)
//   -- barrier
//   A  transition s + 1's draws on the own blocks, as in the one-block form:
//      flips into Gm, masks into M (they read no state)
//   X2 read every other part's words, polling each until it carries this
//      transition's tag: node i of part q becomes h_i, except in the chains
//      perturbed by another part only, which keep S_i
//   -- barrier
// The wait is bounded: a block that polls about a second gives up.  The
// group's status word then decides, once, between the two ends of the
// launch: a block that gives up moves it from 0 to 1 (aborted), block 0 moves
// it from 0 to 2 (complete) after the last transition.  An aborted group never
// writes its state back, so the host re-runs it in the one-block form from the
// state it started from; the other blocks of an aborted group see the word
// and stop polling.  Block 0 records the indicators (state set q by its wave
// q mod G) and writes the state back.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) k_step_split(const StepItem *__restrict__ items)
{
    const StepItem it = load_item(items, blockIdx.x);
    if (it.nchains == 0) return;         // padding of an XCD-aware launch
    const BsView v = load_bs_view(it.sim);
    const PBN_CAS SplitGroup *sg = (const PBN_CAS SplitGroup *)it.grp;
    const uint32_t P = sg->nparts, r = it.part, groups = sg->groups, max_spins = sg->spins;
    const cu32 tab = (cu32)sg->tab;
    PBN_GAS uint64_t *xch = (PBN_GAS uint64_t *)sg->xch;
    PBN_GAS uint32_t *gstat = (PBN_GAS uint32_t *)sg->stat;
    const uint32_t n = v.n, W = v.W, omega = v.omega;
    const uint32_t G = blockDim.x >> 6;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t chain0 = it.chain0;
    const uint32_t c = chain0 + lane;
    const bool active = lane < it.nchains;
    const uint32_t blo = tab[r], bhi = tab[r + 1], glo = tab[P + 1 + r], ghi = tab[P + 2 + r];
    const uint32_t i_lo = 16 * blo, i_hi = min(16 * bhi, n), n_own = i_hi - i_lo;
    const uint32_t m_lo = v.nd_info[2 * i_lo] >> 8;
    const uint32_t m_hi = i_hi < n ? v.nd_info[2 * i_hi] >> 8 : v.msel_total;
    const cu32 fgK = tab + split_head(P);
    const cu32 rec = tab + split_rec_off(P, groups);
    uint64_t *S = lds_bs;
    uint64_t *Gm = S + n;
    uint64_t *Fm = Gm + n_own;
    uint64_t *M = Fm + n_own;
    uint64_t *Pw = M + (m_hi - m_lo);
    uint32_t *Q = (uint32_t *)(Pw + 2 * G) + wave * 3 * kQCap;
    uint32_t *acc = (uint32_t *)(Pw + 2 * G) + G * 3 * kQCap + lane;
    uint32_t *abort_flag = (uint32_t *)(Pw + 2 * G) + G * 3 * kQCap + 64 * kMaxProps;
    uint64_t *xpl = (uint64_t *)(abort_flag + 2);          // the parts' perturbed-chain words, a row per wave
    uint8_t *owner = (uint8_t *)(xpl + kSplitMaxParts * G); // part of each 16-node block
    const uint64_t words_cap = v.d->words_cap;
    const bool recorder = r == 0;

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
    for (uint32_t i = threadIdx.x; i < n_own; i += 64 * G) Gm[i] = Fm[i] = 0ull;
    for (uint32_t i = threadIdx.x; i < m_hi - m_lo; i += 64 * G) M[i] = 0ull;
    if (threadIdx.x < 2 * G) Pw[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) *abort_flag = 0u;
    for (uint32_t b = threadIdx.x; b < v.nblk; b += 64 * G) {
        uint32_t q = 0;
        while (q + 1 < P && tab[q + 1] <= b) ++q;
        owner[b] = (uint8_t)q;
    }
    uint64_t pos = it.pos0;
    const uint32_t nprops = v.nprops;
    if (wave == 0 && recorder) {
        for (uint32_t q = 0; q < nprops; ++q) {
            uint32_t a = 0;
            if (active && it.nrec > 0 && (pos & 31)) {
                gu32 bits = (gu32)v.d->bits;
                const uint32_t old = bits[((size_t)q * words_cap + (pos >> 5)) * omega + c];
                a = old & ((1u << (pos & 31)) - 1u);
            }
            acc[64 * q] = a;
        }
    }
    __syncthreads();

    const uint32_t p_thr = v.p_thr, thr8 = p_thr >> 24, thr8x4 = thr8 * 0x01010101u;
    const uint32_t total = it.nburn + it.nrec * it.thin;
    uint32_t since = 0;
    bool pending = false;
    auto record = [&]() {
        const uint32_t bpos = (uint32_t)(pos & 31);
        for (uint32_t q = wave; q < nprops; q += G) {
            uint64_t xm = ~0ull;
            for (uint32_t m = v.d->pn_off[q]; m < v.d->pn_off[q + 1]; ++m) {
                const uint64_t sv = S[v.d->pn_node[m]];
                xm &= v.d->pn_val[m] ? sv : ~sv;
            }
            const uint32_t a = acc[64 * q] | ((uint32_t)((xm >> lane) & 1ull) << bpos);
            if (bpos == 31) {
                if (active) ((gu32)v.d->bits)[((size_t)q * words_cap + (pos >> 5)) * omega + c] = a;
                acc[64 * q] = 0;
            } else {
                acc[64 * q] = a;
            }
        }
    };
    // ---- A: own blocks, lane = chain.  A draws only from the stream (t,
    // chain, node): it reads no state, so transition s + 1's draws run while
    // this part waits for the other parts' words of transition s.
    auto phase_a = [&](uint32_t s) {
        const uint32_t t = it.t0 + s;
        uint64_t *Pt = Pw + (s & 1) * G;
        uint64_t P_acc = 0;
        uint32_t qlen = 0;
        if (lane == 0) Pt[wave] = 0ull;
        for (uint32_t b = blo + wave;; b += G) {
            const bool last = b >= bhi;
            if (qlen != 0 && (last || qlen + 128 > kQCap)) {
                resolve(v, t, chain0, Q, qlen, Gm, i_lo, M, m_lo, &Pt[wave], lane);
                qlen = 0;
            }
            if (last) break;
            draw_block(v, t, c, lane, b, v.blk_sel[b], thr8, thr8x4, Gm, i_lo, M, m_lo, Q, qlen, P_acc);
        }
        if (P_acc && lane == 0) lds_or(&Pt[wave], P_acc);
    };
    if (total > 0) phase_a(0);
    __syncthreads();
    for (uint32_t s = 0; s < total; ++s) {
        const uint64_t *Pt = Pw + (s & 1) * G;

        // ---- C: own slots, lane = slot
        if (pending && recorder) {
            record();
            ++pos;
        }
        pending = false;
        for (uint32_t g = glo + wave; g < ghi; g += G) {
            const uint32_t K = fgK[g];
            const PBN_CAS u32x4 *rp = (const PBN_CAS u32x4 *)(rec + 8 * ((size_t)64 * g + lane));
            const u32x4 r0 = rp[0], r1 = rp[1];
            const uint32_t node = r0.x, tlo = r0.y, thi = r0.z, mlo = r0.w, mhi = r1.x;
            const uint32_t p01 = r1.y, p23 = r1.z, p45 = r1.w;
            uint64_t x[6];
            x[0] = S[p01 & 0xFFFFu];
            x[1] = K > 1 ? S[p01 >> 16] : 0ull;
            x[2] = K > 2 ? S[p23 & 0xFFFFu] : 0ull;
            x[3] = K > 3 ? S[p23 >> 16] : 0ull;
            x[4] = K > 4 ? S[p45 & 0xFFFFu] : 0ull;
            x[5] = K > 5 ? S[p45 >> 16] : 0ull;
            const uint64_t f = eval_slot(K, tlo, thi, x);
            if (node != kNoNode) {
                const uint64_t below = mlo == kNoMask ? 0ull : M[mlo - m_lo];
                const uint64_t upto = mhi == kNoMask ? ~0ull : M[mhi - m_lo];
                const uint64_t val = f & upto & ~below;
                if (val) lds_or(&Fm[node - i_lo], val);
            }
        }
        __syncthreads();

        // ---- X: exchange through the group's area, parity s & 1.  Own node i
        // is published as h_i = Pr & (S_i ^ flips_i) | ~Pr & f_i with Pr this
        // block's perturbed chains: exact for the chains this block perturbed
        // and for the unperturbed ones; the chains perturbed only in other
        // parts keep S_i, which every reader restores from its own S.
        // Every published 64-bit word is (tag << 32) | one 32-bit half of a
        // mask, tag = s + 1, stored and loaded whole (single-copy atomic), so
        // a reader polls the data itself until each word carries this
        // transition's tag: no counter, no wait for the stores to complete.
        // The area is zero at launch; the word a reader sees before the
        // owner's store is two transitions old (parity) or zero, never this
        // tag.  A reader that polls too long gives up (bounded wait).  A part
        // publishes transition s + 1 only after it has read every word of
        // transition s, so no word of parity s & 1 is overwritten while a
        // reader still needs it.
        PBN_GAS uint64_t *X = xch + (size_t)(s & 1) * 2 * n;
        PBN_GAS uint64_t *XP = xch + (size_t)4 * n + (size_t)(s & 1) * 2 * P;
        const uint64_t tag = (uint64_t)(s + 1) << 32;
        uint64_t Pr = 0;
        for (uint32_t w = 0; w < G; ++w) Pr |= Pt[w];
        for (uint32_t k = threadIdx.x; k < n_own; k += 64 * G) {
            const uint64_t h = (Pr & (S[i_lo + k] ^ Gm[k])) | (~Pr & Fm[k]);
            // h waits in Fm for this block's readers; the flips are consumed
            Fm[k] = h;
            Gm[k] = 0ull;
            __hip_atomic_store(&X[2 * (i_lo + k)], tag | (uint32_t)h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&X[2 * (i_lo + k) + 1], tag | (uint32_t)(h >> 32), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (threadIdx.x == 0) {
            __hip_atomic_store(&XP[2 * r], tag | (uint32_t)Pr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&XP[2 * r + 1], tag | (uint32_t)(Pr >> 32), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        // own words (Fm) complete and the flips cleared before the next draws
        // and before any thread applies them
        __syncthreads();
        if (s + 1 < total) phase_a(s + 1);

        // poll two words (the halves of one mask) until both carry the tag
        bool gave_up = false;
        auto fetch = [&](PBN_GAS uint64_t *w2, uint64_t &out) {
            uint64_t a0 = __hip_atomic_load(&w2[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t a1 = __hip_atomic_load(&w2[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t spins = 0;
            while (((a0 ^ tag) >> 32) | ((a1 ^ tag) >> 32)) {
                // another block of the group gave up: its words will not come
                if ((spins & 63u) == 63u &&
                    __hip_atomic_load(gstat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1u)
                    gave_up = true;
                if (gave_up || ++spins >= max_spins) {
                    gave_up = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                a0 = __hip_atomic_load(&w2[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                a1 = __hip_atomic_load(&w2[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            out = (a1 << 32) | (uint32_t)a0;
        };
        // every wave reads the parts' perturbed-chain words itself (lane q:
        // part q's, kept in the wave's own LDS row), so no barrier separates
        // them from the node words
        uint64_t xw = 0;
        if (lane < P) fetch(&XP[2 * lane], xw);
        uint64_t *xplw = xpl + (size_t)wave * kSplitMaxParts;
        if (lane < P) xplw[lane] = xw;
        uint64_t Pall = 0;
        for (uint32_t q = 0; q < P; ++q) Pall |= xplw[q];
        // node i of part q: h_i, except S_i in the chains perturbed outside q.
        // Every thread issues its next four nodes' loads before any result is
        // used; a batch whose words are not all there yet polls.  The loop is
        // uniform over the wave (lanes past n load nothing).
        constexpr uint32_t U = 4;
        bool quit = __ballot(gave_up) != 0;
        for (uint32_t i0 = threadIdx.x; !quit && i0 - lane < n; i0 += 64 * G * U) {
            uint64_t h[U];
            {
                uint64_t a[2 * U];
#pragma unroll
                for (uint32_t u = 0; u < U; ++u) {
                    const uint32_t i = i0 + u * 64 * G;
                    const bool other = i < n && (i < i_lo || i >= i_hi);
                    a[2 * u] = other ? __hip_atomic_load(&X[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : tag;
                    a[2 * u + 1] =
                        other ? __hip_atomic_load(&X[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : tag;
                }
#pragma unroll
                for (uint32_t u = 0; u < U; ++u) {
                    const uint32_t i = i0 + u * 64 * G;
                    h[u] = (a[2 * u + 1] << 32) | (uint32_t)a[2 * u];
                    if (((a[2 * u] ^ tag) >> 32) | ((a[2 * u + 1] ^ tag) >> 32)) fetch(&X[2 * i], h[u]);
                }
            }
            if (__ballot(gave_up)) {
                quit = true;
                break;
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t i = i0 + u * 64 * G;
                if (i < n) {
                    const uint32_t q = owner[i >> 4];
                    uint64_t hv = h[u];
                    if (q == r) {
                        // own node: h from LDS, cleared for the next C by the
                        // thread that read it (the next flips are already in Gm)
                        hv = Fm[i - i_lo];
                        Fm[i - i_lo] = 0ull;
                    }
                    const uint64_t keep = Pall & ~xplw[q];
                    S[i] = (hv & ~keep) | (S[i] & keep);
                }
            }
        }
        if (quit && lane == 0) {
            // the group ends: the status word records it (at once, so that
            // the other parts stop polling) unless the group already completed
            *abort_flag = 1u;
            uint32_t expect = 0u;
            __hip_atomic_compare_exchange_strong(gstat, &expect, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
        }
        // the state complete (and Fm clear) before the next C reads it
        __syncthreads();
        if (*abort_flag) return;
        if (s >= it.nburn && ++since == it.thin) {
            since = 0;
            pending = true;
        }
    }
    if (pending && recorder) {
        record();
        ++pos;
    }
    if (!recorder) return;
    // the group completed unless a block gave up first: then the state stays
    // as the launch found it, for the host's one-block re-run
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t expect = 0u;
        __hip_atomic_compare_exchange_strong(gstat, &expect, 2u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        *abort_flag = expect == 1u ? 1u : 0u;
    }
    __syncthreads();
    if (*abort_flag) return;
    if (active && it.nrec > 0 && (pos & 31)) {
        gu32 bits = (gu32)v.d->bits;
        for (uint32_t q = wave; q < nprops; q += G)
            bits[((size_t)q * words_cap + (pos >> 5)) * omega + c] = acc[64 * q];
    }
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

// An error left by an earlier runtime call would otherwise be reported as the
// launch's own.
static int no_stale_error(const char *what, std::string &err)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return PBN_OK;
    err = std::string("before ") + what + ", an earlier HIP call failed: " + hipGetErrorString(e);
    return PBN_EDEVICE;
}

static int check_launch(const char *what, uint32_t nitems, uint32_t G, size_t lds, std::string &err)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return PBN_OK;
    err = std::string(what) + " (" + std::to_string(nitems) + " blocks of " + std::to_string(64 * G) +
          " threads, " + std::to_string(lds) + " bytes of LDS): " + hipGetErrorString(e);
    return PBN_EDEVICE;
}

size_t bs_lds_bytes(uint32_t n, uint32_t msel_total, uint32_t G)
{
    return (size_t)8 * (2 * (size_t)n + msel_total + 2 * G) + (size_t)4 * 3 * kQCap * G + (size_t)4 * 64 * kMaxProps;
}

size_t split_lds_bytes(uint32_t n, uint32_t n_own, uint32_t m_own, uint32_t G)
{
    return (size_t)8 * ((size_t)n + 2 * (size_t)n_own + m_own + 2 * G) + (size_t)4 * 3 * kQCap * G +
           (size_t)4 * 64 * kMaxProps + 8 + 8 * kSplitMaxParts * G + ((n + 15) / 16 + 15) / 16 * 16;
}

int launch_step_split(const StepItem *d_items, uint32_t nitems, uint32_t G, size_t lds, void *stream,
                      std::string &err)
{
    if (nitems == 0) return PBN_OK;
    if (G < 1 || G > 16) {
        err = "node-split kernel: waves per block must be 1..16";
        return PBN_EINVAL;
    }
    if (lds > 160 * 1024) {
        err = "node-split state exceeds LDS";
        return PBN_ELIMIT;
    }
    if (lds > 64 * 1024) {
        int rc = allow_full_lds((const void *)k_step_split, err);
        if (rc) return rc;
    }
    if (int rc = no_stale_error("k_step_split launch", err)) return rc;
    hipLaunchKernelGGL(k_step_split, dim3(nitems), dim3(64 * G), lds, (hipStream_t)stream, d_items);
    return check_launch("k_step_split launch", nitems, G, lds, err);
}

int launch_step_bs(const StepItem *d_items, uint32_t nitems, uint32_t G, bool small, size_t lds, void *stream,
                   std::string &err)
{
    if (nitems == 0) return PBN_OK;
    if (G < 1 || G > 16) {
        err = "bit-sliced kernel: waves per block must be 1..16";
        return PBN_EINVAL;
    }
    if (lds > 160 * 1024) {
        err = "bit-sliced state exceeds LDS";
        return PBN_ELIMIT;
    }
    const void *fn = small ? (const void *)k_step_bs<true> : (const void *)k_step_bs<false>;
    if (lds > 64 * 1024) {
        int rc = allow_full_lds(fn, err);
        if (rc) return rc;
    }
    if (int rc = no_stale_error("k_step_bs launch", err)) return rc;
    if (small)
        hipLaunchKernelGGL(k_step_bs<true>, dim3(nitems), dim3(64 * G), lds, (hipStream_t)stream, d_items);
    else
        hipLaunchKernelGGL(k_step_bs<false>, dim3(nitems), dim3(64 * G), lds, (hipStream_t)stream, d_items);
    return check_launch(small ? "k_step_bs<small> launch" : "k_step_bs launch", nitems, G, lds, err);
}

}  // namespace pbn
