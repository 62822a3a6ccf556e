// Device helpers shared by the trajectory kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "pbn_internal.h"

// Read-only network data lives in the constant address space (uniform indices
// become scalar loads); chain state and bit-streams in the global one.  Without
// these casts the compiler falls back to FLAT accesses, which may alias LDS and
// are reloaded after every LDS store.
#define PBN_CAS __attribute__((address_space(4)))
#define PBN_GAS __attribute__((address_space(1)))

namespace pbn {

typedef const PBN_CAS uint32_t *cu32;
typedef const PBN_CAS uint16_t *cu16;
typedef PBN_GAS uint32_t *gu32;

struct Key {
    uint32_t k0, k1;
};

// Philox4x32-10 (Salmon et al., SC'11): ten rounds; each multiplies counter
// words 0 and 2 by the round constants, mixes the high halves with the other
// words and the key, and the key advances by the two Weyl increments.
__device__ __forceinline__ void philox4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, Key key,
                                        uint32_t out[4])
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product per word (v_mad_u64_u32) instead of separate
        // high and low multiplies: about 1.3x the Philox rate on gfx950
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        if (r < 2) {
            // the first rounds mix words that are often wave-uniform (transition,
            // block, stream tag): plain XORs stay on the scalar unit there
            c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        } else {
            // three-input XOR in one v_bitop3_b32 (truth table 0x96)
            c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
            c2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
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

// Low 24 bits of the refinement word of node i (stream tag + 1).
__device__ __forceinline__ uint32_t refine24(Key key, uint32_t t, uint32_t c, uint32_t i, uint32_t tag)
{
    uint32_t w[4];
    philox4(t, c, i >> 2, tag + 1, key, w);
    return pick4(w, i & 3) & 0xFFFFFFu;
}

// Per-launch copy of a simulation's device description, with typed pointers.
struct View {
    cu32 nd_first, fn_thr, fn_desc, fn_tt, tt_ext;
    cu16 par;
    gu32 state, bits;
    uint64_t words_cap;
    uint32_t n, W, p_thr, omega, nprops, F_pad, msel_total, nblk;
    Key key;
    const PBN_CAS DevSim *d;
};

__device__ __forceinline__ View load_view(const DevSim *p)
{
    const PBN_CAS DevSim *d = (const PBN_CAS DevSim *)p;
    View v;
    v.d = d;
    v.nd_first = (cu32)d->nd_first;
    v.fn_thr = (cu32)d->fn_thr;
    v.fn_desc = (cu32)d->fn_desc;
    v.fn_tt = (cu32)d->fn_tt;
    v.tt_ext = (cu32)d->tt_ext;
    v.par = (cu16)d->par;
    v.state = (gu32)d->state;
    v.bits = (gu32)d->bits;
    v.words_cap = d->words_cap;
    v.n = d->n;
    v.W = d->W;
    v.p_thr = d->p_thr;
    v.omega = d->omega;
    v.nprops = d->nprops;
    v.F_pad = d->F_pad;
    v.msel_total = d->msel_total;
    v.nblk = d->nblk;
    v.key = Key{d->key0, d->key1};
    return v;
}

__device__ __forceinline__ StepItem load_item(const StepItem *items, uint32_t b)
{
    const PBN_CAS StepItem *p = (const PBN_CAS StepItem *)items + b;
    StepItem it;
    it.sim = p->sim;
    it.chain0 = p->chain0;
    it.nchains = p->nchains;
    it.t0 = p->t0;
    it.nburn = p->nburn;
    it.nrec = p->nrec;
    it.thin = p->thin;
    it.nodes = p->nodes;
    it.pos0 = p->pos0;
    it.ops_per_step = 0.0f;
    it.philox_per_step = 0.0f;
    it.kernel = p->kernel;
    it.lds = p->lds;
    it.small = 0;
    it.part = p->part;
    it.grp = p->grp;
    return it;
}

__device__ __forceinline__ Query load_query(const Query *qs, uint32_t b)
{
    const PBN_CAS Query *p = (const PBN_CAS Query *)qs + b;
    Query q;
    q.sim = p->sim;
    q.prop = p->prop;
    q.kind = p->kind;
    q.lo = p->lo;
    q.hi = p->hi;
    q.kappa = p->kappa;
    q.m = p->m;
    q.out_off = p->out_off;
    return q;
}

}  // namespace pbn
