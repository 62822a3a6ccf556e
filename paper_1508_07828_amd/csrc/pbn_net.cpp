// Parser and compiler of the canonical network text into the device blob.
//
// The network is the PBN G(V, F) of Sec. 2.2: per node a list of predictor
// functions with selection probabilities c_j and parent sets.  Compilation
// packs parents as CSR (u16 ids), truth tables as 32-bit bitsets (one word for
// k <= 5 parents, ceil(2^k/32) words otherwise) and the selection
// probabilities as cumulative 32-bit thresholds T_j = min(2^32-1,
// floor(2^32 (c_1+..+c_j))), the running sum taken left to right in FP64.
#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "pbn_internal.h"

namespace pbn {
namespace {

struct Lexer {
    const char *p, *end;
    bool next(const char *&tok, size_t &len)
    {
        for (;;) {
            while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
            if (p < end && *p == '#') {
                while (p < end && *p != '\n') ++p;
                continue;
            }
            break;
        }
        if (p >= end) return false;
        tok = p;
        while (p < end && !(*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
        len = size_t(p - tok);
        return true;
    }
    bool word(const char *w)
    {
        const char *t; size_t n;
        return next(t, n) && n == std::strlen(w) && std::memcmp(t, w, n) == 0;
    }
    bool integer(long long &v)
    {
        const char *t; size_t n;
        if (!next(t, n) || n > 30) return false;
        char buf[32]; std::memcpy(buf, t, n); buf[n] = 0;
        char *e; errno = 0; v = std::strtoll(buf, &e, 10);
        return *e == 0 && errno == 0;
    }
    bool real(double &v)
    {
        const char *t; size_t n;
        if (!next(t, n) || n > 60) return false;
        char buf[64]; std::memcpy(buf, t, n); buf[n] = 0;
        char *e; v = std::strtod(buf, &e);
        return *e == 0;
    }
};

int hexdigit(char c)
{
    if (c >= '0' && c <= '9') return c - '0';
    if (c >= 'a' && c <= 'f') return c - 'a' + 10;
    if (c >= 'A' && c <= 'F') return c - 'A' + 10;
    return -1;
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

}  // namespace

void build_bitsliced_schedule(Net &net);

int parse_and_compile(const char *text, size_t len, Net &net, std::string &err)
{
    Lexer lx{text, text + len};
    long long n;
    double p;
    if (!lx.word("PBN") || !lx.integer(n) || !lx.real(p)) { err = "bad header"; return PBN_EFORMAT; }
    if (n < 1 || n > 65535) { err = "n must be in 1..65535"; return n > 65535 ? PBN_ELIMIT : PBN_EFORMAT; }
    if (!(p > 0.0 && p < 1.0)) { err = "p must be in (0,1)"; return PBN_EFORMAT; }
    net = Net();
    net.n = uint32_t(n);
    net.W = (net.n + 31) / 32;
    net.p = p;
    net.p_thr = uint32_t(std::floor(p * 4294967296.0));
    net.nd_first.reserve(n + 1);
    uint64_t total_par = 0;
    std::vector<uint32_t> big_tt_words;
    for (long long i = 0; i < n; ++i) {
        long long idx, l;
        if (!lx.word("N") || !lx.integer(idx) || !lx.integer(l)) { err = "bad node line " + std::to_string(i); return PBN_EFORMAT; }
        if (idx != i) { err = "node " + std::to_string(i) + " out of order"; return PBN_EFORMAT; }
        if (l < 1 || l > 64) { err = "node " + std::to_string(i) + ": function count"; return l > 64 ? PBN_ELIMIT : PBN_EFORMAT; }
        net.nd_first.push_back(net.F);
        if (uint32_t(l) > net.max_l) net.max_l = uint32_t(l);
        double csum = 0.0;
        for (long long j = 0; j < l; ++j) {
            double c;
            long long k;
            if (!lx.word("F") || !lx.real(c) || !lx.integer(k)) { err = "bad function line (node " + std::to_string(i) + ")"; return PBN_EFORMAT; }
            if (!(c >= 0.0 && c <= 1.0)) { err = "bad probability (node " + std::to_string(i) + ")"; return PBN_EFORMAT; }
            if (k < 1 || k > 16) { err = "parent count (node " + std::to_string(i) + ")"; return k > 16 ? PBN_ELIMIT : PBN_EFORMAT; }
            uint32_t po = uint32_t(net.par.size());
            for (long long m = 0; m < k; ++m) {
                long long v;
                if (!lx.integer(v) || v < 0 || v >= n) { err = "bad parent (node " + std::to_string(i) + ")"; return PBN_EFORMAT; }
                for (long long q = 0; q < m; ++q)
                    if (net.par[po + q] == uint16_t(v)) { err = "duplicate parent (node " + std::to_string(i) + ")"; return PBN_EFORMAT; }
                net.par.push_back(uint16_t(v));
            }
            total_par += uint64_t(k);
            const char *hx; size_t hl;
            if (!lx.next(hx, hl)) { err = "missing truth table"; return PBN_EFORMAT; }
            size_t words = ((size_t(1) << k) + 31) / 32;
            std::vector<uint32_t> tt(words, 0u);
            for (size_t d = 0; d < hl; ++d) {
                int hv = hexdigit(hx[hl - 1 - d]);
                if (hv < 0) { err = "bad hex digit"; return PBN_EFORMAT; }
                for (int b = 0; b < 4; ++b) {
                    if (!((hv >> b) & 1)) continue;
                    size_t e = 4 * d + size_t(b);
                    if (e >= (size_t(1) << k)) { err = "truth table longer than 2^k bits"; return PBN_EFORMAT; }
                    tt[e / 32] |= 1u << (e % 32);
                }
            }
            if (k <= 5) {
                net.fn_tt.push_back(tt[0]);
            } else {
                net.fn_tt.push_back(uint32_t(big_tt_words.size()));
                big_tt_words.insert(big_tt_words.end(), tt.begin(), tt.end());
            }
            if (uint32_t(k) > net.max_k) net.max_k = uint32_t(k);
            net.fn_desc.push_back(uint32_t(k) | (po << 5));
            csum = csum + c;
            double scaled = std::floor(csum * 4294967296.0);
            net.fn_thr.push_back(scaled >= 4294967295.0 ? 4294967295u : uint32_t(scaled));
            ++net.F;
        }
        if (std::fabs(csum - 1.0) > 1e-12) { err = "probabilities of node " + std::to_string(i) + " do not sum to 1"; return PBN_EFORMAT; }
    }
    const char *t; size_t tl;
    if (lx.next(t, tl)) { err = "trailing tokens"; return PBN_EFORMAT; }
    if (net.par.size() >= (size_t(1) << 27)) { err = "too many parents"; return PBN_ELIMIT; }
    net.nd_first.push_back(net.F);
    net.tt_ext = std::move(big_tt_words);
    if (net.tt_ext.empty()) net.tt_ext.push_back(0);
    if (net.par.empty()) net.par.push_back(0);
    net.density = double(total_par) / double(net.n);

    // Expected algorithmic work per chain-step (accounting for the roofline):
    // Philox evaluations of the stream (16 primaries per evaluation, a refinement
    // when a primary byte ties a threshold's top byte), comparisons, parent-bit
    // gathers and lookups of the function update (taken when no node is
    // perturbed: probability (1-p)^n).
    {
        const double two32 = 4294967296.0;
        const double pq = (double)net.p_thr / two32;
        const double q_fn = std::pow(1.0 - pq, (double)net.n);
        const uint32_t nblk = (net.n + 15) / 16;
        uint32_t sel_blocks = 0;
        double sel_ref = 0.0, fn_ops = 0.0;
        for (uint32_t b = 0; b < nblk; ++b) {
            bool any = false;
            for (uint32_t i = 16 * b; i < std::min(net.n, 16 * b + 16); ++i)
                if (net.nd_first[i + 1] - net.nd_first[i] > 1) any = true;
            sel_blocks += any ? 1 : 0;
        }
        for (uint32_t i = 0; i < net.n; ++i) {
            const uint32_t a = net.nd_first[i], l = net.nd_first[i + 1] - a;
            sel_ref += (double)(l - 1) / 256.0;
            double ek = 0.0, prev = 0.0;
            for (uint32_t j = 0; j < l; ++j) {
                const double T = (j + 1 == l) ? two32 : (double)net.fn_thr[a + j];
                ek += (T - prev) / two32 * (double)(net.fn_desc[a + j] & 31u);
                prev = T;
            }
            fn_ops += (double)(l - 1) + 2.0 * ek + 1.0;
        }
        net.philox_per_step = (double)nblk + (double)net.n / 256.0 + q_fn * ((double)sel_blocks + sel_ref);
        net.ops_per_step = 100.0 * net.philox_per_step + (double)net.n + q_fn * fn_ops;
    }

    build_bitsliced_schedule(net);

    size_t off = 0;
    auto place = [&](size_t &field, size_t bytes) { field = off; off = align16(off + std::max<size_t>(bytes, 4)); };
    place(net.off_nd_first, 4 * net.nd_first.size());
    place(net.off_fn_thr, 4 * net.fn_thr.size());
    place(net.off_fn_desc, 4 * net.fn_desc.size());
    place(net.off_fn_tt, 4 * net.fn_tt.size());
    place(net.off_tt_ext, 4 * net.tt_ext.size());
    place(net.off_par, 2 * net.par.size());
    // interleaved records for the bit-sliced kernel: per node (meta, top bytes),
    // per predictor slot (node, table lo, table hi, mask below, mask up to,
    // parents 0|1, 2|3, 4|5 as u16 pairs); node records padded with zeros to
    // whole 16-node blocks, so a block's 32 words load without bounds checks
    std::vector<uint32_t> nd_info(32 * (size_t)((net.nd_meta.size() + 15) / 16)), fs_rec(8 * (size_t)net.F_pad);
    for (size_t i = 0; i < net.nd_meta.size(); ++i) {
        nd_info[2 * i] = net.nd_meta[i];
        nd_info[2 * i + 1] = net.nd_tb[i];
    }
    for (size_t s = 0; s < net.F_pad; ++s) {
        uint32_t *r = &fs_rec[8 * s];
        r[0] = net.fs_node[s];
        r[1] = net.fs_tt_lo[s];
        r[2] = net.fs_tt_hi[s];
        r[3] = net.fs_mlo[s];
        r[4] = net.fs_mhi[s];
        for (uint32_t m = 0; m < 3; ++m)
            r[5 + m] = (uint32_t)net.fs_par[(size_t)(2 * m) * net.F_pad + s] |
                       ((uint32_t)net.fs_par[(size_t)(2 * m + 1) * net.F_pad + s] << 16);
    }
    place(net.off_nd_info, 4 * nd_info.size());
    place(net.off_blk_sel, 4 * net.blk_sel.size());
    place(net.off_fs_rec, 4 * fs_rec.size());
    place(net.off_fg_K, 4 * net.fg_K.size());
    net.blob_bytes = off;
    net.blob.assign(off, 0);
    auto put = [&](size_t at, const void *src, size_t bytes) {
        if (bytes) std::memcpy(net.blob.data() + at, src, bytes);
    };
    put(net.off_nd_first, net.nd_first.data(), 4 * net.nd_first.size());
    put(net.off_fn_thr, net.fn_thr.data(), 4 * net.fn_thr.size());
    put(net.off_fn_desc, net.fn_desc.data(), 4 * net.fn_desc.size());
    put(net.off_fn_tt, net.fn_tt.data(), 4 * net.fn_tt.size());
    put(net.off_tt_ext, net.tt_ext.data(), 4 * net.tt_ext.size());
    put(net.off_par, net.par.data(), 2 * net.par.size());
    put(net.off_nd_info, nd_info.data(), 4 * nd_info.size());
    put(net.off_blk_sel, net.blk_sel.data(), 4 * net.blk_sel.size());
    put(net.off_fs_rec, fs_rec.data(), 4 * fs_rec.size());
    put(net.off_fg_K, net.fg_K.data(), 4 * net.fg_K.size());
    return PBN_OK;
}

// Bit-sliced schedule: see the Net comment.  Predictor slots are sorted by
// parent count so that each 64-slot group evaluates one K-input multiplexer
// tree; a predictor with k < K has its table replicated over the extra index
// bits, which makes the padding parents irrelevant.
void build_bitsliced_schedule(Net &net)
{
    net.bitsliced = net.max_k <= kBsMaxK;
    net.nblk = (net.n + 15) / 16;
    net.nd_meta.assign(net.n, 0);
    net.nd_tb.assign(net.n, 0);
    net.blk_sel.assign(net.nblk, 0);
    net.msel_total = 0;
    for (uint32_t i = 0; i < net.n; ++i) {
        const uint32_t a = net.nd_first[i], l = net.nd_first[i + 1] - a;
        net.nd_meta[i] = l | (net.msel_total << 8);
        uint32_t tb = 0;
        for (uint32_t j = 0; j + 1 < l && j < 3; ++j) tb |= (net.fn_thr[a + j] >> 24) << (8 * j);
        net.nd_tb[i] = tb | (std::min<uint32_t>(l, 255) << 24);
        net.blk_sel[i / 16] = std::max(net.blk_sel[i / 16], l);
        net.msel_total += l - 1;
    }
    if (!net.bitsliced) return;
    std::vector<uint32_t> order(net.F);
    for (uint32_t f = 0; f < net.F; ++f) order[f] = f;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return (net.fn_desc[x] & 31u) < (net.fn_desc[y] & 31u); });
    std::vector<uint32_t> fn_node(net.F), fn_j(net.F);
    for (uint32_t i = 0; i < net.n; ++i)
        for (uint32_t f = net.nd_first[i]; f < net.nd_first[i + 1]; ++f) {
            fn_node[f] = i;
            fn_j[f] = f - net.nd_first[i];
        }
    net.F_pad = (net.F + 63) / 64 * 64;
    const uint32_t groups = net.F_pad / 64;
    net.fs_node.assign(net.F_pad, kNoNode);
    net.fs_tt_lo.assign(net.F_pad, 0);
    net.fs_tt_hi.assign(net.F_pad, 0);
    net.fs_mlo.assign(net.F_pad, kNoMask);
    net.fs_mhi.assign(net.F_pad, kNoMask);
    net.fs_par.assign((size_t)kBsMaxK * net.F_pad, 0);
    net.fg_K.assign(groups, 1);
    for (uint32_t g = 0; g < groups; ++g) {
        uint32_t K = 1;
        for (uint32_t s = 64 * g; s < std::min(net.F, 64 * g + 64); ++s) K = std::max(K, net.fn_desc[order[s]] & 31u);
        net.fg_K[g] = K;
        for (uint32_t s = 64 * g; s < std::min(net.F, 64 * g + 64); ++s) {
            const uint32_t f = order[s], k = net.fn_desc[f] & 31u, po = net.fn_desc[f] >> 5;
            const uint32_t i = fn_node[f], j = fn_j[f], l = net.nd_first[i + 1] - net.nd_first[i];
            const uint32_t moff = net.nd_meta[i] >> 8;
            net.fs_node[s] = i;
            for (uint32_t m = 0; m < k; ++m) net.fs_par[(size_t)m * net.F_pad + s] = net.par[po + m];
            // table over 2^K indices, bit e = f(e mod 2^k)
            const uint64_t tt = (k <= 5) ? (uint64_t)net.fn_tt[f]
                                         : ((uint64_t)net.tt_ext[net.fn_tt[f]] | ((uint64_t)net.tt_ext[net.fn_tt[f] + 1] << 32));
            uint64_t rep = 0;
            const uint32_t span = 1u << K, per = 1u << k;
            for (uint32_t e = 0; e < span && e < 64; ++e) rep |= ((tt >> (e % per)) & 1ull) << e;
            if (K <= 5) rep &= 0xFFFFFFFFull;
            net.fs_tt_lo[s] = (uint32_t)rep;
            net.fs_tt_hi[s] = (uint32_t)(rep >> 32);
            net.fs_mlo[s] = j == 0 ? kNoMask : moff + j - 1;
            net.fs_mhi[s] = j + 1 == l ? kNoMask : moff + j;
        }
    }
}

}  // namespace pbn

namespace pbn {

// Node-split tables: 16-node blocks in P contiguous parts of near-equal size;
// each part's predictor slots (its nodes' functions) sorted by parent count
// and padded to whole 64-slot groups, with records as in the one-block
// schedule (the selection-mask indices stay global).
void build_split_tables(const Net &net, uint32_t P, std::vector<uint32_t> &tab)
{
    std::vector<uint32_t> blk(P + 1), grp(P + 1, 0);
    for (uint32_t r = 0; r <= P; ++r) blk[r] = (uint32_t)(((uint64_t)net.nblk * r) / P);
    std::vector<std::vector<uint32_t>> order(P);
    for (uint32_t r = 0; r < P; ++r) {
        const uint32_t i_lo = 16 * blk[r], i_hi = std::min(net.n, 16 * blk[r + 1]);
        for (uint32_t i = i_lo; i < i_hi; ++i)
            for (uint32_t f = net.nd_first[i]; f < net.nd_first[i + 1]; ++f) order[r].push_back(f);
        std::stable_sort(order[r].begin(), order[r].end(),
                         [&](uint32_t x, uint32_t y) { return (net.fn_desc[x] & 31u) < (net.fn_desc[y] & 31u); });
        grp[r + 1] = grp[r] + (uint32_t)((order[r].size() + 63) / 64);
    }
    const uint32_t groups = grp[P];
    const uint32_t rec0 = split_rec_off(P, groups);
    tab.assign((size_t)rec0 + (size_t)groups * 64 * 8, 0);
    for (uint32_t r = 0; r <= P; ++r) {
        tab[r] = blk[r];
        tab[P + 1 + r] = grp[r];
    }
    std::vector<uint32_t> fn_node(net.F), fn_j(net.F);
    for (uint32_t i = 0; i < net.n; ++i)
        for (uint32_t f = net.nd_first[i]; f < net.nd_first[i + 1]; ++f) {
            fn_node[f] = i;
            fn_j[f] = f - net.nd_first[i];
        }
    for (uint32_t r = 0; r < P; ++r) {
        const std::vector<uint32_t> &ord = order[r];
        for (uint32_t g = grp[r]; g < grp[r + 1]; ++g) {
            const size_t s0 = (size_t)(g - grp[r]) * 64, s1 = std::min(ord.size(), s0 + 64);
            uint32_t K = 1;
            for (size_t s = s0; s < s1; ++s) K = std::max(K, net.fn_desc[ord[s]] & 31u);
            tab[split_head(P) + g] = K;
            for (uint32_t m = 0; m < 64; ++m) {
                uint32_t *rec = &tab[rec0 + ((size_t)g * 64 + m) * 8];
                if (s0 + m >= s1) {
                    rec[0] = kNoNode;
                    rec[3] = kNoMask;
                    rec[4] = kNoMask;
                    continue;
                }
                const uint32_t f = ord[s0 + m], k = net.fn_desc[f] & 31u, po = net.fn_desc[f] >> 5;
                const uint32_t i = fn_node[f], j = fn_j[f], l = net.nd_first[i + 1] - net.nd_first[i];
                const uint32_t moff = net.nd_meta[i] >> 8;
                const uint64_t tt = (k <= 5) ? (uint64_t)net.fn_tt[f]
                                             : ((uint64_t)net.tt_ext[net.fn_tt[f]] | ((uint64_t)net.tt_ext[net.fn_tt[f] + 1] << 32));
                uint64_t rep = 0;
                const uint32_t span = 1u << K, per = 1u << k;
                for (uint32_t e = 0; e < span && e < 64; ++e) rep |= ((tt >> (e % per)) & 1ull) << e;
                if (K <= 5) rep &= 0xFFFFFFFFull;
                uint16_t par[kBsMaxK] = {0, 0, 0, 0, 0, 0};
                for (uint32_t q = 0; q < k; ++q) par[q] = net.par[po + q];
                rec[0] = i;
                rec[1] = (uint32_t)rep;
                rec[2] = (uint32_t)(rep >> 32);
                rec[3] = j == 0 ? kNoMask : moff + j - 1;
                rec[4] = j + 1 == l ? kNoMask : moff + j;
                for (uint32_t q = 0; q < 3; ++q) rec[5 + q] = (uint32_t)par[2 * q] | ((uint32_t)par[2 * q + 1] << 16);
            }
        }
    }
}

}  // namespace pbn
