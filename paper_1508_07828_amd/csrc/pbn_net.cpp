// Parser and compiler of the canonical network text into the device blob.
//
// The network is the PBN G(V, F) of Sec. 2.2: per node a list of predictor
// functions with selection probabilities c_j and parent sets.  Compilation
// packs parents as CSR (u16 ids), truth tables as 32-bit bitsets (one word for
// k <= 5 parents, ceil(2^k/32) words otherwise) and the selection
// probabilities as cumulative 32-bit thresholds T_j = min(2^32-1,
// floor(2^32 (c_1+..+c_j))), the running sum taken left to right in FP64.
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

    size_t off = 0;
    net.off_nd_first = off; off = align16(off + 4 * net.nd_first.size());
    net.off_fn_thr = off;   off = align16(off + 4 * net.fn_thr.size());
    net.off_fn_desc = off;  off = align16(off + 4 * net.fn_desc.size());
    net.off_fn_tt = off;    off = align16(off + 4 * net.fn_tt.size());
    net.off_tt_ext = off;   off = align16(off + 4 * net.tt_ext.size());
    net.off_par = off;      off = align16(off + 2 * net.par.size());
    net.blob_bytes = off;
    net.blob.assign(off, 0);
    std::memcpy(net.blob.data() + net.off_nd_first, net.nd_first.data(), 4 * net.nd_first.size());
    std::memcpy(net.blob.data() + net.off_fn_thr, net.fn_thr.data(), 4 * net.fn_thr.size());
    std::memcpy(net.blob.data() + net.off_fn_desc, net.fn_desc.data(), 4 * net.fn_desc.size());
    std::memcpy(net.blob.data() + net.off_fn_tt, net.fn_tt.data(), 4 * net.fn_tt.size());
    std::memcpy(net.blob.data() + net.off_tt_ext, net.tt_ext.data(), 4 * net.tt_ext.size());
    std::memcpy(net.blob.data() + net.off_par, net.par.data(), 2 * net.par.size());
    return PBN_OK;
}

}  // namespace pbn
