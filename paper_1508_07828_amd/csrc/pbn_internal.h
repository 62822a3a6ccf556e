// Internal structures of libpbnssa shared by the host runtime and the kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pbnssa.h"

namespace pbn {

constexpr uint32_t kTagPert = 0, kTagSel = 2, kTagInit = 4;
constexpr uint32_t kMaxProps = PBN_MAX_PROPS;
constexpr uint32_t kMaxTerms = PBN_MAX_TERMS;

// Compiled network (host copy; uploaded verbatim as one blob).
//   nd_first[n+1]  first function of node i (l(i) = nd_first[i+1]-nd_first[i])
//   fn_thr[F]      cumulative selection threshold T_j (unused for the last one)
//   fn_desc[F]     k | (offset of its parents in par[]) << 5
//   fn_tt[F]       truth table for k <= 5, else word offset into tt_ext
//   par[]          parent node ids (u16)
//   tt_ext[]       truth tables of functions with k > 5 (ceil(2^k/32) words)
struct Net {
    uint32_t n = 0, W = 0, F = 0, p_thr = 0, max_k = 0, max_l = 0;
    double p = 0.0, density = 0.0;
    double ops_per_step = 0.0, philox_per_step = 0.0;   // expected, per chain-step
    std::vector<uint32_t> nd_first, fn_thr, fn_desc, fn_tt, tt_ext;
    std::vector<uint16_t> par;
    // Bit-sliced schedule (networks with k <= 6):
    //   nd_meta[n]   l(i) | (offset of node i's selection masks) << 8
    //   nd_tb[n]     top bytes of T_1..T_3, byte j = T_{j+1} >> 24 (j < min(l-1, 3)),
    //                byte 3 = min(l, 255)
    //   blk_sel[nb]  largest predictor count l of the 16-node block b
    //   predictor slots sorted by k, F_pad = 64 * ceil(F/64):
    //   fs_node      node of the slot (kNoNode for padding)
    //   fs_tt_lo/hi  truth table replicated to 2^K bits (K = the slot group's max k)
    //   fs_par[m][s] parent m of slot s (padding parents: node 0)
    //   fs_mlo/mhi   selection-mask indices of T_{j-1} and T_j (kNoMask: none)
    //   fg_K[g]      K of slot group g (64 slots)
    bool bitsliced = false;
    uint32_t F_pad = 0, msel_total = 0, nblk = 0;
    std::vector<uint32_t> nd_meta, nd_tb, blk_sel, fs_node, fs_tt_lo, fs_tt_hi, fs_mlo, fs_mhi, fg_K;
    std::vector<uint16_t> fs_par;
    // blob layout (byte offsets)
    size_t off_nd_first = 0, off_fn_thr = 0, off_fn_desc = 0, off_fn_tt = 0, off_tt_ext = 0,
           off_par = 0, blob_bytes = 0;
    size_t off_nd_info = 0, off_blk_sel = 0, off_fs_rec = 0, off_fg_K = 0;
    std::vector<uint8_t> blob;
};

constexpr uint32_t kNoNode = 0xFFFFFFFFu, kNoMask = 0xFFFFFFFFu;
constexpr uint32_t kBsMaxK = 6;          // bit-sliced evaluation handles k <= 6
constexpr uint32_t kQCap = 192;          // tie-queue entries per wave (bit-sliced kernel)

int parse_and_compile(const char *text, size_t len, Net &out, std::string &err);

// Device-side description of one simulation (lives in the simulation's device
// buffer; kernels receive its device address).
struct DevSim {
    const uint32_t *nd_first;
    const uint32_t *fn_thr;
    const uint32_t *fn_desc;
    const uint32_t *fn_tt;
    const uint32_t *tt_ext;
    const uint16_t *par;
    uint32_t *state;            // [W][omega]
    uint32_t *bits;             // [max_props][words_cap][omega]
    uint64_t words_cap;
    uint32_t n, W, p_thr, omega;
    uint32_t key0, key1;
    uint32_t nprops, nterms;
    uint32_t prop_off[kMaxProps + 1];
    uint32_t term_word[kMaxTerms];
    uint32_t term_mask[kMaxTerms];
    uint32_t term_val[kMaxTerms];
    // node-level form of the same state sets (bit-sliced kernel)
    uint32_t pn_off[kMaxProps + 1];
    uint32_t pn_node[kMaxTerms];
    uint32_t pn_val[kMaxTerms];
    // bit-sliced schedule
    const uint32_t *nd_info;     // [n][2]: l | mask offset << 8, top bytes of T_1..T_3
    const uint32_t *fs_rec;      // [F_pad][8]: node, tt lo, tt hi, mask below, mask up to, parents
    const uint32_t *blk_sel, *fg_K;
    uint32_t F_pad, msel_total, nblk, pad0;
};

// Node-split form of the bit-sliced step: P blocks on P CUs share one 64-chain
// group, block r owning a contiguous range of 16-node blocks and the predictor
// slots of those nodes.  Each transition every block publishes, for its own
// nodes, the perturbation flips and the function values, plus its chains'
// perturbed flags, and reads everyone's as they arrive.
//   tab: u32 [0, P]  first 16-node block of part r (tab[P] = nblk)
//            [P + 1, 2P + 1]  first 64-slot group of part r (tab[2P + 1] = groups)
//            at split_head(P): K of every slot group, then (16-byte aligned) the
//            slot records, 8 words each, as in DevSim::fs_rec
//   xch: u64 [2][n][2] next-state words as published by their owners, then
//        [2][P][2] perturbed-chain words, by transition parity; each u64 holds
//        a 32-bit half of a mask under a 32-bit tag (launch transition + 1);
//        zero at launch
//   stat: 0 at launch; 1 once a block's wait timed out (the group then ends
//         early and leaves its state unchanged), 2 once block 0 completed the
//         last transition (it then writes the state back)
struct SplitGroup {
    const uint32_t *tab;
    uint64_t *xch;
    uint32_t *stat;
    uint32_t nparts, groups;
    uint32_t spins, pad_;        // polls of a word before a part gives up
};
// Exchange-area words of one group.
constexpr size_t split_xch_words(uint32_t n, uint32_t P) { return (size_t)4 * n + (size_t)4 * P; }
// Polls of one exchange word before a block gives up (each poll reads the
// word from memory and sleeps, together well over 100 ns); tests of the
// failure path lower it.
constexpr uint32_t kSplitSpins = 1u << 20;
// Parts of one node-split group, at most.
constexpr uint32_t kSplitMaxParts = 16;
constexpr uint32_t split_head(uint32_t P) { return 2 * (P + 1); }
constexpr uint32_t split_rec_off(uint32_t P, uint32_t groups) { return (split_head(P) + groups + 3) / 4 * 4; }
// The node-split tables of net for P parts (layout of SplitGroup::tab).
void build_split_tables(const Net &net, uint32_t P, std::vector<uint32_t> &tab);

// One unit of step-kernel work: chains [chain0, chain0+nchains) of one sim.
struct StepItem {
    const DevSim *sim;
    uint32_t chain0, nchains;
    uint32_t t0;                 // transition index of the first transition
    uint32_t nburn, nrec, thin;  // unrecorded transitions, recorded positions, spacing
    uint32_t nodes;              // network size (host-side cost and LDS sizing)
    uint64_t pos0;               // first recorded position (0-based)
    float ops_per_step, philox_per_step;   // host-side accounting only
    uint32_t kernel;             // host-side: 0 = lane-per-chain, else waves per block (bit-sliced)
    uint32_t lds;                // host-side: LDS bytes the bit-sliced kernel needs
    uint32_t small;              // host-side: bit-sliced with per-wave metadata in registers
    uint32_t part;               // node-split form: this block's part
    const SplitGroup *grp;       // node-split form: the group (null otherwise)
    void *owner;                 // host-side: the simulation the item advances
    uint32_t parts_hint;         // host-side: node-split parts planned for it (0 = none)
    uint32_t pad_;
};

enum QueryKind : uint32_t { kQueryWindow = 0, kQueryBatch = 1 };

// One reduction query over a sim's bit-streams.
struct Query {
    const DevSim *sim;
    uint32_t prop, kind;
    uint64_t lo, hi;             // window [lo, hi) (0-based positions)
    uint64_t kappa, m;           // batch query: m batches of kappa from lo
    uint64_t out_off;            // batch query: output offset (int32 units)
};

// Results of a window query.
struct WindowResult {
    int64_t T1, T2, n00, n01, n10, n11, pad0, pad1;
};

// ------------------------------------------------------------ launches (.hip)
int launch_init(const DevSim *dsim, uint32_t omega, uint32_t W, void *stream, std::string &err);
// Descriptors staged in device memory copied to their simulations, initial states written.
int launch_setup(const DevSim *d_staging, DevSim *const *d_dst, uint32_t count, void *stream, std::string &err);
// Lane-per-chain step.  Rows of more than 320 words (n > 10240) do not fit in
// LDS: they then live in `rows`, step_rows_words(nitems, max_W) u32 of device
// scratch (0 when LDS suffices; rows may then be null).
size_t step_rows_words(uint32_t nitems, uint32_t max_W);
int launch_step(const StepItem *d_items, uint32_t nitems, uint32_t max_W, uint32_t *rows, void *stream,
                std::string &err);
// Bit-sliced trajectory kernel: G waves per 64-chain block, lds bytes of LDS.
// small: every wave owns at most one 16-node block and one 64-slot group.
int launch_step_bs(const StepItem *d_items, uint32_t nitems, uint32_t G, bool small, size_t lds, void *stream,
                   std::string &err);
size_t bs_lds_bytes(uint32_t n, uint32_t msel_total, uint32_t G);
// Node-split form: LDS of one block owning n_own nodes and m_own selection masks.
size_t split_lds_bytes(uint32_t n, uint32_t n_own, uint32_t m_own, uint32_t G);
int launch_step_split(const StepItem *d_items, uint32_t nitems, uint32_t G, size_t lds, void *stream,
                      std::string &err);
// Dynamic-LDS limit of a kernel raised to 160 KB (once per device).
int allow_full_lds(const void *fn, std::string &err);
int launch_reduce(const Query *d_queries, uint32_t nq, WindowResult *d_win, int32_t *d_bsum,
                  void *stream, std::string &err);

// ------------------------------------------------------------ statistics
double normal_quantile(double p);
double t_quantile(double p, double nu);
double rhat_from_sums(int64_t T1, int64_t T2, uint64_t omega, uint64_t psi, bool *defined);
// Skart: |skewness| > 4 of count 0-1 observations with `ones` ones, exactly.
bool skewness_exceeds_4(uint64_t ones, uint64_t count);
// Exact integer aggregates of batch sums b[c m + j] (pbn_stats.cpp).
struct BatchMoments {
    uint64_t m = 0, P = 0, pairs = 0;
    __int128 S1 = 0, D2 = 0, Q2 = 0, Q3 = 0, QL = 0;
};
BatchMoments batch_moments(const int32_t *b, uint32_t omega, uint64_t m);
bool randomness_passes(const BatchMoments &g, double *C_out = nullptr, double *limit_out = nullptr);
void adjusted_ci(const BatchMoments &g, uint64_t kappa, double conf, double *mu, double *lo, double *hi);
double willink(double zeta, double beta);

}  // namespace pbn
