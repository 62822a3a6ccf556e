/*
 * Plain CPU oracle: trajectories of an instantaneously random PBN with
 * perturbations.  TEST INFRASTRUCTURE ONLY: it is loaded by the tests, by the
 * smoke check and by the benchmark's CPU-baseline leg, never by the product.
 * It shares no code with the GPU library.
 *
 * Semantics (paper Sec. 2.2):
 *   - a PBN has n binary nodes; node i has l(i) predictor functions, function
 *     j chosen with probability c_j^(i), independently per node and per step
 *     (instantaneously random PBN);
 *   - perturbation vector gamma(t): gamma_i ~ Bernoulli(p), i.i.d.;
 *   - if gamma(t) is all zero the next state is f(t)(s(t)) (synchronous
 *     update with the selected predictors); otherwise s(t+1) = s(t) XOR gamma(t).
 *
 * Readings fixed here (the paper leaves them open):
 *   - probabilities are quantised to 32-bit thresholds: p_thr = floor(p 2^32),
 *     T_j = min(2^32-1, floor(2^32 (c_1+..+c_j))) summed left to right in FP64;
 *     gamma_i = (u < p_thr); the selected function is the smallest j < l with
 *     u < T_j, else the last one;
 *   - every uniform u is 32 bits: an 8-bit primary byte (top bits) and a
 *     24-bit refinement (low bits), drawn from Philox4x32-10 as follows, with
 *     key = (seed low 32, seed high 32) and t the 0-based transition index:
 *        primary   byte (i mod 16) of Philox(key, (t, chain, i div 16, tag))
 *                  (byte b of the 16-byte output = bits 8(b mod 4).. of word b div 4)
 *        refinement low 24 bits of word (i mod 4) of Philox(key, (t, chain, i div 4, tag+1))
 *     with tag 0 for perturbation and tag 2 for selection;
 *   - initial state: bit i of chain c is bit (i mod 32) of word (w mod 4) of
 *     Philox(key, (0, c, w div 4, 4)), w = i div 32;
 *   - truth-table index: sum over parents m (0-based, listed order) of v(par_m) << m.
 *
 * Philox4x32-10 follows Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11): ten rounds, each multiplying counter words 0 and
 * 2 by the two round multipliers, mixing the high halves with the key and the
 * other two counter words, and bumping the key by the two Weyl constants
 * between rounds.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define TAG_PERT 0u
#define TAG_SEL 2u
#define TAG_INIT 4u

/* ------------------------------------------------------------- Philox */

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;   /* golden ratio */
            k1 += 0xBB67AE85u;   /* sqrt(3) - 1  */
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_at(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* The 32-bit uniform of node i at transition t for one stream (tag 0 or 2). */
uint32_t orc_uniform(uint64_t seed, uint32_t t, uint32_t chain, uint32_t node, uint32_t tag)
{
    uint32_t prim[4], refi[4];
    philox_at(seed, t, chain, node / 16u, tag, prim);
    uint32_t b = node % 16u;
    uint32_t byte = (prim[b / 4u] >> (8u * (b % 4u))) & 0xFFu;
    philox_at(seed, t, chain, node / 4u, tag + 1u, refi);
    uint32_t low = refi[node % 4u] & 0xFFFFFFu;
    return (byte << 24) | low;
}

/* ------------------------------------------------------------- network */

typedef struct {
    int n;
    double p;
    uint32_t p_thr;
    int nfun;               /* total functions */
    int *nfn;               /* [n] l(i) */
    int *fn_first;          /* [n] first function of node i */
    double *c;              /* [nfun] */
    uint32_t *thr;          /* [nfun] cumulative threshold T_j (last one unused) */
    int *k;                 /* [nfun] */
    int **par;              /* [nfun][k] */
    uint8_t **tt;           /* [nfun][2^k] one byte per entry */
} orc_net;

static char g_err[256];
const char *orc_error(void) { return g_err; }

static void net_release(orc_net *net)
{
    if (!net) return;
    for (int f = 0; f < net->nfun; f++) {
        if (net->par) free(net->par[f]);
        if (net->tt) free(net->tt[f]);
    }
    free(net->par); free(net->tt); free(net->nfn); free(net->fn_first);
    free(net->c); free(net->thr); free(net->k);
    free(net);
}

void orc_free(orc_net *net) { net_release(net); }

static int hexval(char ch)
{
    if (ch >= '0' && ch <= '9') return ch - '0';
    if (ch >= 'a' && ch <= 'f') return ch - 'a' + 10;
    if (ch >= 'A' && ch <= 'F') return ch - 'A' + 10;
    return -1;
}

/* Next whitespace-separated token, skipping '#' comment lines. */
static const char *next_token(const char **cur, size_t *len)
{
    const char *s = *cur;
    for (;;) {
        while (*s == ' ' || *s == '\t' || *s == '\n' || *s == '\r') s++;
        if (*s == '#') { while (*s && *s != '\n') s++; continue; }
        break;
    }
    if (!*s) { *cur = s; return NULL; }
    const char *b = s;
    while (*s && *s != ' ' && *s != '\t' && *s != '\n' && *s != '\r') s++;
    *len = (size_t)(s - b);
    *cur = s;
    return b;
}

static int tok_long(const char **cur, long *v)
{
    size_t len; const char *t = next_token(cur, &len);
    if (!t || len > 30) return -1;
    char buf[32]; memcpy(buf, t, len); buf[len] = 0;
    char *end; *v = strtol(buf, &end, 10);
    return (*end == 0) ? 0 : -1;
}

static int tok_double(const char **cur, double *v)
{
    size_t len; const char *t = next_token(cur, &len);
    if (!t || len > 60) return -1;
    char buf[64]; memcpy(buf, t, len); buf[len] = 0;
    char *end; *v = strtod(buf, &end);
    return (*end == 0) ? 0 : -1;
}

static int tok_word(const char **cur, const char *want)
{
    size_t len; const char *t = next_token(cur, &len);
    return (t && len == strlen(want) && memcmp(t, want, len) == 0) ? 0 : -1;
}

#define FAIL(...) do { snprintf(g_err, sizeof g_err, __VA_ARGS__); net_release(net); return NULL; } while (0)

orc_net *orc_parse(const char *text)
{
    orc_net *net = calloc(1, sizeof *net);
    const char *cur = text;
    long n;
    if (!net) return NULL;
    if (tok_word(&cur, "PBN") || tok_long(&cur, &n) || tok_double(&cur, &net->p)) FAIL("bad header");
    if (n < 1 || n > 65535) FAIL("n out of range");
    if (!(net->p > 0.0 && net->p < 1.0)) FAIL("p must be in (0,1)");
    net->n = (int)n;
    net->p_thr = (uint32_t)floor(net->p * 4294967296.0);
    net->nfn = calloc((size_t)n, sizeof(int));
    net->fn_first = calloc((size_t)n, sizeof(int));
    int cap = (int)n * 2 + 4;
    net->c = malloc(sizeof(double) * cap); net->thr = malloc(sizeof(uint32_t) * cap);
    net->k = malloc(sizeof(int) * cap); net->par = calloc(cap, sizeof(int *));
    net->tt = calloc(cap, sizeof(uint8_t *));
    for (long i = 0; i < n; i++) {
        long idx, l;
        if (tok_word(&cur, "N") || tok_long(&cur, &idx) || tok_long(&cur, &l)) FAIL("bad node line %ld", i);
        if (idx != i) FAIL("node %ld out of order", i);
        if (l < 1 || l > 64) FAIL("node %ld: bad function count", i);
        net->nfn[i] = (int)l;
        net->fn_first[i] = net->nfun;
        double csum = 0.0;
        for (long j = 0; j < l; j++) {
            if (net->nfun == cap) {
                cap *= 2;
                net->c = realloc(net->c, sizeof(double) * cap);
                net->thr = realloc(net->thr, sizeof(uint32_t) * cap);
                net->k = realloc(net->k, sizeof(int) * cap);
                net->par = realloc(net->par, sizeof(int *) * cap);
                net->tt = realloc(net->tt, sizeof(uint8_t *) * cap);
                for (int z = net->nfun; z < cap; z++) { net->par[z] = NULL; net->tt[z] = NULL; }
            }
            int f = net->nfun++;
            long k;
            net->par[f] = NULL; net->tt[f] = NULL;
            if (tok_word(&cur, "F") || tok_double(&cur, &net->c[f]) || tok_long(&cur, &k))
                FAIL("bad function line (node %ld)", i);
            if (!(net->c[f] >= 0.0 && net->c[f] <= 1.0)) FAIL("node %ld: bad probability", i);
            if (k < 1 || k > 16) FAIL("node %ld: parent count out of range", i);
            net->k[f] = (int)k;
            net->par[f] = malloc(sizeof(int) * k);
            for (long m = 0; m < k; m++) {
                long v;
                if (tok_long(&cur, &v) || v < 0 || v >= n) FAIL("node %ld: bad parent", i);
                for (long q = 0; q < m; q++)
                    if (net->par[f][q] == v) FAIL("node %ld: duplicate parent", i);
                net->par[f][m] = (int)v;
            }
            size_t len; const char *hex = next_token(&cur, &len);
            if (!hex) FAIL("node %ld: missing truth table", i);
            size_t entries = (size_t)1 << k;
            net->tt[f] = calloc(entries, 1);
            /* hex digit d (from the right, 0-based) carries table bits 4d..4d+3 */
            for (size_t d = 0; d < len; d++) {
                int hv = hexval(hex[len - 1 - d]);
                if (hv < 0) FAIL("node %ld: bad hex", i);
                for (int b = 0; b < 4; b++) {
                    size_t e = 4 * d + (size_t)b;
                    if ((hv >> b) & 1) {
                        if (e >= entries) FAIL("node %ld: truth table too long", i);
                        net->tt[f][e] = 1;
                    }
                }
            }
            csum = csum + net->c[f];
            double scaled = floor(csum * 4294967296.0);
            net->thr[f] = scaled >= 4294967295.0 ? 4294967295u : (uint32_t)scaled;
        }
        if (fabs(csum - 1.0) > 1e-12) FAIL("node %ld: probabilities sum to %.17g", i, csum);
    }
    size_t len;
    if (next_token(&cur, &len)) FAIL("trailing tokens");
    g_err[0] = 0;
    return net;
}

int orc_n(const orc_net *net) { return net->n; }
uint32_t orc_p_thr(const orc_net *net) { return net->p_thr; }
int orc_nfun(const orc_net *net) { return net->nfun; }
/* Thresholds of node i as the generator defines them (for tests). */
int orc_node_thresholds(const orc_net *net, int i, uint32_t *out)
{
    int l = net->nfn[i];
    for (int j = 0; j < l; j++) out[j] = net->thr[net->fn_first[i] + j];
    return l;
}

/* --------------------------------------------------------- simulation */

/* Initial states s(0) for chains chain0 .. chain0+nchains-1 into states[nchains][n]. */
void orc_init(const orc_net *net, uint64_t seed, uint32_t chain0, uint32_t nchains, uint8_t *states)
{
    int n = net->n;
    for (uint32_t c = 0; c < nchains; c++) {
        for (int i = 0; i < n; i++) {
            uint32_t w = (uint32_t)i / 32u, out[4];
            philox_at(seed, 0u, chain0 + c, w / 4u, TAG_INIT, out);
            states[(size_t)c * n + i] = (uint8_t)((out[w % 4u] >> (i % 32)) & 1u);
        }
    }
}

typedef struct {
    uint32_t nprops;
    const int32_t *offs;     /* [nprops+1] into nodes/vals */
    const int32_t *nodes;
    const uint8_t *vals;
} props_t;

static uint8_t prop_value(const props_t *pr, uint32_t q, const uint8_t *s)
{
    for (int32_t m = pr->offs[q]; m < pr->offs[q + 1]; m++)
        if (s[pr->nodes[m]] != pr->vals[m]) return 0;
    return 1;
}

/* One transition of one chain: s -> s_next at transition index t. */
static void transition(const orc_net *net, uint64_t seed, uint32_t t, uint32_t chain,
                       const uint8_t *s, uint8_t *s_next, uint8_t *gamma)
{
    int n = net->n;
    int perturbed = 0;
    for (int i = 0; i < n; i++) {
        uint32_t u = orc_uniform(seed, t, chain, (uint32_t)i, TAG_PERT);
        gamma[i] = (uint8_t)(u < net->p_thr);
        perturbed |= gamma[i];
    }
    if (perturbed) {
        for (int i = 0; i < n; i++) s_next[i] = s[i] ^ gamma[i];
        return;
    }
    for (int i = 0; i < n; i++) {
        int l = net->nfn[i];
        int j = l - 1;
        if (l > 1) {
            uint32_t u = orc_uniform(seed, t, chain, (uint32_t)i, TAG_SEL);
            for (int jj = 0; jj < l - 1; jj++)
                if (u < net->thr[net->fn_first[i] + jj]) { j = jj; break; }
        }
        int f = net->fn_first[i] + j;
        uint32_t idx = 0;
        for (int m = 0; m < net->k[f]; m++) idx |= (uint32_t)s[net->par[f][m]] << m;
        s_next[i] = net->tt[f][idx];
    }
}

typedef struct {
    const orc_net *net;
    uint64_t seed;
    uint32_t chain0, c_lo, c_hi, nchains;
    uint8_t *states;
    uint64_t t0, nsteps;
    const props_t *props;
    uint8_t *bits;
} job_t;

static void *run_range(void *arg)
{
    job_t *jb = arg;
    int n = jb->net->n;
    uint8_t *tmp = malloc((size_t)n), *gamma = malloc((size_t)n);
    for (uint32_t c = jb->c_lo; c < jb->c_hi; c++) {
        uint8_t *s = jb->states + (size_t)c * n;
        for (uint64_t st = 0; st < jb->nsteps; st++) {
            transition(jb->net, jb->seed, (uint32_t)(jb->t0 + st), jb->chain0 + c, s, tmp, gamma);
            memcpy(s, tmp, (size_t)n);
            if (jb->bits)
                for (uint32_t q = 0; q < jb->props->nprops; q++)
                    jb->bits[((size_t)q * jb->nchains + c) * jb->nsteps + st] = prop_value(jb->props, q, s);
        }
    }
    free(tmp); free(gamma);
    return NULL;
}

/*
 * Advance chains chain0.. by transitions t0 .. t0+nsteps-1.  states[nchains][n]
 * is updated in place; if bits is non-NULL, bits[q][c][st] receives the
 * indicator of property q in the state after transition t0+st.  Properties are
 * conjunctions (node == value) given in CSR form.  Returns 0 or -1.
 */
int orc_run(const orc_net *net, uint64_t seed, uint32_t chain0, uint32_t nchains,
            uint8_t *states, uint64_t t0, uint64_t nsteps,
            uint32_t nprops, const int32_t *offs, const int32_t *nodes, const uint8_t *vals,
            uint8_t *bits, int nthreads)
{
    if (t0 + nsteps > 0xFFFFFFFFull) { snprintf(g_err, sizeof g_err, "step index overflow"); return -1; }
    props_t pr = {nprops, offs, nodes, vals};
    if (nthreads < 1) nthreads = 1;
    if ((uint32_t)nthreads > nchains) nthreads = (int)(nchains ? nchains : 1);
    pthread_t th[256];
    job_t jobs[256];
    if (nthreads > 256) nthreads = 256;
    for (int w = 0; w < nthreads; w++) {
        job_t jb = {net, seed, chain0, (uint32_t)((uint64_t)nchains * w / nthreads),
                    (uint32_t)((uint64_t)nchains * (w + 1) / nthreads), nchains, states,
                    t0, nsteps, &pr, bits};
        jobs[w] = jb;
    }
    for (int w = 1; w < nthreads; w++) pthread_create(&th[w], NULL, run_range, &jobs[w]);
    run_range(&jobs[0]);
    for (int w = 1; w < nthreads; w++) pthread_join(th[w], NULL);
    return 0;
}

/* Single transition with the perturbation vector exposed (for law tests). */
int orc_step_one(const orc_net *net, uint64_t seed, uint32_t t, uint32_t chain,
                 const uint8_t *s, uint8_t *s_next, uint8_t *gamma)
{
    transition(net, seed, t, chain, s, s_next, gamma);
    return 0;
}

/*
 * Sample `count` transitions out of the same state s (transition indices
 * t0 .. t0+count-1 of one chain); out[k] = index sum_i s'_i 2^i of the next
 * state (n <= 30).  Used by the one-step law tests.
 */
int orc_sample_next(const orc_net *net, uint64_t seed, uint32_t chain, const uint8_t *s,
                    uint32_t t0, uint32_t count, uint32_t *out)
{
    int n = net->n;
    if (n > 30) return -1;
    uint8_t *nx = malloc((size_t)n), *g = malloc((size_t)n);
    for (uint32_t k = 0; k < count; k++) {
        transition(net, seed, t0 + k, chain, s, nx, g);
        uint32_t idx = 0;
        for (int i = 0; i < n; i++) idx |= (uint32_t)nx[i] << i;
        out[k] = idx;
    }
    free(nx); free(g);
    return 0;
}
