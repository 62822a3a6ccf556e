// Host FP64 statistics of the method, evaluated from exact integer aggregates
// produced by the device reductions.  Compiled with -ffp-contract=off so that
// every expression rounds exactly as written.
#include <algorithm>
#include <cmath>

#include "pbn_internal.h"

namespace pbn {

// Phi^{-1}(p): Wichura's algorithm AS 241 (PPND16), Applied Statistics 37 (1988).
double normal_quantile(double p)
{
    static const double a[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2,
                                1.9715909503065514427e+3, 1.3731693765509461125e+4,
                                4.5921953931549871457e+4, 6.7265770927008700853e+4,
                                3.3430575583588128105e+4, 2.5090809287301226727e+3};
    static const double b[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
                                5.3941960214247511077e+3, 2.1213794301586595867e+4,
                                3.9307895800092710610e+4, 2.8729085735721942674e+4,
                                5.2264952788528545610e+3};
    static const double c[8] = {1.42343711074968357734e0, 4.63033784615654529590e0,
                                5.76949722146069140550e0, 3.64784832476320460504e0,
                                1.27045825245236838258e0, 2.41780725177450611770e-1,
                                2.27238449892691845833e-2, 7.74545014278341407640e-4};
    static const double d[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
                                6.89767334985100004550e-1, 1.48103976427480074590e-1,
                                1.51986665636164571966e-2, 5.47593808499534494600e-4,
                                1.05075007164441684324e-9};
    static const double e[8] = {6.65790464350110377720e0, 5.46378491116411436990e0,
                                1.78482653991729133580e0, 2.96560571828504891230e-1,
                                2.65321895265761230930e-2, 1.24266094738807843860e-3,
                                2.71155556874348757815e-5, 2.01033439929228813265e-7};
    static const double f[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
                                1.48753612908506148525e-2, 7.86869131145613259100e-4,
                                1.84631831751005468180e-5, 1.42151175831644588870e-7,
                                2.04426310338993978564e-15};
    // Horner evaluation from the highest coefficient down.
    auto horner = [](const double *co, double x) {
        double acc = co[7];
        for (int i = 6; i >= 0; --i) acc = acc * x + co[i];
        return acc;
    };
    double q = p - 0.5;
    if (std::fabs(q) <= 0.425) {
        double r = 0.180625 - q * q;
        return q * horner(a, r) / horner(b, r);
    }
    double r = q < 0.0 ? p : 1.0 - p;
    r = std::sqrt(-std::log(r));
    double val;
    if (r <= 5.0) {
        r = r - 1.6;
        val = horner(c, r) / horner(d, r);
    } else {
        r = r - 5.0;
        val = horner(e, r) / horner(f, r);
    }
    return q < 0.0 ? -val : val;
}

// Student-t quantile by the Cornish-Fisher expansion in 1/nu (Abramowitz and
// Stegun 26.7.5), used only for nu >= 100 (batch counts of Skart are >= 446).
double t_quantile(double p, double nu)
{
    double z = normal_quantile(p);
    double z2 = z * z;
    double g1 = (z2 + 1.0) * z / 4.0;
    double g2 = ((5.0 * z2 + 16.0) * z2 + 3.0) * z / 96.0;
    double g3 = (((3.0 * z2 + 19.0) * z2 + 17.0) * z2 - 15.0) * z / 384.0;
    double g4 = ((((79.0 * z2 + 776.0) * z2 + 1482.0) * z2 - 1920.0) * z2 - 945.0) * z / 92160.0;
    return z + g1 / nu + g2 / (nu * nu) + g3 / (nu * nu * nu) + g4 / (nu * nu * nu * nu);
}

// Gelman-Rubin R of Alg. 3 for 0-1 data from window sums.  With S_c the ones of
// chain c in a window of psi positions, T1 = sum S_c and T2 = sum S_c^2:
//   s_c^2 = S_c (psi - S_c) / (psi (psi-1)),  W = (psi T1 - T2) / (omega psi (psi-1)),
//   B = (omega T2 - T1^2) / (omega (omega-1) psi),
//   R^2 = sigma^2 / W = ((psi-1)/psi) (1 + A/D),  A = omega T2 - T1^2, D = (omega-1)(psi T1 - T2).
// *defined = false when W = 0.
double rhat_from_sums(int64_t T1, int64_t T2, uint64_t omega, uint64_t psi, bool *defined)
{
    __int128 A = (__int128)omega * T2 - (__int128)T1 * T1;
    __int128 D = (__int128)(omega - 1) * ((__int128)psi * T1 - T2);
    if (D <= 0) {
        *defined = false;
        return INFINITY;
    }
    *defined = true;
    double r2 = ((double)(psi - 1) / (double)psi) * (1.0 + (double)A / (double)D);
    return std::sqrt(r2);
}

// ---------------------------------------------------------------- Skart-P
//
// Batch means Y = b / kappa of integer batch sums b[c m + j] (chain c, batch j
// of kappa positions; P = omega m batches).  Every sum over the batches is
// exact (128-bit integers); the moments about the grand mean follow by exact
// integer algebra and floating point enters once per ratio:
//   S1 = sum b, S2 = sum b^2, S3 = sum b^3
//   Q2 = P S2 - S1^2                  = kappa^2 P   sum (Y - mu)^2
//   Q3 = P^2 S3 - 3 P S1 S2 + 2 S1^3  = kappa^3 P^2 sum (Y - mu)^3
//   over the omega (m-1) within-chain pairs (b_j, b_{j+1}):
//   L = sum b_j b_{j+1}, E = sum (b_j + b_{j+1}), D2 = sum (b_{j+1} - b_j)^2
//   QL = P^2 L - P S1 E + pairs S1^2  = kappa^2 P^2 sum (Y_{j+1} - mu)(Y_j - mu)
// With 0 <= b <= kappa and kappa P <= 2^40 every term is below 2^126.

bool skewness_exceeds_4(uint64_t ones, uint64_t count)
{
    // 0-1 data: skewness (1-2q)/sqrt(q(1-q)), q = ones/count; no ones or no
    // zeros: zero variance, unbounded skewness
    if (ones == 0 || ones == count) return true;
    const __int128 d = (__int128)count - 2 * (__int128)ones;
    return d * d > (__int128)16 * ones * (count - ones);
}

BatchMoments batch_moments(const int32_t *b, uint32_t omega, uint64_t m)
{
    BatchMoments g;
    __int128 S1 = 0, S2 = 0, S3 = 0, L = 0, E = 0, D2 = 0;
    for (uint32_t c = 0; c < omega; ++c) {
        const int32_t *row = b + (uint64_t)c * m;
        for (uint64_t j = 0; j < m; ++j) {
            const __int128 v = row[j];
            S1 += v;
            S2 += v * v;
            S3 += v * v * v;
            if (j + 1 < m) {
                const __int128 w = row[j + 1];
                L += v * w;
                E += v + w;
                D2 += (w - v) * (w - v);
            }
        }
    }
    const __int128 P = (__int128)omega * m;
    g.m = m;
    g.P = (uint64_t)P;
    g.pairs = (uint64_t)omega * (m - 1);
    g.S1 = S1;
    g.D2 = D2;
    g.Q2 = P * S2 - S1 * S1;
    g.Q3 = P * P * S3 - 3 * P * S1 * S2 + 2 * S1 * S1 * S1;
    g.QL = P * P * L - P * S1 * E + (__int128)g.pairs * S1 * S1;
    return g;
}

// Von Neumann ratio over within-chain adjacent batch means, one-sided at level
// 0.2: C = 1 - (squared successive differences / pairs) / (2 squared
// deviations / (P-1)) = 1 - D2 P (P-1) / (2 pairs Q2) (the batch size cancels).
bool randomness_passes(const BatchMoments &g, double *C_out, double *limit_out)
{
    if (C_out) *C_out = NAN;
    if (limit_out) *limit_out = NAN;
    if (g.m < 2 || g.Q2 == 0) return true;
    const __int128 P = g.P;
    const double C = 1.0 - (double)(g.D2 * P * (P - 1)) / (double)(2 * (__int128)g.pairs * g.Q2);
    const double limit = normal_quantile(1.0 - 0.2) * std::sqrt(1.0 / (double)g.pairs);
    if (C_out) *C_out = C;
    if (limit_out) *limit_out = limit;
    return C <= limit;
}

// Skewness (Willink) and lag-1 autoregression adjusted t interval on the batch
// means: mu = S1/(kappa P); phi = QL/(pairs Q2), A = (1+phi)/(1-phi) if phi > 0
// else 1; se = sqrt(A S^2/P) with S^2/P = Q2/(kappa^2 P^2 (P-1)); skewness
// Q3/Q2^{3/2}, beta = skew/(6 sqrt P); CI = [mu - G(t) se, mu - G(-t) se] with t
// the Student t quantile 1 - alpha/2 on P-1 degrees of freedom.  All batch
// means equal (Q2 = 0): the point interval at mu.
void adjusted_ci(const BatchMoments &g, uint64_t kappa, double conf, double *mu_out, double *lo_out,
                 double *hi_out)
{
    const __int128 K = kappa, P = g.P;
    const double mu = (double)g.S1 / (double)(K * P);
    *mu_out = *lo_out = *hi_out = mu;
    if (g.Q2 == 0) return;
    const double phi = g.m >= 2 ? (double)g.QL / (double)((__int128)g.pairs * g.Q2) : 0.0;
    const double A = phi > 0.0 ? (1.0 + phi) / (1.0 - phi) : 1.0;
    const double v = (double)g.Q2 / (double)(K * K * P * P * (P - 1));
    const double q2 = (double)g.Q2;
    const double skew = (double)g.Q3 / (q2 * std::sqrt(q2));
    const double beta = skew / (6.0 * std::sqrt((double)g.P));
    const double alpha = 1.0 - conf;
    const double t_hi = t_quantile(1.0 - alpha / 2.0, (double)(g.P - 1));
    const double se = std::sqrt(A * v);
    *lo_out = mu - willink(t_hi, beta) * se;
    *hi_out = mu - willink(-t_hi, beta) * se;
}

// Skewness adjustment of a t critical value (Willink): ((1+6b(z-b))^{1/3}-1)/(2b);
// the cube root minus one is expm1(log1p(x)/3) for |x| < 1/2.
double willink(double zeta, double beta)
{
    if (beta == 0.0) return zeta;
    double x = 6.0 * beta * (zeta - beta);
    double d = std::fabs(x) < 0.5 ? std::expm1(std::log1p(x) / 3.0) : std::cbrt(1.0 + x) - 1.0;
    return d / (2.0 * beta);
}

}  // namespace pbn

extern "C" int pbn_skart_batch_stats(const int32_t *bsum, uint32_t omega, uint64_t m, uint64_t kappa,
                                     double confidence, pbn_skart_stats *out)
{
    if (!bsum || !out || omega < 1 || m < 1 || kappa < 1 || !(confidence > 0.0 && confidence < 1.0))
        return PBN_EINVAL;
    if (m > PBN_SKART_MAX_OBS || (double)omega * (double)m * (double)kappa > (double)PBN_SKART_MAX_OBS)
        return PBN_ELIMIT;
    const uint64_t P = (uint64_t)omega * m;
    if (P < 101) return PBN_EINVAL;                 // the t quantile is taken for P-1 >= 100
    for (uint64_t e = 0; e < P; ++e)
        if (bsum[e] < 0 || (uint64_t)bsum[e] > kappa) return PBN_EINVAL;
    const pbn::BatchMoments g = pbn::batch_moments(bsum, omega, m);
    out->vn_passes = pbn::randomness_passes(g, &out->vn_C, &out->vn_limit) ? 1 : 0;
    pbn::adjusted_ci(g, kappa, confidence, &out->mu, &out->ci_lo, &out->ci_hi);
    out->H = std::max(out->mu - out->ci_lo, out->ci_hi - out->mu);
    out->reserved = 0;
    return PBN_OK;
}

extern "C" double pbn_normal_quantile(double p) { return pbn::normal_quantile(p); }
extern "C" double pbn_t_quantile(double p, double nu) { return pbn::t_quantile(p, nu); }
