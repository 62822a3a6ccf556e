// Host FP64 statistics of the method, evaluated from exact integer aggregates
// produced by the device reductions.  Compiled with -ffp-contract=off so that
// every expression rounds exactly as written.
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

}  // namespace pbn

extern "C" double pbn_normal_quantile(double p) { return pbn::normal_quantile(p); }
extern "C" double pbn_t_quantile(double p, double nu) { return pbn::t_quantile(p, nu); }
