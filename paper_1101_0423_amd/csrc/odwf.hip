// odwf.hip -- the weights of optimal domain-wall fermions (the omega_s that
// Sec. 2.1 fixes for optimal chiral symmetry, with sigma = omega).  Host
// code only.
//
// With sigma = omega the 4D operator on the walls depends on the weights
// through the transfer product Pi(lam) = prod_s (1 - omega_s lam)/(1 + omega_s
// lam) over the spectrum of H = gamma_5 D_w, and it is chirally exact where
// Pi vanishes.  The weights that minimise max |Pi| on an interval
// [lam_min, lam_max] solve Zolotarev's third problem, whose solution places
// the zeros 1 / omega_s at
//     p_j = lam_max dn((2j - 1) K / (2 Ns), k),  k = sqrt(1 - (lam_min / lam_max)^2),
// K = K(k) the complete elliptic integral; equivalently
//     omega_s = dn((2s - 1) K / (2 Ns), k) / lam_min,
// because dn(K - u) = k' / dn(u) with k' = lam_min / lam_max.
// K and dn come from the arithmetic-geometric mean (the descending Landen
// scheme for the Jacobi functions, Abramowitz & Stegun 16.4 and 17.6).
#include <math.h>

#include "dwf_ctx.h"

namespace dwf {
namespace {

constexpr int kAgmMax = 64;

// K(k) = pi / (2 AGM(1, k')), k' = sqrt(1 - k^2) given directly
double ellip_k(double kc) {
    double a = 1.0, b = kc;
    for (int n = 0; n < kAgmMax && fabs(a - b) > 1e-16 * a; ++n) {
        const double an = 0.5 * (a + b);
        b = sqrt(a * b);
        a = an;
    }
    return M_PI / (2.0 * a);
}

// dn(u, k) by the AGM: a_0 = 1, b_0 = k', c_0 = k; phi_N = 2^N a_N u, then
// phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2 and
// dn = cos(phi_0) / cos(phi_1 - phi_0)
double jacobi_dn(double u, double k, double kc) {
    double a[kAgmMax + 1], c[kAgmMax + 1];
    a[0] = 1.0;
    double b = kc;
    c[0] = k;
    int n = 0;
    while (n < kAgmMax && fabs(c[n]) > 1e-16) {
        a[n + 1] = 0.5 * (a[n] + b);
        c[n + 1] = 0.5 * (a[n] - b);
        b = sqrt(a[n] * b);
        ++n;
    }
    double phi = ldexp(a[n] * u, n);
    double phi_next = phi;  // phi_1 once the loop ends
    for (int j = n; j >= 1; --j) {
        phi_next = phi;
        phi = 0.5 * (phi + asin(c[j] * sin(phi) / a[j]));
    }
    if (n == 0) return 1.0;  // k = 0: dn = 1
    return cos(phi) / cos(phi_next - phi);
}

}  // namespace
}  // namespace dwf

extern "C" int dwf_odwf_weights(int Ns, double lambda_min, double lambda_max, double* omega) {
    using namespace dwf;
    if (!omega) return fail(DWF_EINVAL, "NULL omega");
    if (Ns < 1) return fail(DWF_EINVAL, "Ns must be >= 1");
    if (!(lambda_min > 0) || !(lambda_max >= lambda_min) || !std::isfinite(lambda_max))
        return fail(DWF_EINVAL, "need 0 < lambda_min <= lambda_max < inf");
    const double kc = lambda_min / lambda_max;  // k'
    const double k = sqrt((1.0 - kc) * (1.0 + kc));
    const double K = ellip_k(kc);
    for (int s = 0; s < Ns; ++s) {
        const double u = (2.0 * s + 1.0) * K / (2.0 * Ns);
        omega[s] = jacobi_dn(u, k, kc) / lambda_min;
    }
    return DWF_OK;
}
