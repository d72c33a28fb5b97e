// Prefilter constants c(k) on the host, in FP64 (Section 7).
//
// kappa = k'/n with k' the signed FFT index.  Both variants need lattice sums
// S_M(kappa) = sum_i sinc^M(kappa + i), which by Poisson summation equal the
// finite cosine sums sum_s B_M(s) cos(2 pi kappa s) over the integer samples of
// the centred B-spline B_M (zero for |s| >= M/2).  That closed form is what is
// evaluated here:
//   INTERP  c = 1 / S_N(kappa)                      (1 / F_D[B_D](k))
//   L2OPT   c = sinc^N(kappa) / S_2N(kappa)         (F[B] / sum_i F[B](kappa+i)^2)
//   NONE    c = 1                                   (grid values: Lagrange, linear, Hermite)
// and, for the Hermite derivative fields, the real factor 2 pi k'/n of d/ds.
#include <cmath>

#include "common.hpp"

namespace bsi {

namespace {

double lattice_sum(int M, long long ks, int n) {
    // sum over s of B_M(s) cos(2 pi ks s / n); the argument is reduced exactly
    // in integers before the single rounding of the angle.
    double acc = bspline_integer_sample(M, 0);
    for (int s = 1; s < M / 2; ++s) {
        long long m = (ks * s) % n;
        if (m < 0) m += n;
        const double ang = 2.0 * M_PI * double(m) / double(n);
        acc += 2.0 * bspline_integer_sample(M, s) * std::cos(ang);
    }
    return acc;
}

}  // namespace

void prefilter_table(int n, int order, int variant, double* out) {
    for (int k = 0; k < n; ++k) {
        const long long ks = (k <= n / 2) ? k : k - n;
        if (variant == BSI_PREFILTER_NONE) {
            out[k] = 1.0;
        } else if (variant == DERIVATIVE_TABLE) {
            // d/ds of exp(2 pi i ks s / n) in grid units is i 2 pi ks / n times
            // it: the real factor here, i applied by the FFT's first pass; the
            // Nyquist index of a real field has no derivative
            out[k] = (2 * ks == n) ? 0.0 : 2.0 * M_PI * double(ks) / double(n);
        } else if (variant == BSI_PREFILTER_INTERP) {
            out[k] = 1.0 / lattice_sum(order, ks, n);
        } else {
            double sinc = 1.0;
            if (ks != 0) {
                const double x = M_PI * double(ks) / double(n);
                sinc = std::sin(x) / x;
            }
            out[k] = std::pow(sinc, order) / lattice_sum(2 * order, ks, n);
        }
    }
}

}  // namespace bsi
