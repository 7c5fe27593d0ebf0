// Chebyshev coefficients of the ideal low-pass on the device (float64).
#pragma once

#include <hip/hip_runtime.h>

namespace asc {

constexpr double kPi = 3.14159265358979323846;

// a_j = g_j c_j of h_lc on [0, L] (Eq. ideal, Sec. 2.4): with x = 2 lambda / L - 1
// and theta = arccos(2 lc / L - 1), the step 1[x <= x_c] has the Chebyshev
// coefficients c_0 = 1 - theta/pi (not halved) and c_j = -2 sin(j theta)/(j pi);
// g_j are the Jackson damping factors of order p (alpha = pi/(p+2)).
__device__ inline double cheb_coeff_dev(double lc, double L, int p, int j, int jackson) {
    double xc = 2.0 * lc / L - 1.0;
    xc = fmin(fmax(xc, -1.0), 1.0);
    const double th = acos(xc);
    double c = (j == 0) ? 1.0 - th / kPi : -2.0 * sin(j * th) / (j * kPi);
    if (jackson) {
        const double a = kPi / (p + 2);
        const double g = ((p + 2 - j) * cos(j * a) + sin(j * a) / tan(a)) / (p + 2);
        c *= g;
    }
    return c;
}

}  // namespace asc
