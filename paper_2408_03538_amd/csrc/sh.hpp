// Real orthonormal spherical harmonics on the device (FP64), shared by the
// direction tables and the per-splat view basis of the glossy transfer.
#pragma once

#include <hip/hip_runtime.h>

namespace prtgs {

// Real SH through solid-harmonic polynomials: with r^m cos(m phi) and
// r^m sin(m phi) built as the real and imaginary parts of (x + i y)^m, and
// the associated Legendre function divided by (1 - z^2)^(m/2) (a polynomial
// in z, Condon-Shortley phase included) from its recurrence in l, the basis is
//   Y_l^{+m} = sqrt2 K_l^m Pbar_l^m(z) Re(x+iy)^m,   Y_l^{-m} = sqrt2 K_l^m Pbar_l^m(z) Im(x+iy)^m,
//   Y_l^0 = K_l^0 Pbar_l^0(z),   K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
constexpr int kMaxBands = 8;

__device__ inline void real_sh(int bands, double x, double y, double z, double* out)
{
    double re = 1.0, im = 0.0;          // (x + i y)^m
    double pmm = 1.0;                   // Pbar_m^m = (-1)^m (2m-1)!!
    for (int m = 0; m < bands; ++m) {
        if (m > 0) {
            double nre = re * x - im * y;
            im = re * y + im * x;
            re = nre;
            pmm *= -(2.0 * m - 1.0);
        }
        double p_lm2 = 0.0, p_lm1 = pmm;
        for (int l = m; l < bands; ++l) {
            double p;
            if (l == m) p = pmm;
            else if (l == m + 1) p = z * (2.0 * m + 1.0) * pmm;
            else p = ((2.0 * l - 1.0) * z * p_lm1 - (l + m - 1.0) * p_lm2) / (double)(l - m);
            if (l > m) {
                p_lm2 = p_lm1;
                p_lm1 = p;
            }
            double fr = 1.0;            // (l-m)! / (l+m)!
            for (int f = l - m + 1; f <= l + m; ++f) fr /= (double)f;
            double K = sqrt((2.0 * l + 1.0) * fr / (4.0 * 3.14159265358979323846));
            int base = l * l + l;
            if (m == 0) {
                out[base] = K * p;
            } else {
                out[base + m] = 1.41421356237309504880 * K * p * re;
                out[base - m] = 1.41421356237309504880 * K * p * im;
            }
        }
    }
}

}  // namespace prtgs
