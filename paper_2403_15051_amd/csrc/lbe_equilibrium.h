// Discrete equilibrium factors g_{a,k}(u, T) of one momentum axis (Sec. III.C), usable on
// the host and on the device.
//
// The paper writes the half-range factor, eq. (eq_gak_hh), as a sum over half-line moments
// of the 1-D Gaussian times Phi_s^N(|p_k|) (monomial basis).  That sum cancels by up to ~1e6
// in floating point, and so does the three-term recurrence one can derive for the projection
// coefficients, so the same projection is evaluated here in the orthonormal basis with the
// coefficients computed by quadrature:
//   g_k = w_k sum_{l=0}^{N} I_l^{sigma_k} h_l(|p_k|),
//   I_l^+ = int_0^inf G(p; u, T) h_l(p) dp ~= sum_m lam_m G(y_m; u, T) h_l(y_m),   I_l^- = I_l^+(-u, T),
// with a fixed composite Gauss-Legendre rule (y_m, lam_m) on [0, Y] chosen by the host so that
// the Gaussian of every temperature the instance can reach is integrated to rounding.
// The full-range factor, eq. (eq_gak_H), uses c_l = E[He_l(X)]/l! for X ~ N(u, T), which
// obey c_{l+1} = (u c_l + (T - 1) c_{l-1})/(l + 1), c_0 = 1, c_1 = u:
//   g_k = w_k sum_{l=0}^{N} c_l He_l(p_k).
#pragma once

#include <hip/hip_runtime.h>

namespace lbe {

constexpr double kInvSqrt2Pi = 0.398942280401432677939946059934381868;

// Coefficients I_l (l = 0..N) of the half-line projection for one side (uu = +-u), summing
// the quadrature nodes m in [m0, m1) only (the caller may split the sum).
__host__ __device__ inline void half_projection_part(double uu, double T, int N, int m0, int m1, const double* y,
                                                     const double* lam, const double* hy, double* I)
{
    const double c = kInvSqrt2Pi / sqrt(T), inv2T = 1 / (2 * T);
    for (int l = 0; l <= N; l++) I[l] = 0;
    for (int m = m0; m < m1; m++) {
        const double d = y[m] - uu;
        const double g = lam[m] * c * exp(-d * d * inv2T);
        const double* h = hy + (size_t)m * (N + 1);
        for (int l = 0; l <= N; l++) I[l] += g * h[l];
    }
}

template <int NMAX>
__host__ __device__ inline void full_coeffs(double u, double T, int N, double* c)
{
    c[0] = 1;
    if (N >= 1) c[1] = u;
    for (int l = 1; l < N; l++) c[l + 1] = (u * c[l] + (T - 1) * c[l - 1]) / (l + 1);
}

}  // namespace lbe
