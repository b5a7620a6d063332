// mg_cttk.hpp -- kernels of the CTTK and CTTK-Hybrid methods (Summary; Key
// features, "Methods": CTT variants in which the trace K varies in space).
//
// With a varying K, eq. Mom gains -(2/3) psi^6 d_a K.  It carries the psi^6 of the
// momentum density, so the solver takes it as the shifted source
//   S_a -> S_a + D_a K / (12 pi).
// Eq. Ham keeps -(K^2/12) psi^5, which carries the psi^5 of rho5, so a varying K
// enters beside a constant trace K0 as
//   rho5 -> rho5 - (K^2 - K0^2) / (24 pi).
// CTTK-Hybrid: K^2 = 24 pi (rho5 + <rho1>), K0^2 = 24 pi <rho1>, so rho5 -> 0: the
// psi-independent energy density sits in K, the gradient energy in psi.
// CTTK: psi is free data; after every W step eq. Ham is solved for K,
// K^2 = 12 H0 / psi^5 with H0 the Hamiltonian residual at K = 0 (K0 = 0).
#pragma once

#include "mg_device.hpp"

namespace grtmg {

// Block partial sums of an FP64 field, grid-stride: partials[blockIdx.x].
__global__ void __launch_bounds__(kBlock) k_sum_field(const double *__restrict__ a, int64_t m,
                                                      double *__restrict__ partials)
{
    double v[1] = {0.0};
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < m; q += (int64_t)gridDim.x * kBlock)
        v[0] += a[q];
    block_reduce_store<1>(v, 0u, partials + blockIdx.x);
}

// CTTK-Hybrid trace: K = sqrt(24 pi (rho5 + mean)) with mean = <rho1> (a device
// scalar), and rho5 -> 0.
__global__ void __launch_bounds__(kBlock) k_cttk_hybrid_K(int64_t m, const double *__restrict__ mean,
                                                          double *__restrict__ rho5, double *__restrict__ K)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= m) return;
    K[q] = sqrt(24.0 * M_PI * (rho5[q] + *mean));
    rho5[q] = 0.0;
}

// CTTK trace from the K = 0 Hamiltonian residual held in K on entry:
// K^2 = 12 H0 / psi^5 with psi = 1 + u (NaN where K^2 < 0: no real trace), and the
// shifted rho5_eff = rho5 - K^2 / (24 pi).
__global__ void __launch_bounds__(kBlock) k_cttk_K(int64_t m, const double *__restrict__ u,
                                                   const double *__restrict__ rho5, double *__restrict__ K,
                                                   double *__restrict__ rho5_eff)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= m) return;
    const double psi = 1.0 + u[q];
    const double psi2 = psi * psi;
    double K2 = 12.0 * K[q] / (psi2 * psi2 * psi);
    if (!(K2 >= 0.0)) K2 = __builtin_nan("");
    K[q] = sqrt(K2);
    rho5_eff[q] = rho5[q] - K2 / (24.0 * M_PI);
}

// Shifted momentum density S_out = S_in + D K / (12 pi), D the fourth-order first
// derivative under the boundary rule (S_in null: zero; S_out may be S_in).
template <int BC>
__global__ void __launch_bounds__(kBlock) k_cttk_shift_S(Geo g, const double *__restrict__ K, const double *S_in,
                                                         double *S_out)
{
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= m) return;
    const int k = (int)(q % n), j = (int)((q / n) % n), i = (int)(q / ((int64_t)n * n));
    const Acc<BC, double> A{K, g};
    const double s = 1.0 / (12.0 * g.h * 12.0 * M_PI);
    const double dx = (A(i - 2, j, k) - 8.0 * A(i - 1, j, k)) + (8.0 * A(i + 1, j, k) - A(i + 2, j, k));
    const double dy = (A(i, j - 2, k) - 8.0 * A(i, j - 1, k)) + (8.0 * A(i, j + 1, k) - A(i, j + 2, k));
    const double dz = (A(i, j, k - 2) - 8.0 * A(i, j, k - 1)) + (8.0 * A(i, j, k + 1) - A(i, j, k + 2));
    const double d[3] = {dx, dy, dz};
#pragma unroll
    for (int a = 0; a < 3; a++) S_out[a * m + q] = (S_in ? S_in[a * m + q] : 0.0) + d[a] * s;
}

// ---- Anderson mixing of the CTTK fixed point ------------------------------------------
// The K-W coupling makes the CTTK outer iteration a fixed-point iteration whose
// contraction grows with resolution; consecutive W steps are combined by one-step
// Anderson mixing (a secant method on the fixed point).  With f = d - mean(d) the
// W step's correction, dF = f - f_prev and dW = W - W_prev from the previous
// iteration:  gamma = <dF, f> / <dF, dF>,  W -> W + f - gamma (dW + dF).
// aa: device scalars {<dF, f>, <dF, dF>, steps taken, gamma}.

// Block partial sums of <dF, f> and <dF, dF> over the three components (grid-stride).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_aa_dots(const T *__restrict__ d, const double *__restrict__ mean,
                                                    const double *__restrict__ f_prev, int64_t m,
                                                    double *__restrict__ partials)
{
    double v[2] = {0.0, 0.0};
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < 3 * m; q += (int64_t)gridDim.x * kBlock) {
        const double f = (double)d[q] - mean[q / m];
        const double dF = f - f_prev[q];
        v[0] += dF * f;
        v[1] += dF * dF;
    }
    block_reduce_store<2>(v, 0u, partials + 2 * (int64_t)blockIdx.x);
}

// gamma from the reduced sums (0 on the first step or when dF = 0); counts the step.
__global__ void k_aa_gamma(double *aa)
{
    if (threadIdx.x != 0) return;
    aa[3] = (aa[2] > 0.0 && aa[1] > 0.0) ? aa[0] / aa[1] : 0.0;
    aa[2] += 1.0;
}

// W -> W + f - gamma (dW + dF); the history becomes W_prev = W, f_prev = f.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_aa_update(double *__restrict__ W, const T *__restrict__ d,
                                                      const double *__restrict__ mean, double *__restrict__ W_prev,
                                                      double *__restrict__ f_prev, const double *__restrict__ aa,
                                                      int64_t m)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= 3 * m) return;
    const double gamma = aa[3];
    const double f = (double)d[q] - mean[q / m];
    const double w = W[q];
    const double mix = gamma != 0.0 ? gamma * ((w - W_prev[q]) + (f - f_prev[q])) : 0.0;
    W[q] = w + f - mix;
    W_prev[q] = w;
    f_prev[q] = f;
}

} // namespace grtmg
