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

// Anderson mixing over the last D >= 2 steps.  Ring slots j < D hold, for consecutive
// steps, dF_j = f - f_prev and dG_j = dW_j + dF_j with dW_j = W - W_prev (slot j at
// j * 3m; the update needs only their sum), stored in the context's working type T (FP32
// in FP32 contexts: they steer the iteration, not its fixed point); the newest pair
// replaces the oldest.  st = {pairs stored, slot of the next pair, steps
// taken, unused x5, gamma_0 .. gamma_{D-1}, unused up to 16, the reduced sums}.  gamma minimises |f - sum_j gamma_j dF_j|
// through its normal equations: the secant quotient for one stored pair; for more, a
// ridge of 1e-12 of the largest Gram diagonal entry and Gaussian elimination with
// partial pivoting (gamma = 0 if that entry is 0); W -> W + f - sum_j gamma_j (dW_j + dF_j).
constexpr int kMixMax = 6; // mix_nv<6>() = 27 sums: within the 32 of one reduction mask
template <int D>
constexpr int mix_nv()
{
    return D + D * (D + 1) / 2;
}
constexpr int kMixRed = 16; // offset of the reduced sums in the state
constexpr int kMixState = kMixRed + mix_nv<kMixMax>();

// One pass over the 3m values: from the second step on the newest pair (dG, dF) into its slot,
// and block partials of <dF_i, f> (i < D), then <dF_i, dF_j> (j <= i), over the
// stored pairs (zero for slots not yet filled).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_aa_push_dots(const T *__restrict__ d, const double *__restrict__ mean,
                                                         const double *__restrict__ W,
                                                         const double *__restrict__ W_prev,
                                                         const double *__restrict__ f_prev, T *__restrict__ dG_ring,
                                                         T *__restrict__ dF_ring, const double *__restrict__ st,
                                                         int64_t m, double *__restrict__ partials)
{
    constexpr int NV = mix_nv<D>();
    static_assert(NV <= 32, "block_reduce_store's max_mask holds one bit per value");
    const int64_t n3 = 3 * m;
    const bool push = st[2] > 0.0;
    const int head = (int)st[1];
    const int cnt = min((int)st[0] + (push ? 1 : 0), D);
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n3; q += (int64_t)gridDim.x * kBlock) {
        const double f = (double)d[q] - mean[q / m];
        const double dFn = push ? (double)(T)(f - f_prev[q]) : 0.0; // the stored value
        if (push) {
            dF_ring[head * n3 + q] = (T)dFn;
            dG_ring[head * n3 + q] = (T)((W[q] - W_prev[q]) + dFn);
        }
        double F[D];
#pragma unroll
        for (int i = 0; i < D; i++) F[i] = i >= cnt ? 0.0 : (push && i == head) ? dFn : (double)dF_ring[i * n3 + q];
        int k = D;
#pragma unroll
        for (int i = 0; i < D; i++) {
            v[i] += F[i] * f;
#pragma unroll
            for (int j = 0; j <= i; j++) v[k++] += F[i] * F[j];
        }
    }
    block_reduce_store<NV>(v, 0u, partials + (int64_t)NV * blockIdx.x);
}

// gamma from the reduced sums red (layout of k_aa_push_dots); counts the pair and the step.
template <int D>
__global__ void k_aa_solve(const double *__restrict__ red, double *__restrict__ st)
{
    if (threadIdx.x != 0) return;
    const bool push = st[2] > 0.0;
    const int cnt = min((int)st[0] + (push ? 1 : 0), D);
    double A[D * D], b[D], g[D];
    for (int i = 0; i < D; i++) g[i] = 0.0;
    for (int i = 0; i < cnt; i++) {
        b[i] = red[i];
        for (int j = 0; j <= i; j++) A[i * cnt + j] = A[j * cnt + i] = red[D + i * (i + 1) / 2 + j];
    }
    if (cnt == 1) {
        g[0] = A[0] > 0.0 ? b[0] / A[0] : 0.0;
    } else if (cnt > 1) {
        double dmax = 0.0;
        for (int i = 0; i < cnt; i++) dmax = fmax(dmax, A[i * cnt + i]);
        if (dmax > 0.0) {
            for (int i = 0; i < cnt; i++) A[i * cnt + i] += 1e-12 * dmax;
            for (int k = 0; k < cnt; k++) {
                int piv = k;
                for (int i = k + 1; i < cnt; i++)
                    if (fabs(A[i * cnt + k]) > fabs(A[piv * cnt + k])) piv = i;
                if (piv != k) {
                    for (int j = 0; j < cnt; j++) {
                        const double t = A[k * cnt + j];
                        A[k * cnt + j] = A[piv * cnt + j];
                        A[piv * cnt + j] = t;
                    }
                    const double t = b[k];
                    b[k] = b[piv];
                    b[piv] = t;
                }
                for (int i = k + 1; i < cnt; i++) {
                    const double l = A[i * cnt + k] / A[k * cnt + k];
                    for (int j = k; j < cnt; j++) A[i * cnt + j] -= l * A[k * cnt + j];
                    b[i] -= l * b[k];
                }
            }
            for (int i = cnt - 1; i >= 0; i--) {
                double x = b[i];
                for (int j = i + 1; j < cnt; j++) x -= A[i * cnt + j] * g[j];
                g[i] = x / A[i * cnt + i];
            }
        }
    }
    for (int i = 0; i < D; i++) st[8 + i] = g[i];
    st[0] = (double)cnt;
    if (push) st[1] = (double)((int)(st[1] + 0.5) + 1 == D ? 0 : (int)(st[1] + 0.5) + 1);
    st[2] += 1.0;
}

// W -> W + f - sum_j gamma_j dG_j over the stored pairs; the history becomes
// W_prev = W, f_prev = f.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock) k_aa_update_ring(double *__restrict__ W, const T *__restrict__ d,
                                                           const double *__restrict__ mean,
                                                           double *__restrict__ W_prev, double *__restrict__ f_prev,
                                                           const T *__restrict__ dG_ring,
                                                           const double *__restrict__ st, int64_t m)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n3 = 3 * m;
    if (q >= n3) return;
    const int cnt = (int)st[0];
    const double f = (double)d[q] - mean[q / m];
    const double w = W[q];
    double mix = 0.0;
#pragma unroll
    for (int j = 0; j < D; j++)
        if (j < cnt) mix += st[8 + j] * (double)dG_ring[j * n3 + q];
    W[q] = w + f - mix;
    W_prev[q] = w;
    f_prev[q] = f;
}

} // namespace grtmg
