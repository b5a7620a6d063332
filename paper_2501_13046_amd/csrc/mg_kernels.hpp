// mg_kernels.hpp -- HIP kernels of the constraint multigrid (gfx950).
//
// Every multigrid kernel here is bound by HBM bandwidth: one thread per cell
// (z fastest, so a wavefront reads 64 consecutive cells of a z-line), stencil
// neighbours served by the L1/L2 caches.  The residual and the update stay
// FP64; the V-cycle kernels are templated on the working type T (float for
// the FP32 V-cycle inside FP64 iterative refinement, double otherwise).
#pragma once

#include "mg_device.hpp"

namespace grtmg {

constexpr double kPi = 3.14159265358979323846;

// Cell (i, j, k) of linear index tid (z fastest); false past the grid.  The
// grids hold fewer than 2^32 cells (validated at the API), so the division
// runs in 32 bits: a 64-bit division by a runtime n costs ~10x the instructions.
__device__ __forceinline__ bool cell_of(int64_t tid, int n, int &i, int &j, int &k)
{
    const int64_t cells = (int64_t)n * n * n;
    if (tid >= cells) return false;
    const unsigned t = (unsigned)tid, un = (unsigned)n;
    const unsigned r = t / un;
    k = (int)(t - r * un);
    const unsigned s = r / un;
    j = (int)(r - s * un);
    i = (int)s;
    return true;
}

__device__ __forceinline__ double psi0_at(const Geo &g, double pmass, int i, int j, int k)
{
    return pmass > 0.0 ? 1.0 + pmass / (2.0 * cell_radius(g, i, j, k)) : 1.0;
}

// ---------------------------------------------------------------------------------------
// Nonlinear residuals (FP64).  Per cell: psi = psi0 + u,
//   H = L_h u + 2 pi rho5 psi^5 + 2 pi rho1 psi - (K^2/12) psi^5 + A2 psi^-7/8 + f
//   c = 10 pi rho5 psi^4 + 2 pi rho1 - (5 K^2/12) psi^4 - (7/8) A2 psi^-8
//   M_a = (Delta_L W)_a - (8 pi psi^6 S_a - meanS_a)
// Outputs are optional: H, M, c as FP64 fields; r = -H, rc = c, rW = -M in T;
// per-block partials (sum H^2, max |H|, sum |M|^2, max |M|).
// ---------------------------------------------------------------------------------------
struct ResArgs {
    const double *u, *W, *rho5, *rho1, *S, *f;
    // optional background (may be null): psi0 in place of 1 + M/(2r), and the A2
    // of an analytic traceless extrinsic curvature added to the one of W
    const double *psi0f, *A2bg;
    const double *meanS; // device, 3 values (periodic momentum source mean)
    const double *K2p;   // device K^2 of the member (grouped batches), else null: K2
    double K2, pmass;
    double *H, *M, *c;
    void *r, *rc, *rW; // T
    double *partials;  // 4 per block
    // first colour pass of the finest level from a zero correction (T; may be
    // null): d1 from r and rc (psi), d1W from rW times idiagW (W)
    void *d1, *d1W;
    double idiagW;
    int want_M;        // compute momentum residual
    int conformal;     // matter given as rho_bar = psi^8 rho, S_bar = psi^6 S
};

// Every array of a ResArgs moved to this block's member of a grouped launch.
__device__ __forceinline__ ResArgs res_shift(ResArgs a, long long zs)
{
    if (zs == 0) return a;
    a.u = zsh(a.u, zs);
    a.W = zsh(a.W, zs);
    a.rho5 = zsh(a.rho5, zs);
    a.rho1 = zsh(a.rho1, zs);
    a.S = zsh(a.S, zs);
    a.f = zsh(a.f, zs);
    a.psi0f = zsh(a.psi0f, zs);
    a.A2bg = zsh(a.A2bg, zs);
    a.meanS = zsh(a.meanS, zs);
    a.K2p = zsh(a.K2p, zs);
    a.H = zsh(a.H, zs);
    a.M = zsh(a.M, zs);
    a.c = zsh(a.c, zs);
    a.r = zsh(a.r, zs);
    a.rc = zsh(a.rc, zs);
    a.rW = zsh(a.rW, zs);
    a.partials = zsh(a.partials, zs);
    a.d1 = zsh(a.d1, zs);
    a.d1W = zsh(a.d1W, zs);
    return a;
}

// The finest level's first colour pass from a zero correction at cell (x, y, z),
// written beside the right-hand side (colour 0: r / diag as the pass kernels
// form it; colour 1: 0) so that the V-cycle starts with the second pass.
template <int BC, typename T>
__device__ __forceinline__ void first_pass_fine(const Geo &g, const ResArgs &a, unsigned q, int x, int y, int z,
                                                T r, T rc, const T *rW)
{
    const bool first = ((x + y + z) & 1) == 0;
    if (a.d1) {
        T diag;
        if constexpr (BC == kBcPeriodic)
            diag = pinned((T)(-90.0 * g.inv12h2)) + rc;
        else
            diag = pinned((T)(lap_diag_sum<BC>(g, x, y, z) * g.inv12h2)) + rc;
        elt((T *)a.d1, q) = first ? T(0) + (r - T(0)) / diag : T(0);
    }
    if (a.d1W) {
        const unsigned m = (unsigned)g.n * g.n * g.n;
#pragma unroll
        for (int s2 = 0; s2 < 3; s2++) elt((T *)a.d1W + (size_t)s2 * m, q) = first ? rW[s2] * (T)a.idiagW : T(0);
    }
}

template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_residual(Geo g, ResArgs a)
{
    a = res_shift(a, g.zs);
    if (a.K2p) a.K2 = *a.K2p;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    int i, j, k;
    double hv = 0.0, m2 = 0.0;
    if (cell_of(tid, n, i, j, k)) {
        const int64_t q = tid;
        const double psi = (a.psi0f ? a.psi0f[q] : psi0_at(g, a.pmass, i, j, k)) + a.u[q];
        Acc<BC, double> U{a.u, g};
        double A2 = a.A2bg ? a.A2bg[q] : 0.0;
        double Mv[3] = {0.0, 0.0, 0.0};
        if (a.W) {
            Acc<BC, double> W0{a.W, g}, W1{a.W + m, g}, W2{a.W + 2 * m, g};
            // dW[a][b] = D_a W_b
            double dW[3][3];
            dW[0][0] = d1_sum<0, double>(W0, i, j, k) * g.inv12h;
            dW[1][0] = d1_sum<1, double>(W0, i, j, k) * g.inv12h;
            dW[2][0] = d1_sum<2, double>(W0, i, j, k) * g.inv12h;
            dW[0][1] = d1_sum<0, double>(W1, i, j, k) * g.inv12h;
            dW[1][1] = d1_sum<1, double>(W1, i, j, k) * g.inv12h;
            dW[2][1] = d1_sum<2, double>(W1, i, j, k) * g.inv12h;
            dW[0][2] = d1_sum<0, double>(W2, i, j, k) * g.inv12h;
            dW[1][2] = d1_sum<1, double>(W2, i, j, k) * g.inv12h;
            dW[2][2] = d1_sum<2, double>(W2, i, j, k) * g.inv12h;
            const double div = dW[0][0] + dW[1][1] + dW[2][2];
#pragma unroll
            for (int p = 0; p < 3; p++)
#pragma unroll
                for (int s = 0; s < 3; s++) {
                    double Ab = dW[p][s] + dW[s][p] - (p == s ? 2.0 * div / 3.0 : 0.0);
                    A2 += Ab * Ab;
                }
            if (a.want_M) {
                const double w0 = a.W[q], w1 = a.W[m + q], w2 = a.W[2 * m + q];
                const double xx0 = d2_sum<0, double>(W0, i, j, k, w0);
                const double xx1 = d2_sum<1, double>(W1, i, j, k, w1);
                const double xx2 = d2_sum<2, double>(W2, i, j, k, w2);
                const double l0 = (xx0 + d2_sum<1, double>(W0, i, j, k, w0) +
                                   d2_sum<2, double>(W0, i, j, k, w0)) * g.inv12h2;
                const double l1 = (d2_sum<0, double>(W1, i, j, k, w1) + xx1 +
                                   d2_sum<2, double>(W1, i, j, k, w1)) * g.inv12h2;
                const double l2 = (d2_sum<0, double>(W2, i, j, k, w2) +
                                   d2_sum<1, double>(W2, i, j, k, w2) + xx2) * g.inv12h2;
                const double t0 = xx0 * g.inv12h2 + (dmix_sum<0, 1, double>(W1, i, j, k) +
                                                     dmix_sum<0, 2, double>(W2, i, j, k)) * g.inv144h2;
                const double t1 = xx1 * g.inv12h2 + (dmix_sum<1, 0, double>(W0, i, j, k) +
                                                     dmix_sum<1, 2, double>(W2, i, j, k)) * g.inv144h2;
                const double t2 = xx2 * g.inv12h2 + (dmix_sum<2, 0, double>(W0, i, j, k) +
                                                     dmix_sum<2, 1, double>(W1, i, j, k)) * g.inv144h2;
                Mv[0] = l0 + t0 / 3.0;
                Mv[1] = l1 + t1 / 3.0;
                Mv[2] = l2 + t2 / 3.0;
            }
        }
        if (a.want_M && a.S) {
            const double psi2 = psi * psi;
            const double w6 = a.conformal ? 1.0 : psi2 * psi2 * psi2;
#pragma unroll
            for (int s = 0; s < 3; s++) Mv[s] -= 8.0 * kPi * w6 * a.S[s * m + q] - a.meanS[s];
        }
        const double psi2 = psi * psi, psi4 = psi2 * psi2, psi5 = psi4 * psi;
        const double ipsi = 1.0 / psi, ipsi4 = 1.0 / psi4;
        const double ipsi7 = ipsi4 * ipsi * ipsi * ipsi, ipsi8 = ipsi7 * ipsi;
        const double r5 = a.rho5[q], r1 = a.rho1[q];
        double matter, dmatter;
        if (a.conformal) {
            const double rbar = r5 + r1;
            matter = 2.0 * kPi * rbar * (ipsi4 * psi);
            dmatter = -6.0 * kPi * rbar * ipsi4;
        } else {
            matter = 2.0 * kPi * r5 * psi5 + 2.0 * kPi * r1 * psi;
            dmatter = 10.0 * kPi * r5 * psi4 + 2.0 * kPi * r1;
        }
        double H = lap_sum<double>(U, i, j, k, a.u[q]) * g.inv12h2 + matter -
                   (a.K2 / 12.0) * psi5 + 0.125 * A2 * ipsi7;
        if (a.f) H += a.f[q];
        const double c = dmatter - (5.0 * a.K2 / 12.0) * psi4 - 0.875 * A2 * ipsi8;
        const T rT = pinned((T)(-H)), rcT = pinned((T)c);
        const T rW[3] = {pinned((T)(-Mv[0])), pinned((T)(-Mv[1])), pinned((T)(-Mv[2]))};
        if (a.H) a.H[q] = H;
        if (a.c) a.c[q] = c;
        if (a.r) ((T *)a.r)[q] = rT;
        if (a.rc) ((T *)a.rc)[q] = rcT;
        if (a.want_M) {
            if (a.M) {
                a.M[q] = Mv[0];
                a.M[m + q] = Mv[1];
                a.M[2 * m + q] = Mv[2];
            }
            if (a.rW) {
                ((T *)a.rW)[q] = rW[0];
                ((T *)a.rW)[m + q] = rW[1];
                ((T *)a.rW)[2 * m + q] = rW[2];
            }
            m2 = Mv[0] * Mv[0] + Mv[1] * Mv[1] + Mv[2] * Mv[2];
        }
        if (a.d1 || a.d1W) first_pass_fine<BC, T>(g, a, (unsigned)q, i, j, k, rT, rcT, rW);
        hv = H;
    }
    if (a.partials) {
        double v[4] = {hv * hv, fabs(hv), m2, sqrt(m2)};
        block_reduce_store<4>(v, 0xAu, a.partials + 4 * (int64_t)blockIdx.x);
    }
}

// Cells per thread of the whole-grid sums below (fewer, fuller partial sums
// for the single-block final reduction).
constexpr int kSumCells = 8;
inline unsigned sum_blocks(int64_t m) { return (unsigned)((m + kBlock * kSumCells - 1) / (kBlock * kSumCells)); }

// Per-block partial sums of 8 pi psi^6 S_a (for the periodic mean removal).
template <int BC>
__global__ void __launch_bounds__(kBlock) k_source_sum(Geo g, const double *u, const double *S,
                                                       double pmass, int conformal,
                                                       double *partials)
{
    u = zsh(u, g.zs);
    S = zsh(S, g.zs);
    partials = zsh(partials, g.zs);
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < kSumCells; c++) {
        const int64_t tid = ((int64_t)blockIdx.x * kSumCells + c) * kBlock + threadIdx.x;
        int i, j, k;
        if (cell_of(tid, n, i, j, k)) {
            const double psi = psi0_at(g, pmass, i, j, k) + u[tid];
            const double p2 = psi * psi, p6 = conformal ? 1.0 : p2 * p2 * p2;
#pragma unroll
            for (int s = 0; s < 3; s++) v[s] += 8.0 * kPi * p6 * S[s * m + tid];
        }
    }
    block_reduce_store<3>(v, 0u, partials + 3 * (int64_t)blockIdx.x);
}

// Per-block partial sums of the three components of a vector field.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sum3(const T *a, int64_t m, double *partials, long long zs)
{
    a = zsh(a, zs);
    partials = zsh(partials, zs);
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < kSumCells; c++) {
        const int64_t q = ((int64_t)blockIdx.x * kSumCells + c) * kBlock + threadIdx.x;
        if (q < m) {
            v[0] += (double)a[q];
            v[1] += (double)a[m + q];
            v[2] += (double)a[2 * m + q];
        }
    }
    block_reduce_store<3>(v, 0u, partials + 3 * (int64_t)blockIdx.x);
}

// Single-block final reduction: out[v] = combine over blocks of partials[b*NV+v];
// scale (if non-zero) multiplies the sums.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_reduce_final(const double *partials, int64_t nblocks,
                                                         unsigned max_mask, double scale,
                                                         double *out, long long zs)
{
    static_assert(NV >= 1 && NV <= 32, "max_mask holds one bit per value");
    partials = zsh(partials, zs);
    out = zsh(out, zs);
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = 0.0;
#pragma unroll 4
    for (int64_t b = threadIdx.x; b < nblocks; b += kBlock)
#pragma unroll
        for (int q = 0; q < NV; q++) {
            double x = partials[b * NV + q];
            v[q] = ((max_mask >> q) & 1u) ? fmax(v[q], x) : v[q] + x;
        }
    __shared__ double res[NV];
    double tmp[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) tmp[q] = v[q];
    block_reduce_store<NV>(tmp, max_mask, res);
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; q++)
            out[q] = ((max_mask >> q) & 1u) || scale == 0.0 ? res[q] : res[q] * scale;
}

// ---------------------------------------------------------------------------------------
// Smoothers: one colour pass of double-buffered red-black Gauss-Seidel.  Cells
// of the active colour ((i+j+k) mod 2) get d + (r - A d)/diag(A); the others
// are copied.  Every read is from `in` (the state before the pass).
// ---------------------------------------------------------------------------------------
// One colour pass of the psi smoother at cell q = (i, j, k) (double-buffered:
// reads in, writes out; the other colour is copied).
template <int BC, typename T>
__device__ __forceinline__ void psi_pass_cell(const Geo &g, const T *__restrict__ in, T *__restrict__ out,
                                              const T *__restrict__ r, const T *__restrict__ c, int colour,
                                              int64_t q, int i, int j, int k)
{
    const T x = in[q];
    if (((i + j + k) & 1) != colour) {
        out[q] = x;
        return;
    }
    Acc<BC, T> D{in, g};
    const T cv = c[q];
    const T h2 = (T)g.inv12h2;
    const T Ad = lap_sum<T>(D, i, j, k, x) * h2 + cv * x;
    const T diag = pinned((T)(lap_diag_sum<BC>(g, i, j, k) * g.inv12h2)) + cv;
    out[q] = x + (r[q] - Ad) / diag;
}

template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_pass_psi(Geo g, const T *__restrict__ in,
                                                     T *__restrict__ out, const T *__restrict__ r,
                                                     const T *__restrict__ c, int colour)
{
    in = zsh(in, g.zs);
    out = zsh(out, g.zs);
    r = zsh(r, g.zs);
    c = zsh(c, g.zs);
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int i, j, k;
    if (!cell_of(tid, g.n, i, j, k)) return;
    psi_pass_cell<BC, T>(g, in, out, r, c, colour, tid, i, j, k);
}

// (Delta_L d)_a at a cell for the three components (periodic), from taps at
// wrapped offsets computed once per cell.
template <typename T>
__device__ __forceinline__ void deltaL_at(const Geo &g, const T *d, unsigned m, const WrapOff &o, T out[3])
{
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2, third = T(1) / T(3);
    WPart<T> P;
    W_field_parts<T, 0, 0>(WrapTaps<T>{d, o}, h2, P);
    W_field_parts<T, 1, 0>(WrapTaps<T>{d + m, o}, h2, P);
    W_field_parts<T, 2, 0>(WrapTaps<T>{d + 2 * (size_t)m, o}, h2, P);
#pragma unroll
    for (int f = 0; f < 3; f++) out[f] = P.lap[f] + (P.dd[f] + P.mix[f] * m2) * third;
}

template <typename T>
__device__ __forceinline__ void deltaL_apply(const Geo &g, const T *d, int64_t m, int i, int j,
                                             int k, int64_t q, T out[3])
{
    (void)q;
    deltaL_at<T>(g, d, (unsigned)m, WrapOff(g.n, i, j, k), out);
}

// One colour pass of the W smoother at cell q (periodic, double-buffered).
template <typename T>
__device__ __forceinline__ void W_pass_cell(const Geo &g, const T *__restrict__ in, T *__restrict__ out,
                                            const T *__restrict__ r, int colour, int64_t q,
                                            int i, int j, int k)
{
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    if (((i + j + k) & 1) != colour) {
        out[q] = in[q];
        out[m + q] = in[m + q];
        out[2 * m + q] = in[2 * m + q];
        return;
    }
    T Ad[3];
    deltaL_apply<T>(g, in, m, i, j, k, q, Ad);
    // diagonal of Delta_L,h: (-90 - 30/3) / (12 h^2) = -25 / (3 h^2)
    const T diag = (T)(-100.0 * g.inv12h2);
#pragma unroll
    for (int s = 0; s < 3; s++) out[s * m + q] = in[s * m + q] + (r[s * m + q] - Ad[s]) / diag;
}

// Colour passes on levels without bricks (periodic): thread p owns the z pair
// (2 kp, 2 kp + 1) of row (i, j), updates the member of the active colour and
// copies the other (no idle lanes on the checkerboard).
__device__ __forceinline__ bool pair_of(unsigned p, int n, int colour, int &i, int &j, int &ka, int &kb)
{
    const unsigned np = (unsigned)n >> 1;
    if (p >= (unsigned)n * (unsigned)n * np) return false;
    const unsigned kp = p % np, rest = p / np;
    j = (int)(rest % (unsigned)n);
    i = (int)(rest / (unsigned)n);
    const int par = (colour + i + j) & 1;
    ka = 2 * (int)kp + par;
    kb = 2 * (int)kp + (par ^ 1);
    return true;
}

// W colour pass with four lanes per z pair: lane f < 3 evaluates the taps of
// component f (its Laplacian and second derivative, and its two mixed
// derivatives, which belong to the other two rows of Delta_L), so each lane
// issues 45 loads instead of 135 and all loads of a lane are in flight at once.
// The planes of the mixed derivatives are chosen per lane through offset
// tables, so the lanes run one instruction stream; the cross terms reach
// their rows through a butterfly over the four lanes (lane 3 contributes
// zeros), which adds them in the order of the single-lane evaluation.
// Row f of (Delta_L d) at cell (i, j, k) evaluated by the four lanes of a quad
// (lane f = t & 3 < 3 holds row f on return; lane 3 takes part in the
// exchange only).  *c receives component f of d at the cell.
template <typename T>
__device__ __forceinline__ T quad_deltaL_row(const Geo &g, const T *__restrict__ d, unsigned m, int f,
                                             const WrapOff &o, T *c)
{
    const int fc = f < 3 ? f : 2;
    const T *a = d + (size_t)fc * m;
    // plane 1 of the mixed derivatives: xy (f = 0, 1) or xz (f = 2); plane 2: xz (f = 0) or yz (f = 1, 2)
    unsigned b1[5], a2[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        b1[q] = fc == 2 ? o.y[2] + o.z[q] : o.y[q] + o.z[2];
        a2[q] = fc == 0 ? o.x[q] + o.y[2] : o.x[2] + o.y[q];
    }
    auto tap = [&](unsigned off) { return elt(a, off); };
    const T cv = tap(o.x[2] + o.y[2] + o.z[2]);
    auto d2 = [&](T m2v, T p2v, T m1v, T p1v) { return T(16) * (m1v + p1v) - (m2v + p2v) - T(30) * cv; };
    const T xx = d2(tap(o.x[0] + o.y[2] + o.z[2]), tap(o.x[4] + o.y[2] + o.z[2]), tap(o.x[1] + o.y[2] + o.z[2]),
                    tap(o.x[3] + o.y[2] + o.z[2]));
    const T yy = d2(tap(o.x[2] + o.y[0] + o.z[2]), tap(o.x[2] + o.y[4] + o.z[2]), tap(o.x[2] + o.y[1] + o.z[2]),
                    tap(o.x[2] + o.y[3] + o.z[2]));
    const T zz = d2(tap(o.x[2] + o.y[2] + o.z[0]), tap(o.x[2] + o.y[2] + o.z[4]), tap(o.x[2] + o.y[2] + o.z[1]),
                    tap(o.x[2] + o.y[2] + o.z[3]));
    // D_A D_B: first-derivative weights along B inside, along A outside
    auto dB1 = [&](int da) {
        const unsigned xa = o.x[da];
        return (tap(xa + b1[0]) - tap(xa + b1[4])) + T(8) * (tap(xa + b1[3]) - tap(xa + b1[1]));
    };
    auto dB2 = [&](int da) {
        const unsigned aa = a2[da];
        return (tap(aa + o.z[0]) - tap(aa + o.z[4])) + T(8) * (tap(aa + o.z[3]) - tap(aa + o.z[1]));
    };
    const T mixA = (dB1(0) - dB1(4)) + T(8) * (dB1(3) - dB1(1));
    const T mixB = (dB2(0) - dB2(4)) + T(8) * (dB2(3) - dB2(1));
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2, third = T(1) / T(3);
    const T lap = (xx + yy + zz) * h2;
    const T dd = (fc == 0 ? xx : fc == 1 ? yy : zz) * h2;
    // cross terms by target row: field 0 -> rows 1 (xy), 2 (xz); field 1 -> rows 0 (xy), 2 (yz);
    // field 2 -> rows 0 (xz), 1 (yz)
    T mt[3];
    mt[0] = f == 1 || f == 2 ? mixA : T(0);
    mt[1] = f == 0 ? mixA : (f == 2 ? mixB : T(0));
    mt[2] = f == 0 ? mixB : (f == 1 ? mixB : T(0));
#pragma unroll
    for (int q = 0; q < 3; q++) {
        mt[q] += __shfl_xor(mt[q], 1, kWave);
        mt[q] += __shfl_xor(mt[q], 2, kWave);
    }
    const T mix = f == 0 ? mt[0] : (f == 1 ? mt[1] : mt[2]);
    *c = cv;
    return lap + (dd + mix * m2) * third;
}

// W colour pass with four lanes per z pair (levels of at most 32^3 cells, where
// a pass is bound by rounds of memory latency): lane f < 3 evaluates the taps
// of component f (its Laplacian and second derivative, and its two mixed
// derivatives, which belong to the other two rows of Delta_L), so each lane
// issues 45 loads instead of 135 and all of them are in flight at once.  The
// planes of the mixed derivatives are chosen per lane through offset tables,
// so the lanes run one instruction stream; the cross terms reach their rows
// through a butterfly over the four lanes (lane 3 contributes zeros), which
// adds them in the order of the single-lane evaluation.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pass_W_quad(Geo g, const T *__restrict__ in, T *__restrict__ out,
                                                        const T *__restrict__ r, int colour)
{
    in = zsh(in, g.zs);
    out = zsh(out, g.zs);
    r = zsh(r, g.zs);
    const int n = g.n;
    const unsigned t = blockIdx.x * kBlock + threadIdx.x;
    const int f = (int)(t & 3u);
    int i, j, ka, kb;
    const bool live = pair_of(t >> 2, n, colour, i, j, ka, kb);
    if (!live) { // whole quads are live or not; dead ones read cell 0 and store nothing
        i = j = ka = 0;
        kb = 1;
    }
    const unsigned m = (unsigned)n * n * n, row = ((unsigned)i * n + (unsigned)j) * (unsigned)n;
    const unsigned qa = row + (unsigned)ka, qb = row + (unsigned)kb;
    T c;
    const T Ad = quad_deltaL_row<T>(g, in, m, f, WrapOff(n, i, j, ka), &c);
    if (!live || f == 3) return;
    const T *inf = in + (size_t)f * m, *rf = r + (size_t)f * m;
    T *of = out + (size_t)f * m;
    elt(of, qb) = elt(inf, qb);
    elt(of, qa) = c + (elt(rf, qa) - Ad) * (T)(1.0 / (-100.0 * g.inv12h2));
}

// W defect r - Delta_L d restricted to the next coarser level, four lanes per
// fine cell and the 8 children of a coarse cell in 32 adjacent lanes: lane
// 4 child + f; the child sum runs over lanes of the same f.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_defect_restrict_W_quad(Geo g, const T *__restrict__ d,
                                                                   const T *__restrict__ r, T *__restrict__ rc_out,
                                                                   T *__restrict__ d1_out, T idiag_c)
{
    d = zsh(d, g.zs);
    r = zsh(r, g.zs);
    rc_out = zsh(rc_out, g.zs);
    d1_out = zsh(d1_out, g.zs);
    const int n = g.n, nc = n / 2;
    const unsigned t = blockIdx.x * kBlock + threadIdx.x;
    const int f = (int)(t & 3u), ch = (int)((t >> 2) & 7u);
    const unsigned qc = t >> 5, mc = (unsigned)nc * nc * nc, m = (unsigned)n * n * n;
    const bool live = qc < mc;
    const unsigned qq = live ? qc : 0u;
    const int K = (int)(qq % (unsigned)nc), J = (int)((qq / (unsigned)nc) % (unsigned)nc),
              I = (int)(qq / ((unsigned)nc * nc));
    const int i = 2 * I + (ch >> 2), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch & 1);
    T c;
    const T Ad = quad_deltaL_row<T>(g, d, m, f, WrapOff(n, i, j, k), &c);
    const unsigned q = ((unsigned)i * n + (unsigned)j) * (unsigned)n + (unsigned)k;
    const int fc = f < 3 ? f : 2;
    T v = elt(r + (size_t)fc * m, q) - Ad;
    v += __shfl_xor(v, 4, kWave);
    v += __shfl_xor(v, 8, kWave);
    v += __shfl_xor(v, 16, kWave);
    if (live && ch == 0 && f < 3) {
        const T rcv = v * T(0.125);
        elt(rc_out + (size_t)f * mc, qc) = rcv;
        if (d1_out) elt(d1_out + (size_t)f * mc, qc) = ((I + J + K) & 1) == 0 ? rcv * idiag_c : T(0);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_pass_psi_pairs(Geo g, const T *__restrict__ in, T *__restrict__ out,
                                                           const T *__restrict__ r, const T *__restrict__ c,
                                                           int colour)
{
    in = zsh(in, g.zs);
    out = zsh(out, g.zs);
    r = zsh(r, g.zs);
    c = zsh(c, g.zs);
    const int n = g.n;
    int i, j, ka, kb;
    if (!pair_of(blockIdx.x * kBlock + threadIdx.x, n, colour, i, j, ka, kb)) return;
    const unsigned row = ((unsigned)i * n + (unsigned)j) * (unsigned)n;
    const unsigned qa = row + (unsigned)ka, qb = row + (unsigned)kb;
    const WrapOff o(n, i, j, ka);
    RegTaps<T, false> D;
    D.get_lap(WrapTaps<T>{in, o});
    const T v = D.c(), cv = elt(c, qa);
    const T Ad = (D.dxx(v) + D.dyy(v) + D.dzz(v)) * (T)g.inv12h2 + cv * v;
    const T diag = pinned((T)(-90.0 * g.inv12h2)) + cv;
    elt(out, qb) = elt(in, qb);
    elt(out, qa) = v + (elt(r, qa) - Ad) / diag;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_pass_W(Geo g, const T *__restrict__ in,
                                                   T *__restrict__ out, const T *__restrict__ r,
                                                   int colour)
{
    in = zsh(in, g.zs);
    out = zsh(out, g.zs);
    r = zsh(r, g.zs);
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int i, j, k;
    if (!cell_of(tid, g.n, i, j, k)) return;
    W_pass_cell<T>(g, in, out, r, colour, tid, i, j, k);
}

// ---------------------------------------------------------------------------------------
// Defect + restriction: coarse(I) = average over the 8 children of r - A d;
// optionally the coefficient c is restricted the same way.
// ---------------------------------------------------------------------------------------
// Sum of a value over the 8 lanes of an aligned lane group (the 8 children of
// one coarse cell), in a fixed butterfly order; every lane of the group gets it.
template <typename T>
__device__ __forceinline__ T child_sum(T v)
{
    v += __shfl_xor(v, 1, kWave);
    v += __shfl_xor(v, 2, kWave);
    v += __shfl_xor(v, 4, kWave);
    return v;
}

// One thread per fine cell: thread 8 qc + (4 di + 2 dj + dk) owns child
// (di, dj, dk) of coarse cell qc, so the 8 children are adjacent lanes.
__device__ __forceinline__ bool child_of(int64_t tid, int nc, int64_t &qc, int &i, int &j, int &k)
{
    qc = tid >> 3;
    int I, J, K;
    if (!cell_of(qc, nc, I, J, K)) return false;
    const int ch = (int)(tid & 7);
    i = 2 * I + (ch >> 2);
    j = 2 * J + ((ch >> 1) & 1);
    k = 2 * K + (ch & 1);
    return true;
}

// Defect r - A d restricted to the coarse grid (8-child average), and the
// coefficient c restricted the same way (cc_out may be null).  Two forms:
// one thread per coarse cell (the 8 children's overlapping stencils share
// loads in registers: large grids), or one thread per fine cell with a lane
// group per coarse cell (8x the parallelism: small, latency-bound grids).
// First colour pass of the coarse level from a zero correction at coarse cell
// (I, J, K): r / diag on colour 0 and 0 on colour 1, with the diagonal as the
// pass kernels form it.
template <int BC, typename T>
__device__ __forceinline__ T first_pass_psi(const Geo &gc, int I, int J, int K, T rcv, T ccv)
{
    if (((I + J + K) & 1) != 0) return T(0);
    T diag;
    if constexpr (BC == kBcPeriodic)
        diag = pinned((T)(-90.0 * gc.inv12h2)) + ccv;
    else
        diag = pinned((T)(lap_diag_sum<BC>(gc, I, J, K) * gc.inv12h2)) + ccv;
    return T(0) + (rcv - T(0)) / diag;
}

template <int BC, typename T>
__device__ __forceinline__ void defect_restrict_psi_coarse(const Geo &g, const T *__restrict__ d, const T *__restrict__ r,
                                                           const T *__restrict__ c, T *__restrict__ rc_out,
                                                           T *__restrict__ cc_out, int64_t qc, int I, int J, int K,
                                                           T *__restrict__ d1_out = nullptr, const Geo *gc = nullptr)
{
    Acc<BC, T> D{d, g};
    const T h2 = (T)g.inv12h2;
    T sd = T(0), sc = T(0);
#pragma unroll
    for (int di = 0; di < 2; di++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int dk = 0; dk < 2; dk++) {
                const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                const int64_t q = lidx(g.n, i, j, k);
                const T x = d[q], cv = c[q];
                sd += r[q] - (lap_sum<T>(D, i, j, k, x) * h2 + cv * x);
                sc += cv;
            }
    const T rcv = sd * T(0.125), ccv = sc * T(0.125);
    rc_out[qc] = rcv;
    if (cc_out) cc_out[qc] = ccv;
    if (d1_out) d1_out[qc] = first_pass_psi<BC, T>(*gc, I, J, K, rcv, ccv);
}

// d1_out (may be null; needs cc_out): the coarse level's first colour pass
// from zero, so that its smoothing starts with the second pass.
template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_defect_restrict_psi(Geo g, const T *__restrict__ d,
                                                                const T *__restrict__ r,
                                                                const T *__restrict__ c,
                                                                T *__restrict__ rc_out,
                                                                T *__restrict__ cc_out, T *__restrict__ d1_out,
                                                                Geo gc)
{
    d = zsh(d, g.zs);
    r = zsh(r, g.zs);
    c = zsh(c, g.zs);
    rc_out = zsh(rc_out, g.zs);
    cc_out = zsh(cc_out, g.zs);
    d1_out = zsh(d1_out, g.zs);
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int I, J, K;
    if (!cell_of(tid, g.n / 2, I, J, K)) return;
    defect_restrict_psi_coarse<BC, T>(g, d, r, c, rc_out, cc_out, tid, I, J, K, d1_out, &gc);
}

// Fine-cell form: fine cell tid of the grid of 8 nc^3 threads (child_of), group
// sums in a fixed order; lane 8 qc writes coarse cell qc.
template <int BC, typename T>
__device__ __forceinline__ void defect_restrict_psi_child(const Geo &g, const T *__restrict__ d, const T *__restrict__ r,
                                                          const T *__restrict__ c, T *__restrict__ rc_out,
                                                          T *__restrict__ cc_out, int64_t tid,
                                                          T *__restrict__ d1_out = nullptr, const Geo *gc = nullptr)
{
    int64_t qc;
    int i, j, k;
    const bool live = child_of(tid, g.n / 2, qc, i, j, k);
    T sd = T(0), cv = T(0);
    if (live) {
        Acc<BC, T> D{d, g};
        const T h2 = (T)g.inv12h2;
        const int64_t q = lidx(g.n, i, j, k);
        const T x = d[q];
        cv = c[q];
        sd = r[q] - (lap_sum<T>(D, i, j, k, x) * h2 + cv * x);
    }
    sd = child_sum(sd);
    const T sc = child_sum(cv);
    if (live && (tid & 7) == 0) {
        const T rcv = sd * T(0.125), ccv = sc * T(0.125);
        rc_out[qc] = rcv;
        if (cc_out) cc_out[qc] = ccv;
        if (d1_out) d1_out[qc] = first_pass_psi<BC, T>(*gc, i >> 1, j >> 1, k >> 1, rcv, ccv);
    }
}

template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_defect_restrict_psi_fine(Geo g, const T *__restrict__ d,
                                                                     const T *__restrict__ r,
                                                                     const T *__restrict__ c,
                                                                     T *__restrict__ rc_out,
                                                                     T *__restrict__ cc_out, T *__restrict__ d1_out,
                                                                     Geo gc)
{
    d = zsh(d, g.zs);
    r = zsh(r, g.zs);
    c = zsh(c, g.zs);
    rc_out = zsh(rc_out, g.zs);
    cc_out = zsh(cc_out, g.zs);
    d1_out = zsh(d1_out, g.zs);
    defect_restrict_psi_child<BC, T>(g, d, r, c, rc_out, cc_out, (int64_t)blockIdx.x * kBlock + threadIdx.x, d1_out,
                                     &gc);
}

template <typename T>
__device__ __forceinline__ void defect_restrict_W_coarse(const Geo &g, const T *__restrict__ d, const T *__restrict__ r,
                                                         T *__restrict__ rc_out,
                                                         int64_t qc, int I, int J, int K)
{
    const int nc = g.n / 2;
    const int64_t mf = (int64_t)g.n * g.n * g.n, mc = (int64_t)nc * nc * nc;
    T s[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int di = 0; di < 2; di++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int dk = 0; dk < 2; dk++) {
                const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                const int64_t q = lidx(g.n, i, j, k);
                T Ad[3];
                deltaL_apply<T>(g, d, mf, i, j, k, q, Ad);
#pragma unroll
                for (int a = 0; a < 3; a++) s[a] += r[a * mf + q] - Ad[a];
            }
#pragma unroll
    for (int a = 0; a < 3; a++) rc_out[a * mc + qc] = s[a] * T(0.125);
}

// Grid kernel with the body written out (not through defect_restrict_W_coarse):
// at the 256-register limit the inlined form is scheduled with far fewer
// loads in flight (mean outstanding loads per wait 4 instead of 21; 1.45x the
// time at 128^3).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_defect_restrict_W(Geo g, const T *__restrict__ d,
                                                              const T *__restrict__ r,
                                                              T *__restrict__ rc_out, T *__restrict__ d1_out,
                                                              T idiag_c)
{
    d = zsh(d, g.zs);
    r = zsh(r, g.zs);
    rc_out = zsh(rc_out, g.zs);
    d1_out = zsh(d1_out, g.zs);
    const int nc = g.n / 2;
    const int64_t mf = (int64_t)g.n * g.n * g.n, mc = (int64_t)nc * nc * nc;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int I, J, K;
    if (!cell_of(tid, nc, I, J, K)) return;
    T s[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int di = 0; di < 2; di++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int dk = 0; dk < 2; dk++) {
                const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                const int64_t q = lidx(g.n, i, j, k);
                T Ad[3];
                deltaL_apply<T>(g, d, mf, i, j, k, q, Ad);
#pragma unroll
                for (int a = 0; a < 3; a++) s[a] += r[a * mf + q] - Ad[a];
            }
    const bool first = ((I + J + K) & 1) == 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const T v = s[a] * T(0.125);
        rc_out[a * mc + tid] = v;
        if (d1_out) d1_out[a * mc + tid] = first ? v * idiag_c : T(0);
    }
}

template <typename T>
__device__ __forceinline__ void defect_restrict_W_child(const Geo &g, const T *__restrict__ d, const T *__restrict__ r,
                                                        T *__restrict__ rc_out, int64_t tid)
{
    const int nc = g.n / 2;
    const int64_t mf = (int64_t)g.n * g.n * g.n, mc = (int64_t)nc * nc * nc;
    int64_t qc;
    int i, j, k;
    const bool live = child_of(tid, nc, qc, i, j, k);
    T s[3] = {T(0), T(0), T(0)};
    if (live) {
        const int64_t q = lidx(g.n, i, j, k);
        T Ad[3];
        deltaL_apply<T>(g, d, mf, i, j, k, q, Ad);
#pragma unroll
        for (int a = 0; a < 3; a++) s[a] = r[a * mf + q] - Ad[a];
    }
#pragma unroll
    for (int a = 0; a < 3; a++) s[a] = child_sum(s[a]);
    if (live && (tid & 7) == 0) {
#pragma unroll
        for (int a = 0; a < 3; a++) rc_out[a * mc + qc] = s[a] * T(0.125);
    }
}

// ---------------------------------------------------------------------------------------
// Trilinear cell-centred prolongation: fine += P coarse (weights 3/4, 1/4 per
// axis toward the nearer coarse neighbour), ncomp components.  gc: coarse grid.
// ---------------------------------------------------------------------------------------
template <int BC, typename T>
__device__ __forceinline__ void prolong_cell(const Geo &gc, const T *__restrict__ coarse, T *__restrict__ fine, int ncomp,
                                             int64_t q, int i,
                                             int j, int k)
{
    const int nf = 2 * gc.n;
    const int64_t mf = (int64_t)nf * nf * nf, mc = (int64_t)gc.n * gc.n * gc.n;
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int I1 = (i & 1) ? I + 1 : I - 1;
    const int J1 = (j & 1) ? J + 1 : J - 1;
    const int K1 = (k & 1) ? K + 1 : K - 1;
    const T a = T(0.75), b = T(0.25);
    for (int s = 0; s < ncomp; s++) {
        Acc<BC, T> C{coarse + s * mc, gc};
        const T v = a * (a * (a * C(I, J, K) + b * C(I, J, K1)) + b * (a * C(I, J1, K) + b * C(I, J1, K1))) +
                    b * (a * (a * C(I1, J, K) + b * C(I1, J, K1)) + b * (a * C(I1, J1, K) + b * C(I1, J1, K1)));
        fine[s * mf + q] += v;
    }
}

template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_add(Geo gc, const T *__restrict__ coarse,
                                                        T *__restrict__ fine, int ncomp)
{
    coarse = zsh(coarse, gc.zs);
    fine = zsh(fine, gc.zs);
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int i, j, k;
    if (!cell_of(tid, 2 * gc.n, i, j, k)) return;
    prolong_cell<BC, T>(gc, coarse, fine, ncomp, tid, i, j, k);
}

// Four-point cubic interpolation (FP64), fine = Q coarse.  One thread per coarse cell
// (I, J, K) writes its 8 fine children from the 5^3 coarse neighbourhood I-2 .. I+2:
// child parity p along an axis uses nodes p .. p+3 of that window with the weights
// (-5, 35, 105, -7)/128 (p = 0, offset -1/4) or their mirror (p = 1, offset +1/4).  The
// sums are separable and taken in the order of the plain triple sum over (x, y, z)
// nodes: z innermost, then y, then x.
template <int BC>
__global__ void __launch_bounds__(kBlock) k_interp_cubic(Geo gc, const double *__restrict__ coarse,
                                                         double *__restrict__ fine)
{
    const int nc = gc.n, nf = 2 * nc;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int I, J, K;
    if (!cell_of(tid, nc, I, J, K)) return;
    const double w[2][4] = {{-5.0 / 128.0, 35.0 / 128.0, 105.0 / 128.0, -7.0 / 128.0},
                            {-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0}};
    Acc<BC, double> C{coarse, gc};
    double yz[2][2][5]; // [z parity][y parity][x node]
#pragma unroll
    for (int a = 0; a < 5; a++) {
        double zc[2][5]; // [z parity][y node] at x node a
#pragma unroll
        for (int b = 0; b < 5; b++) {
            double v[5];
#pragma unroll
            for (int e = 0; e < 5; e++) v[e] = C(I - 2 + a, J - 2 + b, K - 2 + e);
#pragma unroll
            for (int pk = 0; pk < 2; pk++) {
                double sb = 0.0;
#pragma unroll
                for (int e = 0; e < 4; e++) sb += w[pk][e] * v[e + pk];
                zc[pk][b] = sb;
            }
        }
#pragma unroll
        for (int pk = 0; pk < 2; pk++)
#pragma unroll
            for (int pj = 0; pj < 2; pj++) {
                double sa = 0.0;
#pragma unroll
                for (int b = 0; b < 4; b++) sa += w[pj][b] * zc[pk][b + pj];
                yz[pk][pj][a] = sa;
            }
    }
#pragma unroll
    for (int pi = 0; pi < 2; pi++)
#pragma unroll
        for (int pj = 0; pj < 2; pj++) {
            double out[2];
#pragma unroll
            for (int pk = 0; pk < 2; pk++) {
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < 4; a++) s += w[pi][a] * yz[pk][pj][a + pi];
                out[pk] = s;
            }
            const int64_t q = ((int64_t)(2 * I + pi) * nf + (2 * J + pj)) * nf + 2 * K;
            *reinterpret_cast<double2 *>(fine + q) = make_double2(out[0], out[1]);
        }
}

// ---------------------------------------------------------------------------------------
// Cubic prolongation of corrections (MG_FLAG_CUBIC_PROLONG): fine += Q coarse with Q the
// 4-point cubic of the FMG start (tensor product of the weights (-5, 35, 105, -7)/128 and
// their mirror), ghosts by the level's rule.  A coarse cell writes its 8 children from its
// 5^3 neighbourhood with the separable sums of k_interp_cubic (z, then y, then x).
// ---------------------------------------------------------------------------------------
template <typename T, typename Src>
__device__ __forceinline__ void cubic_children_add(const Src &S, T *__restrict__ fine, int nf, int I, int J, int K)
{
    const T w[2][4] = {{T(-5.0 / 128.0), T(35.0 / 128.0), T(105.0 / 128.0), T(-7.0 / 128.0)},
                       {T(-7.0 / 128.0), T(105.0 / 128.0), T(35.0 / 128.0), T(-5.0 / 128.0)}};
    T yz[2][2][5]; // [z parity][y parity][x node]
#pragma unroll
    for (int a = 0; a < 5; a++) {
        T zc[2][5]; // [z parity][y node] at x node a
#pragma unroll
        for (int b = 0; b < 5; b++) {
            T v[5];
#pragma unroll
            for (int e = 0; e < 5; e++) v[e] = S(a, b, e);
#pragma unroll
            for (int pk = 0; pk < 2; pk++) {
                T sb = T(0);
#pragma unroll
                for (int e = 0; e < 4; e++) sb += w[pk][e] * v[e + pk];
                zc[pk][b] = sb;
            }
        }
#pragma unroll
        for (int pk = 0; pk < 2; pk++)
#pragma unroll
            for (int pj = 0; pj < 2; pj++) {
                T sa = T(0);
#pragma unroll
                for (int b = 0; b < 4; b++) sa += w[pj][b] * zc[pk][b + pj];
                yz[pk][pj][a] = sa;
            }
    }
    using V2 = std::conditional_t<sizeof(T) == 4, float2, double2>;
#pragma unroll
    for (int pi = 0; pi < 2; pi++)
#pragma unroll
        for (int pj = 0; pj < 2; pj++) {
            T out[2];
#pragma unroll
            for (int pk = 0; pk < 2; pk++) {
                T acc = T(0);
#pragma unroll
                for (int a = 0; a < 4; a++) acc += w[pi][a] * yz[pk][pj][a + pi];
                out[pk] = acc;
            }
            V2 *f = reinterpret_cast<V2 *>(fine + ((int64_t)(2 * I + pi) * nf + (2 * J + pj)) * nf + 2 * K);
            V2 v = *f;
            v.x += out[0];
            v.y += out[1];
            *f = v;
        }
}

// Any coarse size: one thread per coarse cell, neighbours through the boundary rule.
template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_cubic_add(Geo gc, const T *__restrict__ coarse,
                                                              T *__restrict__ fine, int ncomp)
{
    coarse = zsh(coarse, gc.zs);
    fine = zsh(fine, gc.zs);
    const int nc = gc.n, nf = 2 * nc;
    const int64_t mc = (int64_t)nc * nc * nc, mf = 8 * mc;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int I, J, K;
    if (!cell_of(tid, nc, I, J, K)) return;
    for (int s = 0; s < ncomp; s++) {
        const Acc<BC, T> C{coarse + s * mc, gc};
        cubic_children_add<T>([&](int a, int b, int e) { return C(I - 2 + a, J - 2 + b, K - 2 + e); }, fine + s * mf,
                              nf, I, J, K);
    }
}

// Coarse sizes divisible by 16: a block of 4 x 4 x 16 coarse cells stages their 8 x 8 x 20
// neighbourhood in LDS (each value loaded once) and reads the 5^3 taps from there.  A wave
// reads four z rows of 16 values at once; with rows kCubSZP = 48 values apart the rows
// served together land on disjoint banks (float: word offsets 0, 48, 96, 144 fill four
// distinct 16-bank quarters of 64 banks; double: consecutive rows 96 words apart fill the
// two halves), where the unpadded stride of 20 put 2-4 rows on the same banks.
constexpr int kCubX = 4, kCubY = 4, kCubZ = 16;
constexpr int kCubSX = kCubX + 4, kCubSY = kCubY + 4, kCubSZ = kCubZ + 4, kCubSZP = 48;
template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_cubic_add_staged(Geo gc, const T *__restrict__ coarse,
                                                                     T *__restrict__ fine, int ncomp)
{
    static_assert(kCubX * kCubY * kCubZ == kBlock, "one coarse cell per thread");
    coarse = zsh(coarse, gc.zs);
    fine = zsh(fine, gc.zs);
    __shared__ T S[kCubSX][kCubSY][kCubSZP];
    const int nc = gc.n, nf = 2 * nc;
    const int64_t mc = (int64_t)nc * nc * nc, mf = 8 * mc;
    const int nby = nc / kCubY, nbz = nc / kCubZ;
    const int bz = blockIdx.x % nbz, by = (blockIdx.x / nbz) % nby, bx = blockIdx.x / (nbz * nby);
    const int I0 = bx * kCubX, J0 = by * kCubY, K0 = bz * kCubZ;
    const int t = threadIdx.x, kz = t % kCubZ, jy = (t / kCubZ) % kCubY, ix = t / (kCubZ * kCubY);
    constexpr int kStaged = kCubSX * kCubSY * kCubSZ;
    for (int s = 0; s < ncomp; s++) {
        const Acc<BC, T> C{coarse + s * mc, gc};
        if (s > 0) __syncthreads(); // the previous component's taps are read
        for (int q = t; q < kStaged; q += kBlock) {
            const int a = q / (kCubSY * kCubSZ), rem = q % (kCubSY * kCubSZ), b = rem / kCubSZ, e = rem % kCubSZ;
            S[a][b][e] = C(I0 - 2 + a, J0 - 2 + b, K0 - 2 + e);
        }
        __syncthreads();
        cubic_children_add<T>([&](int a, int b, int e) { return S[ix + a][jy + b][kz + e]; }, fine + s * mf, nf,
                              I0 + ix, J0 + jy, K0 + kz);
    }
}

// ---------------------------------------------------------------------------------------
// Coarsest level: dense operator assembly, Gauss-Jordan inverse (partial
// pivoting, FP64, one workgroup), and x = A^-1 r as a column-major mat-vec.
// ---------------------------------------------------------------------------------------

// Row `row` of (L_h + c): A[row][col] accumulated over the 13 taps, boundary
// rule included.  A is zeroed by the caller.
template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_assemble_psi(Geo g, const T *c, double *A)
{
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int i, j, k;
    if (!cell_of(row, n, i, j, k)) return;
    const double w[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    for (int ax = 0; ax < 3; ax++)
        for (int d = -2; d <= 2; d++) {
            int bi, bj, bk;
            const double fac =
                ghost_source<BC>(g, i + (ax == 0 ? d : 0), j + (ax == 1 ? d : 0), k + (ax == 2 ? d : 0), bi, bj, bk);
            A[row * m + lidx(n, bi, bj, bk)] += w[d + 2] * g.inv12h2 * fac;
        }
    A[row * m + row] += (double)c[row];
}

// Rows of Delta_L,h on a periodic grid (3 n^3 unknowns) plus -(1/(n^3 h^2))
// on every same-component entry, which fixes each component's mean to zero.
__global__ void __launch_bounds__(kBlock) k_assemble_W(Geo g, double *A)
{
    const int n = g.n;
    const int64_t cn = (int64_t)n * n * n, m = 3 * cn;
    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row >= m) return;
    const int a = (int)(row / cn);
    int i, j, k;
    cell_of(row % cn, n, i, j, k);
    double *Ar = A + row * m;
    const double reg = 1.0 / ((double)cn * g.h * g.h);
    for (int64_t col = a * cn; col < (a + 1) * cn; col++) Ar[col] -= reg;
    const double w2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
    const double w1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
    for (int ax = 0; ax < 3; ax++) {
        const double s = (ax == a) ? 1.0 + 1.0 / 3.0 : 1.0;
        for (int d = -2; d <= 2; d++) {
            int ii = wrap(i + (ax == 0 ? d : 0), n), jj = wrap(j + (ax == 1 ? d : 0), n),
                kk = wrap(k + (ax == 2 ? d : 0), n);
            Ar[a * cn + lidx(n, ii, jj, kk)] += s * w2[d + 2] * g.inv12h2;
        }
    }
    for (int b = 0; b < 3; b++) {
        if (b == a) continue;
        for (int d = -2; d <= 2; d++)
            for (int e = -2; e <= 2; e++) {
                if (d == 0 || e == 0) continue;
                int o[3] = {0, 0, 0};
                o[a] += d;
                o[b] += e;
                int ii = wrap(i + o[0], n), jj = wrap(j + o[1], n), kk = wrap(k + o[2], n);
                Ar[b * cn + lidx(n, ii, jj, kk)] += w1[d + 2] * w1[e + 2] * g.inv144h2 / 3.0;
            }
    }
}

// Gauss-Jordan inversion with partial pivoting of the m x m row-major matrix
// A (destroyed); writes the inverse column-major into Ainv.  One workgroup of
// 1024 threads; aug is an m x 2m scratch.  *flag = 1 if a pivot is zero.
constexpr int kGjThreads = 1024;
__global__ void __launch_bounds__(kGjThreads) k_gauss_jordan(const double *A, double *aug,
                                                             double *Ainv, int m, double *flag)
{
    const int tid = threadIdx.x;
    const int64_t w = 2 * (int64_t)m;
    for (int64_t e = tid; e < (int64_t)m * w; e += kGjThreads) {
        const int64_t r = e / w, col = e % w;
        aug[e] = col < m ? A[r * m + col] : (col - m == r ? 1.0 : 0.0);
    }
    __shared__ double sv[kGjThreads / kWave];
    __shared__ int si[kGjThreads / kWave];
    __shared__ int piv_row;
    __shared__ int bad;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int kcol = 0; kcol < m; kcol++) {
        // pivot search over rows kcol..m-1 (lowest index wins ties)
        double best = -1.0;
        int bi = m;
        for (int r = kcol + tid; r < m; r += kGjThreads) {
            double v = fabs(aug[(int64_t)r * w + kcol]);
            if (v > best) {
                best = v;
                bi = r;
            }
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            double ov = __shfl_xor(best, o, kWave);
            int oi = __shfl_xor(bi, o, kWave);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if (tid % kWave == 0) {
            sv[tid / kWave] = best;
            si[tid / kWave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double b = sv[0];
            int idx = si[0];
            for (int q = 1; q < kGjThreads / kWave; q++)
                if (sv[q] > b || (sv[q] == b && si[q] < idx)) {
                    b = sv[q];
                    idx = si[q];
                }
            piv_row = idx;
            if (!(b > 0.0)) bad = 1;
        }
        __syncthreads();
        if (bad) break;
        const int pr = piv_row;
        if (pr != kcol)
            for (int64_t col = tid; col < w; col += kGjThreads) {
                double t = aug[(int64_t)kcol * w + col];
                aug[(int64_t)kcol * w + col] = aug[(int64_t)pr * w + col];
                aug[(int64_t)pr * w + col] = t;
            }
        __syncthreads();
        const double inv = 1.0 / aug[(int64_t)kcol * w + kcol];
        __syncthreads();
        for (int64_t col = tid; col < w; col += kGjThreads) aug[(int64_t)kcol * w + col] *= inv;
        __syncthreads();
        // eliminate column kcol from every other row
        for (int64_t e = tid; e < (int64_t)m * w; e += kGjThreads) {
            const int64_t r = e / w, col = e % w;
            if (r == kcol || col == kcol) continue;
            aug[e] -= aug[r * w + kcol] * aug[(int64_t)kcol * w + col];
        }
        __syncthreads();
        for (int64_t r = tid; r < m; r += kGjThreads)
            if (r != kcol) aug[r * w + kcol] = 0.0;
        __syncthreads();
    }
    if (tid == 0) *flag = bad ? 1.0 : 0.0;
    for (int64_t e = tid; e < (int64_t)m * m; e += kGjThreads) {
        const int64_t r = e / m, col = e % m;
        Ainv[col * m + r] = aug[r * w + m + col]; // column-major
    }
}

// x = Ainv (r - mean r per component when ncomp_project > 0), Ainv column-major.
// Each block covers 16 rows with 16 threads per row (interleaved columns).
constexpr int kApplySplit = 16;
constexpr int kApplyRows = kBlock / kApplySplit;

// sum over col = part, part + STRIDE, ... < m of Ainv[col * m + row] * rs[col], in
// that order; the loads of each chunk of columns are issued together, so that a
// thread waits for global memory once per chunk instead of once per column.
template <int STRIDE>
__device__ __forceinline__ double inv_row_dot(const double *Ainv, int m, int row, int part, const double *rs)
{
    constexpr int kChunk = 12;
    double s = 0.0;
    for (int c0 = part; c0 < m; c0 += kChunk * STRIDE) {
        double v[kChunk];
#pragma unroll
        for (int e = 0; e < kChunk; e++) {
            const int col = c0 + e * STRIDE;
            v[e] = col < m ? Ainv[(int64_t)col * m + row] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < kChunk; e++) {
            const int col = c0 + e * STRIDE;
            if (col < m) s += v[e] * rs[col];
        }
    }
    return s;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse_apply(const double *Ainv, int m,
                                                         const T *r, T *x, int ncomp_project, long long zs)
{
    Ainv = zsh(Ainv, zs);
    r = zsh(r, zs);
    x = zsh(x, zs);
    extern __shared__ double rs[];
    for (int q = threadIdx.x; q < m; q += kBlock) rs[q] = (double)r[q];
    __syncthreads();
    if (ncomp_project > 0) {
        __shared__ double mean[3];
        const int cn = m / ncomp_project;
        if (threadIdx.x < ncomp_project) {
            double s = 0.0;
            for (int q = 0; q < cn; q++) s += rs[threadIdx.x * cn + q];
            mean[threadIdx.x] = s / (double)cn;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += kBlock) rs[q] -= mean[q / cn];
        __syncthreads();
    }
    const int row = blockIdx.x * kApplyRows + threadIdx.x % kApplyRows;
    const int part = threadIdx.x / kApplyRows;
    const double s = row < m ? inv_row_dot<kApplySplit>(Ainv, m, row, part, rs) : 0.0;
    __shared__ double red[kApplySplit][kApplyRows];
    red[part][threadIdx.x % kApplyRows] = s;
    __syncthreads();
    if (threadIdx.x < kApplyRows && row < m) {
        double t = 0.0;
        for (int q = 0; q < kApplySplit; q++) t += red[q][threadIdx.x];
        x[row] = (T)t;
    }
}

// coarse = average of the 8 children of fine (coefficient restriction alone);
// same summation order as the fused defect-restriction kernels.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(int nf, const T *__restrict__ fine, T *__restrict__ coarse, long long zs)
{
    fine = zsh(fine, zs);
    coarse = zsh(coarse, zs);
    const int nc = nf / 2;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int I, J, K;
    if (!cell_of(tid, nc, I, J, K)) return;
    T s = T(0);
#pragma unroll
    for (int di = 0; di < 2; di++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int dk = 0; dk < 2; dk++) s += fine[lidx(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
    coarse[tid] = s * T(0.125);
}

// ---------------------------------------------------------------------------------------
// Coarsest psi solve (m = M unknowns, M <= 64, a compile-time constant that
// fixes the number of columns each wave holds in registers): Gauss-Jordan with
// partial pivoting on [A | r], A assembled from the level's stencil and c.
// Pivot: the largest |a_ik| over unused rows, found with one wave max of a
// packed key (float bits of |a_ik|, low 6 bits replaced by 63 - row so ties go
// to the lowest row).  *flag = 1 if no non-zero pivot exists (published as
// pivot row -1).
// The pivot rows are not scaled: step k subtracts (a_ik / a_pk) times row p
// from every other row, and the end divides the right-hand side of pivot row
// perm[q] by that row's pivot a_{perm[q], q} (recorded at its step), so each
// step is one FMA per matrix element.  Columns already eliminated keep
// receiving the update (their values are never read again), so no element
// needs a select.
// The solve is spread over a block of 16 waves: lanes hold rows, the columns
// of [A | r] are dealt round-robin to the waves (wave w holds columns w,
// w + 16, ...).  At step k the wave owning column k picks the pivot and
// publishes the pivot row index and the row factors in LDS (double-buffered:
// one barrier per step); every wave then updates its own columns, reading the
// pivot row's values from lane p of its own registers (v_readlane: p is
// uniform).  The step loop is not unrolled: the kernel runs once per launch,
// and an unrolled body of every step would not stay in the instruction cache.
// ---------------------------------------------------------------------------------------
constexpr int kGjWaves = 16;

// Maximum of an unsigned value over the 64 lanes of a wave, returned in a
// scalar register: DPP exchanges inside each row of 16 lanes (quad swaps, then
// the half-row and row mirrors), then the four row results read lane by lane.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false));  // quad_perm 2,3,0,1
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false)); // row_half_mirror
    v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false)); // row_mirror
    const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
    const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
    const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
    const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
    return max(max(r0, r1), max(r2, r3));
}

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------------------
// Krylov solves of the coarsest psi system (L_h + c) x = r in FP64.  Periodic grids
// give a symmetric matrix: conjugate gradients (Hestenes-Stiefel); Robin ghosts make
// it slightly non-symmetric: BiCGSTAB (van der Vorst).  Either is accepted only when
// the true residual |r - A x| is below 1e-12 |r| afterwards; the caller otherwise
// solves by elimination.
//
// The 12 off-centre taps of L_h at a cell, as (source cell, weight) pairs with the
// boundary rule folded in (ghost_source).  A tap may name the cell itself.
// ---------------------------------------------------------------------------------------
template <int BC>
__device__ __forceinline__ void coarse_taps(const Geo &g, int q, int src[12], double w[12])
{
    const int n = g.n;
    const int k = q % n, j = (q / n) % n, i = q / (n * n);
    const double wt[4] = {-1.0, 16.0, 16.0, -1.0}; // offsets -2, -1, +1, +2
    const int dof[4] = {-2, -1, 1, 2};
    int t = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ax++)
#pragma unroll
        for (int e = 0; e < 4; e++, t++) {
            int bi, bj, bk;
            const double fac = ghost_source<BC>(g, i + (ax == 0 ? dof[e] : 0), j + (ax == 1 ? dof[e] : 0),
                                                k + (ax == 2 ? dof[e] : 0), bi, bj, bk);
            src[t] = (bi * n + bj) * n + bk;
            w[t] = wt[e] * g.inv12h2 * fac;
        }
}

// One 64-bit DPP lane move (both halves with the same control).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed order, the same value in every lane:
// DPP exchanges inside rows of 16 lanes, then the four row sums read lane by lane.
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_f64<0xB1>(v);  // quad_perm 1,0,3,2
    v += dpp_f64<0x4E>(v);  // quad_perm 2,3,0,1
    v += dpp_f64<0x141>(v); // row_half_mirror
    v += dpp_f64<0x140>(v); // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// One wave, one cell per lane (M <= 64 cells); lanes >= M carry zeros.  Needs no
// barrier: the taps come from the owning lanes by cross-lane permutes.  Writes x and
// returns true when accepted.
template <int BC, typename T, int M>
__device__ __forceinline__ bool coarse_psi_krylov_wave(const Geo &g, const T *c, const T *r, T *x)
{
    static_assert(M <= kWave, "one cell per lane");
    const int lane = threadIdx.x & (kWave - 1);
    const bool own = lane < M;
    int src[12];
    double w[12];
    if (own) {
        coarse_taps<BC>(g, lane, src, w);
    } else {
#pragma unroll
        for (int t = 0; t < 12; t++) {
            src[t] = lane;
            w[t] = 0.0;
        }
    }
    const double cq = own ? (double)c[lane] : 0.0;
    const double dg = own ? -90.0 * g.inv12h2 + cq : 0.0;
    auto apply = [&](double v) {
        double y = dg * v;
#pragma unroll
        for (int t = 0; t < 12; t++) y += w[t] * __shfl(v, src[t], kWave);
        return y;
    };
    const double b = own ? (double)r[lane] : 0.0;
    const double bb = wave_sum_dpp(b * b);
    if (!(bb > 0.0)) {
        if (own) x[lane] = T(0);
        return bb == 0.0;
    }
    const double tol2 = 1e-28 * bb;
    double xv = 0.0;
    bool ok = false;
    if constexpr (BC == kBcPeriodic) {
        // conjugate gradients end within M steps in exact arithmetic; a system that needs
        // many more is ill-conditioned or indefinite, and elimination is then quicker
        double rr = b, p = b, rz = bb;
#pragma unroll 1
        for (int it = 0; it < M + 16; it++) {
            const double ap = apply(p);
            const double pap = wave_sum_dpp(p * ap);
            if (!(pap != 0.0)) break;
            const double alpha = rz / pap;
            xv += alpha * p;
            rr -= alpha * ap;
            const double rz1 = wave_sum_dpp(rr * rr);
            if (rz1 <= tol2) {
                ok = true;
                break;
            }
            p = rr + (rz1 / rz) * p;
            rz = rz1;
        }
    } else {
        double rr = b, rh = b, p = 0.0, v = 0.0, rho = 1.0, alpha = 1.0, omega = 1.0;
#pragma unroll 1
        for (int it = 0; it < 4 * M + 32; it++) {
            const double rho1 = wave_sum_dpp(rh * rr);
            if (!(rho1 != 0.0)) break;
            p = rr + (rho1 / rho) * (alpha / omega) * (p - omega * v);
            v = apply(p);
            const double rv = wave_sum_dpp(rh * v);
            if (!(rv != 0.0)) break;
            alpha = rho1 / rv;
            const double sv = rr - alpha * v;
            if (wave_sum_dpp(sv * sv) <= tol2) {
                xv += alpha * p;
                ok = true;
                break;
            }
            const double t = apply(sv);
            const double ts = wave_sum_dpp(t * sv), tt = wave_sum_dpp(t * t);
            if (!(tt > 0.0)) break;
            omega = ts / tt;
            xv += alpha * p + omega * sv;
            rr = sv - omega * t;
            rho = rho1;
            if (wave_sum_dpp(rr * rr) <= tol2) {
                ok = true;
                break;
            }
            if (!(omega != 0.0)) break;
        }
    }
    const double tr = b - apply(xv);
    const double trr = wave_sum_dpp(tr * tr);
    ok = ok && trr <= 1e-24 * bb;
    if (ok && own) x[lane] = (T)xv;
    return ok;
}

// The same for up to kGjWaves * kWave * CPT cells on a block of kGjWaves waves: every
// thread owns CPT cells (q = tid + kGjWaves * kWave * e), the vector being multiplied
// is staged in LDS, and inner products are block reductions.  Writes x and returns
// true (in every thread) when accepted; called by every thread of the block.
constexpr int kKrylovCpt = 2;
constexpr int kKrylovMax = kGjWaves * kWave * kKrylovCpt;

template <int NV>
__device__ __forceinline__ void block_sums(double v[NV], double (*part)[kGjWaves])
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = wave_sum_dpp(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; q++) part[q][wave] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kGjWaves; w++) s += part[q][w];
        v[q] = s;
    }
    __syncthreads();
}

template <int BC, typename T>
__device__ __forceinline__ bool coarse_psi_krylov_block(const Geo &g, int m, const T *c, const T *r, T *x)
{
    constexpr int E = kKrylovCpt;
    constexpr int NT = kGjWaves * kWave;
    __shared__ double vec[kKrylovMax];
    __shared__ double part[3][kGjWaves];
    int src[E][12];
    double w[E][12], dg[E], b[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const int q = threadIdx.x + NT * e;
        if (q < m) {
            coarse_taps<BC>(g, q, src[e], w[e]);
            dg[e] = -90.0 * g.inv12h2 + (double)c[q];
            b[e] = (double)r[q];
        } else {
#pragma unroll
            for (int t = 0; t < 12; t++) {
                src[e][t] = 0;
                w[e][t] = 0.0;
            }
            dg[e] = 0.0;
            b[e] = 0.0;
        }
    }
    // y = A v for the owned cells (v staged in LDS by every thread first)
    auto apply = [&](const double v[E], double y[E]) {
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int q = threadIdx.x + NT * e;
            if (q < m) vec[q] = v[e];
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; e++) {
            double s = dg[e] * v[e];
#pragma unroll
            for (int t = 0; t < 12; t++) s += w[e][t] * vec[src[e][t]];
            y[e] = s;
        }
        __syncthreads();
    };
    double t3[3];
    t3[0] = 0.0;
#pragma unroll
    for (int e = 0; e < E; e++) t3[0] += b[e] * b[e];
    block_sums<1>(t3, part);
    const double bb = t3[0];
    const int q0 = threadIdx.x;
    if (!(bb > 0.0)) {
#pragma unroll
        for (int e = 0; e < E; e++)
            if (q0 + NT * e < m) x[q0 + NT * e] = T(0);
        return bb == 0.0;
    }
    const double tol2 = 1e-28 * bb;
    double xv[E], rr[E], p[E], ap[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        xv[e] = 0.0;
        rr[e] = b[e];
    }
    bool ok = false;
    if constexpr (BC == kBcPeriodic) {
        double rz = bb;
#pragma unroll
        for (int e = 0; e < E; e++) p[e] = b[e];
#pragma unroll 1
        for (int it = 0; it < 2 * m + 32; it++) {
            apply(p, ap);
            t3[0] = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) t3[0] += p[e] * ap[e];
            block_sums<1>(t3, part);
            if (!(t3[0] != 0.0)) break;
            const double alpha = rz / t3[0];
            t3[0] = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) {
                xv[e] += alpha * p[e];
                rr[e] -= alpha * ap[e];
                t3[0] += rr[e] * rr[e];
            }
            block_sums<1>(t3, part);
            if (t3[0] <= tol2) {
                ok = true;
                break;
            }
            const double beta = t3[0] / rz;
            rz = t3[0];
#pragma unroll
            for (int e = 0; e < E; e++) p[e] = rr[e] + beta * p[e];
        }
    } else {
        double rh[E], v[E], sv[E], tv[E];
        double rho = 1.0, alpha = 1.0, omega = 1.0;
#pragma unroll
        for (int e = 0; e < E; e++) {
            rh[e] = b[e];
            p[e] = 0.0;
            v[e] = 0.0;
        }
#pragma unroll 1
        for (int it = 0; it < 2 * m + 32; it++) {
            t3[0] = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) t3[0] += rh[e] * rr[e];
            block_sums<1>(t3, part);
            const double rho1 = t3[0];
            if (!(rho1 != 0.0)) break;
            const double beta = (rho1 / rho) * (alpha / omega);
#pragma unroll
            for (int e = 0; e < E; e++) p[e] = rr[e] + beta * (p[e] - omega * v[e]);
            apply(p, v);
            t3[0] = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) t3[0] += rh[e] * v[e];
            block_sums<1>(t3, part);
            if (!(t3[0] != 0.0)) break;
            alpha = rho1 / t3[0];
            t3[0] = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) {
                sv[e] = rr[e] - alpha * v[e];
                t3[0] += sv[e] * sv[e];
            }
            block_sums<1>(t3, part);
            if (t3[0] <= tol2) {
#pragma unroll
                for (int e = 0; e < E; e++) xv[e] += alpha * p[e];
                ok = true;
                break;
            }
            apply(sv, tv);
            t3[0] = t3[1] = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) {
                t3[0] += tv[e] * sv[e];
                t3[1] += tv[e] * tv[e];
            }
            block_sums<2>(t3, part);
            if (!(t3[1] > 0.0)) break;
            omega = t3[0] / t3[1];
            t3[0] = 0.0;
#pragma unroll
            for (int e = 0; e < E; e++) {
                xv[e] += alpha * p[e] + omega * sv[e];
                rr[e] = sv[e] - omega * tv[e];
                t3[0] += rr[e] * rr[e];
            }
            rho = rho1;
            block_sums<1>(t3, part);
            if (t3[0] <= tol2) {
                ok = true;
                break;
            }
            if (!(omega != 0.0)) break;
        }
    }
    double tr[E];
    apply(xv, tr);
    t3[0] = 0.0;
#pragma unroll
    for (int e = 0; e < E; e++) {
        tr[e] = b[e] - tr[e];
        t3[0] += tr[e] * tr[e];
    }
    block_sums<1>(t3, part);
    ok = ok && t3[0] <= 1e-24 * bb;
    if (ok)
#pragma unroll
        for (int e = 0; e < E; e++)
            if (q0 + NT * e < m) x[q0 + NT * e] = (T)xv[e];
    return ok;
}

// Coarsest psi levels of more than 64 cells: the block Krylov solve; a system it
// does not solve raises the singular flag.
template <int BC, typename T>
__global__ void __launch_bounds__(kGjWaves *kWave) k_coarse_psi_krylov(Geo g, int m, const T *c, const T *r, T *x,
                                                                      double *flag)
{
    c = zsh(c, g.zs);
    r = zsh(r, g.zs);
    x = zsh(x, g.zs);
    flag = zsh(flag, g.zs);
    const bool ok = coarse_psi_krylov_block<BC, T>(g, m, c, r, x);
    if (!ok && threadIdx.x == 0) *flag = 1.0;
}

// Called by every thread of a block of kGjWaves waves.
template <int BC, typename T, int M>
__device__ __forceinline__ void coarse_psi_block_solve(const Geo &g, const T *c, const T *r, T *x, double *flag)
{
    constexpr int NC = M + 1;
    constexpr int S = (NC + kGjWaves - 1) / kGjWaves;
    __shared__ double A[M][NC + 1];
    __shared__ double fac[2][kWave];
    __shared__ int piv[2];
    __shared__ int perm[M];
    __shared__ double pdiag[M];
    __shared__ int krylov_ok;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int n = g.n;
    // first the Krylov solve on wave 0 alone; elimination only if it is not accepted
    if (wave == 0) {
        const bool ok = coarse_psi_krylov_wave<BC, T, M>(g, c, r, x);
        if (lane == 0) krylov_ok = ok ? 1 : 0;
    }
    __syncthreads();
    if (krylov_ok) return;
    if (threadIdx.x < M) {
        const int row = threadIdx.x;
        for (int j = 0; j < NC; j++) A[row][j] = 0.0;
        const int k = row % n, j = (row / n) % n, i = row / (n * n);
        const double wt[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};
        for (int ax = 0; ax < 3; ax++)
            for (int d = -2; d <= 2; d++) {
                int bi, bj, bk;
                const double fac_bc = ghost_source<BC>(g, i + (ax == 0 ? d : 0), j + (ax == 1 ? d : 0),
                                                       k + (ax == 2 ? d : 0), bi, bj, bk);
                A[row][(bi * n + bj) * n + bk] += wt[d + 2] * g.inv12h2 * fac_bc;
            }
        A[row][row] += (double)c[row];
        A[row][M] = (double)r[row];
    }
    __syncthreads();
    double v[S];
#pragma unroll
    for (int q = 0; q < S; q++) {
        const int col = wave + kGjWaves * q;
        v[q] = (lane < M && col < NC) ? A[lane][col] : 0.0;
    }
    // step k = kGjWaves * qk + w: pivot column k is register qk of wave w
    constexpr int QK = (M + kGjWaves - 1) / kGjWaves;
    uint64_t used = 0;
    bool singular = false;
    static_for<QK>([&](auto qc) {
        constexpr int qk = decltype(qc)::value;
        if (singular) return;
#pragma unroll 1
        for (int w = 0; w < kGjWaves; w++) {
            const int k = kGjWaves * qk + w;
            if (k >= M) break;
            const int buf = k & 1;
            if (wave == w) {
                const double a = v[qk];
                unsigned key = 0u;
                if (lane < M && !((used >> lane) & 1ull)) {
                    const unsigned bits = __float_as_uint((float)fabs(a));
                    key = (bits & ~63u) | (63u - (unsigned)lane);
                }
                const unsigned kmax = wave_max_u32(key);
                if ((kmax >> 6) == 0u) {
                    if (lane == 0) piv[buf] = -1; // no non-zero pivot left
                } else {
                    const int p = 63 - (int)(kmax & 63u);
                    const double ap = readlane_f64(a, p);
                    const double inv = 1.0 / ap;
                    fac[buf][lane] = lane == p ? 0.0 : a * inv;
                    if (lane == 0) {
                        piv[buf] = p;
                        pdiag[k] = ap;
                        perm[k] = p;
                    }
                }
                __builtin_amdgcn_s_setprio(0);
            }
            __syncthreads();
            const int p = __builtin_amdgcn_readfirstlane(piv[buf]);
            double f = fac[buf][lane];
            asm volatile("" : "+v"(f)); // both LDS reads in flight together
            if (p < 0) {
                singular = true;
                break;
            }
            // the owner of the next pivot column goes first on its SIMD
            if (wave == (w + 1) % kGjWaves) __builtin_amdgcn_s_setprio(2);
            used |= 1ull << p;
#pragma unroll
            for (int q = 0; q < S; q++) v[q] = fma(-f, readlane_f64(v[q], p), v[q]);
        }
    });
    if (singular) {
        if (threadIdx.x == 0) *flag = 1.0;
        return;
    }
    // the right-hand side column (held by one wave) through LDS
#pragma unroll
    for (int q = 0; q < S; q++)
        if (wave + kGjWaves * q == M && lane < M) A[lane][M] = v[q];
    __syncthreads();
    if (threadIdx.x < M) x[threadIdx.x] = (T)(A[perm[threadIdx.x]][M] / pdiag[threadIdx.x]);
}

template <int BC, typename T, int M>
__global__ void __launch_bounds__(kGjWaves * kWave) k_coarse_psi_block(Geo g, const T *c, const T *r, T *x,
                                                                      double *flag)
{
    c = zsh(c, g.zs);
    r = zsh(r, g.zs);
    x = zsh(x, g.zs);
    flag = zsh(flag, g.zs);
    coarse_psi_block_solve<BC, T, M>(g, c, r, x, flag);
}

// ---------------------------------------------------------------------------------------
// V-cycle tails: the coarse levels of one V-cycle (from level ls down to the
// coarsest and back) run in one workgroup of kGjWaves waves, phase by phase
// with block barriers, on arrays resident in LDS (these levels are too small
// to fill the GPU: as separate launches every phase would cost a launch).
// The tail reads its first level's right-hand side (and psi coefficient) from
// global memory, keeps every level's corrections, right-hand sides and
// coefficients in LDS, and writes its first level's correction back.  Each
// phase calls the same per-cell functions as the grid kernels.
// ---------------------------------------------------------------------------------------
constexpr int kTailThreads = kGjWaves * kWave;
constexpr int kMaxTail = 4;

// Cells of a tail summed over its levels: psi keeps d, r and c of every level
// in LDS, W d and r of three components (the passes update in place).  One
// workgroup runs a whole level per phase, so a tail pays off only while its
// first level is small: a W colour pass over 16^3 cells takes longer on one
// CU than as a grid launch, a psi pass (13 taps) does not.
template <typename T>
struct TailCap {
    static constexpr int kPsi = sizeof(T) == 4 ? 4680 : 1971; // 16^3 + 8^3 + 4^3 + 2^3 ; 12^3 + 6^3 + 3^3
    static constexpr int kPsiRobin = 1971;
    static constexpr int kW = 1971;
};

template <typename T>
struct TailArgs {
    int nl;      // levels in the tail (the last one is the coarsest)
    int nu_pre, nu_post;
    Geo geo[kMaxTail];
    const T *r0, *c0; // first level: right-hand side (3 components for W), psi coefficient
    T *d0;            // first level: the correction (output)
    const double *inv; // W: coarsest inverse (column-major m x m), m = 3 cells
    double *flag;      // psi: set when the coarsest matrix is singular
};

__device__ __forceinline__ int tail_cells(const Geo &g) { return g.n * g.n * g.n; }

// New value of an active cell of a psi colour pass (the arithmetic of the
// grid pass kernels: k_pass_psi_pairs when periodic, psi_pass_cell otherwise).
template <int BC, typename T>
__device__ __forceinline__ T psi_new_value(const Geo &g, const T *in, const T *r, const T *c, unsigned q, int i,
                                           int j, int k)
{
    if constexpr (BC == kBcPeriodic) {
        const WrapOff o(g.n, i, j, k);
        RegTaps<T, false> D;
        D.get_lap(WrapTaps<T>{in, o});
        const T v = D.c(), cv = c[q];
        const T Ad = (D.dxx(v) + D.dyy(v) + D.dzz(v)) * (T)g.inv12h2 + cv * v;
        const T diag = pinned((T)(-90.0 * g.inv12h2)) + cv;
        return v + (r[q] - Ad) / diag;
    } else {
        Acc<BC, T> D{in, g};
        const T x = in[q], cv = c[q];
        const T Ad = lap_sum<T>(D, i, j, k, x) * (T)g.inv12h2 + cv * x;
        const T diag = pinned((T)(lap_diag_sum<BC>(g, i, j, k) * g.inv12h2)) + cv;
        return x + (r[q] - Ad) / diag;
    }
}

// Active cells of a psi tail pass per thread: half the cells of a first level
// of at most 16^3 (periodic) or 12^3 (Robin: its ghost-cell taps need the
// registers of a second item).
template <int BC>
constexpr int tail_psi_items()
{
    return BC == kBcPeriodic ? 2 : 1;
}

// One colour pass of the psi smoother on an LDS-resident level, in place: the
// active cells' new values are formed from d into registers, the block waits,
// then they are written (the double-buffered pass's values).
template <int BC, typename T>
__device__ __forceinline__ void tail_psi_pass(const Geo &g, T *d, const T *r, const T *c, int colour)
{
    const int n = g.n, np = n >> 1, half = (n * n * n) >> 1;
    constexpr int NI = tail_psi_items<BC>();
    T val[NI];
    unsigned dst[NI];
#pragma unroll
    for (int s = 0; s < NI; s++) {
        const int it = (int)threadIdx.x + s * kTailThreads;
        dst[s] = ~0u;
        val[s] = T(0);
        if (it < half) {
            const int row = it / np, kp = it - row * np, i = row / n, j = row - i * n;
            const int k = 2 * kp + ((i + j + colour) & 1);
            const unsigned q = (unsigned)((i * n + j) * n + k);
            val[s] = psi_new_value<BC, T>(g, d, r, c, q, i, j, k);
            dst[s] = q;
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NI; s++)
        if (dst[s] != ~0u) d[dst[s]] = val[s];
    __syncthreads();
}

// psi tail: restricts c below its first level, then the V-cycle from the
// tail's first level.  LDS: per level d | r | c, levels consecutive.
template <int BC, typename T, int M>
__global__ void __launch_bounds__(kTailThreads) k_tail_psi(TailArgs<T> a)
{
    {
        const long long zs = a.geo[0].zs;
        a.r0 = zsh(a.r0, zs);
        a.c0 = zsh(a.c0, zs);
        a.d0 = zsh(a.d0, zs);
        a.inv = zsh(a.inv, zs);
        a.flag = zsh(a.flag, zs);
    }
    __shared__ T buf[3 * TailCap<T>::kPsi];
    const int L = a.nl;
    int off[kMaxTail] = {0, 0, 0, 0};
    {
        int o = 0;
        for (int l = 0; l < L && l < kMaxTail; l++) {
            off[l] = o;
            o += 3 * tail_cells(a.geo[l]);
        }
        if (L < 2 || L > kMaxTail || o > 3 * TailCap<T>::kPsi ||
            tail_cells(a.geo[0]) / 2 > tail_psi_items<BC>() * kTailThreads)
            return; // the host picks tails that fit
    }
    auto D = [&](int l) { return buf + off[l]; };
    auto R = [&](int l) { return buf + off[l] + tail_cells(a.geo[l]); };
    auto C = [&](int l) { return buf + off[l] + 2 * tail_cells(a.geo[l]); };
    {
        const int m0 = tail_cells(a.geo[0]);
        T *r0 = R(0), *c0 = C(0);
        for (int q = threadIdx.x; q < m0; q += kTailThreads) {
            r0[q] = a.r0[q];
            c0[q] = a.c0[q];
        }
    }
    __syncthreads();
    for (int l = 0; l + 1 < L; l++) {
        const int nf = a.geo[l].n, nc = a.geo[l + 1].n, mc = tail_cells(a.geo[l + 1]);
        const T *cf = C(l);
        T *cc = C(l + 1);
        for (int q = threadIdx.x; q < mc; q += kTailThreads) {
            int I, J, K;
            cell_of(q, nc, I, J, K);
            T s = T(0);
#pragma unroll
            for (int di = 0; di < 2; di++)
#pragma unroll
                for (int dj = 0; dj < 2; dj++)
#pragma unroll
                    for (int dk = 0; dk < 2; dk++) s += cf[lidx(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
            cc[q] = s * T(0.125);
        }
        __syncthreads();
    }
    for (int l = 0; l + 1 < L; l++) {
        const Geo &g = a.geo[l];
        const int mf = tail_cells(g);
        T *d = D(l);
        for (int q = threadIdx.x; q < mf; q += kTailThreads) d[q] = T(0);
        __syncthreads();
        for (int s = 0; s < a.nu_pre; s++) {
            tail_psi_pass<BC, T>(g, D(l), R(l), C(l), 0);
            tail_psi_pass<BC, T>(g, D(l), R(l), C(l), 1);
        }
        for (int q = threadIdx.x; q < mf + (kTailThreads - 1); q += kTailThreads) {
            if (q - (int)threadIdx.x >= mf) break; // the whole block leaves together
            defect_restrict_psi_child<BC, T>(g, D(l), R(l), C(l), R(l + 1), (T *)nullptr, q);
        }
        __syncthreads();
    }
    {
        const int mc = tail_cells(a.geo[L - 1]);
        T *x = D(L - 1);
        for (int q = threadIdx.x; q < mc; q += kTailThreads) x[q] = T(0); // stays 0 if singular
        __syncthreads();
        coarse_psi_block_solve<BC, T, M>(a.geo[L - 1], C(L - 1), R(L - 1), x, a.flag);
        __syncthreads();
    }
    for (int l = L - 2; l >= 0; l--) {
        const int nf = a.geo[l].n, mf = tail_cells(a.geo[l]);
        for (int q = threadIdx.x; q < mf; q += kTailThreads) {
            int i, j, k;
            cell_of(q, nf, i, j, k);
            prolong_cell<BC, T>(a.geo[l + 1], D(l + 1), D(l), 1, q, i, j, k);
        }
        __syncthreads();
        for (int s = 0; s < a.nu_post; s++) {
            tail_psi_pass<BC, T>(a.geo[l], D(l), R(l), C(l), 0);
            tail_psi_pass<BC, T>(a.geo[l], D(l), R(l), C(l), 1);
        }
    }
    {
        const int m0 = tail_cells(a.geo[0]);
        const T *d0 = D(0);
        for (int q = threadIdx.x; q < m0; q += kTailThreads) a.d0[q] = d0[q];
    }
}

// (Delta_L d)_A at a cell from wrapped offsets, component A alone: the terms
// W_field_parts forms for that component, in the same order.  centre: d_A at
// the cell.
template <typename T, int A>
__device__ __forceinline__ T deltaL_comp(const T *d, unsigned m, const WrapOff &o, T h2, T m2, T third, T &centre)
{
    RegTaps<T, false> D;
    D.get_lap(WrapTaps<T>{d + A * m, o});
    const T c = D.c();
    centre = c;
    const T xx = D.dxx(c), yy = D.dyy(c), zz = D.dzz(c);
    const T lap = (xx + yy + zz) * h2;
    const T dd = (A == 0 ? xx : (A == 1 ? yy : zz)) * h2;
    RegTaps<T, false> E, G;
    T mix;
    if constexpr (A == 0) {
        E.template get_mixed<0, 1>(WrapTaps<T>{d + m, o});
        G.template get_mixed<0, 2>(WrapTaps<T>{d + 2 * m, o});
        mix = E.dxy();
        mix = mix + G.dxz();
    } else if constexpr (A == 1) {
        E.template get_mixed<0, 1>(WrapTaps<T>{d, o});
        G.template get_mixed<1, 2>(WrapTaps<T>{d + 2 * m, o});
        mix = E.dxy();
        mix = mix + G.dyz();
    } else {
        E.template get_mixed<0, 2>(WrapTaps<T>{d, o});
        G.template get_mixed<1, 2>(WrapTaps<T>{d + m, o});
        mix = E.dxz();
        mix = mix + G.dyz();
    }
    return lap + (dd + mix * m2) * third;
}

// Work items of a W tail pass: three components of half the cells of a first
// level of at most TailCap<T>::kW cells in all (12^3).
constexpr int kTailWStage = 3 * 1728 / 2;

// One colour pass of the W smoother on an LDS-resident level, in place: the
// threads evaluate the (component, active cell) items from d into the LDS
// stage, the block waits, then the values go to d (the same values as the
// double-buffered pass: the other colour is unchanged).  Items are
// component-major, so a wave handles one component.
template <typename T>
__device__ __forceinline__ void tail_W_pass(const Geo &g, T *d, const T *r, T *stage, int colour)
{
    const int n = g.n, np = n >> 1;
    const unsigned m = (unsigned)(n * n * n);
    const int half = (int)(m >> 1), items = 3 * half;
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2, third = T(1) / T(3);
    const T diag = (T)(-100.0 * g.inv12h2);
    // item it: component a, active cell h of the colour, (i, j, k) and index q
    auto cell = [&](int it, int &a, int &i, int &j, int &k) {
        a = it / half;
        const int h = it - a * half, row = h / np, kp = h - row * np;
        i = row / n;
        j = row - i * n;
        k = 2 * kp + ((i + j + colour) & 1);
        return (unsigned)((i * n + j) * n + k);
    };
#pragma unroll 1
    for (int it = threadIdx.x; it < items; it += kTailThreads) {
        int a, i, j, k;
        const unsigned q = cell(it, a, i, j, k);
        const WrapOff o(n, i, j, k);
        T centre, Ad;
        if (a == 0)
            Ad = deltaL_comp<T, 0>(d, m, o, h2, m2, third, centre);
        else if (a == 1)
            Ad = deltaL_comp<T, 1>(d, m, o, h2, m2, third, centre);
        else
            Ad = deltaL_comp<T, 2>(d, m, o, h2, m2, third, centre);
        stage[it] = centre + (r[a * m + q] - Ad) / diag;
    }
    __syncthreads();
#pragma unroll 1
    for (int it = threadIdx.x; it < items; it += kTailThreads) {
        int a, i, j, k;
        const unsigned q = cell(it, a, i, j, k);
        d[a * m + q] = stage[it];
    }
    __syncthreads();
}

// W tail (periodic): V-cycle from the tail's first level; the coarsest solve
// applies the precomputed inverse to the mean-free residual (as
// k_coarse_apply, rows in blocks of 64 with the columns split over 16 parts).
// LDS: per level d | r (three components each), levels consecutive.
template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail_W(TailArgs<T> a)
{
    {
        const long long zs = a.geo[0].zs;
        a.r0 = zsh(a.r0, zs);
        a.c0 = zsh(a.c0, zs);
        a.d0 = zsh(a.d0, zs);
        a.inv = zsh(a.inv, zs);
        a.flag = zsh(a.flag, zs);
    }
    __shared__ T buf[6 * TailCap<T>::kW];
    __shared__ T stage[kTailWStage];
    __shared__ double rs[1536];
    __shared__ double red[kTailThreads / kWave][kWave];
    __shared__ double mean[3];
    const int L = a.nl;
    int off[kMaxTail] = {0, 0, 0, 0};
    {
        int o = 0;
        for (int l = 0; l < L && l < kMaxTail; l++) {
            off[l] = o;
            o += 6 * tail_cells(a.geo[l]);
        }
        if (L < 2 || L > kMaxTail || o > 6 * TailCap<T>::kW || 3 * tail_cells(a.geo[0]) / 2 > kTailWStage ||
            3 * tail_cells(a.geo[L - 1]) > 1536)
            return; // the host picks tails that fit
    }
    auto D = [&](int l) { return buf + off[l]; };
    auto R = [&](int l) { return buf + off[l] + 3 * tail_cells(a.geo[l]); };
    {
        const int m0 = 3 * tail_cells(a.geo[0]);
        T *r0 = R(0);
        for (int q = threadIdx.x; q < m0; q += kTailThreads) r0[q] = a.r0[q];
    }
    __syncthreads();
    for (int l = 0; l + 1 < L; l++) {
        const Geo &g = a.geo[l];
        const int m = tail_cells(g);
        T *d = D(l);
        for (int q = threadIdx.x; q < 3 * m; q += kTailThreads) d[q] = T(0);
        __syncthreads();
        for (int s = 0; s < a.nu_pre; s++) {
            tail_W_pass<T>(g, D(l), R(l), stage, 0);
            tail_W_pass<T>(g, D(l), R(l), stage, 1);
        }
        for (int q = threadIdx.x; q < m + (kTailThreads - 1); q += kTailThreads) {
            if (q - (int)threadIdx.x >= m) break; // the whole block leaves together
            defect_restrict_W_child<T>(g, D(l), R(l), R(l + 1), q);
        }
        __syncthreads();
    }
    {
        const int cn = tail_cells(a.geo[L - 1]), m = 3 * cn;
        const T *rc = R(L - 1);
        for (int q = threadIdx.x; q < m; q += kTailThreads) rs[q] = (double)rc[q];
        __syncthreads();
        if (threadIdx.x < 3) {
            double s = 0.0;
            for (int q = 0; q < cn; q++) s += rs[threadIdx.x * cn + q];
            mean[threadIdx.x] = s / (double)cn;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < m; q += kTailThreads) rs[q] -= mean[q / cn];
        __syncthreads();
        T *x = D(L - 1);
        constexpr int kParts = kTailThreads / kWave;
        const int rl = threadIdx.x % kWave, part = threadIdx.x / kWave;
        for (int rb = 0; rb < m; rb += kWave) {
            const int row = rb + rl;
            const double s = row < m ? inv_row_dot<kParts>(a.inv, m, row, part, rs) : 0.0;
            red[part][rl] = s;
            __syncthreads();
            if (threadIdx.x < kWave && row < m) {
                double t = 0.0;
                for (int q = 0; q < kParts; q++) t += red[q][rl];
                x[row] = (T)t;
            }
            __syncthreads();
        }
    }
    for (int l = L - 2; l >= 0; l--) {
        const Geo &g = a.geo[l];
        const int nf = g.n, mf = tail_cells(g);
        for (int q = threadIdx.x; q < mf; q += kTailThreads) {
            int i, j, k;
            cell_of(q, nf, i, j, k);
            prolong_cell<kBcPeriodic, T>(a.geo[l + 1], D(l + 1), D(l), 3, q, i, j, k);
        }
        __syncthreads();
        for (int s = 0; s < a.nu_post; s++) {
            tail_W_pass<T>(g, D(l), R(l), stage, 0);
            tail_W_pass<T>(g, D(l), R(l), stage, 1);
        }
    }
    {
        const int m0 = 3 * tail_cells(a.geo[0]);
        const T *d0 = D(0);
        for (int q = threadIdx.x; q < m0; q += kTailThreads) a.d0[q] = d0[q];
    }
}

// ---------------------------------------------------------------------------------------
// Elementwise helpers
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T *a, int64_t count, T v, long long zs)
{
    a = zsh(a, zs);
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < count) a[q] = v;
}

// u += d.  gate (nullable): the update is skipped when *gate == 0 (an instance
// of a batch that has already converged).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update_u(double *u, const T *d, int64_t m, const double *gate, long long zs)
{
    u = zsh(u, zs);
    d = zsh(d, zs);
    gate = zsh(gate, zs);
    if (gate && *gate == 0.0) return;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < m) u[q] += (double)d[q];
}

// k_update_u followed by k_source_sum's partial sums of 8 pi psi^6 S_a at the
// updated state, in one pass (same cells per thread and summation order as
// k_source_sum).
template <int BC, typename T>
__global__ void __launch_bounds__(kBlock) k_update_u_source(Geo g, double *u, const T *d, const double *gate,
                                                            const double *S, double pmass, int conformal,
                                                            double *partials)
{
    u = zsh(u, g.zs);
    d = zsh(d, g.zs);
    gate = zsh(gate, g.zs);
    S = zsh(S, g.zs);
    partials = zsh(partials, g.zs);
    const bool upd = !(gate && *gate == 0.0);
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < kSumCells; c++) {
        const int64_t tid = ((int64_t)blockIdx.x * kSumCells + c) * kBlock + threadIdx.x;
        int i, j, k;
        if (cell_of(tid, n, i, j, k)) {
            double uq = u[tid];
            if (upd) {
                uq += (double)d[tid];
                u[tid] = uq;
            }
            const double psi = psi0_at(g, pmass, i, j, k) + uq;
            const double p2 = psi * psi, p6 = conformal ? 1.0 : p2 * p2 * p2;
#pragma unroll
            for (int s = 0; s < 3; s++) v[s] += 8.0 * kPi * p6 * S[s * m + tid];
        }
    }
    block_reduce_store<3>(v, 0u, partials + 3 * (int64_t)blockIdx.x);
}

// W_a += dW_a - mean_a (mean: device, 3 values); gate as for k_update_u
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update_W(double *W, const T *d, const double *mean,
                                                     int64_t m, const double *gate, long long zs)
{
    W = zsh(W, zs);
    d = zsh(d, zs);
    mean = zsh(mean, zs);
    gate = zsh(gate, zs);
    if (gate && *gate == 0.0) return;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= m) return;
#pragma unroll
    for (int s = 0; s < 3; s++) W[s * m + q] += (double)d[s * m + q] - mean[s];
}

// Convergence bookkeeping of one batch instance after an evaluation.
// scal: the instance's scalar block (norm sums / maxima at 0..3).  If the
// instance was active, its update count is incremented (the evaluation follows
// an update step, except the first one, which passes count_update = 0); the
// instance stays active while rms H > tol or (momentum) rms |M| > tol and the
// norms are finite; a non-finite norm marks it diverged.
__global__ void k_batch_check(double *scal, int active_slot, int iters_slot, int div_slot, double inv_cells,
                              double tol, int momentum, int count_update, long long zs)
{
    scal = zsh(scal, zs);
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double was = scal[active_slot];
    if (was == 0.0) return;
    if (count_update) scal[iters_slot] += 1.0;
    const double h = sqrt(scal[0] * inv_cells), mm = sqrt(scal[2] * inv_cells);
    if (!isfinite(h) || !isfinite(mm)) {
        scal[div_slot] = 1.0;
        scal[active_slot] = 0.0;
        return;
    }
    if (h <= tol && (!momentum || mm <= tol)) scal[active_slot] = 0.0;
}

// The device scalars of the members of a group (block z: the member zs bytes after
// member 0's block src) copied to consecutive blocks of dst, for one host copy.
__global__ void k_gather_scal(const double *src, long long zs, int count, double *dst)
{
    src = zsh(src, zs);
    if ((int)threadIdx.x < count) dst[(int64_t)blockIdx.z * count + threadIdx.x] = src[threadIdx.x];
}

// ---------------------------------------------------------------------------------------
// Scalar-field sources from Fourier modes and the puncture shell.
// ---------------------------------------------------------------------------------------
constexpr int kMaxModes = 32;
struct ModeTable {
    int nphi, npi;
    double phi[kMaxModes][5];
    double pi[kMaxModes][5];
};

__global__ void __launch_bounds__(kBlock) k_sources_modes(Geo g, double length, ModeTable t,
                                                          double mass, double *rho5, double *rho1,
                                                          double *S, double *partials)
{
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    const double tw = 2.0 * kPi / length;
    double acc[1] = {0.0};
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < m;
         q += (int64_t)gridDim.x * kBlock) {
        int i, j, k;
        cell_of(q, n, i, j, k);
        const double x = g.org[0] + (i + 0.5) * g.h, y = g.org[1] + (j + 0.5) * g.h,
                     z = g.org[2] + (k + 0.5) * g.h;
        double phi = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0, Pi = 0.0;
        for (int p = 0; p < t.nphi; p++) {
            const double *md = t.phi[p];
            double s, c;
            sincos(tw * (md[0] * x + md[1] * y + md[2] * z) + md[4], &s, &c);
            phi += md[3] * c;
            d0 -= md[3] * tw * md[0] * s;
            d1 -= md[3] * tw * md[1] * s;
            d2 -= md[3] * tw * md[2] * s;
        }
        for (int p = 0; p < t.npi; p++) {
            const double *md = t.pi[p];
            Pi += md[3] * cos(tw * (md[0] * x + md[1] * y + md[2] * z) + md[4]);
        }
        const double r5 = 0.5 * Pi * Pi + 0.5 * mass * mass * phi * phi;
        const double r1 = 0.5 * (d0 * d0 + d1 * d1 + d2 * d2);
        rho5[q] = r5;
        rho1[q] = r1;
        S[q] = -Pi * d0;
        S[m + q] = -Pi * d1;
        S[2 * m + q] = -Pi * d2;
        acc[0] += r5 + r1;
    }
    if (partials) block_reduce_store<1>(acc, 0u, partials + blockIdx.x);
}

// Bowen-York punctures: psi0 = 1 + sum m / (2 r) and A2 = Abar_ij Abar_ij of the sum over
// punctures of (3 / (2 r^2)) [P_i n_j + P_j n_i - (delta_ij - n_i n_j) P.n]
// + (3 / r^3) [(S x n)_i n_j + (S x n)_j n_i], n = (x - C) / r, at every cell centre.
constexpr int kMaxPunctures = 8;
struct PunctureTable {
    int count;
    double t[kMaxPunctures][10]; // m, C[3], P[3], S[3]
};

__global__ void __launch_bounds__(kBlock) k_bowen_york(Geo g, PunctureTable pt, double *psi0, double *A2)
{
    const int n = g.n;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int i, j, k;
    if (!cell_of(q, n, i, j, k)) return;
    const double x[3] = {g.org[0] + (i + 0.5) * g.h, g.org[1] + (j + 0.5) * g.h, g.org[2] + (k + 0.5) * g.h};
    double A[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    double s = 1.0;
    for (int p = 0; p < pt.count; p++) {
        const double *t = pt.t[p];
        const double d[3] = {x[0] - t[1], x[1] - t[2], x[2] - t[3]};
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double ir = 1.0 / r;
        const double nv[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
        const double pn = t[4] * nv[0] + t[5] * nv[1] + t[6] * nv[2];
        const double sxn[3] = {t[8] * nv[2] - t[9] * nv[1], t[9] * nv[0] - t[7] * nv[2], t[7] * nv[1] - t[8] * nv[0]};
        const double cb = 1.5 * ir * ir, cs = 3.0 * ir * ir * ir;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const double boost = t[4 + a] * nv[b] + t[4 + b] * nv[a] - ((a == b ? 1.0 : 0.0) - nv[a] * nv[b]) * pn;
                A[a][b] += cb * boost + cs * (sxn[a] * nv[b] + sxn[b] * nv[a]);
            }
        s += t[0] * 0.5 * ir;
    }
    double a2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) a2 += A[a][b] * A[a][b];
    psi0[q] = s;
    A2[q] = a2;
}

__global__ void __launch_bounds__(kBlock) k_sources_shell(Geo g, double amp, double r0,
                                                          double width2, double mass, double *rho5,
                                                          double *rho1, double *S)
{
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int i, j, k;
    if (!cell_of(q, n, i, j, k)) return;
    const double x[3] = {g.org[0] + (i + 0.5) * g.h - g.ctr[0], g.org[1] + (j + 0.5) * g.h - g.ctr[1],
                         g.org[2] + (k + 0.5) * g.h - g.ctr[2]};
    const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double ylm = sqrt(3.0 / (4.0 * kPi));
    const double fr = amp * exp(-(r - r0) * (r - r0) / width2);
    const double dfr = -2.0 * (r - r0) / width2 * fr;
    const double phi = fr * ylm * x[0] / r;
    double g2 = 0.0;
    for (int a = 0; a < 3; a++) {
        // d_a [f(r) x/r] = f'(r) (x_a/r)(x/r) + f(r) (delta_a0/r - x x_a/r^3)
        const double da = ylm * (dfr * (x[a] / r) * (x[0] / r) +
                                 fr * ((a == 0 ? 1.0 : 0.0) / r - x[0] * x[a] / (r * r * r)));
        g2 += da * da;
    }
    rho5[q] = 0.5 * mass * mass * phi * phi;
    rho1[q] = 0.5 * g2;
    S[q] = 0.0;
    S[m + q] = 0.0;
    S[2 * m + q] = 0.0;
}

} // namespace grtmg
