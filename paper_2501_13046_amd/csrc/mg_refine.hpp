// mg_refine.hpp -- kernels of the static mesh refinement by nested boxes (Key
// features, "Adaptive Mesh Refinement": refined boxes over the base grid; "Fast").
//
// Levels: a base grid, then boxes, each refined by 2 over m^3 cells of its parent
// whose corner is parent cell (b0, b0, b0) (nf = 2m cells per axis).  A parent
// cell under a box holds the average of its 8 children; a box's two ghost layers
// are the children of the parent cells around it by the 4-point cubic (weights
// (-5, 35, 105, -7)/128 and mirror).  A box is solved as a grid of its own under
// the zero ghost rule with a forcing that carries the interpolated ghosts,
// f = sum over stencil taps outside the box of w g / (12 h_box^2); a parent takes
// the FAS forcing tau = R H_box - H_parent(R u_box) on the cells under the box.  A
// box keeps a margin of at least 3 parent cells, so every cubic stencil stays inside
// the parent and no boundary rule is needed here.  BoxGeo names a parent-box pair:
// nc is the parent's cells per axis.
#pragma once

#include "mg_device.hpp"

namespace grtmg {

struct BoxGeo {
    int nc;   // base cells per axis
    int b0;   // base index of the box's first cell on every axis
    int m;    // base cells covered per axis (the box has 2m fine cells per axis)
};

__device__ __forceinline__ int64_t cidx(int n, int i, int j, int k) { return ((int64_t)i * n + j) * n + k; }

// Cubic weights of the child of parity p (0: nearer the lower neighbour) on the four
// base nodes I - 2 + p .. I + 1 + p.
__device__ __forceinline__ double cubic_w(int p, int e)
{
    const double w0[4] = {-5.0 / 128.0, 35.0 / 128.0, 105.0 / 128.0, -7.0 / 128.0};
    const double w1[4] = {-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0};
    return p ? w1[e] : w0[e];
}

// Value at box cell (fi, fj, fk) (indices may lie up to 2 cells outside the box) of the
// cubic interpolation of the base field a (difference a - b when b is not null).
__device__ __forceinline__ double box_cubic_at(const BoxGeo &bx, const double *a, const double *b, int fi, int fj,
                                               int fk)
{
    const int f[3] = {fi, fj, fk};
    int lo[3], par[3];
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        const int q = 2 * bx.b0 + f[ax]; // fine index on the base grid's refinement
        const int I = q >> 1;            // q >= 0: the margin keeps the box inside
        par[ax] = q & 1;
        lo[ax] = I - 2 + par[ax];
    }
    double s = 0.0;
#pragma unroll
    for (int x = 0; x < 4; x++) {
        double sy = 0.0;
#pragma unroll
        for (int y = 0; y < 4; y++) {
            double sz = 0.0;
#pragma unroll
            for (int z = 0; z < 4; z++) {
                const int64_t q = cidx(bx.nc, lo[0] + x, lo[1] + y, lo[2] + z);
                sz += cubic_w(par[2], z) * (b ? a[q] - b[q] : a[q]);
            }
            sy += cubic_w(par[1], y) * sz;
        }
        s += cubic_w(par[0], x) * sy;
    }
    return s;
}

// Base cells under the box take the average of their 8 children: uc[b0 + I..] = R uf.
__global__ void __launch_bounds__(kBlock) k_box_restrict(BoxGeo bx, const double *__restrict__ uf,
                                                         double *__restrict__ uc)
{
    const int m = bx.m, nf = 2 * m;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)m * m * m) return;
    const int K = (int)(t % m), J = (int)((t / m) % m), I = (int)(t / ((int64_t)m * m));
    double s = 0.0;
#pragma unroll
    for (int di = 0; di < 2; di++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int dk = 0; dk < 2; dk++) s += uf[cidx(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
    uc[cidx(bx.nc, bx.b0 + I, bx.b0 + J, bx.b0 + K)] = 0.125 * s;
}

// Forcing of the box under the zero rule: the taps of every fine cell that fall
// outside the box, on the interpolated ghosts, times 1/(12 (h/2)^2), plus the box's
// own FAS forcing tau from a finer box inside it (null: none).
__global__ void __launch_bounds__(kBlock) k_box_ghost_forcing(BoxGeo bx, double inv12h2, const double *__restrict__ uc,
                                                              const double *__restrict__ tau, double *__restrict__ ff)
{
    const int nf = 2 * bx.m;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)nf * nf * nf) return;
    const int k = (int)(t % nf), j = (int)((t / nf) % nf), i = (int)(t / ((int64_t)nf * nf));
    const double wt[5] = {-1.0, 16.0, 0.0, 16.0, -1.0};
    const int c[3] = {i, j, k};
    double f = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
        if (c[ax] >= 2 && c[ax] < nf - 2) continue; // every tap along this axis is inside
#pragma unroll
        for (int d = -2; d <= 2; d++) {
            const int q = c[ax] + d;
            if (d == 0 || (q >= 0 && q < nf)) continue;
            const int gi = ax == 0 ? q : i, gj = ax == 1 ? q : j, gk = ax == 2 ? q : k;
            f += wt[d + 2] * box_cubic_at(bx, uc, nullptr, gi, gj, gk);
        }
    }
    ff[t] = f * inv12h2 + (tau ? tau[t] : 0.0);
}

// FAS forcing of the base grid: tau = R H_f - H_c on covered cells, zero elsewhere.
__global__ void __launch_bounds__(kBlock) k_box_tau(BoxGeo bx, const double *__restrict__ Hf,
                                                    const double *__restrict__ Hc, double *__restrict__ fc)
{
    const int nc = bx.nc, m = bx.m, nf = 2 * m;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)nc * nc * nc) return;
    const int K = (int)(t % nc) - bx.b0, J = (int)((t / nc) % nc) - bx.b0, I = (int)(t / ((int64_t)nc * nc)) - bx.b0;
    if ((unsigned)I >= (unsigned)m || (unsigned)J >= (unsigned)m || (unsigned)K >= (unsigned)m) {
        fc[t] = 0.0;
        return;
    }
    double s = 0.0;
#pragma unroll
    for (int di = 0; di < 2; di++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int dk = 0; dk < 2; dk++) s += Hf[cidx(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
    fc[t] = 0.125 * s - Hc[t];
}

// Box correction by the base grid's change: uf += cubic interpolation of uc - uc_old,
// one thread per covered base cell writing its 8 children.
__global__ void __launch_bounds__(kBlock) k_box_correct(BoxGeo bx, const double *__restrict__ uc,
                                                        const double *__restrict__ uc_old, double *__restrict__ uf)
{
    const int m = bx.m, nf = 2 * m;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)m * m * m) return;
    const int K = (int)(t % m), J = (int)((t / m) % m), I = (int)(t / ((int64_t)m * m));
#pragma unroll
    for (int di = 0; di < 2; di++)
#pragma unroll
        for (int dj = 0; dj < 2; dj++)
#pragma unroll
            for (int dk = 0; dk < 2; dk++) {
                const int fi = 2 * I + di, fj = 2 * J + dj, fk = 2 * K + dk;
                uf[cidx(nf, fi, fj, fk)] += box_cubic_at(bx, uc, uc_old, fi, fj, fk);
            }
}

// Composite norm partials of one level: sum of H^2 times the cell volume over the
// cells no finer box covers (child.m = 0: no finer box), and max |H|; grid-stride.
__global__ void __launch_bounds__(kBlock) k_level_norm(int n, BoxGeo child, double vol, const double *__restrict__ H,
                                                       double *__restrict__ partials)
{
    const int64_t m3 = (int64_t)n * n * n;
    double v[2] = {0.0, 0.0};
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < m3; q += (int64_t)gridDim.x * kBlock) {
        const int K = (int)(q % n) - child.b0, J = (int)((q / n) % n) - child.b0, I = (int)(q / ((int64_t)n * n)) - child.b0;
        if ((unsigned)I < (unsigned)child.m && (unsigned)J < (unsigned)child.m && (unsigned)K < (unsigned)child.m)
            continue;
        const double h = H[q];
        v[0] += vol * h * h;
        v[1] = fmax(v[1], fabs(h));
    }
    block_reduce_store<2>(v, 0x2u, partials + 2 * (int64_t)blockIdx.x);
}

} // namespace grtmg
