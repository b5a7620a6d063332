// mg_tiled.hpp -- LDS-tiled kernels for the finest multigrid levels.
//
// A workgroup of 64 (z) x 4 (y) threads owns a brick of TX x 4 x 64 cells
// (each thread TX cells along x).  It stages the brick plus a 2-cell halo on
// every side of each stencil field in LDS with one coalesced pass (boundary
// rule applied by the accessor), synchronises once, and evaluates its cells
// from LDS.  Global traffic per cell is one read per field plus halo
// re-reads that neighbouring bricks share through L2, instead of one cached
// load per stencil tap; one pass per brick keeps thousands of independent
// workgroups in flight.
//
// Workgroups are renumbered so that each XCD (hardware workgroup ids are
// dealt round-robin to the 8 XCDs) receives a contiguous slab of bricks,
// whose shared halos stay in that XCD's L2.
#pragma once

#include "mg_kernels.hpp"

namespace grtmg {

constexpr int kTY = 4;    // brick rows (y) = waves per workgroup
constexpr int kLanes = 64; // lanes per wave
constexpr int kBZ = 128;   // brick depth along z: each lane owns a z pair
constexpr int kPY = kTY + 4;
constexpr int kPZ = kBZ + 4;     // staged z extent (2-cell halo each side)
constexpr int kHalf = kPZ / 2;   // LDS rows are split by z parity
constexpr int kXCD = 8;

struct TileMap {
    int nx, ny, nz; // bricks along x, y, z
    int tx;         // brick depth along x; 0: level not tiled
};

__device__ __forceinline__ void brick_of(const TileMap &t, int &x0, int &y0, int &z0)
{
    const int total = t.nx * t.ny * t.nz;
    const int b = blockIdx.x;
    int logical = b;
    if (total % kXCD == 0) logical = (b % kXCD) * (total / kXCD) + b / kXCD;
    const int bz = logical % t.nz;
    const int rest = logical / t.nz;
    const int by = rest % t.ny;
    const int bx = rest / t.ny;
    x0 = bx * t.tx;
    y0 = by * kTY;
    z0 = bz * kBZ;
}

// Staged layout: lds[xx][yy][h * kHalf + j] holds the value at staged z index
// zz = 2 j + h (zz = z - z0 + 2): even and odd z in separate halves, so lanes
// that read z = 2 lane + const hit consecutive words.

template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

// Stage brick + halo of one field.  Wave w stages rows w, w + kTY, ... of the
// (TX + 4) x kPY row grid; a lane moves the interior pair z0 + 2 lane, +1 with
// one aligned vector load, lanes 0..3 the four z-halo cells.  All of a wave's
// global loads are issued before any LDS store, so their latencies overlap.
template <int BC, typename T, int TX>
__device__ __forceinline__ void load_brick(T (*s)[kPY][kPZ], const Acc<BC, T> &A, int x0, int y0, int z0)
{
    using V2 = typename Vec2<T>::type;
    constexpr int RPW = (TX + 4) * kPY / kTY; // rows per wave
    static_assert((TX + 4) * kPY % kTY == 0, "rows must divide among the waves");
    const int n = A.g.n;
    const int w = threadIdx.y, lane = threadIdx.x;
    // lane 0: zz 0 (z0-2), 1: zz 1 (z0-1), 2: zz 130 (z0+128), 3: zz 131 (z0+129)
    const int hz = lane < 2 ? lane : kBZ + lane;
    V2 v[RPW];
    T hv[RPW];
#pragma unroll
    for (int i = 0; i < RPW; i++) {
        const int row = w + i * kTY;
        const int xg = x0 + row / kPY - 2, yg = y0 + row % kPY - 2;
        const bool inside = (unsigned)xg < (unsigned)n && (unsigned)yg < (unsigned)n;
        if (BC == kBcPeriodic || inside) {
            const T *src = A.a + ((int64_t)wrap(xg, n) * n + wrap(yg, n)) * n;
            v[i] = *reinterpret_cast<const V2 *>(src + z0 + 2 * lane);
        } else {
            v[i].x = A(xg, yg, z0 + 2 * lane);
            v[i].y = A(xg, yg, z0 + 2 * lane + 1);
        }
        hv[i] = lane < 4 ? A(xg, yg, z0 + hz - 2) : T(0);
    }
#pragma unroll
    for (int i = 0; i < RPW; i++) {
        const int row = w + i * kTY;
        T *dst = s[row / kPY][row % kPY];
        dst[lane + 1] = v[i].x;
        dst[kHalf + lane + 1] = v[i].y;
        if (lane < 4) dst[(hz & 1) * kHalf + (hz >> 1)] = hv[i];
    }
}

// Compile-time LDS offset of staged z index (2 lane + PAR + 2 + DZ) relative to
// the lane's word lane (PAR: z parity of the evaluated cell).
template <int PAR, int DZ>
constexpr int zoff()
{
    return ((PAR + DZ) & 1) * kHalf + ((PAR + 2 + DZ) >> 1);
}

constexpr int kRow = kPZ;        // words between y rows
constexpr int kPlane = kPY * kPZ; // words between x planes

// Taps around the thread's cell: base points at word (xx, yy, lane) of a field.
template <typename T, int PAR>
struct Taps {
    const T *b;
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T at() const
    {
        return b[DX * kPlane + DY * kRow + zoff<PAR, DZ>()];
    }
    __device__ __forceinline__ T c() const { return at<0, 0, 0>(); }
    __device__ __forceinline__ T dxx(T v) const
    {
        return T(16) * (at<-1, 0, 0>() + at<1, 0, 0>()) - (at<-2, 0, 0>() + at<2, 0, 0>()) - T(30) * v;
    }
    __device__ __forceinline__ T dyy(T v) const
    {
        return T(16) * (at<0, -1, 0>() + at<0, 1, 0>()) - (at<0, -2, 0>() + at<0, 2, 0>()) - T(30) * v;
    }
    __device__ __forceinline__ T dzz(T v) const
    {
        return T(16) * (at<0, 0, -1>() + at<0, 0, 1>()) - (at<0, 0, -2>() + at<0, 0, 2>()) - T(30) * v;
    }
    // first-difference sums f(-2) - 8 f(-1) + 8 f(+1) - f(+2), at an offset
    template <int DX, int DZ>
    __device__ __forceinline__ T dy_at() const
    {
        return (at<DX, -2, DZ>() - at<DX, 2, DZ>()) + T(8) * (at<DX, 1, DZ>() - at<DX, -1, DZ>());
    }
    template <int DX, int DY>
    __device__ __forceinline__ T dz_at() const
    {
        return (at<DX, DY, -2>() - at<DX, DY, 2>()) + T(8) * (at<DX, DY, 1>() - at<DX, DY, -1>());
    }
    // products of two first-difference stencils (144 h^2 D_p D_q)
    __device__ __forceinline__ T dxy() const
    {
        return (dy_at<-2, 0>() - dy_at<2, 0>()) + T(8) * (dy_at<1, 0>() - dy_at<-1, 0>());
    }
    __device__ __forceinline__ T dxz() const
    {
        return (dz_at<-2, 0>() - dz_at<2, 0>()) + T(8) * (dz_at<1, 0>() - dz_at<-1, 0>());
    }
    __device__ __forceinline__ T dyz() const
    {
        return (dz_at<0, -2>() - dz_at<0, 2>()) + T(8) * (dz_at<0, 1>() - dz_at<0, -1>());
    }
};

// (Delta_L d)_a at the thread's cell from three staged fields
template <typename T, int PAR>
__device__ __forceinline__ void deltaL_taps(const Taps<T, PAR> &F0, const Taps<T, PAR> &F1,
                                            const Taps<T, PAR> &F2, T h2, T m2, T out[3])
{
    const T c0 = F0.c(), c1 = F1.c(), c2 = F2.c();
    const T xx0 = F0.dxx(c0), yy1 = F1.dyy(c1), zz2 = F2.dzz(c2);
    const T l0 = (xx0 + F0.dyy(c0) + F0.dzz(c0)) * h2;
    const T l1 = (F1.dxx(c1) + yy1 + F1.dzz(c1)) * h2;
    const T l2 = (F2.dxx(c2) + F2.dyy(c2) + zz2) * h2;
    const T third = T(1) / T(3);
    const T t0 = xx0 * h2 + (F1.dxy() + F2.dxz()) * m2;
    const T t1 = yy1 * h2 + (F0.dxy() + F2.dyz()) * m2;
    const T t2 = zz2 * h2 + (F0.dxz() + F1.dyz()) * m2;
    out[0] = l0 + t0 * third;
    out[1] = l1 + t1 * third;
    out[2] = l2 + t2 * third;
}

// ---------------------------------------------------------------------------------------
// psi smoother colour pass on a brick.  For every (x, y) row a lane owns the z
// pair (z0 + 2 lane, z0 + 2 lane + 1): it updates the member of the active
// colour and copies the other, so no lane idles on the checkerboard.
// ---------------------------------------------------------------------------------------
template <int BC, typename T, int PAR>
__device__ __forceinline__ void psi_cell(const Geo &g, const T *lds_row, const T *__restrict__ r,
                                         const T *__restrict__ c, T *__restrict__ out, int x, int y, int z0,
                                         int lane, T h2, T dlap)
{
    Taps<T, PAR> D{lds_row + lane};
    const int za = z0 + 2 * lane + PAR, zb = z0 + 2 * lane + (PAR ^ 1);
    const int64_t qrow = ((int64_t)x * g.n + y) * g.n;
    const T v = D.c();
    const T cv = c[qrow + za];
    const T Ad = (D.dxx(v) + D.dyy(v) + D.dzz(v)) * h2 + cv * v;
    T diag;
    if constexpr (BC == kBcPeriodic)
        diag = dlap + cv;
    else
        diag = (T)(lap_diag_sum<BC>(g, x, y, za) * g.inv12h2) + cv;
    out[qrow + za] = v + (r[qrow + za] - Ad) / diag;
    out[qrow + zb] = D.template at<0, 0, (PAR ? -1 : 1)>();
}

template <int BC, typename T, int TX>
__global__ void __launch_bounds__(kTY *kLanes) k_pass_psi_tiled(Geo g, TileMap tm, const T *__restrict__ in,
                                                               T *__restrict__ out, const T *__restrict__ r,
                                                               const T *__restrict__ c, int colour)
{
    __shared__ T lds[TX + 4][kPY][kPZ];
    int x0, y0, z0;
    brick_of(tm, x0, y0, z0);
    const int ty = threadIdx.y, lane = threadIdx.x;
    const int y = y0 + ty;
    load_brick<BC, T, TX>(lds, Acc<BC, T>{in, g}, x0, y0, z0);
    __syncthreads();
    const T h2 = (T)g.inv12h2;
    const T dlap = (T)(-90.0 * g.inv12h2);
#pragma unroll
    for (int t = 0; t < TX; t++) {
        const int x = x0 + t;
        const T *row = &lds[t + 2][ty + 2][0];
        if (((colour + x + y + z0) & 1) == 0)
            psi_cell<BC, T, 0>(g, row, r, c, out, x, y, z0, lane, h2, dlap);
        else
            psi_cell<BC, T, 1>(g, row, r, c, out, x, y, z0, lane, h2, dlap);
    }
}

// ---------------------------------------------------------------------------------------
// W smoother colour pass (periodic) on a brick: three staged fields, same
// checkerboard lane mapping.
// ---------------------------------------------------------------------------------------
template <typename T, int PAR>
__device__ __forceinline__ void W_cell(const T *row0, const T *row1, const T *row2, const T *__restrict__ r,
                                       T *__restrict__ out, int64_t m, int64_t qrow, int z0, int lane, T h2, T m2,
                                       T diag)
{
    Taps<T, PAR> F0{row0 + lane}, F1{row1 + lane}, F2{row2 + lane};
    const int za = z0 + 2 * lane + PAR, zb = z0 + 2 * lane + (PAR ^ 1);
    T Ad[3];
    deltaL_taps<T, PAR>(F0, F1, F2, h2, m2, Ad);
    const int64_t qa = qrow + za, qb = qrow + zb;
    out[qa] = F0.c() + (r[qa] - Ad[0]) / diag;
    out[m + qa] = F1.c() + (r[m + qa] - Ad[1]) / diag;
    out[2 * m + qa] = F2.c() + (r[2 * m + qa] - Ad[2]) / diag;
    constexpr int DZ = PAR ? -1 : 1;
    out[qb] = F0.template at<0, 0, DZ>();
    out[m + qb] = F1.template at<0, 0, DZ>();
    out[2 * m + qb] = F2.template at<0, 0, DZ>();
}

template <typename T, int TX>
__global__ void __launch_bounds__(kTY *kLanes) k_pass_W_tiled(Geo g, TileMap tm, const T *__restrict__ in,
                                                             T *__restrict__ out, const T *__restrict__ r,
                                                             int colour)
{
    __shared__ T lds[3][TX + 4][kPY][kPZ];
    int x0, y0, z0;
    brick_of(tm, x0, y0, z0);
    const int n = g.n;
    const int64_t m = (int64_t)n * n * n;
    const int ty = threadIdx.y, lane = threadIdx.x;
    const int y = y0 + ty;
    load_brick<kBcPeriodic, T, TX>(lds[0], Acc<kBcPeriodic, T>{in, g}, x0, y0, z0);
    load_brick<kBcPeriodic, T, TX>(lds[1], Acc<kBcPeriodic, T>{in + m, g}, x0, y0, z0);
    load_brick<kBcPeriodic, T, TX>(lds[2], Acc<kBcPeriodic, T>{in + 2 * m, g}, x0, y0, z0);
    __syncthreads();
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2;
    const T diag = (T)(-100.0 * g.inv12h2);
#pragma unroll
    for (int t = 0; t < TX; t++) {
        const int x = x0 + t;
        const int64_t qrow = ((int64_t)x * n + y) * n;
        const T *r0 = &lds[0][t + 2][ty + 2][0], *r1 = &lds[1][t + 2][ty + 2][0], *r2 = &lds[2][t + 2][ty + 2][0];
        if (((colour + x + y + z0) & 1) == 0)
            W_cell<T, 0>(r0, r1, r2, r, out, m, qrow, z0, lane, h2, m2, diag);
        else
            W_cell<T, 1>(r0, r1, r2, r, out, m, qrow, z0, lane, h2, m2, diag);
    }
}

// Brick map for a level (tx == 0 when the level is not tiled).
template <int TX>
inline TileMap make_tilemap(int n)
{
    TileMap t{0, 0, 0, 0};
    if (n % kBZ != 0 || n % kTY != 0 || n % TX != 0) return t;
    t.nx = n / TX;
    t.ny = n / kTY;
    t.nz = n / kBZ;
    t.tx = TX;
    return t;
}

} // namespace grtmg
