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

// Stage brick + halo of one field.  A staged row (fixed x, y) holds the 66
// aligned z pairs (z0 - 2 + 2P, z0 - 1 + 2P), P = 0..65; pair P lands at
// words P (even z) and kHalf + P (odd z).  Every lane of wave w moves pair
// P = lane of rows w, w + kTY, ...; the two remaining pairs of every row are
// spread over the whole block.  All global loads are issued before any LDS
// store.  Offsets are 32-bit (fields up to 2^31 elements).
template <int BC, typename T, int TX>
__device__ __forceinline__ void load_brick(T (*s)[kPY][kPZ], const Acc<BC, T> &A, int x0, int y0, int z0)
{
    using V2 = typename Vec2<T>::type;
    constexpr int NROW = (TX + 4) * kPY;
    constexpr int RPW = NROW / kTY; // rows per wave
    static_assert(NROW % kTY == 0, "rows must divide among the waves");
    static_assert(2 * NROW <= kTY * kLanes, "one extra pair per thread at most");
    const int n = A.g.n;
    const int w = threadIdx.y, lane = threadIdx.x;
    const int tid = w * kLanes + lane;
    auto row_base = [&](int row, bool &inside) -> int {
        const int xg = x0 + row / kPY - 2, yg = y0 + row % kPY - 2;
        inside = (unsigned)xg < (unsigned)n && (unsigned)yg < (unsigned)n;
        return (wrap(xg, n) * n + wrap(yg, n)) * n;
    };
    auto pair_z = [&](int P) { return wrap(z0 - 2 + 2 * P, n); };
    V2 v[RPW];
#pragma unroll
    for (int i = 0; i < RPW; i++) {
        const int row = w + i * kTY;
        bool inside;
        const int base = row_base(row, inside);
        const int zp = pair_z(lane);
        if (BC == kBcPeriodic || (inside && z0 - 2 + 2 * lane >= 0)) {
            v[i] = *reinterpret_cast<const V2 *>(A.a + base + zp);
        } else {
            const int xg = x0 + row / kPY - 2, yg = y0 + row % kPY - 2;
            v[i].x = A(xg, yg, z0 - 2 + 2 * lane);
            v[i].y = A(xg, yg, z0 - 1 + 2 * lane);
        }
    }
    // extra pairs: thread tid < 2 NROW moves pair 64 + (tid & 1) of row tid / 2
    V2 e;
    const int erow = tid >> 1, ep = kLanes + (tid & 1);
    if (tid < 2 * NROW) {
        bool inside;
        const int base = row_base(erow, inside);
        if (BC == kBcPeriodic || (inside && z0 - 2 + 2 * ep + 1 < n)) {
            e = *reinterpret_cast<const V2 *>(A.a + base + pair_z(ep));
        } else {
            const int xg = x0 + erow / kPY - 2, yg = y0 + erow % kPY - 2;
            e.x = A(xg, yg, z0 - 2 + 2 * ep);
            e.y = A(xg, yg, z0 - 1 + 2 * ep);
        }
    }
#pragma unroll
    for (int i = 0; i < RPW; i++) {
        const int row = w + i * kTY;
        T *dst = s[row / kPY][row % kPY];
        dst[lane] = v[i].x;
        dst[kHalf + lane] = v[i].y;
    }
    if (tid < 2 * NROW) {
        T *dst = s[erow / kPY][erow % kPY];
        dst[ep] = e.x;
        dst[kHalf + ep] = e.y;
    }
}

// Compile-time LDS offset (words) of staged z index (2 lane + PAR + 2 + DZ)
// relative to word `lane` of a row (PAR: z parity of the evaluated cell).
template <int PAR, int DZ>
constexpr int zoff()
{
    return ((PAR + DZ) & 1) * kHalf + ((PAR + 2 + DZ) >> 1);
}

constexpr int kRow = kPZ;         // words between y rows
constexpr int kPlane = kPY * kPZ; // words between x planes

// Taps around the cell (x0 + TT, y0 + ty, .) of a staged field; b points at
// word lane of staged row (plane 0, row ty), so every offset is non-negative.
template <typename T, int PAR, int TT>
struct Taps {
    const T *b;
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T at() const
    {
        return b[(TT + 2 + DX) * kPlane + (2 + DY) * kRow + zoff<PAR, DZ>()];
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
template <typename T, int PAR, int TT>
__device__ __forceinline__ void deltaL_taps(const Taps<T, PAR, TT> &F0, const Taps<T, PAR, TT> &F1,
                                            const Taps<T, PAR, TT> &F2, T h2, T m2, T out[3])
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
template <int BC, typename T, int PAR, int TT>
__device__ __forceinline__ void psi_cell(const Geo &g, const T *row0, const T *__restrict__ r,
                                         const T *__restrict__ c, T *__restrict__ out, int x, int y, int z0,
                                         int lane, T h2, T dlap)
{
    Taps<T, PAR, TT> D{row0 + lane};
    const int za = z0 + 2 * lane + PAR, zb = z0 + 2 * lane + (PAR ^ 1);
    const int qrow = (x * g.n + y) * g.n;
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

template <int BC, typename T, int TX, int TT>
__device__ __forceinline__ void psi_cells(const Geo &g, const T *row0, const T *__restrict__ r,
                                          const T *__restrict__ c, T *__restrict__ out, int x0, int y, int z0,
                                          int lane, int colour, T h2, T dlap)
{
    if constexpr (TT < TX) {
        const int x = x0 + TT;
        if (((colour + x + y + z0) & 1) == 0)
            psi_cell<BC, T, 0, TT>(g, row0, r, c, out, x, y, z0, lane, h2, dlap);
        else
            psi_cell<BC, T, 1, TT>(g, row0, r, c, out, x, y, z0, lane, h2, dlap);
        psi_cells<BC, T, TX, TT + 1>(g, row0, r, c, out, x0, y, z0, lane, colour, h2, dlap);
    }
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
    load_brick<BC, T, TX>(lds, Acc<BC, T>{in, g}, x0, y0, z0);
    __syncthreads();
    const T h2 = (T)g.inv12h2;
    const T dlap = (T)(-90.0 * g.inv12h2);
    psi_cells<BC, T, TX, 0>(g, &lds[0][ty][0], r, c, out, x0, y0 + ty, z0, lane, colour, h2, dlap);
}

// ---------------------------------------------------------------------------------------
// W smoother colour pass (periodic) on a brick: three staged fields, same
// checkerboard lane mapping.
// ---------------------------------------------------------------------------------------
template <typename T, int PAR, int TT>
__device__ __forceinline__ void W_cell(const T *row0, const T *row1, const T *row2, const T *__restrict__ r,
                                       T *__restrict__ out, int m, int qrow, int z0, int lane, T h2, T m2,
                                       T inv_diag)
{
    Taps<T, PAR, TT> F0{row0 + lane}, F1{row1 + lane}, F2{row2 + lane};
    const int za = z0 + 2 * lane + PAR, zb = z0 + 2 * lane + (PAR ^ 1);
    T Ad[3];
    deltaL_taps<T, PAR, TT>(F0, F1, F2, h2, m2, Ad);
    const int qa = qrow + za, qb = qrow + zb;
    out[qa] = F0.c() + (r[qa] - Ad[0]) * inv_diag;
    out[m + qa] = F1.c() + (r[m + qa] - Ad[1]) * inv_diag;
    out[2 * m + qa] = F2.c() + (r[2 * m + qa] - Ad[2]) * inv_diag;
    constexpr int DZ = PAR ? -1 : 1;
    out[qb] = F0.template at<0, 0, DZ>();
    out[m + qb] = F1.template at<0, 0, DZ>();
    out[2 * m + qb] = F2.template at<0, 0, DZ>();
}

template <typename T, int TX, int TT>
__device__ __forceinline__ void W_cells(const T *row0, const T *row1, const T *row2, const T *__restrict__ r,
                                        T *__restrict__ out, int n, int x0, int y, int z0, int lane, int colour,
                                        T h2, T m2, T inv_diag)
{
    if constexpr (TT < TX) {
        const int x = x0 + TT;
        const int m = n * n * n, qrow = (x * n + y) * n;
        if (((colour + x + y + z0) & 1) == 0)
            W_cell<T, 0, TT>(row0, row1, row2, r, out, m, qrow, z0, lane, h2, m2, inv_diag);
        else
            W_cell<T, 1, TT>(row0, row1, row2, r, out, m, qrow, z0, lane, h2, m2, inv_diag);
        W_cells<T, TX, TT + 1>(row0, row1, row2, r, out, n, x0, y, z0, lane, colour, h2, m2, inv_diag);
    }
}

// The diagonal of Delta_L,h is the constant -100/(12 h^2); its reciprocal
// multiplies the defect.
template <typename T, int TX>
__global__ void __launch_bounds__(kTY *kLanes) k_pass_W_tiled(Geo g, TileMap tm, const T *__restrict__ in,
                                                             T *__restrict__ out, const T *__restrict__ r,
                                                             int colour)
{
    __shared__ T lds[3][TX + 4][kPY][kPZ];
    int x0, y0, z0;
    brick_of(tm, x0, y0, z0);
    const int n = g.n;
    const int m = n * n * n;
    const int ty = threadIdx.y, lane = threadIdx.x;
    load_brick<kBcPeriodic, T, TX>(lds[0], Acc<kBcPeriodic, T>{in, g}, x0, y0, z0);
    load_brick<kBcPeriodic, T, TX>(lds[1], Acc<kBcPeriodic, T>{in + m, g}, x0, y0, z0);
    load_brick<kBcPeriodic, T, TX>(lds[2], Acc<kBcPeriodic, T>{in + 2 * m, g}, x0, y0, z0);
    __syncthreads();
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2;
    const T inv_diag = (T)(1.0 / (-100.0 * g.inv12h2));
    W_cells<T, TX, 0>(&lds[0][0][ty][0], &lds[1][0][ty][0], &lds[2][0][ty][0], r, out, n, x0, y0 + ty, z0, lane,
                      colour, h2, m2, inv_diag);
}

// ---------------------------------------------------------------------------------------
// Residual on bricks of TX x 4 x 64 cells, one cell per lane per x plane (no
// colouring here).  The three W fields are staged in LDS (z contiguous, 2-cell
// halo); u is read through L1 (13 taps).  Outputs as k_residual.
// ---------------------------------------------------------------------------------------
constexpr int kRZ = 64;
constexpr int kRPZ = kRZ + 4;
constexpr int kRRow = kRPZ;
constexpr int kRPlane = kPY * kRPZ;

// Stage brick + halo of one field for the residual: a row holds z0 - 2 ..
// z0 + 65 at words 0..67; lanes move z0 - 2 + lane, the 4 remaining values of
// every row are spread over the block.
template <int BC, typename T, int TX>
__device__ __forceinline__ void load_rbrick(T (*s)[kPY][kRPZ], const Acc<BC, T> &A, int x0, int y0, int z0)
{
    constexpr int NROW = (TX + 4) * kPY;
    constexpr int RPW = NROW / kTY;
    static_assert(4 * NROW <= kTY * kLanes, "one extra value per thread at most");
    const int n = A.g.n;
    const int w = threadIdx.y, lane = threadIdx.x, tid = w * kLanes + lane;
    auto fetch = [&](int row, int zz) -> T {
        const int xg = x0 + row / kPY - 2, yg = y0 + row % kPY - 2, zg = z0 - 2 + zz;
        if (BC == kBcPeriodic)
            return A.a[(wrap(xg, n) * n + wrap(yg, n)) * n + wrap(zg, n)];
        return A(xg, yg, zg);
    };
    T v[RPW];
#pragma unroll
    for (int i = 0; i < RPW; i++) v[i] = fetch(w + i * kTY, lane);
    const int erow = tid >> 2, ez = kRZ + (tid & 3);
    T e = T(0);
    if (tid < 4 * NROW) e = fetch(erow, ez);
#pragma unroll
    for (int i = 0; i < RPW; i++) {
        const int row = w + i * kTY;
        s[row / kPY][row % kPY][lane] = v[i];
    }
    if (tid < 4 * NROW) s[erow / kPY][erow % kPY][ez] = e;
}

// 4th-order Laplacian sum of a periodic field at (x, y, z) with wrapped
// neighbour offsets (the centre value passed in).
__device__ __forceinline__ double lap_periodic(const double *__restrict__ a, int n, int x, int y, int z, double c)
{
    const int nn = n * n;
    const int q = (x * n + y) * n + z;
    auto off = [n](int i, int d, int stride) { // stride offset of coordinate i + d, wrapped
        const int j = i + d;
        return (j < 0 ? j + n : (j >= n ? j - n : j)) * stride - i * stride;
    };
    double s = -90.0 * c;
    s += 16.0 * (a[q + off(x, -1, nn)] + a[q + off(x, 1, nn)] + a[q + off(y, -1, n)] + a[q + off(y, 1, n)] +
                 a[q + off(z, -1, 1)] + a[q + off(z, 1, 1)]);
    s -= a[q + off(x, -2, nn)] + a[q + off(x, 2, nn)] + a[q + off(y, -2, n)] + a[q + off(y, 2, n)] +
         a[q + off(z, -2, 1)] + a[q + off(z, 2, 1)];
    return s;
}

template <typename T>
struct RTaps {
    const T *b; // word (xx, yy, lane + 2) of a staged field
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T at() const
    {
        return b[DX * kRPlane + DY * kRRow + DZ];
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
    template <int DY, int DZ>
    __device__ __forceinline__ T dx_at() const
    {
        return (at<-2, DY, DZ>() - at<2, DY, DZ>()) + T(8) * (at<1, DY, DZ>() - at<-1, DY, DZ>());
    }
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
    __device__ __forceinline__ T dx() const { return dx_at<0, 0>(); }
    __device__ __forceinline__ T dy() const { return dy_at<0, 0>(); }
    __device__ __forceinline__ T dz() const { return dz_at<0, 0>(); }
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

template <int BC, typename T, int TX, bool HAS_W>
__global__ void __launch_bounds__(kTY *kLanes) k_residual_tiled(Geo g, TileMap tm, ResArgs a)
{
    __shared__ double lds[HAS_W ? 3 : 1][TX + 4][kPY][kRPZ];
    const int total = tm.nx * tm.ny * tm.nz;
    int logical = blockIdx.x;
    if (total % kXCD == 0) logical = (blockIdx.x % kXCD) * (total / kXCD) + blockIdx.x / kXCD;
    const int bz = logical % tm.nz, rest = logical / tm.nz;
    const int x0 = (rest / tm.ny) * TX, y0 = (rest % tm.ny) * kTY, z0 = bz * kRZ;
    const int n = g.n;
    const int m = n * n * n;
    const int ty = threadIdx.y, lane = threadIdx.x;
    const int y = y0 + ty, z = z0 + lane;
    if constexpr (HAS_W) {
        load_rbrick<BC, double, TX>(lds[0], Acc<BC, double>{a.W, g}, x0, y0, z0);
        load_rbrick<BC, double, TX>(lds[1], Acc<BC, double>{a.W + m, g}, x0, y0, z0);
        load_rbrick<BC, double, TX>(lds[2], Acc<BC, double>{a.W + 2 * m, g}, x0, y0, z0);
        __syncthreads();
    }
    Acc<BC, double> U{a.u, g};
    const double K2 = a.K2;
    double hsum = 0.0, hmax = 0.0, msum = 0.0, mmax = 0.0;
#pragma unroll
    for (int t = 0; t < TX; t++) {
        const int x = x0 + t;
        const int q = (x * n + y) * n + z;
        const double uc = a.u[q];
        const double psi = psi0_at(g, a.pmass, x, y, z) + uc;
        double A2 = 0.0;
        double Mv[3] = {0.0, 0.0, 0.0};
        if constexpr (HAS_W) {
            const int off = ((t + 2) * kPY + (ty + 2)) * kRPZ + lane + 2;
            RTaps<double> F0{&lds[0][0][0][0] + off}, F1{&lds[1][0][0][0] + off}, F2{&lds[2][0][0][0] + off};
            double dW[3][3];
            dW[0][0] = F0.dx() * g.inv12h;
            dW[1][0] = F0.dy() * g.inv12h;
            dW[2][0] = F0.dz() * g.inv12h;
            dW[0][1] = F1.dx() * g.inv12h;
            dW[1][1] = F1.dy() * g.inv12h;
            dW[2][1] = F1.dz() * g.inv12h;
            dW[0][2] = F2.dx() * g.inv12h;
            dW[1][2] = F2.dy() * g.inv12h;
            dW[2][2] = F2.dz() * g.inv12h;
            const double div = dW[0][0] + dW[1][1] + dW[2][2];
#pragma unroll
            for (int p = 0; p < 3; p++)
#pragma unroll
                for (int s2 = 0; s2 < 3; s2++) {
                    const double Ab = dW[p][s2] + dW[s2][p] - (p == s2 ? 2.0 * div / 3.0 : 0.0);
                    A2 += Ab * Ab;
                }
            if (a.want_M) {
                const double c0 = F0.c(), c1 = F1.c(), c2 = F2.c();
                const double xx0 = F0.dxx(c0), yy1 = F1.dyy(c1), zz2 = F2.dzz(c2);
                const double l0 = (xx0 + F0.dyy(c0) + F0.dzz(c0)) * g.inv12h2;
                const double l1 = (F1.dxx(c1) + yy1 + F1.dzz(c1)) * g.inv12h2;
                const double l2 = (F2.dxx(c2) + F2.dyy(c2) + zz2) * g.inv12h2;
                const double t0 = xx0 * g.inv12h2 + (F1.dxy() + F2.dxz()) * g.inv144h2;
                const double t1 = yy1 * g.inv12h2 + (F0.dxy() + F2.dyz()) * g.inv144h2;
                const double t2 = zz2 * g.inv12h2 + (F0.dxz() + F1.dyz()) * g.inv144h2;
                Mv[0] = l0 + t0 / 3.0;
                Mv[1] = l1 + t1 / 3.0;
                Mv[2] = l2 + t2 / 3.0;
            }
        }
        if (a.want_M && a.S) {
            const double p2 = psi * psi;
            const double w6 = a.conformal ? 1.0 : p2 * p2 * p2;
#pragma unroll
            for (int s2 = 0; s2 < 3; s2++) Mv[s2] -= 8.0 * kPi * w6 * a.S[s2 * m + q] - a.meanS[s2];
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
        double lu;
        if constexpr (BC == kBcPeriodic)
            lu = lap_periodic(a.u, n, x, y, z, uc);
        else
            lu = lap_sum<double>(U, x, y, z, uc);
        double H = lu * g.inv12h2 + matter - (K2 / 12.0) * psi5 + 0.125 * A2 * ipsi7;
        if (a.f) H += a.f[q];
        const double cc = dmatter - (5.0 * K2 / 12.0) * psi4 - 0.875 * A2 * ipsi8;
        if (a.H) a.H[q] = H;
        if (a.c) a.c[q] = cc;
        if (a.r) ((T *)a.r)[q] = (T)(-H);
        if (a.rc) ((T *)a.rc)[q] = (T)cc;
        if (a.want_M) {
            if (a.M) {
                a.M[q] = Mv[0];
                a.M[m + q] = Mv[1];
                a.M[2 * m + q] = Mv[2];
            }
            if (a.rW) {
                ((T *)a.rW)[q] = (T)(-Mv[0]);
                ((T *)a.rW)[m + q] = (T)(-Mv[1]);
                ((T *)a.rW)[2 * m + q] = (T)(-Mv[2]);
            }
            const double m2 = Mv[0] * Mv[0] + Mv[1] * Mv[1] + Mv[2] * Mv[2];
            msum += m2;
            mmax = fmax(mmax, sqrt(m2));
        }
        hsum += H * H;
        hmax = fmax(hmax, fabs(H));
    }
    if (a.partials) {
        double v[4] = {hsum, hmax, msum, mmax};
        // 256 threads per block, as block_reduce_store assumes
        block_reduce_store<4>(v, 0xAu, a.partials + 4 * (int64_t)blockIdx.x);
    }
}

template <int TX>
inline TileMap make_rtilemap(int n)
{
    TileMap t{0, 0, 0, 0};
    if (n % kRZ != 0 || n % kTY != 0 || n % TX != 0 || n < 64) return t;
    t.nx = n / TX;
    t.ny = n / kTY;
    t.nz = n / kRZ;
    t.tx = TX;
    return t;
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
