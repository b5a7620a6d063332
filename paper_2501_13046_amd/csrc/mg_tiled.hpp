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

#include <type_traits>
#include <utility>

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

// ---------------------------------------------------------------------------------------
// Periodic trilinear prolongation for a z pair of fine cells (2K, 2K + 1):
// both share coarse z K and their coarse x and y neighbours, and take coarse z
// K - 1 and K + 1 respectively, so a pair reads 12 coarse values instead of
// 16 and updates its two fine values with one vector load and store.  Each
// value is prolong_cell's expression.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_add_pairs(Geo gc, const T *__restrict__ coarse,
                                                             T *__restrict__ fine, int ncomp)
{
    coarse = zsh(coarse, gc.zs);
    fine = zsh(fine, gc.zs);
    using V2 = typename Vec2<T>::type;
    const int nc = gc.n, nf = 2 * nc;
    const unsigned pairs = (unsigned)nf * nf * nc;
    const unsigned t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= pairs) return;
    const unsigned row = t / (unsigned)nc;
    const int K = (int)(t - row * (unsigned)nc);
    const int i = (int)(row / (unsigned)nf), j = (int)(row - (unsigned)i * nf);
    const int I = i >> 1, J = j >> 1;
    const int I1 = wrap((i & 1) ? I + 1 : I - 1, nc), J1 = wrap((j & 1) ? J + 1 : J - 1, nc);
    const int Km = wrap(K - 1, nc), Kp = wrap(K + 1, nc);
    const T a = T(0.75), b = T(0.25);
    const size_t mf = (size_t)nf * nf * nf, mc = (size_t)nc * nc * nc;
    const unsigned r00 = ((unsigned)I * nc + J) * nc, r01 = ((unsigned)I * nc + J1) * nc;
    const unsigned r10 = ((unsigned)I1 * nc + J) * nc, r11 = ((unsigned)I1 * nc + J1) * nc;
    for (int s = 0; s < ncomp; s++) {
        const T *C = coarse + s * mc;
        const T c00 = C[r00 + K], c01 = C[r01 + K], c10 = C[r10 + K], c11 = C[r11 + K];
        const T m00 = C[r00 + Km], m01 = C[r01 + Km], m10 = C[r10 + Km], m11 = C[r11 + Km];
        const T p00 = C[r00 + Kp], p01 = C[r01 + Kp], p10 = C[r10 + Kp], p11 = C[r11 + Kp];
        const T v0 = a * (a * (a * c00 + b * m00) + b * (a * c01 + b * m01)) +
                     b * (a * (a * c10 + b * m10) + b * (a * c11 + b * m11));
        const T v1 = a * (a * (a * c00 + b * p00) + b * (a * c01 + b * p01)) +
                     b * (a * (a * c10 + b * p10) + b * (a * c11 + b * p11));
        V2 *F = reinterpret_cast<V2 *>(fine + s * mf + ((size_t)i * nf + j) * nf + 2 * K);
        V2 f = *F;
        f.x += v0;
        f.y += v1;
        *F = f;
    }
}

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
    static constexpr bool kOrdered = true;
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
        diag = pinned((T)(lap_diag_sum<BC>(g, x, y, za) * g.inv12h2)) + cv;
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
    in = zsh(in, g.zs);
    out = zsh(out, g.zs);
    r = zsh(r, g.zs);
    c = zsh(c, g.zs);
    __shared__ T lds[TX + 4][kPY][kPZ];
    int x0, y0, z0;
    brick_of(tm, x0, y0, z0);
    const int ty = threadIdx.y, lane = threadIdx.x;
    load_brick<BC, T, TX>(lds, Acc<BC, T>{in, g}, x0, y0, z0);
    __syncthreads();
    const T h2 = (T)g.inv12h2;
    const T dlap = pinned((T)(-90.0 * g.inv12h2));
    psi_cells<BC, T, TX, 0>(g, &lds[0][ty][0], r, c, out, x0, y0 + ty, z0, lane, colour, h2, dlap);
}

// ---------------------------------------------------------------------------------------
// W smoother colour pass (periodic) on a brick, one field at a time.  The
// three components are staged through two LDS buffers of one field each: the
// global loads of field f + 1 are in flight while the lanes evaluate the taps
// of field f, and a brick needs a third of the LDS of staging all three fields
// at once (more workgroups per CU).  The contributions of each field to the
// three rows of Delta_L are accumulated in registers:
//   field 0: Laplacian row 0, D_xx (row 0), D_xy (row 1), D_xz (row 2)
//   field 1: Laplacian row 1, D_yy (row 1), D_xy (row 0), D_yz (row 2)
//   field 2: Laplacian row 2, D_zz (row 2), D_xz (row 0), D_yz (row 1)
// Same lane mapping as the psi pass: the lane owning a z pair updates the
// member of the active colour and copies the other.
// ---------------------------------------------------------------------------------------

// Staging rows of one periodic field, held in registers between the global
// loads and the LDS stores.  Pair layout as in load_brick.
template <typename T, int TX>
struct BrickRegs {
    using V2 = typename Vec2<T>::type;
    static constexpr int NROW = (TX + 4) * kPY;
    static constexpr int RPW = NROW / kTY;
    static_assert(NROW % kTY == 0 && 2 * NROW <= kTY * kLanes, "staging rows must spread over the block");
    static_assert(kPY == 2 * kTY, "each wave stages two y rows of every x plane");
    V2 v[RPW];
    V2 e;
    __device__ __forceinline__ void fetch(const T *__restrict__ a, int n, int x0, int y0, int z0)
    {
        const int w = threadIdx.y, lane = threadIdx.x, tid = w * kLanes + lane;
        auto row_off = [&](int row) -> unsigned {
            return (unsigned)(wrap(x0 + row / kPY - 2, n) * n + wrap(y0 + row % kPY - 2, n)) * (unsigned)n;
        };
        const unsigned zp = (unsigned)wrap(z0 - 2 + 2 * lane, n);
        // row w + 4 i is y row w + 4 (i & 1) of x plane i / 2 (uniform x wrap)
        const unsigned yw[2] = {(unsigned)wrap(y0 + w - 2, n), (unsigned)wrap(y0 + w + 2, n)};
#pragma unroll
        for (int i = 0; i < RPW; i++)
            v[i] = *reinterpret_cast<const V2 *>(
                reinterpret_cast<const char *>(a) +
                (((unsigned)wrap(x0 + i / 2 - 2, n) * (unsigned)n + yw[i & 1]) * (unsigned)n + zp) * (unsigned)sizeof(T));
        if (tid < 2 * NROW) {
            const int erow = tid >> 1, ep = kLanes + (tid & 1);
            const unsigned ze = (unsigned)wrap(z0 - 2 + 2 * ep, n);
            e = *reinterpret_cast<const V2 *>(reinterpret_cast<const char *>(a) +
                                              (row_off(erow) + ze) * (unsigned)sizeof(T));
        }
    }
    __device__ __forceinline__ void store(T (*s)[kPY][kPZ]) const
    {
        const int w = threadIdx.y, lane = threadIdx.x, tid = w * kLanes + lane;
#pragma unroll
        for (int i = 0; i < RPW; i++) {
            const int row = w + i * kTY;
            T *dst = s[row / kPY][row % kPY];
            dst[lane] = v[i].x;
            dst[kHalf + lane] = v[i].y;
        }
        if (tid < 2 * NROW) {
            const int erow = tid >> 1, ep = kLanes + (tid & 1);
            T *dst = s[erow / kPY][erow % kPY];
            dst[ep] = e.x;
            dst[kHalf + ep] = e.y;
        }
    }
};

// Per-cell partial sums of the W pass: Laplacian rows (times 1/(12 h^2)), the
// diagonal second derivatives (times 1/(12 h^2)), the mixed-derivative sums of
// each row, the centre values.
// W_field_parts, and the other member of the z pair copied to out.
template <typename T, int F, int PAR, typename Src>
__device__ __forceinline__ void W_field_taps(const Src &S, T *__restrict__ out, unsigned qb, T h2, WPart<T> &P)
{
    elt(out, qb) = W_field_parts<T, F, PAR>(S, h2, P);
}

template <typename T, int F, int PAR, int TT>
__device__ __forceinline__ void W_field_cell(const T *row0, T *__restrict__ out, unsigned qb, T h2, WPart<T> &P)
{
    W_field_taps<T, F, PAR>(Taps<T, PAR, TT>{row0}, out, qb, h2, P);
}

// Contributions of field F to every cell of the thread; P0 is the parity of
// the active member of the thread's z pair at x = x0 (it alternates with x).
template <typename T, int TX, int F, int P0>
__device__ __forceinline__ void W_field(const T *row0, T *__restrict__ outF, const unsigned *qb, T h2, WPart<T> *P)
{
    static_for<TX>([&](auto tt) {
        constexpr int TT = decltype(tt)::value;
        W_field_cell<T, F, P0 ^ (TT & 1), TT>(row0, outF, qb[TT], h2, P[TT]);
    });
}

// The diagonal of Delta_L,h is the constant -100/(12 h^2); its reciprocal
// multiplies the defect.
template <typename T, int TX>
__global__ void __launch_bounds__(kTY *kLanes) k_pass_W_tiled(Geo g, TileMap tm, const T *__restrict__ in,
                                                             T *__restrict__ out, const T *__restrict__ r,
                                                             int colour)
{
    in = zsh(in, g.zs);
    out = zsh(out, g.zs);
    r = zsh(r, g.zs);
    __shared__ T lds[2][TX + 4][kPY][kPZ];
    int x0, y0, z0;
    brick_of(tm, x0, y0, z0);
    const int n = g.n;
    const unsigned m = (unsigned)n * n * n;
    const int ty = threadIdx.y, lane = threadIdx.x;
    const int y = y0 + ty;
    const int p0 = (colour + x0 + y + z0) & 1;
    // flat indices of the active (qa) and copied (qb) member of the pair at each x
    unsigned qa[TX], qb[TX];
#pragma unroll
    for (int t = 0; t < TX; t++) {
        const unsigned row = (unsigned)((x0 + t) * n + y) * (unsigned)n + (unsigned)(z0 + 2 * lane);
        const unsigned pa = (unsigned)(p0 ^ (t & 1));
        qa[t] = row + pa;
        qb[t] = row + (pa ^ 1u);
    }
    BrickRegs<T, TX> st;
    st.fetch(in, n, x0, y0, z0);
    // 32-bit byte offsets from uniform per-component pointers (one address VGPR per access)
    const T *rf[3] = {r, r + m, r + 2 * (size_t)m};
    T *of[3] = {out, out + m, out + 2 * (size_t)m};
    T rv[3][TX];
#pragma unroll
    for (int f = 0; f < 3; f++)
#pragma unroll
        for (int t = 0; t < TX; t++)
            rv[f][t] = *reinterpret_cast<const T *>(reinterpret_cast<const char *>(rf[f]) + qa[t] * (unsigned)sizeof(T));
    st.store(lds[0]);
    __syncthreads();
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2;
    const T inv_diag = (T)(1.0 / (-100.0 * g.inv12h2));
    const T third = T(1) / T(3);
    WPart<T> P[TX];
    const T *b0 = &lds[0][0][ty][0] + lane, *b1 = &lds[1][0][ty][0] + lane;

    st.fetch(in + m, n, x0, y0, z0);
    if (p0) W_field<T, TX, 0, 1>(b0, of[0], qb, h2, P);
    else W_field<T, TX, 0, 0>(b0, of[0], qb, h2, P);
    st.store(lds[1]);
    __syncthreads();

    st.fetch(in + 2 * (size_t)m, n, x0, y0, z0);
    if (p0) W_field<T, TX, 1, 1>(b1, of[1], qb, h2, P);
    else W_field<T, TX, 1, 0>(b1, of[1], qb, h2, P);
    st.store(lds[0]); // every lane finished reading field 0 before the barrier above
    __syncthreads();

    if (p0) W_field<T, TX, 2, 1>(b0, of[2], qb, h2, P);
    else W_field<T, TX, 2, 0>(b0, of[2], qb, h2, P);

#pragma unroll
    for (int t = 0; t < TX; t++)
#pragma unroll
        for (int f = 0; f < 3; f++) {
            const T Ad = P[t].lap[f] + (P[t].dd[f] + P[t].mix[f] * m2) * third;
            *reinterpret_cast<T *>(reinterpret_cast<char *>(of[f]) + qa[t] * (unsigned)sizeof(T)) =
                P[t].c[f] + (rv[f][t] - Ad) * inv_diag;
        }
}

// ---------------------------------------------------------------------------------------
// W smoother colour pass marching along x.  A workgroup owns a column of TYB (y)
// x BZ (z) cells and LX consecutive x planes (BZ = 128: one brick row per wave,
// 4 rows; BZ = 64: two rows per wave, 32 lanes each, 8 rows).  The three
// components of each staged x plane (rows y0 - 2 .. y0 + TYB + 1, z0 - 2 ..
// z0 + BZ + 1, the pair layout of the bricks) live in a ring of six LDS
// slots: while the lanes evaluate plane x from the slots of x - 2 .. x + 2,
// the registers hold plane x + 4 in flight from HBM and plane x + 3 is
// written into the slot that plane x - 3 vacated, so global loads, LDS
// traffic and arithmetic overlap for the whole column and each staged plane
// is loaded once per column (x halo amortised over LX).
// ---------------------------------------------------------------------------------------
constexpr int kRing = 6;

template <int BZ>
struct ZGeom {
    static_assert(BZ == 128 || BZ == 64, "brick rows of 128 or 64 cells");
    static constexpr int kRPW = 128 / BZ;       // brick rows per wave
    static constexpr int kLPR = BZ / 2;         // lanes (z pairs) per row
    static constexpr int kTYB = kTY * kRPW;     // brick rows (y) per workgroup
    static constexpr int kPYB = kTYB + 4;       // staged rows per component
    static constexpr int kPZB = BZ + 4;         // staged words per row
    static constexpr int kHalfB = kPZB / 2;     // odd z start here
    static constexpr int kPlaneB = kPYB * kPZB; // one component of a staged plane
    static constexpr int kNR = 3 * kPYB;        // staged rows of a plane
    // LDS word of staged z index (2 p + PAR + 2 + DZ) relative to word p of a row
    template <int PAR, int DZ>
    static constexpr int zoff()
    {
        return ((PAR + DZ) & 1) * kHalfB + ((PAR + 2 + DZ) >> 1);
    }
    __device__ static int row() { return threadIdx.y * kRPW + (int)threadIdx.x / kLPR; }
    __device__ static int pair() { return (int)threadIdx.x % kLPR; }
};

template <int BZ>
__device__ __forceinline__ void column_of(const TileMap &t, int &x0, int &y0, int &z0)
{
    const int total = t.nx * t.ny * t.nz;
    const int b = blockIdx.x;
    int logical = b;
    if (total % kXCD == 0) logical = (b % kXCD) * (total / kXCD) + b / kXCD;
    const int bz = logical % t.nz;
    const int rest = logical / t.nz;
    x0 = (rest / t.ny) * t.tx;
    y0 = (rest % t.ny) * ZGeom<BZ>::kTYB;
    z0 = bz * BZ;
}

// One staged x plane of the three components (kNR rows of kLPR + 2 pairs):
// load i of a thread moves main pair p of row i kTYB + (its brick row), threads
// tid < 2 kNR the two remaining pairs of row tid / 2.
template <typename T, int BZ>
struct PlaneRegs {
    using G = ZGeom<BZ>;
    using V2 = typename Vec2<T>::type;
    static constexpr int NL = (G::kNR + G::kTYB - 1) / G::kTYB;
    static_assert(2 * G::kNR <= kTY * kLanes, "extra pairs must spread over the block");
    V2 v[NL];
    V2 e;
    __device__ __forceinline__ void fetch(const T *__restrict__ in, unsigned m, int n, int x, int y0, int z0)
    {
        const int tid = threadIdx.y * kLanes + threadIdx.x, ty = G::row(), p = G::pair();
        const unsigned xo = (unsigned)wrap(x, n) * (unsigned)n;
        const unsigned zp = (unsigned)wrap(z0 - 2 + 2 * p, n);
#pragma unroll
        for (int i = 0; i < NL; i++) {
            const int row = i * G::kTYB + ty;
            if (G::kNR % G::kTYB == 0 || row < G::kNR) {
                const int f = row / G::kPYB, yr = row - f * G::kPYB;
                const unsigned off = (xo + (unsigned)wrap(y0 + yr - 2, n)) * (unsigned)n + zp;
                v[i] = elt(reinterpret_cast<const V2 *>(in + (size_t)f * m), off >> 1);
            }
        }
        if (tid < 2 * G::kNR) {
            const int erow = tid >> 1, ep = G::kLPR + (tid & 1);
            const int f = erow / G::kPYB, yr = erow - f * G::kPYB;
            const unsigned off = (xo + (unsigned)wrap(y0 + yr - 2, n)) * (unsigned)n + (unsigned)wrap(z0 - 2 + 2 * ep, n);
            e = elt(reinterpret_cast<const V2 *>(in + (size_t)f * m), off >> 1);
        }
    }
    __device__ __forceinline__ void store(T (*s)[G::kPZB]) const // s: the staged rows of one slot
    {
        const int tid = threadIdx.y * kLanes + threadIdx.x, ty = G::row(), p = G::pair();
#pragma unroll
        for (int i = 0; i < NL; i++) {
            const int row = i * G::kTYB + ty;
            if (G::kNR % G::kTYB == 0 || row < G::kNR) {
                s[row][p] = v[i].x;
                s[row][G::kHalfB + p] = v[i].y;
            }
        }
        if (tid < 2 * G::kNR) {
            const int erow = tid >> 1, ep = G::kLPR + (tid & 1);
            s[erow][ep] = e.x;
            s[erow][G::kHalfB + ep] = e.y;
        }
    }
};

// Ring prologue of a marched column: planes x0 - 2 .. x0 + 2 into slots 0..4,
// plane x0 + 3 left in st; all six fetches are issued before the first store.
template <typename T, int BZ>
__device__ __forceinline__ void march_prologue(T (*lds)[ZGeom<BZ>::kNR][ZGeom<BZ>::kPZB], PlaneRegs<T, BZ> &st,
                                               const T *__restrict__ in, unsigned m, int n, int x0, int y0, int z0,
                                               bool fetch_next = true)
{
    PlaneRegs<T, BZ> w[5];
#pragma unroll
    for (int j = 0; j < 5; j++) w[j].fetch(in, m, n, x0 - 2 + j, y0, z0);
    if (fetch_next) st.fetch(in, m, n, x0 + 3, y0, z0); // a column of one plane needs no sixth
#pragma unroll
    for (int j = 0; j < 5; j++) w[j].store(lds[j]);
}

// Taps of component F around the thread's cell: pb[DX + 2] is word p of the
// thread's staged row of the slot holding plane x + DX.
template <typename T, int PAR, int F, int BZ>
struct RingTaps {
    using G = ZGeom<BZ>;
    static constexpr bool kOrdered = true;
    const T *const *pb;
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T at() const
    {
        return pb[DX + 2][F * G::kPlaneB + (2 + DY) * G::kPZB + G::template zoff<PAR, DZ>()];
    }
};

template <typename T, int PAR, int BZ>
__device__ __forceinline__ void W_march_cell(const T *const *pb, T *const *of, unsigned qb, T h2, WPart<T> &P)
{
    W_field_taps<T, 0, PAR>(RingTaps<T, PAR, 0, BZ>{pb}, of[0], qb, h2, P);
    W_field_taps<T, 1, PAR>(RingTaps<T, PAR, 1, BZ>{pb}, of[1], qb, h2, P);
    W_field_taps<T, 2, PAR>(RingTaps<T, PAR, 2, BZ>{pb}, of[2], qb, h2, P);
}

template <typename T, int LX, int BZ>
__global__ void __launch_bounds__(kTY *kLanes) k_pass_W_march(Geo g, TileMap tm, const T *__restrict__ in,
                                                             T *__restrict__ out, const T *__restrict__ r,
                                                             int colour)
{
    in = zsh(in, g.zs);
    out = zsh(out, g.zs);
    r = zsh(r, g.zs);
    using G = ZGeom<BZ>;
    __shared__ T lds[kRing][G::kNR][G::kPZB];
    int x0, y0, z0;
    column_of<BZ>(tm, x0, y0, z0);
    const int n = g.n;
    const unsigned m = (unsigned)n * n * n;
    const int ty = G::row(), p = G::pair();
    const int y = y0 + ty;
    const T *rf[3] = {r, r + m, r + 2 * (size_t)m};
    T *of[3] = {out, out + m, out + 2 * (size_t)m};
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2;
    const T inv_diag = (T)(1.0 / (-100.0 * g.inv12h2));
    const T third = T(1) / T(3);

    // staged plane j (0 .. LX + 3) is x = x0 - 2 + j, in slot j % kRing; the
    // first six planes are all in flight at once
    PlaneRegs<T, BZ> st;
    march_prologue<T, BZ>(lds, st, in, m, n, x0, y0, z0, LX > 1);
    auto row_of = [&](int x) { return (unsigned)(x * n + y) * (unsigned)n + (unsigned)(z0 + 2 * p); };
    auto par_of = [&](int x) { return (unsigned)((colour + x + y + z0) & 1); };
    T rv[3];
#pragma unroll
    for (int f = 0; f < 3; f++) rv[f] = elt(rf[f], row_of(x0) + par_of(x0));
    __syncthreads();

#pragma unroll 1
    for (int k = 0; k < LX; k++) {
        const int x = x0 + k;
        const unsigned pa = par_of(x);
        const unsigned qa = row_of(x) + pa, qb = row_of(x) + (pa ^ 1u);
        const T *pb[5];
#pragma unroll
        for (int d = 0; d < 5; d++) pb[d] = &lds[(k + d) % kRing][ty][p];
        T rn[3] = {T(0), T(0), T(0)};
        if (k + 1 < LX) { // r of the next plane's active cells
            const unsigned qn = row_of(x + 1) + (pa ^ 1u);
#pragma unroll
            for (int f = 0; f < 3; f++) rn[f] = elt(rf[f], qn);
        }
        WPart<T> P;
        if (pa) W_march_cell<T, 1, BZ>(pb, of, qb, h2, P);
        else W_march_cell<T, 0, BZ>(pb, of, qb, h2, P);
#pragma unroll
        for (int f = 0; f < 3; f++) {
            const T Ad = P.lap[f] + (P.dd[f] + P.mix[f] * m2) * third;
            elt(of[f], qa) = P.c[f] + (rv[f] - Ad) * inv_diag;
            rv[f] = rn[f];
        }
        if (k + 5 <= LX + 3) { // plane x + 3 into the slot plane x - 3 left
            st.store(lds[(k + 5) % kRing]);
            if (k + 6 <= LX + 3) st.fetch(in, m, n, x + 4, y0, z0);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// W defect r - Delta_L d and its restriction (mean of the 8 children) to the
// next coarser level, marching along x like k_pass_W_march.  Each lane
// evaluates both members of its z pair on two consecutive x planes; the
// paired y rows (brick rows 2 w' and 2 w' + 1) are added through LDS and the
// even row writes one coarse cell per lane (coarse z = z0 / 2 + p, coalesced).
// ---------------------------------------------------------------------------------------
template <typename T, int PAR, int BZ>
__device__ __forceinline__ void W_defect_cell(const T *const *pb, const T (&rv)[3], T h2, T m2, T third, T (&acc)[3])
{
    WPart<T> P;
    W_field_parts<T, 0, PAR>(RingTaps<T, PAR, 0, BZ>{pb}, h2, P);
    W_field_parts<T, 1, PAR>(RingTaps<T, PAR, 1, BZ>{pb}, h2, P);
    W_field_parts<T, 2, PAR>(RingTaps<T, PAR, 2, BZ>{pb}, h2, P);
#pragma unroll
    for (int f = 0; f < 3; f++) acc[f] += rv[f] - (P.lap[f] + (P.dd[f] + P.mix[f] * m2) * third);
}

template <typename T, int LX, int BZ>
__global__ void __launch_bounds__(kTY *kLanes) k_defect_restrict_W_march(Geo g, TileMap tm, const T *__restrict__ d,
                                                                        const T *__restrict__ r,
                                                                        T *__restrict__ rc_out, T *__restrict__ d1_out,
                                                                        T idiag_c)
{
    d = zsh(d, g.zs);
    r = zsh(r, g.zs);
    rc_out = zsh(rc_out, g.zs);
    d1_out = zsh(d1_out, g.zs);
    using G = ZGeom<BZ>;
    static_assert(LX % 2 == 0 && G::kTYB % 2 == 0, "whole coarse cells per column");
    using V2 = typename Vec2<T>::type;
    __shared__ T lds[kRing][G::kNR][G::kPZB];
    __shared__ T red[3][G::kTYB / 2][G::kLPR];
    int x0, y0, z0;
    column_of<BZ>(tm, x0, y0, z0);
    const int n = g.n, nc = n / 2;
    const unsigned m = (unsigned)n * n * n, mc = (unsigned)nc * nc * nc;
    const int ty = G::row(), p = G::pair();
    const int y = y0 + ty;
    const T *rf[3] = {r, r + m, r + 2 * (size_t)m};
    const T h2 = (T)g.inv12h2, m2 = (T)g.inv144h2;
    const T third = T(1) / T(3);

    PlaneRegs<T, BZ> st;
    march_prologue<T, BZ>(lds, st, d, m, n, x0, y0, z0);
    auto pair_at = [&](int x) { return (unsigned)(x * n + y) * (unsigned)n + (unsigned)(z0 + 2 * p); };
    V2 rv[3];
#pragma unroll
    for (int f = 0; f < 3; f++) rv[f] = elt(reinterpret_cast<const V2 *>(rf[f]), pair_at(x0) >> 1);
    __syncthreads();

    T acc[3] = {T(0), T(0), T(0)};
#pragma unroll 1
    for (int k = 0; k < LX; k++) {
        const int x = x0 + k;
        const T *pb[5];
#pragma unroll
        for (int dd = 0; dd < 5; dd++) pb[dd] = &lds[(k + dd) % kRing][ty][p];
        V2 rn[3];
        if (k + 1 < LX) {
#pragma unroll
            for (int f = 0; f < 3; f++) rn[f] = elt(reinterpret_cast<const V2 *>(rf[f]), pair_at(x + 1) >> 1);
        }
        const T ra[3] = {rv[0].x, rv[1].x, rv[2].x}, rb[3] = {rv[0].y, rv[1].y, rv[2].y};
        W_defect_cell<T, 0, BZ>(pb, ra, h2, m2, third, acc);
        W_defect_cell<T, 1, BZ>(pb, rb, h2, m2, third, acc);
        if ((k & 1) && (ty & 1)) {
#pragma unroll
            for (int f = 0; f < 3; f++) red[f][ty >> 1][p] = acc[f];
        }
        if (k + 5 <= LX + 3) {
            st.store(lds[(k + 5) % kRing]);
            if (k + 6 <= LX + 3) st.fetch(d, m, n, x + 4, y0, z0);
        }
        __syncthreads();
        if (k & 1) {
            if (!(ty & 1)) {
                const unsigned qc = ((unsigned)(x >> 1) * (unsigned)nc + (unsigned)(y >> 1)) * (unsigned)nc +
                                    (unsigned)((z0 >> 1) + p);
                const bool first = (((x >> 1) + (y >> 1) + (z0 >> 1) + p) & 1) == 0;
#pragma unroll
                for (int f = 0; f < 3; f++) {
                    const T v = (acc[f] + red[f][ty >> 1][p]) * T(0.125);
                    elt(rc_out + (size_t)f * mc, qc) = v;
                    if (d1_out) elt(d1_out + (size_t)f * mc, qc) = first ? v * idiag_c : T(0);
                }
            }
#pragma unroll
            for (int f = 0; f < 3; f++) acc[f] = T(0);
        }
        if (k + 1 < LX) {
#pragma unroll
            for (int f = 0; f < 3; f++) rv[f] = rn[f];
        }
    }
}

// Column map of the marched kernels (tx == 0: the level does not fit).
template <int LX, int BZ>
inline TileMap make_marchmap(int n)
{
    TileMap t{0, 0, 0, 0};
    constexpr int TYB = ZGeom<BZ>::kTYB;
    if (n % BZ != 0 || n % TYB != 0 || n % LX != 0) return t;
    t.nx = n / LX;
    t.ny = n / TYB;
    t.nz = n / BZ;
    t.tx = LX;
    return t;
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
    static_assert(kPY == 2 * kTY, "each wave stages two y rows of every x plane");
    const int n = A.g.n;
    const int w = threadIdx.y, lane = threadIdx.x, tid = w * kLanes + lane;
    auto fetch = [&](int row, int zz) -> T {
        const int xg = x0 + row / kPY - 2, yg = y0 + row % kPY - 2, zg = z0 - 2 + zz;
        if (BC == kBcPeriodic)
            return elt(A.a, ((unsigned)wrap(xg, n) * (unsigned)n + (unsigned)wrap(yg, n)) * (unsigned)n +
                                (unsigned)wrap(zg, n));
        return A(xg, yg, zg);
    };
    T v[RPW];
    if constexpr (BC == kBcPeriodic) {
        // row w + 4 i of the block is y row w + 4 (i & 1) of x plane i / 2: the x
        // wrap is uniform, the y and z wraps are two and one per thread
        const unsigned un = (unsigned)n, zw = (unsigned)wrap(z0 - 2 + lane, n);
        const unsigned yw[2] = {(unsigned)wrap(y0 + w - 2, n), (unsigned)wrap(y0 + w + 2, n)};
#pragma unroll
        for (int i = 0; i < RPW; i++)
            v[i] = elt(A.a, ((unsigned)wrap(x0 + i / 2 - 2, n) * un + yw[i & 1]) * un + zw);
    } else {
#pragma unroll
        for (int i = 0; i < RPW; i++) v[i] = fetch(w + i * kTY, lane);
    }
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
// neighbour indices (the centre value passed in).
__device__ __forceinline__ double lap_periodic(const double *__restrict__ a, int n, int x, int y, int z, double c)
{
    const unsigned un = (unsigned)n, nn = un * un;
    const unsigned q = ((unsigned)x * un + (unsigned)y) * un + (unsigned)z;
    auto at = [&](int i, int d, unsigned stride) { // value at coordinate i + d (wrapped) along one axis
        const int j = i + d;
        const int w = j < 0 ? j + n : (j >= n ? j - n : j);
        return elt(a, q + (unsigned)w * stride - (unsigned)i * stride);
    };
    double s = -90.0 * c;
    s += 16.0 * (at(x, -1, nn) + at(x, 1, nn) + at(y, -1, un) + at(y, 1, un) + at(z, -1, 1u) + at(z, 1, 1u));
    s -= at(x, -2, nn) + at(x, 2, nn) + at(y, -2, un) + at(y, 2, un) + at(z, -2, 1u) + at(z, 2, 1u);
    return s;
}

// Taps of a residual brick field relative to the staged word of the stencil
// corner (x - 2, y - 2, z - 2): every offset is non-negative.
template <typename T>
struct RCorner {
    static constexpr bool kOrdered = true;
    const T *b;
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T at() const
    {
        return b[(DX + 2) * kRPlane + (DY + 2) * kRRow + DZ + 2];
    }
};

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

// Residual at cell (x, y, z), linear index q, with the W taps of field F
// from src_of(integral_constant F) (a RegTaps source, stencil corner at
// (x - 2, y - 2, z - 2)); accumulates the norm partials.  Outputs as
// k_residual.
struct ResSums {
    double hsum = 0.0, hmax = 0.0, msum = 0.0, mmax2 = 0.0;
};

// BG: the background fields (psi0f, A2bg) may be set; the marched columns of the
// periodic coupled solve are compiled without them (the host does not route a
// context with a background to them).
template <int BC, typename T, bool HAS_W, bool BG = true, typename SrcOf>
__device__ __forceinline__ void residual_cell(const Geo &g, const ResArgs &a, int x, int y, int z, const SrcOf &src_of,
                                              ResSums &acc)
{
    const int n = g.n;
    const int m = n * n * n;
    const double K2 = a.K2p ? *a.K2p : a.K2;
    const double third = 1.0 / 3.0, two_thirds = 2.0 / 3.0;
    const unsigned q = ((unsigned)x * (unsigned)n + (unsigned)y) * (unsigned)n + (unsigned)z;
    const double uc = elt(a.u, q);
    const double psi = ((BG && a.psi0f) ? elt(a.psi0f, q) : psi0_at(g, a.pmass, x, y, z)) + uc;
    double A2 = (BG && a.A2bg) ? elt(a.A2bg, q) : 0.0;
    double Mv[3] = {0.0, 0.0, 0.0};
    if constexpr (HAS_W) {
        double dW[3][3]; // dW[p][s]: d_p W_s
        double lap[3], dd[3], mix[3];
        auto field = [&](auto fc) {
            constexpr int F = decltype(fc)::value;
            const auto S = src_of(fc);
            RegTaps<double> D;
            D.get_lap(S);
            if (a.want_M) {
                if constexpr (F == 0) {
                    D.template get_mixed<0, 1>(S);
                    D.template get_mixed<0, 2>(S);
                } else if constexpr (F == 1) {
                    D.template get_mixed<0, 1>(S);
                    D.template get_mixed<1, 2>(S);
                } else {
                    D.template get_mixed<0, 2>(S);
                    D.template get_mixed<1, 2>(S);
                }
            }
            dW[0][F] = D.dx() * g.inv12h;
            dW[1][F] = D.dy() * g.inv12h;
            dW[2][F] = D.dz() * g.inv12h;
            if (a.want_M) {
                const double c = D.c();
                const double xx = D.dxx(c), yy = D.dyy(c), zz = D.dzz(c);
                lap[F] = (xx + yy + zz) * g.inv12h2;
                if constexpr (F == 0) {
                    dd[0] = xx * g.inv12h2;
                    mix[1] = D.dxy();
                    mix[2] = D.dxz();
                } else if constexpr (F == 1) {
                    dd[1] = yy * g.inv12h2;
                    mix[0] = D.dxy();
                    mix[2] = mix[2] + D.dyz();
                } else {
                    dd[2] = zz * g.inv12h2;
                    mix[0] = mix[0] + D.dxz();
                    mix[1] = mix[1] + D.dyz();
                }
            }
        };
        static_for<3>(field);
        const double tdiv = (dW[0][0] + dW[1][1] + dW[2][2]) * two_thirds;
#pragma unroll
        for (int p = 0; p < 3; p++)
#pragma unroll
            for (int s2 = 0; s2 < 3; s2++) {
                const double Ab = dW[p][s2] + dW[s2][p] - (p == s2 ? tdiv : 0.0);
                A2 += Ab * Ab;
            }
        if (a.want_M) {
#pragma unroll
            for (int f = 0; f < 3; f++) Mv[f] = lap[f] + (dd[f] + mix[f] * g.inv144h2) * third;
        }
    }
    if (a.want_M && a.S) {
        const double p2 = psi * psi;
        const double w6 = a.conformal ? 1.0 : p2 * p2 * p2;
#pragma unroll
        for (int s2 = 0; s2 < 3; s2++) Mv[s2] -= 8.0 * kPi * w6 * elt(a.S + (size_t)s2 * m, q) - a.meanS[s2];
    }
    const double psi2 = psi * psi, psi4 = psi2 * psi2, psi5 = psi4 * psi;
    const double ipsi = 1.0 / psi, ipsi2 = ipsi * ipsi, ipsi4 = ipsi2 * ipsi2;
    const double ipsi7 = ipsi4 * ipsi2 * ipsi, ipsi8 = ipsi4 * ipsi4;
    const double r5 = elt(a.rho5, q), r1 = elt(a.rho1, q);
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
        lu = lap_sum<double>(Acc<BC, double>{a.u, g}, x, y, z, uc);
    double H = lu * g.inv12h2 + matter - (K2 / 12.0) * psi5 + 0.125 * A2 * ipsi7;
    if (a.f) H += elt(a.f, q);
    const double cc = dmatter - (5.0 * K2 / 12.0) * psi4 - 0.875 * A2 * ipsi8;
    if (a.H) elt(a.H, q) = H;
    if (a.c) elt(a.c, q) = cc;
    const T rT = pinned((T)(-H)), rcT = pinned((T)cc);
    if (a.r) elt((T *)a.r, q) = rT;
    if (a.rc) elt((T *)a.rc, q) = rcT;
    if (a.d1) {
        ResArgs ap = a;
        ap.d1W = nullptr;
        first_pass_fine<BC, T>(g, ap, q, x, y, z, rT, rcT, nullptr);
    }
    if (a.want_M) {
        if (a.M) {
#pragma unroll
            for (int s2 = 0; s2 < 3; s2++) elt(a.M + (size_t)s2 * m, q) = Mv[s2];
        }
        const T rW[3] = {pinned((T)(-Mv[0])), pinned((T)(-Mv[1])), pinned((T)(-Mv[2]))};
        if (a.rW) {
#pragma unroll
            for (int s2 = 0; s2 < 3; s2++) elt((T *)a.rW + (size_t)s2 * m, q) = rW[s2];
        }
        if (a.d1W) {
            ResArgs aw = a;
            aw.d1 = nullptr;
            first_pass_fine<BC, T>(g, aw, q, x, y, z, T(0), T(0), rW);
        }
        const double m2 = Mv[0] * Mv[0] + Mv[1] * Mv[1] + Mv[2] * Mv[2];
        acc.msum += m2;
        acc.mmax2 = fmax(acc.mmax2, m2);
    }
    acc.hsum += H * H;
    acc.hmax = fmax(acc.hmax, fabs(H));
}

template <int BC, typename T, int TX, bool HAS_W>
__global__ void __launch_bounds__(kTY *kLanes) k_residual_tiled(Geo g, TileMap tm, ResArgs a)
{
    a = res_shift(a, g.zs);
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
    ResSums acc;
#pragma unroll
    for (int t = 0; t < TX; t++) {
        // staged word of the stencil corner (x - 2, y - 2, z - 2) of this cell
        const int off = (t * kPY + ty) * kRPZ + lane;
        residual_cell<BC, T, HAS_W>(
            g, a, x0 + t, y, z,
            [&](auto fc) { return RCorner<double>{&lds[HAS_W ? decltype(fc)::value : 0][0][0][0] + off}; }, acc);
    }
    if (a.partials) {
        double v[4] = {acc.hsum, acc.hmax, acc.msum, sqrt(acc.mmax2)};
        // 256 threads per block, as block_reduce_store assumes
        block_reduce_store<4>(v, 0xAu, a.partials + 4 * (int64_t)blockIdx.x);
    }
}

// ---------------------------------------------------------------------------------------
// Residual marching along x (periodic): a workgroup owns a column of 4 (y) x
// 64 (z) cells and LX consecutive x planes, one cell per lane per plane.  The
// three W fields of each staged x plane (rows y0 - 2 .. y0 + 5, z0 - 2 ..
// z0 + 65, FP64) live in a ring of six LDS slots: while the lanes evaluate
// plane x from the slots of x - 2 .. x + 2, the registers hold plane x + 4 in
// flight from HBM and plane x + 3 is written into the slot plane x - 3
// vacated.  Each staged plane is loaded once per column, so the x halo costs
// 4 / LX instead of 4 / TX of the bricks.  Same per-cell arithmetic.
// ---------------------------------------------------------------------------------------
constexpr int kRPlaneF = kPY * kRPZ; // one field of a staged plane
constexpr int kRSlot = 3 * kRPlaneF; // one ring slot

// One staged x plane of the three W fields: 3 kPY rows of kRPZ words; load i
// of a thread moves word `lane` of row w + kTY i, threads tid < 4 * 3 kPY the
// four remaining words of row tid / 4.
struct RPlaneRegs {
    static constexpr int NROW = 3 * kPY;
    static constexpr int RPW = NROW / kTY;
    static_assert(NROW % kTY == 0 && 4 * NROW <= kTY * kLanes, "rows of a plane over the block");
    double v[RPW];
    double e;
    __device__ __forceinline__ void fetch(const double *__restrict__ W, unsigned m, int n, int x, int y0, int z0)
    {
        const int w = threadIdx.y, lane = threadIdx.x, tid = w * kLanes + lane;
        const unsigned un = (unsigned)n, xo = (unsigned)wrap(x, n) * un;
        const unsigned zw = (unsigned)wrap(z0 - 2 + lane, n);
#pragma unroll
        for (int i = 0; i < RPW; i++) {
            const int row = w + kTY * i, f = row / kPY, yr = row - f * kPY;
            v[i] = elt(W + (size_t)f * m, (xo + (unsigned)wrap(y0 + yr - 2, n)) * un + zw);
        }
        e = 0.0;
        if (tid < 4 * NROW) {
            const int row = tid >> 2, f = row / kPY, yr = row - f * kPY;
            e = elt(W + (size_t)f * m, (xo + (unsigned)wrap(y0 + yr - 2, n)) * un + (unsigned)wrap(z0 + kRZ - 2 + (tid & 3), n));
        }
    }
    __device__ __forceinline__ void store(double *slot) const
    {
        const int w = threadIdx.y, lane = threadIdx.x, tid = w * kLanes + lane;
#pragma unroll
        for (int i = 0; i < RPW; i++) slot[(w + kTY * i) * kRPZ + lane] = v[i];
        if (tid < 4 * NROW) slot[(tid >> 2) * kRPZ + kRZ + (tid & 3)] = e;
    }
};

// Taps of field F around the thread's cell: pb[DX + 2] is the word of the
// stencil corner row (y - 2, z - 2) in the slot of plane x + DX.
template <int F>
struct RRing {
    static constexpr bool kOrdered = true;
    const double *const *pb;
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ double at() const
    {
        return pb[DX + 2][F * kRPlaneF + (DY + 2) * kRPZ + DZ + 2];
    }
};

template <typename T, int LX, bool HAS_W>
__global__ void __launch_bounds__(kTY *kLanes) k_residual_march(Geo g, TileMap tm, ResArgs a)
{
    a = res_shift(a, g.zs);
    __shared__ double ring[HAS_W ? kRing : 1][HAS_W ? kRSlot : 1];
    const int total = tm.nx * tm.ny * tm.nz;
    int logical = blockIdx.x;
    if (total % kXCD == 0) logical = (blockIdx.x % kXCD) * (total / kXCD) + blockIdx.x / kXCD;
    const int bz = logical % tm.nz, rest = logical / tm.nz;
    const int x0 = (rest / tm.ny) * LX, y0 = (rest % tm.ny) * kTY, z0 = bz * kRZ;
    const int n = g.n;
    const unsigned m = (unsigned)n * n * n;
    const int ty = threadIdx.y, lane = threadIdx.x;
    const int y = y0 + ty, z = z0 + lane;
    RPlaneRegs st;
    if constexpr (HAS_W) {
        // staged plane j (0 .. LX + 3) is x = x0 - 2 + j, in slot j % kRing; the
        // first six planes are all in flight at once
        RPlaneRegs w5[5];
#pragma unroll
        for (int j = 0; j < 5; j++) w5[j].fetch(a.W, m, n, x0 - 2 + j, y0, z0);
        if (LX > 1) st.fetch(a.W, m, n, x0 + 3, y0, z0);
#pragma unroll
        for (int j = 0; j < 5; j++) w5[j].store(ring[j]);
        __syncthreads();
    }
    ResSums acc;
#pragma unroll 1
    for (int k = 0; k < LX; k++) {
        const double *pb[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        if constexpr (HAS_W) {
#pragma unroll
            for (int d = 0; d < 5; d++) pb[d] = &ring[(k + d) % kRing][ty * kRPZ + lane];
        }
        residual_cell<kBcPeriodic, T, HAS_W, false>(
            g, a, x0 + k, y, z, [&](auto fc) { return RRing<decltype(fc)::value>{pb}; }, acc);
        if constexpr (HAS_W) {
            if (k + 5 <= LX + 3) { // plane x + 3 into the slot plane x - 3 left
                st.store(ring[(k + 5) % kRing]);
                if (k + 6 <= LX + 3) st.fetch(a.W, m, n, x0 + k + 4, y0, z0);
            }
            __syncthreads();
        }
    }
    if (a.partials) {
        double v[4] = {acc.hsum, acc.hmax, acc.msum, sqrt(acc.mmax2)};
        // 256 threads per block, as block_reduce_store assumes
        block_reduce_store<4>(v, 0xAu, a.partials + 4 * (int64_t)blockIdx.x);
    }
}

// Column map of the marched residual (tx == 0: the level does not fit).
template <int LX>
inline TileMap make_rmarchmap(int n)
{
    TileMap t{0, 0, 0, 0};
    if (n % kRZ != 0 || n % kTY != 0 || n % LX != 0) return t;
    if ((double)n * n * n * sizeof(double) >= 4294967296.0) return t; // 32-bit byte offsets per field
    t.nx = n / LX;
    t.ny = n / kTY;
    t.nz = n / kRZ;
    t.tx = LX;
    return t;
}

template <int TX>
inline TileMap make_rtilemap(int n)
{
    TileMap t{0, 0, 0, 0};
    if (n % kRZ != 0 || n % kTY != 0 || n % TX != 0 || n < 64) return t;
    if ((double)n * n * n * sizeof(double) >= 4294967296.0) return t; // 32-bit byte offsets per field
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
