// mg_device.hpp -- device-side building blocks of the constraint multigrid:
// grid geometry, boundary accessors, 4th-order stencils and block reductions.
//
// Layout: cell-centred N^3 fields, z fastest, element (i,j,k) at (i*N+j)*N+k;
// 3-vector fields are three consecutive N^3 blocks.  Boundary values come
// from the accessor: periodic wrap, or the 1/r Robin rule a(g) = a(b)|x_b|/|x_g|
// with b the nearest grid cell (coordinates clamped) and radii measured from
// the puncture position.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace grtmg {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kBcPeriodic = 0;
constexpr int kBcRobin = 1;
constexpr int kBcReflect = 2; // mirror image across each boundary face (even parity)
constexpr int kBcExtrap = 3;  // zeroth-order extrapolation along the face normal
constexpr int kBcZero = 4;    // homogeneous ghosts (a refined box: its interface ghosts enter as a forcing)

struct Geo {
    int n;
    int bc;
    double h;
    double inv12h;   // 1 / (12 h)
    double inv12h2;  // 1 / (12 h^2)
    double inv144h2; // 1 / (144 h^2)
    double org[3];
    double ctr[3];
    // Grouped launches of a batch: gz members of one size run in one launch, member
    // blockIdx.z on arrays zs bytes after member 0's (every array of a member lies in
    // one workspace region, the regions of a group zs bytes apart).  gz = 1, zs = 0
    // for a single instance.
    int gz;
    long long zs;
};

__host__ __device__ inline Geo make_geo(int n, int bc, double length, const double org[3],
                                        const double ctr[3])
{
    Geo g;
    g.n = n;
    g.bc = bc;
    g.h = length / n;
    g.inv12h = 1.0 / (12.0 * g.h);
    g.inv12h2 = 1.0 / (12.0 * g.h * g.h);
    g.inv144h2 = 1.0 / (144.0 * g.h * g.h);
    for (int a = 0; a < 3; a++) {
        g.org[a] = org[a];
        g.ctr[a] = ctr[a];
    }
    g.gz = 1;
    g.zs = 0;
    return g;
}

// Pointer p of member 0 moved to this block's member (blockIdx.z) of a grouped
// launch; null stays null.
// The move is byte arithmetic on the pointer itself, so that the result stays based
// on the (restrict-qualified) argument for the compiler's aliasing analysis.
template <typename P>
__device__ __forceinline__ P *zsh(P *p, long long zs)
{
    using B = std::conditional_t<std::is_const_v<P>, const char, char>;
    return p ? reinterpret_cast<P *>(reinterpret_cast<B *>(p) + (long long)blockIdx.z * zs) : p;
}

__device__ __forceinline__ int64_t lidx(int n, int i, int j, int k)
{
    return ((int64_t)i * n + j) * n + k;
}

__device__ __forceinline__ double cell_radius(const Geo &g, int i, int j, int k)
{
    double x = g.org[0] + (i + 0.5) * g.h - g.ctr[0];
    double y = g.org[1] + (j + 0.5) * g.h - g.ctr[1];
    double z = g.org[2] + (k + 0.5) * g.h - g.ctr[2];
    return sqrt(x * x + y * y + z * z);
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
__device__ __forceinline__ int clampc(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

// Cell index that a position i (possibly a ghost, at most two cells outside) reads
// along one axis under the mirror rule (-1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2).
__device__ __forceinline__ int mirror(int i, int n) { return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i); }

// Grid cell (bi, bj, bk) and weight whose product gives the boundary-ruled value
// at (i, j, k): the cell itself inside the grid; outside it, the periodic image
// (weight 1), the nearest grid cell scaled by |x_b| / |x_g| (Robin), the mirror
// image (reflective, weight 1) or the nearest grid cell (extrapolating, weight 1).
template <int BC>
__device__ __forceinline__ double ghost_source(const Geo &g, int i, int j, int k, int &bi, int &bj, int &bk)
{
    const int n = g.n;
    if constexpr (BC == kBcPeriodic) {
        bi = wrap(i, n);
        bj = wrap(j, n);
        bk = wrap(k, n);
        return 1.0;
    } else {
        if ((unsigned)i < (unsigned)n && (unsigned)j < (unsigned)n && (unsigned)k < (unsigned)n) {
            bi = i;
            bj = j;
            bk = k;
            return 1.0;
        }
        if constexpr (BC == kBcReflect) {
            bi = mirror(i, n);
            bj = mirror(j, n);
            bk = mirror(k, n);
            return 1.0;
        } else if constexpr (BC == kBcZero) {
            bi = clampc(i, n); // any grid cell: the ghost depends on none
            bj = clampc(j, n);
            bk = clampc(k, n);
            return 0.0;
        } else {
            bi = clampc(i, n);
            bj = clampc(j, n);
            bk = clampc(k, n);
            if constexpr (BC == kBcRobin) return cell_radius(g, bi, bj, bk) / cell_radius(g, i, j, k);
            return 1.0;
        }
    }
}

// Read-only field accessor with the boundary rule applied.
template <int BC, typename T>
struct Acc {
    const T *__restrict__ a;
    Geo g;
    __device__ __forceinline__ T operator()(int i, int j, int k) const
    {
        const int n = g.n;
        if constexpr (BC == kBcPeriodic) {
            return a[lidx(n, wrap(i, n), wrap(j, n), wrap(k, n))];
        } else {
            if ((unsigned)i < (unsigned)n && (unsigned)j < (unsigned)n && (unsigned)k < (unsigned)n)
                return a[lidx(n, i, j, k)];
            if constexpr (BC == kBcRobin) {
                int bi = clampc(i, n), bj = clampc(j, n), bk = clampc(k, n);
                double v = (double)a[lidx(n, bi, bj, bk)] * cell_radius(g, bi, bj, bk);
                return (T)(v / cell_radius(g, i, j, k));
            } else if constexpr (BC == kBcZero) {
                return T(0);
            } else if constexpr (BC == kBcReflect) {
                return a[lidx(n, mirror(i, n), mirror(j, n), mirror(k, n))];
            } else {
                return a[lidx(n, clampc(i, n), clampc(j, n), clampc(k, n))];
            }
        }
    }
};

// Weight with which the boundary-ruled value at (i,j,k)+offset depends on the
// stored value at (i,j,k) itself (1 for the centre tap).
template <int BC>
__device__ __forceinline__ double self_weight(const Geo &g, int i, int j, int k, int di, int dj,
                                              int dk)
{
    int bi, bj, bk;
    const double w = ghost_source<BC>(g, i + di, j + dj, k + dk, bi, bj, bk);
    return (bi == i && bj == j && bk == k) ? w : 0.0;
}

// ---- stencils (unscaled sums; the caller multiplies by 1/(12h) or 1/(12h^2)) ----

template <int AX>
__device__ __forceinline__ void off(int d, int &di, int &dj, int &dk)
{
    di = (AX == 0) ? d : 0;
    dj = (AX == 1) ? d : 0;
    dk = (AX == 2) ? d : 0;
}

// f(-2) - 8 f(-1) + 8 f(+1) - f(+2) along AX
template <int AX, typename T, typename F>
__device__ __forceinline__ T d1_sum(const F &f, int i, int j, int k)
{
    int a, b, c;
    off<AX>(1, a, b, c);
    return (f(i - 2 * a, j - 2 * b, k - 2 * c) - f(i + 2 * a, j + 2 * b, k + 2 * c)) +
           T(8) * (f(i + a, j + b, k + c) - f(i - a, j - b, k - c));
}

// -f(-2) + 16 f(-1) - 30 f(0) + 16 f(+1) - f(+2) along AX (centre passed in)
template <int AX, typename T, typename F>
__device__ __forceinline__ T d2_sum(const F &f, int i, int j, int k, T centre)
{
    int a, b, c;
    off<AX>(1, a, b, c);
    return T(16) * (f(i - a, j - b, k - c) + f(i + a, j + b, k + c)) -
           (f(i - 2 * a, j - 2 * b, k - 2 * c) + f(i + 2 * a, j + 2 * b, k + 2 * c)) -
           T(30) * centre;
}

template <typename T, typename F>
__device__ __forceinline__ T lap_sum(const F &f, int i, int j, int k, T centre)
{
    return d2_sum<0, T>(f, i, j, k, centre) + d2_sum<1, T>(f, i, j, k, centre) +
           d2_sum<2, T>(f, i, j, k, centre);
}

// sum_{d,e} w1[d] w1[e] f(x + d e_P + e e_Q), w1 = (1, -8, 0, 8, -1): D_P D_Q * 144 h^2
template <int P, int Q, typename T, typename F>
__device__ __forceinline__ T dmix_sum(const F &f, int i, int j, int k)
{
    int pa, pb, pc, qa, qb, qc;
    off<P>(1, pa, pb, pc);
    off<Q>(1, qa, qb, qc);
    T s = T(0);
#pragma unroll
    for (int d = -2; d <= 2; d++) {
        if (d == 0) continue;
        const T wd = (d == -2) ? T(1) : (d == -1) ? T(-8) : (d == 1) ? T(8) : T(-1);
        T t = T(0);
#pragma unroll
        for (int e = -2; e <= 2; e++) {
            if (e == 0) continue;
            const T we = (e == -2) ? T(1) : (e == -1) ? T(-8) : (e == 1) ? T(8) : T(-1);
            t += we * f(i + d * pa + e * qa, j + d * pb + e * qb, k + d * pc + e * qc);
        }
        s += wd * t;
    }
    return s;
}

// Diagonal of the unscaled Laplacian sum at (i,j,k) with the boundary rule.
template <int BC>
__device__ __forceinline__ double lap_diag_sum(const Geo &g, int i, int j, int k)
{
    if constexpr (BC == kBcPeriodic) {
        return -90.0;
    } else {
        const int n = g.n;
        double s = -90.0;
        // only cells on the boundary see their own value through a ghost
        if (i == 0 || i == n - 1 || j == 0 || j == n - 1 || k == 0 || k == n - 1) {
            const double w[5] = {-1.0, 16.0, 0.0, 16.0, -1.0};
#pragma unroll
            for (int d = -2; d <= 2; d++) {
                if (d == 0) continue;
                s += w[d + 2] * self_weight<BC>(g, i, j, k, d, 0, 0);
                s += w[d + 2] * self_weight<BC>(g, i, j, k, 0, d, 0);
                s += w[d + 2] * self_weight<BC>(g, i, j, k, 0, 0, d);
            }
        }
        return s;
    }
}

// ---- reductions ---------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Deterministic block reduction of NV values (bit v of max_mask set: max,
// else sum) over a block of kBlock threads (1D or 2D); thread 0 writes the
// block's results to out[0..NV).
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], unsigned max_mask,
                                                   double *out)
{
    __shared__ double sh[NV][kBlock / kWave];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid % kWave, wid = tid / kWave;
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = ((max_mask >> q) & 1u) ? wave_max(v[q]) : wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) sh[q][wid] = v[q];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; q++) {
            double a = sh[q][0];
            for (int w = 1; w < kBlock / kWave; w++)
                a = ((max_mask >> q) & 1u) ? fmax(a, sh[q][w]) : a + sh[q][w];
            out[q] = a;
        }
    }
}

// A value held in one register from here on, rounded on its own: the compiler
// can neither recompute it nor fuse the operation that produced it into the
// next one (a diagonal term -90/(12 h^2) + c must round the product first in
// every kernel, or FP64 results would depend on how often a kernel reuses it).
template <typename T>
__device__ __forceinline__ T pinned(T v)
{
    asm("" : "+v"(v));
    return v;
}

// Element i of an array addressed by a 32-bit byte offset from its (uniform)
// base: one address register per access instead of a 64-bit sum.
template <typename P>
__device__ __forceinline__ P &elt(P *base, unsigned i)
{
    return *reinterpret_cast<P *>(reinterpret_cast<char *>(const_cast<std::remove_const_t<P> *>(base)) +
                                  i * (unsigned)sizeof(P));
}

template <int... I, typename Fn>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, I...>, Fn &&f)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void static_for(Fn &&f)
{
    static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// The taps of one cell read into registers first, then evaluated.  For LDS
// sources (ORDER) each read is followed by a compiler-only ordering point: the
// taps stay single ds_read_b32 with an immediate offset (instead of being
// paired into ds_read2_b32, whose 8-bit offsets need a fresh base address per
// pair of these taps), and all of them are in flight before the arithmetic.
template <typename T, bool ORDER = true>
struct RegTaps {
    T v[5][5][5]; // (DX + 2, DY + 2, DZ + 2); only the entries read are kept
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T at() const
    {
        return v[DX + 2][DY + 2][DZ + 2];
    }
    template <int DX, int DY, int DZ, typename Src>
    __device__ __forceinline__ void get(const Src &S)
    {
        v[DX + 2][DY + 2][DZ + 2] = S.template at<DX, DY, DZ>();
        if constexpr (ORDER) asm volatile("" ::: "memory");
    }
    // centre, D_xx, D_yy, D_zz taps
    template <typename Src>
    __device__ __forceinline__ void get_lap(const Src &S)
    {
        get<0, 0, 0>(S);
        get<-1, 0, 0>(S), get<1, 0, 0>(S), get<-2, 0, 0>(S), get<2, 0, 0>(S);
        get<0, -1, 0>(S), get<0, 1, 0>(S), get<0, -2, 0>(S), get<0, 2, 0>(S);
        get<0, 0, -1>(S), get<0, 0, 1>(S), get<0, 0, -2>(S), get<0, 0, 2>(S);
    }
    // the 16 off-axis taps of D_ab in the plane of axes A < B (0 = x, 1 = y, 2 = z)
    template <int A, int B, typename Src>
    __device__ __forceinline__ void get_mixed(const Src &S)
    {
        static_for<4>([&](auto i) {
            constexpr int da = (decltype(i)::value & 1 ? 1 : -1) * (decltype(i)::value < 2 ? 1 : 2);
            static_for<4>([&](auto j) {
                constexpr int db = (decltype(j)::value & 1 ? 1 : -1) * (decltype(j)::value < 2 ? 1 : 2);
                constexpr int dx = A == 0 ? da : 0;
                constexpr int dy = A == 1 ? da : (B == 1 ? db : 0);
                constexpr int dz = B == 2 ? db : 0;
                get<dx, dy, dz>(S);
            });
        });
    }
    __device__ __forceinline__ T c() const { return at<0, 0, 0>(); }
    __device__ __forceinline__ T dxx(T c) const
    {
        return T(16) * (at<-1, 0, 0>() + at<1, 0, 0>()) - (at<-2, 0, 0>() + at<2, 0, 0>()) - T(30) * c;
    }
    __device__ __forceinline__ T dyy(T c) const
    {
        return T(16) * (at<0, -1, 0>() + at<0, 1, 0>()) - (at<0, -2, 0>() + at<0, 2, 0>()) - T(30) * c;
    }
    __device__ __forceinline__ T dzz(T c) const
    {
        return T(16) * (at<0, 0, -1>() + at<0, 0, 1>()) - (at<0, 0, -2>() + at<0, 0, 2>()) - T(30) * c;
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
    // first derivatives at the centre (times 12 h)
    __device__ __forceinline__ T dx() const
    {
        return (at<-2, 0, 0>() - at<2, 0, 0>()) + T(8) * (at<1, 0, 0>() - at<-1, 0, 0>());
    }
    __device__ __forceinline__ T dy() const { return dy_at<0, 0>(); }
    __device__ __forceinline__ T dz() const { return dz_at<0, 0>(); }
};

template <typename T>
struct WPart {
    T lap[3], dd[3], mix[3], c[3];
};

// Contributions of field F at one cell whose taps the source S reads (S.at<DX, DY, DZ>
// relative to the cell); returns the value of the other member of the z pair.
template <typename T, int F, int PAR, typename Src>
__device__ __forceinline__ T W_field_parts(const Src &S, T h2, WPart<T> &P)
{
    RegTaps<T, Src::kOrdered> D;
    D.get_lap(S);
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
    const T c = D.c();
    const T xx = D.dxx(c), yy = D.dyy(c), zz = D.dzz(c);
    P.c[F] = c;
    P.lap[F] = (xx + yy + zz) * h2;
    if constexpr (F == 0) {
        P.dd[0] = xx * h2;
        P.mix[1] = D.dxy();
        P.mix[2] = D.dxz();
    } else if constexpr (F == 1) {
        P.dd[1] = yy * h2;
        P.mix[0] = D.dxy();
        P.mix[2] = P.mix[2] + D.dyz();
    } else {
        P.dd[2] = zz * h2;
        P.mix[0] = P.mix[0] + D.dxz();
        P.mix[1] = P.mix[1] + D.dyz();
    }
    constexpr int DZ = PAR ? -1 : 1;
    return D.template at<0, 0, DZ>();
}


// Taps of a periodic field around cell (i, j, k) from wrapped plane, row and
// column offsets computed once per cell: two integer adds per tap.
struct WrapOff {
    unsigned x[5], y[5], z[5];
    __device__ __forceinline__ WrapOff(int n, int i, int j, int k)
    {
        const unsigned un = (unsigned)n;
#pragma unroll
        for (int d = -2; d <= 2; d++) {
            x[d + 2] = (unsigned)wrap(i + d, n) * un * un;
            y[d + 2] = (unsigned)wrap(j + d, n) * un;
            z[d + 2] = (unsigned)wrap(k + d, n);
        }
    }
};

template <typename T>
struct WrapTaps {
    static constexpr bool kOrdered = false;
    const T *a;
    const WrapOff &o;
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T at() const
    {
        return elt(a, o.x[DX + 2] + o.y[DY + 2] + o.z[DZ + 2]);
    }
};

} // namespace grtmg
