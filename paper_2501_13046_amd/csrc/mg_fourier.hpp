// mg_fourier.hpp -- exact solve of the momentum equation's defect equation on a
// coarse periodic level: the bottom of the W V-cycle of the FP32 contexts (Key
// features, "Fast").  Delta_L,h has constant coefficients on a periodic grid, so each
// discrete Fourier mode of the three components decouples into a 3x3 system built
// from the stencils' symbols; with t_a = 2 pi k_a / N,
//   D_aa -> lam_a = (-2 cos 2t_a + 32 cos t_a - 30) / (12 h^2)
//   D_a  -> i s_a,   s_a = (8 sin t_a - sin 2t_a) / (6 h)
//   (Delta_L)_aa = sum_c lam_c + lam_a / 3,   (Delta_L)_ab = -s_a s_b / 3  (a != b)
// (the mixed derivatives are products of the first-derivative stencils).  The zero
// mode is set to 0: the result is the mean-free solution for r - mean(r), as the
// coarsest-level inverse gives.
//
// Line transforms run in registers (radix 2, decimation in time, twiddles fixed at
// compile time).  Two forms:
//  * N = 16: one workgroup per batch member holds all 3 N^3 complex values in LDS
//    (z transforms on the way in from and out to global memory, y and x as LDS passes);
//  * N = 32, 64: three launches over a complex buffer Z of 3 N^3 values: k_spec_fwd (one
//    workgroup per x plane and component: z then y transforms), k_spec_solve (pencils along
//    x, three components: x transforms, the 3x3 solves, inverse x transforms), k_spec_inv
//    (per x plane and component: inverse y then z transforms, real parts scaled by 1/N^3);
//    each line transform is shared by the four threads of a quad (below), and the launches
//    hold 3 N or N^2 / 16 workgroups so that the work spreads over the chip.
// Every LDS row that neighbouring lanes read or write whole is padded to N + 1 entries so
// that the rows start in different banks.
#pragma once

#include "mg_device.hpp"

namespace grtmg {

// cos and sin of x in [0, pi] from their Taylor series (compile time only).
__host__ __device__ constexpr double series_cos(double x)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 40; k++) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
__host__ __device__ constexpr double series_sin(double x)
{
    double term = x, sum = x;
    for (int k = 1; k < 40; k++) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double kTwoPi = 6.283185307179586476925286766559;

__host__ __device__ constexpr int bit_reverse(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; b++) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}
__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// In-place FFT of N complex values in registers: v[k] <- sum_j v[j] exp(-+ 2 pi i jk / N)
// (INV: the + sign; no scaling).
template <int N, bool INV>
__device__ __forceinline__ void fft_reg(float2 (&v)[N])
{
    constexpr int B = ilog2(N);
    static_assert((1 << B) == N, "power-of-two lines");
    static_for<N>([&](auto ii) {
        constexpr int i = decltype(ii)::value, j = bit_reverse(i, B);
        if constexpr (i < j) {
            const float2 t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    });
    static_for<B>([&](auto ss) {
        constexpr int half = 1 << decltype(ss)::value, len = 2 * half;
        static_for<N / 2>([&](auto bb) {
            constexpr int b = decltype(bb)::value, j = b % half, lo = (b / half) * len + j, hi = lo + half;
            constexpr int t = j * (N / len); // twiddle exp(-+ 2 pi i t / N)
            const float2 a = v[lo], x = v[hi];
            float2 wx;
            if constexpr (t == 0) {
                wx = x;
            } else if constexpr (4 * t == N) { // times -i (forward) or +i (inverse)
                wx = INV ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
            } else {
                constexpr float wr = (float)series_cos(kTwoPi * t / N);
                constexpr float wi = (float)(INV ? series_sin(kTwoPi * t / N) : -series_sin(kTwoPi * t / N));
                wx = make_float2(x.x * wr - x.y * wi, x.x * wi + x.y * wr);
            }
            v[lo] = make_float2(a.x + wx.x, a.y + wx.y);
            v[hi] = make_float2(a.x - wx.x, a.y - wx.y);
        });
    });
}

// cos and sin of 2 pi q / 64, q < 64, fixed at compile time (the unit circle of every
// transform length that divides 64).
struct UnitCircle64 {
    double c[64], s[64];
};
constexpr UnitCircle64 make_unit_circle64()
{
    UnitCircle64 u{};
    for (int q = 0; q < 64; q++) {
        const int r = q <= 32 ? q : 64 - q; // angle reduced to [0, pi]
        u.c[q] = series_cos(kTwoPi * r / 64);
        u.s[q] = q <= 32 ? series_sin(kTwoPi * r / 64) : -series_sin(kTwoPi * r / 64);
    }
    return u;
}
__constant__ const UnitCircle64 kUnit64 = make_unit_circle64();

// Symbols of the second and first derivative stencils at t = 2 pi q / N (N divides 64).
__device__ __forceinline__ void stencil_symbols(int q, int N, double h, float &lam, float &s)
{
    const int i1 = q * (64 / N), i2 = (2 * i1) & 63;
    lam = (float)((-2.0 * kUnit64.c[i2] + 32.0 * kUnit64.c[i1] - 30.0) / (12.0 * h * h));
    s = (float)((8.0 * kUnit64.s[i1] - kUnit64.s[i2]) / (6.0 * h));
}

// b <- (Delta_L symbol)^-1 b for one mode (the symmetric 3x3 system through its adjugate).
__device__ __forceinline__ void mode_solve(float la, float lb, float lc, float sa, float sb, float sc, float2 &b0,
                                           float2 &b1, float2 &b2)
{
    const float ls = la + lb + lc, third = 1.f / 3.f;
    const float a00 = ls + la * third, a11 = ls + lb * third, a22 = ls + lc * third;
    const float a01 = -sa * sb * third, a02 = -sa * sc * third, a12 = -sb * sc * third;
    const float c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    const float c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
    const float inv = 1.f / (a00 * c00 + a01 * c01 + a02 * c02);
    const float2 x0 = b0, x1 = b1, x2 = b2;
    b0 = make_float2((c00 * x0.x + c01 * x1.x + c02 * x2.x) * inv, (c00 * x0.y + c01 * x1.y + c02 * x2.y) * inv);
    b1 = make_float2((c01 * x0.x + c11 * x1.x + c12 * x2.x) * inv, (c01 * x0.y + c11 * x1.y + c12 * x2.y) * inv);
    b2 = make_float2((c02 * x0.x + c12 * x1.x + c22 * x2.x) * inv, (c02 * x0.y + c12 * x1.y + c22 * x2.y) * inv);
}

template <int N>
__device__ __forceinline__ void load_real_row(const float *src, float2 (&v)[N])
{
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
#pragma unroll
    for (int e = 0; e < N / 4; e++) {
        const float4 q = s4[e];
        v[4 * e] = make_float2(q.x, 0.f);
        v[4 * e + 1] = make_float2(q.y, 0.f);
        v[4 * e + 2] = make_float2(q.z, 0.f);
        v[4 * e + 3] = make_float2(q.w, 0.f);
    }
}

template <int N>
__device__ __forceinline__ void store_real_row(float *dst, const float2 (&v)[N], float scale)
{
    float4 *d4 = reinterpret_cast<float4 *>(dst);
#pragma unroll
    for (int e = 0; e < N / 4; e++)
        d4[e] = make_float4(v[4 * e].x * scale, v[4 * e + 1].x * scale, v[4 * e + 2].x * scale, v[4 * e + 3].x * scale);
}

// ---- N = 16: one workgroup ---------------------------------------------------------------

constexpr int kFourierN = 16;
constexpr int kFourierThreads = 1024;

// One pass of line transforms along y (AXIS = 1) or x (AXIS = 0) over the three
// components in LDS (component stride P, cell (i, j, k) at (i N + j)(N + 1) + k).
template <int AXIS, bool INV>
__device__ __forceinline__ void fourier_pass_lds(float2 *F)
{
    constexpr int N = kFourierN, R = N + 1, P = N * N * R;
    for (int L = threadIdx.x; L < 3 * N * N; L += kFourierThreads) {
        const int comp = L / (N * N), p = (L / N) % N, q = L % N;
        // lanes with consecutive q read consecutive entries of LDS
        const int base = comp * P + (AXIS == 1 ? p * N * R + q : p * R + q);
        constexpr int stride = AXIS == 1 ? R : N * R;
        float2 v[N];
#pragma unroll
        for (int t = 0; t < N; t++) v[t] = F[base + t * stride];
        fft_reg<N, INV>(v);
#pragma unroll
        for (int t = 0; t < N; t++) F[base + t * stride] = v[t];
    }
}

// x = mean-free solution of Delta_L,h x = r - mean(r) on a 16^3 periodic level g (r, x:
// three components of 16^3 FP32 values, 16-byte aligned).  One workgroup per batch
// member (blockIdx.z).
__global__ void __launch_bounds__(kFourierThreads) k_fourier_W(Geo g, const float *__restrict__ r,
                                                                float *__restrict__ x)
{
    constexpr int N = kFourierN, R = N + 1, P = N * N * R, M = N * N * N;
    r = zsh(r, g.zs);
    x = zsh(x, g.zs);
    __shared__ float2 F[3 * P];
    __shared__ float lam[N], sv[N];
    if (threadIdx.x < N) stencil_symbols(threadIdx.x, N, g.h, lam[threadIdx.x], sv[threadIdx.x]);
    // z transforms of the rows of r, into LDS
    for (int L = threadIdx.x; L < 3 * N * N; L += kFourierThreads) {
        const int comp = L / (N * N), row = L % (N * N);
        float2 v[N];
        load_real_row<N>(r + (size_t)comp * M + (size_t)row * N, v);
        fft_reg<N, false>(v);
        float2 *dst = F + comp * P + row * R;
#pragma unroll
        for (int t = 0; t < N; t++) dst[t] = v[t];
    }
    __syncthreads();
    fourier_pass_lds<1, false>(F);
    __syncthreads();
    fourier_pass_lds<0, false>(F);
    __syncthreads();
    for (int q = threadIdx.x; q < M; q += kFourierThreads) {
        const int i = q / (N * N), j = (q / N) % N, k = q % N;
        const int o = (i * N + j) * R + k;
        if (q == 0) {
            F[o] = F[P + o] = F[2 * P + o] = make_float2(0.f, 0.f);
            continue;
        }
        mode_solve(lam[i], lam[j], lam[k], sv[i], sv[j], sv[k], F[o], F[P + o], F[2 * P + o]);
    }
    __syncthreads();
    fourier_pass_lds<0, true>(F);
    __syncthreads();
    fourier_pass_lds<1, true>(F);
    __syncthreads();
    // inverse z transforms out of LDS; the real parts, scaled by 1/N^3, to x
    for (int L = threadIdx.x; L < 3 * N * N; L += kFourierThreads) {
        const int comp = L / (N * N), row = L % (N * N);
        const float2 *srcl = F + comp * P + row * R;
        float2 v[N];
#pragma unroll
        for (int t = 0; t < N; t++) v[t] = srcl[t];
        fft_reg<N, true>(v);
        store_real_row<N>(x + (size_t)comp * M + (size_t)row * N, v, 1.f / (float)M);
    }
}

// ---- N = 32, 64: three launches over the complex buffer Z ---------------------------------
//
// A line of N = 4Q points is shared by the four threads t of a quad (adjacent lanes): thread t
// holds x[4m + t] (m < Q) and transforms it with Q points in registers (F_t); with
// G_t[k1] = w^(t k1) F_t[k1], w = exp(-+ 2 pi i / N), the outputs are the 4-point transforms
// X[k1 + Q k2] = sum_t (-+i)^(t k2) G_t[k1] (k2 < 4), formed after an exchange of the G through
// the line's N slots in LDS: thread t takes k1 = E t .. E t + E - 1 (E = Q / 4).  Each thread
// runs a quarter of the line's arithmetic, so a transform's latency is a quarter of one thread's.

constexpr int kSpecPencils = 16; // pencils along x per workgroup of k_spec_solve

// tw[q] = exp(-2 pi i q / N), q < N (the inverse takes the conjugate).
__device__ __forceinline__ float2 spec_twiddle(int q, int N)
{
    const int i = q * (64 / N);
    return make_float2((float)kUnit64.c[i], (float)-kUnit64.s[i]);
}

// The quad transform above.  In: v[m] = x[4m + t].  Out: v[k2 E + e] = X[E t + e + Q k2].
// xch: the line's N slots in LDS (stride xs), used by this quad alone; every thread of the
// block calls this equally often (two barriers).
template <int N, bool INV>
__device__ __forceinline__ void fft_quad(float2 (&v)[N / 4], int t, float2 *xch, int xs, const float2 *tw)
{
    constexpr int Q = N / 4, E = Q / 4;
    fft_reg<Q, INV>(v);
#pragma unroll
    for (int k1 = 0; k1 < Q; k1++) {
        float2 w = tw[t * k1];
        if (INV) w.y = -w.y;
        const float2 a = v[k1];
        xch[(t * Q + k1) * xs] = make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
    }
    __syncthreads();
    float2 gq[E][4];
#pragma unroll
    for (int e = 0; e < E; e++)
#pragma unroll
        for (int u = 0; u < 4; u++) gq[e][u] = xch[(u * Q + E * t + e) * xs];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; e++) {
        const float2 a0 = gq[e][0], a1 = gq[e][1], a2 = gq[e][2], a3 = gq[e][3];
        const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y), d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
        const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y), d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
        // -i d13 (forward) or +i d13 (inverse)
        const float2 jd = INV ? make_float2(-d13.y, d13.x) : make_float2(d13.y, -d13.x);
        v[e] = make_float2(s02.x + s13.x, s02.y + s13.y);
        v[E + e] = make_float2(d02.x + jd.x, d02.y + jd.y);
        v[2 * E + e] = make_float2(s02.x - s13.x, s02.y - s13.y);
        v[3 * E + e] = make_float2(d02.x - jd.x, d02.y - jd.y);
    }
}

// One workgroup (4 N threads: a quad per line) per x plane i and component (blockIdx.y): z
// transforms of the plane's rows of r, then y transforms of its columns, into Z
// (component-major, (i N + j) N + k).
template <int N>
__global__ void __launch_bounds__(4 * N) k_spec_fwd(Geo g, const float *__restrict__ r, float2 *__restrict__ Z)
{
    constexpr int Q = N / 4, E = Q / 4, R = N + 1, M = N * N * N;
    r = zsh(r, g.zs);
    Z = zsh(Z, g.zs);
    __shared__ float2 S[N * R];
    __shared__ float2 tw[N];
    const int i = blockIdx.x, comp = blockIdx.y, tid = threadIdx.x;
    const int t = tid & 3, line = tid >> 2;
    if (tid < N) tw[tid] = spec_twiddle(tid, N);
    float2 v[Q];
    const float *row = r + (size_t)comp * M + ((size_t)i * N + line) * N; // row j = line
#pragma unroll
    for (int m = 0; m < Q; m++) v[m] = make_float2(row[4 * m + t], 0.f);
    __syncthreads();
    float2 *Sr = S + line * R;
    fft_quad<N, false>(v, t, Sr, 1, tw);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++)
#pragma unroll
        for (int e = 0; e < E; e++) Sr[E * t + e + Q * k2] = v[k2 * E + e];
    __syncthreads();
    float2 *Sc = S + line; // column k = line
#pragma unroll
    for (int m = 0; m < Q; m++) v[m] = Sc[(4 * m + t) * R];
    __syncthreads();
    fft_quad<N, false>(v, t, Sc, R, tw);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++)
#pragma unroll
        for (int e = 0; e < E; e++) {
            const int j = E * t + e + Q * k2;
            Z[(size_t)comp * M + ((size_t)i * N + j) * N + line] = v[k2 * E + e];
        }
}

// One workgroup (12 kSpecPencils threads) per run of kSpecPencils pencils along x at fixed j:
// x transforms, the 3x3 solve of every mode, inverse x transforms, in place.
template <int N>
__global__ void __launch_bounds__(12 * kSpecPencils) k_spec_solve(Geo g, float2 *__restrict__ Z)
{
    constexpr int KW = kSpecPencils, RW = KW + 1, P = N * RW, Q = N / 4, E = Q / 4, M = N * N * N;
    Z = zsh(Z, g.zs);
    __shared__ float2 QB[3 * P];
    __shared__ float2 tw[N];
    __shared__ float lam[N], sv[N];
    const int j = blockIdx.x / (N / KW), k0 = (blockIdx.x % (N / KW)) * KW;
    const int tid = threadIdx.x, t = tid & 3, kk = (tid >> 2) % KW, comp = tid / (4 * KW);
    if (tid < N) {
        tw[tid] = spec_twiddle(tid, N);
        stencil_symbols(tid, N, g.h, lam[tid], sv[tid]);
    }
    float2 *line = Z + (size_t)comp * M + (size_t)j * N + k0 + kk; // x stride N^2
    float2 v[Q];
#pragma unroll
    for (int m = 0; m < Q; m++) v[m] = line[(size_t)(4 * m + t) * N * N];
    __syncthreads();
    float2 *xq = QB + comp * P + kk; // the pencil's slots, stride RW
    fft_quad<N, false>(v, t, xq, RW, tw);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++)
#pragma unroll
        for (int e = 0; e < E; e++) xq[(E * t + e + Q * k2) * RW] = v[k2 * E + e];
    __syncthreads();
    for (int q = tid; q < N * KW; q += 12 * KW) {
        const int ix = q / KW, kq = q % KW, k = k0 + kq, o = ix * RW + kq;
        if (ix == 0 && j == 0 && k == 0) {
            QB[o] = QB[P + o] = QB[2 * P + o] = make_float2(0.f, 0.f);
            continue;
        }
        mode_solve(lam[ix], lam[j], lam[k], sv[ix], sv[j], sv[k], QB[o], QB[P + o], QB[2 * P + o]);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < Q; m++) v[m] = xq[(4 * m + t) * RW];
    __syncthreads();
    fft_quad<N, true>(v, t, xq, RW, tw);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++)
#pragma unroll
        for (int e = 0; e < E; e++) line[(size_t)(E * t + e + Q * k2) * N * N] = v[k2 * E + e];
}

// One workgroup (4 N threads) per x plane i and component: inverse y transforms of the
// plane's columns of Z, then inverse z transforms of its rows; real parts / N^3 into x.
template <int N>
__global__ void __launch_bounds__(4 * N) k_spec_inv(Geo g, const float2 *__restrict__ Z, float *__restrict__ x)
{
    constexpr int Q = N / 4, E = Q / 4, R = N + 1, M = N * N * N;
    Z = zsh(Z, g.zs);
    x = zsh(x, g.zs);
    __shared__ float2 S[N * R];
    __shared__ float2 tw[N];
    const int i = blockIdx.x, comp = blockIdx.y, tid = threadIdx.x;
    const int t = tid & 3, line = tid >> 2;
    if (tid < N) tw[tid] = spec_twiddle(tid, N);
    float2 v[Q];
#pragma unroll
    for (int m = 0; m < Q; m++) v[m] = Z[(size_t)comp * M + ((size_t)i * N + 4 * m + t) * N + line]; // column k = line
    __syncthreads();
    float2 *Sc = S + line;
    fft_quad<N, true>(v, t, Sc, R, tw);
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++)
#pragma unroll
        for (int e = 0; e < E; e++) Sc[(E * t + e + Q * k2) * R] = v[k2 * E + e];
    __syncthreads();
    float2 *Sr = S + line * R; // row j = line
#pragma unroll
    for (int m = 0; m < Q; m++) v[m] = Sr[4 * m + t];
    __syncthreads();
    fft_quad<N, true>(v, t, Sr, 1, tw);
    constexpr float kScale = 1.f / (float)M;
    float *row = x + (size_t)comp * M + ((size_t)i * N + line) * N;
#pragma unroll
    for (int k2 = 0; k2 < 4; k2++)
#pragma unroll
        for (int e = 0; e < E; e++) row[E * t + e + Q * k2] = v[k2 * E + e].x * kScale;
}

} // namespace grtmg
