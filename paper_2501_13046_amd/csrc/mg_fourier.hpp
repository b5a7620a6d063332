// mg_fourier.hpp -- exact solve of the momentum equation's defect equation on a small
// periodic level inside one workgroup: the bottom of the W V-cycle of the FP32
// contexts (Key features, "Fast").  Delta_L,h has constant coefficients on a periodic
// grid, so each discrete Fourier mode of the three components decouples into a 3x3
// system built from the stencils' symbols; with t_a = 2 pi k_a / N,
//   D_aa -> lam_a = (-2 cos 2t_a + 32 cos t_a - 30) / (12 h^2)
//   D_a  -> i s_a,   s_a = (8 sin t_a - sin 2t_a) / (6 h)
//   (Delta_L)_aa = sum_c lam_c + lam_a / 3,   (Delta_L)_ab = -s_a s_b / 3  (a != b)
// (the mixed derivatives are products of the first-derivative stencils).  The zero
// mode is set to 0: the result is the mean-free solution for r - mean(r), as the
// coarsest-level inverse gives.
//
// Layout: the three components' N^3 complex values stay in LDS, each z row padded to
// N + 1 entries so that rows read by neighbouring lanes start in different banks.  The
// z transforms run on the way in from global memory and on the way out; the y and x
// transforms are passes over LDS, one line of N points per thread, as a radix-2 FFT
// in registers.
#pragma once

#include "mg_device.hpp"

namespace grtmg {

constexpr int kFourierN = 16;
constexpr int kFourierThreads = 1024;

__host__ __device__ constexpr int bit_reverse(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; b++) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

// In-place FFT of N = 16 complex values: v[k] <- sum_j v[j] exp(-+ 2 pi i jk / N)
// (INV: the + sign, no scaling).  Radix 2, decimation in time.
template <bool INV>
__device__ __forceinline__ void fft16(float2 (&v)[kFourierN])
{
    constexpr int N = kFourierN, kBits = 4;
    // cos and sin of 2 pi t / 16, t = 0 .. 7
    constexpr float kC[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                             0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
    constexpr float kS[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                             1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};
#pragma unroll
    for (int i = 0; i < N; i++) {
        const int j = bit_reverse(i, kBits);
        if (i < j) {
            const float2 t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
        for (int st = 0; st < N; st += len) {
#pragma unroll
            for (int j = 0; j < len / 2; j++) {
                const int t = j * (N / len);
                const float2 a = v[st + j], b = v[st + j + len / 2];
                float2 tb;
                if (t == 0) {
                    tb = b;
                } else {
                    const float wr = kC[t], wi = INV ? kS[t] : -kS[t];
                    tb = make_float2(b.x * wr - b.y * wi, b.x * wi + b.y * wr);
                }
                v[st + j] = make_float2(a.x + tb.x, a.y + tb.y);
                v[st + j + len / 2] = make_float2(a.x - tb.x, a.y - tb.y);
            }
        }
    }
}

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
        fft16<INV>(v);
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
    if (threadIdx.x < N) {
        const double t = 2.0 * M_PI * threadIdx.x / N;
        lam[threadIdx.x] = (float)((-2.0 * cos(2.0 * t) + 32.0 * cos(t) - 30.0) / (12.0 * g.h * g.h));
        sv[threadIdx.x] = (float)((8.0 * sin(t) - sin(2.0 * t)) / (6.0 * g.h));
    }
    // z transforms of the rows of r, into LDS
    for (int L = threadIdx.x; L < 3 * N * N; L += kFourierThreads) {
        const int comp = L / (N * N), row = L % (N * N);
        const float4 *src = reinterpret_cast<const float4 *>(r + (size_t)comp * M + (size_t)row * N);
        float2 v[N];
#pragma unroll
        for (int e = 0; e < N / 4; e++) {
            const float4 q = src[e];
            v[4 * e] = make_float2(q.x, 0.f);
            v[4 * e + 1] = make_float2(q.y, 0.f);
            v[4 * e + 2] = make_float2(q.z, 0.f);
            v[4 * e + 3] = make_float2(q.w, 0.f);
        }
        fft16<false>(v);
        float2 *dst = F + comp * P + row * R;
#pragma unroll
        for (int t = 0; t < N; t++) dst[t] = v[t];
    }
    __syncthreads();
    fourier_pass_lds<1, false>(F);
    __syncthreads();
    fourier_pass_lds<0, false>(F);
    __syncthreads();
    // every mode: the symmetric 3x3 symbol system, solved through its adjugate
    for (int q = threadIdx.x; q < M; q += kFourierThreads) {
        const int i = q / (N * N), j = (q / N) % N, k = q % N;
        const int o = (i * N + j) * R + k;
        if (q == 0) {
            F[o] = F[P + o] = F[2 * P + o] = make_float2(0.f, 0.f);
            continue;
        }
        const float la = lam[i], lb = lam[j], lc = lam[k], sa = sv[i], sb = sv[j], sc = sv[k];
        const float ls = la + lb + lc, third = 1.f / 3.f;
        const float a00 = ls + la * third, a11 = ls + lb * third, a22 = ls + lc * third;
        const float a01 = -sa * sb * third, a02 = -sa * sc * third, a12 = -sb * sc * third;
        const float c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
        const float c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
        const float inv = 1.f / (a00 * c00 + a01 * c01 + a02 * c02);
        const float2 b0 = F[o], b1 = F[P + o], b2 = F[2 * P + o];
        F[o] = make_float2((c00 * b0.x + c01 * b1.x + c02 * b2.x) * inv, (c00 * b0.y + c01 * b1.y + c02 * b2.y) * inv);
        F[P + o] = make_float2((c01 * b0.x + c11 * b1.x + c12 * b2.x) * inv,
                               (c01 * b0.y + c11 * b1.y + c12 * b2.y) * inv);
        F[2 * P + o] = make_float2((c02 * b0.x + c12 * b1.x + c22 * b2.x) * inv,
                                   (c02 * b0.y + c12 * b1.y + c22 * b2.y) * inv);
    }
    __syncthreads();
    fourier_pass_lds<0, true>(F);
    __syncthreads();
    fourier_pass_lds<1, true>(F);
    __syncthreads();
    // inverse z transforms out of LDS; the real parts, scaled by 1/N^3, to x
    constexpr float kScale = 1.f / (float)M;
    for (int L = threadIdx.x; L < 3 * N * N; L += kFourierThreads) {
        const int comp = L / (N * N), row = L % (N * N);
        const float2 *srcl = F + comp * P + row * R;
        float2 v[N];
#pragma unroll
        for (int t = 0; t < N; t++) v[t] = srcl[t];
        fft16<true>(v);
        float4 *dst = reinterpret_cast<float4 *>(x + (size_t)comp * M + (size_t)row * N);
#pragma unroll
        for (int e = 0; e < N / 4; e++)
            dst[e] = make_float4(v[4 * e].x * kScale, v[4 * e + 1].x * kScale, v[4 * e + 2].x * kScale,
                                 v[4 * e + 3].x * kScale);
    }
}

} // namespace grtmg
