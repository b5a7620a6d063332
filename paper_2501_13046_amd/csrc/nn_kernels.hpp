// nn_kernels.hpp -- device kernels of the warm-start network.
//
// Activations are BF16, channels-last: element c of cell v = (i*n + j)*n + k
// of a C-channel tensor is at v*C + c (C a multiple of 8, so one channel
// octet is one aligned 16-byte load).  Convolutions are implicit GEMMs on
// the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulate):
//   M = cells (16 consecutive cells per tile), N = output channels (16 per
//   tile), K = 27 taps x input channels, enumerated as channel octets
//   (tap-major, octet-minor) and consumed 4 octets (32 values) per step.
// Lane l of a wave supplies row l%16 of A and column l%16 of B, each with
// the 8 consecutive K values of octet l/16 of the step; it receives rows
// 4*(l/16) .. 4*(l/16)+3 of column l%16 of the 16x16 result.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grtnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

constexpr int kNBlock = 256; // threads per block (4 waves)
constexpr int kRows = 4;     // 16-cell M tiles per wave in the convolution

// ---- BF16 helpers -------------------------------------------------------------------

__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float((uint32_t)b << 16); }

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint32_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ uint32_t pack2(float lo, float hi) { return f2bf(lo) | (f2bf(hi) << 16); }

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigm(z);
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ u32x4 silu8(u32x4 w)
{
    u32x4 o;
#pragma unroll
    for (int q = 0; q < 4; q++) o[q] = pack2(silu(bf_lo(w[q])), silu(bf_hi(w[q])));
    return o;
}

__device__ __forceinline__ void unpack8(u32x4 w, float (&f)[8])
{
#pragma unroll
    for (int q = 0; q < 4; q++) {
        f[2 * q] = bf_lo(w[q]);
        f[2 * q + 1] = bf_hi(w[q]);
    }
}

__device__ __forceinline__ u32x4 pack8(const float (&f)[8])
{
    u32x4 o;
#pragma unroll
    for (int q = 0; q < 4; q++) o[q] = pack2(f[2 * q], f[2 * q + 1]);
    return o;
}

__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ---- convolution (forward; backward data with flipped transposed weights) ----------

enum { kEpStoreBf16 = 0, kEpStoreF32 = 1, kEpAddF32 = 2, kEpDsiluBf16 = 3 };

struct ConvArgs {
    const u16 *in1, *in2; // input = concatenation [in1, in2] along channels
    int c1, c2;           // channels (= strides) of in1 / in2 (c2 = 0: no in2)
    int act1, act2;       // apply SiLU to values read from in1 / in2
    const u32x4 *w;       // packed weights [tile][chunk][64 lanes] of 8 BF16
    const float *bias;    // per output channel, or null
    int n;                // cells per axis
    int nchunk;           // K steps of 32
    int ntile;            // 16-wide output channel tiles of the layer
    int cout;             // output channels written = oc1 + oc2
    int oc1, oc2;         // output channels [0, oc1) -> out1, [oc1, cout) -> out2
    int mode1, mode2;     // epilogue per destination (kEp*)
    void *out1, *out2;
    const u16 *zref1, *zref2; // pre-activations (layout of out1 / out2) for kEpDsiluBf16
};

template <int NTB>
__global__ void __launch_bounds__(kNBlock) k_conv3(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n;
    const int64_t V = (int64_t)n * n * n;
    const int64_t vb = ((int64_t)blockIdx.x * (kNBlock / 64) + wave) * (16 * kRows);
    if (vb >= V) return; // no block-level synchronisation in this kernel
    const int t0 = blockIdx.y * NTB;
    int px[kRows], py[kRows], pz[kRows];
#pragma unroll
    for (int q = 0; q < kRows; q++) {
        int64_t v = vb + q * 16 + r;
        if (v >= V) v = V - 1; // rows past the end are computed but not stored
        pz[q] = (int)(v % n);
        const int64_t t = v / n;
        py[q] = (int)(t % n);
        px[q] = (int)(t / n);
    }
    f32x4 acc[kRows][NTB];
#pragma unroll
    for (int q = 0; q < kRows; q++)
#pragma unroll
        for (int t = 0; t < NTB; t++) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int opt = (a.c1 + a.c2) >> 3; // channel octets per tap
    const int G = 27 * opt;
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (int ch = 0; ch < a.nchunk; ch++) {
        u32x4 b[NTB];
#pragma unroll
        for (int t = 0; t < NTB; t++)
            b[t] = (t0 + t < a.ntile) ? a.w[((int64_t)(t0 + t) * a.nchunk + ch) * 64 + lane] : zero;
        const int oct = ch * 4 + g;
        u32x4 av[kRows];
        if (oct < G) {
            const int tap = oct / opt, o8 = oct - tap * opt;
            const int dx = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dz = tap % 3 - 1;
            const u16 *src;
            int cs, c0, act;
            if (o8 * 8 < a.c1) {
                src = a.in1;
                cs = a.c1;
                c0 = o8 * 8;
                act = a.act1;
            } else {
                src = a.in2;
                cs = a.c2;
                c0 = o8 * 8 - a.c1;
                act = a.act2;
            }
#pragma unroll
            for (int q = 0; q < kRows; q++) {
                const int x = wrapn(px[q] + dx, n), y = wrapn(py[q] + dy, n), z = wrapn(pz[q] + dz, n);
                const int64_t v = ((int64_t)x * n + y) * n + z;
                av[q] = *(const u32x4 *)(src + v * cs + c0);
                if (act) av[q] = silu8(av[q]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < kRows; q++) av[q] = zero;
        }
#pragma unroll
        for (int q = 0; q < kRows; q++)
#pragma unroll
            for (int t = 0; t < NTB; t++) acc[q][t] = mfma(av[q], b[t], acc[q][t]);
    }
#pragma unroll
    for (int t = 0; t < NTB; t++) {
        const int co = (t0 + t) * 16 + r;
        if (co >= a.cout) continue;
        const float bias = a.bias ? a.bias[co] : 0.0f;
        const bool first = co < a.oc1;
        void *out = first ? a.out1 : a.out2;
        const int cc = first ? co : co - a.oc1;
        const int oc = first ? a.oc1 : a.oc2;
        const int mode = first ? a.mode1 : a.mode2;
        const u16 *zr = first ? a.zref1 : a.zref2;
#pragma unroll
        for (int q = 0; q < kRows; q++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t v = vb + q * 16 + 4 * g + i;
                if (v >= V) continue;
                const float val = acc[q][t][i] + bias;
                const int64_t idx = v * oc + cc;
                if (mode == kEpStoreBf16)
                    ((u16 *)out)[idx] = (u16)f2bf(val);
                else if (mode == kEpStoreF32)
                    ((float *)out)[idx] = val;
                else if (mode == kEpAddF32)
                    ((float *)out)[idx] += val;
                else
                    ((u16 *)out)[idx] = (u16)f2bf(val * dsilu(bf2f(zr[idx])));
            }
    }
}

// ---- weight gradient ------------------------------------------------------------------
//
// dW[co][ci][t] = sum_v dy[v][co] a[v + d_t][ci]: an MFMA with M = output
// channels, N = input channels, K = cells (32 per step, 8 per lane group).
// Block (co tile, ci tile, split) sums the cells of its split (waves take
// every fourth step), the waves' partial tiles are added in LDS in a fixed
// order and the block writes its partial [co][ci][27] (and the bias partial
// sum_v dy[v][co] when it is the first ci tile) for a deterministic reduction.

struct WgtArgs {
    const u16 *in1, *in2;
    int c1, c2, act1, act2; // layer input as in ConvArgs
    const u16 *dy;          // output gradient, BF16, stride cy
    int cy, cout;           // stride and real output channels
    int n;
    int steps_per_split;    // 32-cell steps per split
    int cot, cit;           // co / ci tiles of the layer
    float *part;            // [split][cot*16][cit*16][27]
    float *partb;           // [split][cot*16]
};

__global__ void __launch_bounds__(kNBlock) k_conv3_wgrad(WgtArgs a)
{
    __shared__ float red[16 * 16 * 27 + 16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n;
    const int64_t V = (int64_t)n * n * n;
    const int64_t nsteps = (V + 31) / 32;
    const int cotile = blockIdx.x, citile = blockIdx.y, split = blockIdx.z;
    const int co = cotile * 16 + r, ci = citile * 16 + r;
    const int cin = a.c1 + a.c2;
    const u16 *src = nullptr;
    int cs = 0, c0 = 0, act = 0;
    if (ci < a.c1) {
        src = a.in1;
        cs = a.c1;
        c0 = ci;
        act = a.act1;
    } else if (ci < cin) {
        src = a.in2;
        cs = a.c2;
        c0 = ci - a.c1;
        act = a.act2;
    }
    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.0f;
    const int64_t s0 = (int64_t)split * a.steps_per_split;
    int64_t s1 = s0 + a.steps_per_split;
    if (s1 > nsteps) s1 = nsteps;
    for (int64_t s = s0 + wave; s < s1; s += kNBlock / 64) {
        const int64_t v0 = s * 32 + 8 * g;
        int px[8], py[8], pz[8];
        bool ok[8];
        float av[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            int64_t v = v0 + j;
            ok[j] = v < V;
            if (!ok[j]) v = 0;
            pz[j] = (int)(v % n);
            const int64_t t = v / n;
            py[j] = (int)(t % n);
            px[j] = (int)(t / n);
            av[j] = (ok[j] && co < a.cout) ? bf2f(a.dy[v * a.cy + co]) : 0.0f;
            dbias += av[j];
        }
        const u32x4 A = pack8(av); // exact: av are BF16 values
#pragma unroll 1
        for (int t = 0; t < 27; t++) {
            const int dx = t / 9 - 1, dyy = (t / 3) % 3 - 1, dz = t % 3 - 1;
            float bv[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                float x = 0.0f;
                if (src && ok[j]) {
                    const int64_t v = ((int64_t)wrapn(px[j] + dx, n) * n + wrapn(py[j] + dyy, n)) * n +
                                      wrapn(pz[j] + dz, n);
                    x = bf2f(src[v * cs + c0]);
                    if (act) x = bf2f((u16)f2bf(silu(x)));
                }
                bv[j] = x;
            }
            acc[t] = mfma(A, pack8(bv), acc[t]);
        }
    }
    // bias: lanes with the same r hold the same co; sum the four lane groups
    dbias += __shfl_xor(dbias, 16, 64);
    dbias += __shfl_xor(dbias, 32, 64);
    // add the waves' tiles in LDS in a fixed order
    for (int w = 0; w < kNBlock / 64; w++) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < 27; t++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int idx = ((4 * g + i) * 16 + r) * 27 + t;
                    red[idx] = (w == 0 ? 0.0f : red[idx]) + acc[t][i];
                }
            if (g == 0) red[16 * 16 * 27 + r] = (w == 0 ? 0.0f : red[16 * 16 * 27 + r]) + dbias;
        }
        __syncthreads();
    }
    const int64_t ldco = (int64_t)a.cit * 16 * 27;
    float *dst = a.part + (int64_t)split * a.cot * 16 * ldco;
    for (int e = threadIdx.x; e < 16 * 16 * 27; e += kNBlock) {
        const int rco = e / (16 * 27), rem = e - rco * 16 * 27;
        dst[(int64_t)(cotile * 16 + rco) * ldco + (int64_t)citile * 16 * 27 + rem] = red[e];
    }
    if (citile == 0 && threadIdx.x < 16)
        a.partb[(int64_t)split * a.cot * 16 + cotile * 16 + threadIdx.x] = red[16 * 16 * 27 + threadIdx.x];
}

// grad[(co*cin + ci)*27 + t] (+)= sum_s part[s][co][ci][t]; gradb[co] (+)= sum_s partb[s][co]
__global__ void __launch_bounds__(kNBlock) k_wgrad_reduce(const float *part, const float *partb, int nsplit,
                                                         int cot, int cit, int cout, int cin, float *grad,
                                                         float *gradb, int accumulate)
{
    const int64_t nw = (int64_t)cout * cin * 27;
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    const int64_t per = (int64_t)cot * 16 * cit * 16 * 27;
    if (e < nw) {
        const int co = (int)(e / ((int64_t)cin * 27));
        const int rem = (int)(e - (int64_t)co * cin * 27);
        const int ci = rem / 27, t = rem - ci * 27;
        const int64_t off = ((int64_t)co * cit * 16 + ci) * 27 + t;
        float s = 0.0f;
        for (int q = 0; q < nsplit; q++) s += part[q * per + off];
        grad[e] = accumulate ? grad[e] + s : s;
    } else if (e < nw + cout) {
        const int co = (int)(e - nw);
        float s = 0.0f;
        for (int q = 0; q < nsplit; q++) s += partb[(int64_t)q * cot * 16 + co];
        gradb[co] = accumulate ? gradb[co] + s : s;
    }
}

// ---- weight packing -------------------------------------------------------------------
//
// Forward pack of a layer W[co][ci][27] (cin_real real input channels stored in
// cin_pad channels): element (tile, chunk, lane) holds, for the octet
// oct = 4*chunk + lane/16 (tap = oct / (cin_pad/8)), the 8 weights
// W[tile*16 + lane%16][8*(oct % (cin_pad/8)) + j][tap].  The transposed pack
// (backward data) does the same for W'[ci][co][26 - tap], i.e. the layer with
// inputs and outputs exchanged and the taps mirrored.
__global__ void __launch_bounds__(kNBlock) k_pack_weights(const float *W, int cin_real, int cout, int cin_pad,
                                                         int nchunk, int ntile, int transposed, u32x4 *out)
{
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    const int64_t total = (int64_t)ntile * nchunk * 64;
    if (e >= total) return;
    const int lane = (int)(e % 64);
    const int64_t tc = e / 64;
    const int chunk = (int)(tc % nchunk), tile = (int)(tc / nchunk);
    const int opt = cin_pad / 8;
    const int oct = chunk * 4 + lane / 16;
    const int col = tile * 16 + lane % 16; // output channel of the (possibly transposed) layer
    float f[8];
#pragma unroll
    for (int j = 0; j < 8; j++) f[j] = 0.0f;
    if (oct < 27 * opt) {
        const int tap = oct / opt, o8 = oct - tap * opt;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = o8 * 8 + j; // input channel of the (possibly transposed) layer
            if (!transposed) {
                if (col < cout && k < cin_real) f[j] = W[((int64_t)col * cin_real + k) * 27 + tap];
            } else {
                // layer (cin_real -> cout) seen as (cout -> cin_real): col = ci, k = co
                if (col < cin_real && k < cout) f[j] = W[((int64_t)k * cin_real + col) * 27 + (26 - tap)];
            }
        }
    }
    out[e] = pack8(f);
}

// ---- pooling, upsampling and their adjoints ---------------------------------------------

// out[coarse][c] = mean of the 8 children of act(z); one thread per (coarse cell, octet)
__global__ void __launch_bounds__(kNBlock) k_pool(const u16 *z, int C, int nc, int act, u16 *out)
{
    const int oc = C / 8;
    const int64_t Vc = (int64_t)nc * nc * nc;
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (e >= Vc * oc) return;
    const int o = (int)(e % oc);
    const int64_t v = e / oc;
    const int k = (int)(v % nc), j = (int)((v / nc) % nc), i = (int)(v / ((int64_t)nc * nc));
    const int nf = 2 * nc;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int c = 0; c < 2; c++) {
                const int64_t vf = ((int64_t)(2 * i + a) * nf + (2 * j + b)) * nf + (2 * k + c);
                u32x4 w = *(const u32x4 *)(z + vf * C + 8 * o);
                if (act) w = silu8(w);
                float f[8];
                unpack8(w, f);
#pragma unroll
                for (int q = 0; q < 8; q++) s[q] += f[q];
            }
#pragma unroll
    for (int q = 0; q < 8; q++) s[q] *= 0.125f;
    *(u32x4 *)(out + v * C + 8 * o) = pack8(s);
}

// Per-axis weights of cell-centred x2 interpolation: fine 2I+a takes 3/4 of
// coarse I and 1/4 of coarse I-1 (a = 0) or I+1 (a = 1).
__global__ void __launch_bounds__(kNBlock) k_up(const u16 *z, int C, int nc, int act, u16 *out)
{
    const int oc = C / 8;
    const int nf = 2 * nc;
    const int64_t Vf = (int64_t)nf * nf * nf;
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (e >= Vf * oc) return;
    const int o = (int)(e % oc);
    const int64_t v = e / oc;
    const int k = (int)(v % nf), j = (int)((v / nf) % nf), i = (int)(v / ((int64_t)nf * nf));
    int ci[2], cj[2], ck[2];
    ci[0] = i >> 1;
    ci[1] = wrapn((i >> 1) + ((i & 1) ? 1 : -1), nc);
    cj[0] = j >> 1;
    cj[1] = wrapn((j >> 1) + ((j & 1) ? 1 : -1), nc);
    ck[0] = k >> 1;
    ck[1] = wrapn((k >> 1) + ((k & 1) ? 1 : -1), nc);
    const float wt[2] = {0.75f, 0.25f};
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int c = 0; c < 2; c++) {
                const int64_t vc = ((int64_t)ci[a] * nc + cj[b]) * nc + ck[c];
                u32x4 w = *(const u32x4 *)(z + vc * C + 8 * o);
                if (act) w = silu8(w);
                float f[8];
                unpack8(w, f);
                const float ww = wt[a] * wt[b] * wt[c];
#pragma unroll
                for (int q = 0; q < 8; q++) s[q] += ww * f[q];
            }
    *(u32x4 *)(out + v * C + 8 * o) = pack8(s);
}

// Adjoint of k_up followed by the SiLU derivative: for coarse cell I and
// channel c, sum over the 4 fine cells per axis that read I (2I-1, 2I, 2I+1,
// 2I+2 with weights 1/4, 3/4, 3/4, 1/4) of g_fine, times SiLU'(zref[I][c]).
__global__ void __launch_bounds__(kNBlock) k_up_adjoint_dsilu(const float *gf, int C, int nc, const u16 *zref,
                                                             u16 *dz)
{
    const int64_t Vc = (int64_t)nc * nc * nc;
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (e >= Vc * C) return;
    const int c = (int)(e % C);
    const int64_t v = e / C;
    const int k = (int)(v % nc), j = (int)((v / nc) % nc), i = (int)(v / ((int64_t)nc * nc));
    const int nf = 2 * nc;
    const int off[4] = {-1, 0, 1, 2};
    const float wt[4] = {0.25f, 0.75f, 0.75f, 0.25f};
    float s = 0.0f;
    for (int a = 0; a < 4; a++) {
        const int fi = wrapn(2 * i + off[a], nf);
        for (int b = 0; b < 4; b++) {
            const int fj = wrapn(2 * j + off[b], nf);
            const float wab = wt[a] * wt[b];
            for (int q = 0; q < 4; q++) {
                const int fk = wrapn(2 * k + off[q], nf);
                s += wab * wt[q] * gf[(((int64_t)fi * nf + fj) * nf + fk) * C + c];
            }
        }
    }
    dz[e] = (u16)f2bf(s * dsilu(bf2f(zref[e])));
}

// dz[fine] = (skip[fine] + g_coarse[parent] / 8) * SiLU'(zref[fine]); skip may be null
__global__ void __launch_bounds__(kNBlock) k_pool_adjoint_dsilu(const float *gc, const float *skip, int C, int nc,
                                                               const u16 *zref, u16 *dz)
{
    const int nf = 2 * nc;
    const int64_t Vf = (int64_t)nf * nf * nf;
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (e >= Vf * C) return;
    const int c = (int)(e % C);
    const int64_t v = e / C;
    const int k = (int)(v % nf), j = (int)((v / nf) % nf), i = (int)(v / ((int64_t)nf * nf));
    const int64_t vc = ((int64_t)(i >> 1) * nc + (j >> 1)) * nc + (k >> 1);
    float s = 0.125f * gc[vc * C + c];
    if (skip) s += skip[e];
    dz[e] = (u16)f2bf(s * dsilu(bf2f(zref[e])));
}

// ---- loss, optimiser, packing of fields -------------------------------------------------

// dz[v][c] = 2 (out - t) / (V * cout) for c < cout, 0 for cout <= c < 8 (BF16);
// block partial sums of (out - t)^2.
__global__ void __launch_bounds__(kNBlock) k_mse(const float *out, const u16 *target, int cout, int64_t V,
                                                u16 *dz, double *partials)
{
    __shared__ double sh[kNBlock / 64];
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    const float scale = (float)(2.0 / ((double)V * cout));
    double sq = 0.0;
    if (e < V * 8) {
        const int c = (int)(e % 8);
        const int64_t v = e / 8;
        float d = 0.0f;
        if (c < cout) {
            d = out[v * cout + c] - bf2f(target[v * cout + c]);
            sq = (double)d * d;
        }
        dz[e] = (u16)f2bf(scale * d);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Deterministic sum of count doubles by one block; out[0] = sum.
__global__ void __launch_bounds__(kNBlock) k_sum_final(const double *x, int64_t count, double *out)
{
    __shared__ double sh[kNBlock];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < count; q += kNBlock) s += x[q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kNBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Block partial sums of x and x^2 (grid-stride): partials[block] and
// partials[gridDim.x + block]
__global__ void __launch_bounds__(kNBlock) k_moments(const double *x, int64_t count, double *partials)
{
    __shared__ double sh[2][kNBlock / 64];
    double s = 0.0, s2 = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kNBlock + threadIdx.x; q < count; q += (int64_t)gridDim.x * kNBlock) {
        const double v = x[q];
        s += v;
        s2 += v * v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        s2 += __shfl_xor(s2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = s;
        sh[1][threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        partials[gridDim.x + blockIdx.x] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    }
}

__global__ void __launch_bounds__(kNBlock) k_adam(float *p, const float *g, float *m, float *v, int64_t count,
                                                 float lr, float b1, float b2, float eps, float c1, float c2,
                                                 float gscale)
{
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (e >= count) return;
    const float gr = gscale * g[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gr;
    const float vv = b2 * v[e] + (1.0f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

struct Norm8 {
    float in_mean[4], in_inv[4], out_mean[4], out_std[4];
};

// x[v][c]: (rho5 + rho1, S_x, S_y, S_z) standardised, channels 4..7 zero
__global__ void __launch_bounds__(kNBlock) k_pack_input(const double *rho5, const double *rho1, const double *S,
                                                       int64_t V, Norm8 nm, u16 *x)
{
    const int64_t v = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (v >= V) return;
    float f[8];
    f[0] = (float)((rho5[v] + rho1[v] - nm.in_mean[0]) * nm.in_inv[0]);
    for (int a = 0; a < 3; a++) f[1 + a] = (float)((S[a * V + v] - nm.in_mean[1 + a]) * nm.in_inv[1 + a]);
    f[4] = f[5] = f[6] = f[7] = 0.0f;
    *(u32x4 *)(x + v * 8) = pack8(f);
}

__global__ void __launch_bounds__(kNBlock) k_pack_target(const double *u, const double *W, int64_t V, Norm8 nm,
                                                        u16 *t)
{
    const int64_t v = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (v >= V) return;
    float f[4];
    f[0] = (float)((u[v] - nm.out_mean[0]) / nm.out_std[0]);
    for (int a = 0; a < 3; a++) f[1 + a] = (float)((W[a * V + v] - nm.out_mean[1 + a]) / nm.out_std[1 + a]);
    uint2 o;
    o.x = pack2(f[0], f[1]);
    o.y = pack2(f[2], f[3]);
    *(uint2 *)(t + v * 4) = o;
}

__global__ void __launch_bounds__(kNBlock) k_unpack_output(const float *out, int64_t V, Norm8 nm, double *u,
                                                          double *W)
{
    const int64_t v = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (v >= V) return;
    u[v] = (double)out[v * 4] * nm.out_std[0] + nm.out_mean[0];
    for (int a = 0; a < 3; a++) W[a * V + v] = (double)out[v * 4 + 1 + a] * nm.out_std[1 + a] + nm.out_mean[1 + a];
}

} // namespace grtnn
