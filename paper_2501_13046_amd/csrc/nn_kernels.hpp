// nn_kernels.hpp -- device kernels of the warm-start network.
//
// Activations are BF16, channels-last: element c of cell v = (i*n + j)*n + k
// of a C-channel tensor is at v*C + c (C a multiple of 8, so one channel
// octet is one aligned 16-byte load).  Convolutions are implicit GEMMs on
// the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulate):
//   M = cells (16 per tile), N = output channels (16 per tile), K = 27 taps x
//   input channels, enumerated as channel octets (see KOrder) and consumed
//   4 octets (32 values) per step.
// Lane l of a wave supplies row l%16 of A and column l%16 of B, each with
// the 8 consecutive K values of octet l/16 of the step; it receives rows
// 4*(l/16) .. 4*(l/16)+3 of column l%16 of the 16x16 result.
#pragma once

#include <utility>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grtnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

constexpr int kNBlock = 256; // threads per block (4 waves)

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

// logistic function with the hardware reciprocal (about 1 ulp; the results are
// rounded to BF16)
__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
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

// ---- K order shared by the packed weights and the convolution kernels --------------
//
// The input channels are processed in slices of cs channels (32, 16 or 8: the
// largest that divides both concatenated inputs).  K step ch belongs to slice
// ch / spp (spp = ceil(27 cs / 32) steps per slice); within the slice, lane
// group g of step ch takes octet o = 4 (ch % spp) + g (octets o >= 27 cs / 8
// are zero padding), i.e. tap o / (cs/8) and channels
// slice * cs + 8 (o % (cs/8)) .. + 7.  Tap t = 9 kx + 3 ky + kz is the offset
// (kx - 1, ky - 1, kz - 1).

struct KOrder {
    int cs, spp;
    __device__ __forceinline__ bool at(int ch, int g, int &tap, int &c0) const
    {
        const int sl = ch / spp, o = (ch - sl * spp) * 4 + g;
        const int per = cs >> 3;
        if (o >= 27 * per) return false;
        tap = o / per;
        c0 = sl * cs + (o - tap * per) * 8;
        return true;
    }
};

// ---- convolution (forward; backward data with mirrored transposed weights) ----------

enum { kEpStoreBf16 = 0, kEpStoreF32 = 1, kEpAddF32 = 2, kEpDsiluBf16 = 3, kEpSiluBf16 = 4 };

struct ConvArgs {
    const u16 *in1, *in2; // input = concatenation [in1, in2] along channels
    int c1, c2;           // channels (= strides) of in1 / in2 (c2 = 0: no in2)
    int act1, act2;       // apply SiLU to values read from in1 / in2 (general kernel only)
    const u32x4 *w;       // packed weights [tile][chunk][64 lanes] of 8 BF16
    const float *bias;    // per output channel, or null
    int n;                // cells per axis
    KOrder ko;            // K order of the packed weights
    int nchunk;           // K steps
    int ntile;            // 16-wide output channel tiles of the layer
    int cout;             // output channels written = oc1 + oc2
    int oc1, oc2;         // output channels [0, oc1) -> out1, [oc1, cout) -> out2
    int mode1, mode2;     // epilogue per destination (kEp*)
    void *out1, *out2;
    const u16 *zref1, *zref2; // pre-activations (layout of out1 / out2) for kEpDsiluBf16
    u16 *zout1;           // kEpSiluBf16: pre-activations of destination 1 (may be null)
};

// Epilogue of one value: output channel co of cell v
__device__ __forceinline__ void conv_store(const ConvArgs &a, int co, int64_t v, float acc)
{
    const float val = acc + (a.bias ? a.bias[co] : 0.0f);
    const bool first = co < a.oc1;
    const int cc = first ? co : co - a.oc1;
    const int oc = first ? a.oc1 : a.oc2;
    const int mode = first ? a.mode1 : a.mode2;
    void *out = first ? a.out1 : a.out2;
    const int64_t idx = v * oc + cc;
    if (mode == kEpSiluBf16) {
        ((u16 *)out)[idx] = (u16)f2bf(silu(val));
        if (a.zout1) a.zout1[idx] = (u16)f2bf(val);
    } else if (mode == kEpStoreBf16) {
        ((u16 *)out)[idx] = (u16)f2bf(val);
    } else if (mode == kEpStoreF32) {
        ((float *)out)[idx] = val;
    } else if (mode == kEpAddF32) {
        ((float *)out)[idx] += val;
    } else {
        const u16 *zr = first ? a.zref1 : a.zref2;
        ((u16 *)out)[idx] = (u16)f2bf(val * dsilu(bf2f(zr[idx])));
    }
}

// General kernel (any n): every wave computes ROWS M tiles of 16 consecutive
// cells and reads its A operands straight from global memory.
template <int NTB, int ROWS = kRows>
__global__ void __launch_bounds__(kNBlock) k_conv3(ConvArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n;
    const int64_t V = (int64_t)n * n * n;
    const int64_t vb = ((int64_t)blockIdx.x * (kNBlock / 64) + wave) * (16 * ROWS);
    if (vb >= V) return; // no block-level synchronisation in this kernel
    const int t0 = blockIdx.y * NTB;
    int px[ROWS], py[ROWS], pz[ROWS];
#pragma unroll
    for (int q = 0; q < ROWS; q++) {
        int64_t v = vb + q * 16 + r;
        if (v >= V) v = V - 1; // rows past the end are computed but not stored
        const unsigned uv = (unsigned)v, un = (unsigned)n, t = uv / un; // n^3 < 2^32
        pz[q] = (int)(uv - t * un);
        py[q] = (int)(t % un);
        px[q] = (int)(t / un);
    }
    f32x4 acc[ROWS][NTB];
#pragma unroll
    for (int q = 0; q < ROWS; q++)
#pragma unroll
        for (int t = 0; t < NTB; t++) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (int ch = 0; ch < a.nchunk; ch++) {
        u32x4 b[NTB];
#pragma unroll
        for (int t = 0; t < NTB; t++)
            b[t] = (t0 + t < a.ntile) ? a.w[((int64_t)(t0 + t) * a.nchunk + ch) * 64 + lane] : zero;
        int tap, cg;
        u32x4 av[ROWS];
        if (a.ko.at(ch, g, tap, cg)) {
            const int dx = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dz = tap % 3 - 1;
            const bool one = cg < a.c1;
            const u16 *src = one ? a.in1 : a.in2;
            const int cs = one ? a.c1 : a.c2, c0 = one ? cg : cg - a.c1, act = one ? a.act1 : a.act2;
#pragma unroll
            for (int q = 0; q < ROWS; q++) {
                const int x = wrapn(px[q] + dx, n), y = wrapn(py[q] + dy, n), z = wrapn(pz[q] + dz, n);
                const int64_t v = ((int64_t)x * n + y) * n + z;
                av[q] = *(const u32x4 *)(src + v * cs + c0);
                if (act) av[q] = silu8(av[q]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < ROWS; q++) av[q] = zero;
        }
#pragma unroll
        for (int q = 0; q < ROWS; q++)
#pragma unroll
            for (int t = 0; t < NTB; t++) acc[q][t] = mfma(av[q], b[t], acc[q][t]);
    }
#pragma unroll
    for (int t = 0; t < NTB; t++) {
        const int co = (t0 + t) * 16 + r;
        if (co >= a.cout) continue;
#pragma unroll
        for (int q = 0; q < ROWS; q++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t v = vb + q * 16 + 4 * g + i;
                if (v < V) conv_store(a, co, v, acc[q][t][i]);
            }
    }
}

// Brick kernel (n a multiple of 16): a block computes a brick of 4 x 4 x 16
// cells (wave w: x0 + w; M tile q: y0 + q; row r: z0 + r).  For every channel
// slice the block stages the brick's halo (6 x 6 x 18 cells x CS channels,
// wrapped periodically) in LDS; every A operand is then one 16-byte LDS read,
// and the 16 rows x 4 octets of a step are contiguous (conflict-free).
constexpr int kHX = 6, kHY = 6, kHZ = 18;
constexpr int kHalo = kHX * kHY * kHZ;

__device__ __forceinline__ int brick_block(int nblocks)
{
    // consecutive bricks (which share halo cells) go to the same XCD
    const int b = blockIdx.x;
    return (nblocks % 8 == 0) ? (b % 8) * (nblocks / 8) + b / 8 : b;
}

// Epilogue of 8 consecutive output channels co0 .. co0+7 of cell v (values
// without bias); vector stores where the octet is whole.
__device__ __forceinline__ void conv_store8(const ConvArgs &a, int co0, int64_t v, const float (&acc)[8])
{
    if (co0 >= a.cout) return;
    const bool first = co0 < a.oc1;
    const int cc = first ? co0 : co0 - a.oc1;
    const int oc = first ? a.oc1 : a.oc2;
    const int mode = first ? a.mode1 : a.mode2;
    void *out = first ? a.out1 : a.out2;
    const int nv = min(8, a.cout - co0);
    float f[8];
#pragma unroll
    for (int j = 0; j < 8; j++) f[j] = acc[j] + ((a.bias && j < nv) ? a.bias[co0 + j] : 0.0f);
    const int64_t idx = v * oc + cc;
    if (nv == 8 && mode != kEpStoreF32 && mode != kEpAddF32) {
        if (mode == kEpSiluBf16) {
            float s8[8];
#pragma unroll
            for (int j = 0; j < 8; j++) s8[j] = silu(f[j]);
            *(u32x4 *)((u16 *)out + idx) = pack8(s8);
            if (a.zout1) *(u32x4 *)(a.zout1 + idx) = pack8(f);
        } else if (mode == kEpStoreBf16) {
            *(u32x4 *)((u16 *)out + idx) = pack8(f);
        } else {
            const u16 *zr = first ? a.zref1 : a.zref2;
            float z[8];
            unpack8(*(const u32x4 *)(zr + idx), z);
#pragma unroll
            for (int j = 0; j < 8; j++) f[j] *= dsilu(z[j]);
            *(u32x4 *)((u16 *)out + idx) = pack8(f);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
        if (j >= nv) break;
        if (mode == kEpStoreF32)
            ((float *)out)[idx + j] = f[j];
        else if (mode == kEpAddF32)
            ((float *)out)[idx + j] += f[j];
        else if (mode == kEpStoreBf16)
            ((u16 *)out)[idx + j] = (u16)f2bf(f[j]);
        else if (mode == kEpSiluBf16) {
            ((u16 *)out)[idx + j] = (u16)f2bf(silu(f[j]));
            if (a.zout1) a.zout1[idx + j] = (u16)f2bf(f[j]);
        } else {
            const u16 *zr = first ? a.zref1 : a.zref2;
            ((u16 *)out)[idx + j] = (u16)f2bf(f[j] * dsilu(bf2f(zr[idx + j])));
        }
    }
}

// Halo element (16-byte units) of K octet o of a slice of P octets per tap,
// relative to the lane's element ((wave kHY + q) kHZ + r) P; octets past the 27
// taps point at element 0 (their operands are zeroed).
template <int P>
struct TapOffsets {
    static constexpr int kSteps = (27 * P + 3) / 4;
    int v[kSteps * 4];
    constexpr TapOffsets() : v()
    {
        for (int o = 0; o < kSteps * 4; o++) {
            const int oo = o < 27 * P ? o : 0;
            const int tap = oo / P, o8 = oo % P;
            v[o] = (((tap / 9) * kHY + (tap / 3) % 3) * kHZ + tap % 3) * P + o8;
        }
    }
};

// Offset of K step ST for lane group g (octet 4 ST + g).
template <int P, int ST>
__device__ __forceinline__ int tap_offset(int g)
{
    constexpr TapOffsets<P> T{};
    if constexpr (P == 4)
        return T.v[4 * ST] + g; // one tap per step, the lane group picks the octet
    else if constexpr (P == 2)
        return ((g & 2) ? T.v[4 * ST + 2] : T.v[4 * ST]) + (g & 1);
    else
        return g == 0 ? T.v[4 * ST] : g == 1 ? T.v[4 * ST + 1] : g == 2 ? T.v[4 * ST + 2] : T.v[4 * ST + 3];
}

// PD: weight prefetch depth in K steps (2 for grids that fill the chip, deeper
// for the small levels whose few blocks wait on every weight fetch).
template <int NTB, int CS, int PD>
__global__ void __launch_bounds__(kNBlock) k_conv3_brick(ConvArgs a)
{
    constexpr int P = CS / 8;
    constexpr int kTile = kHalo * P;                     // 16-byte halo elements
    constexpr int kOutRow = 17;                          // floats per staged output cell (padded)
    constexpr int kOut = (256 * kOutRow + 3) / 4;        // 16-byte elements of the output stage
    constexpr int kSmem = kTile > kOut ? kTile : kOut;
    constexpr int NE = (kTile + kNBlock - 1) / kNBlock;  // staging loads per thread
    __shared__ u32x4 smem[kSmem];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n;
    const int nbz = n / 16, nby = n / 4;
    int b = brick_block(gridDim.x);
    const int bz = b % nbz;
    b /= nbz;
    const int by = b % nby, bx = b / nby;
    const int x0 = bx * 4, y0 = by * 4, z0 = bz * 16;
    const int t0 = blockIdx.y * NTB;
    f32x4 acc[4][NTB];
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
        for (int t = 0; t < NTB; t++) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    const int nslice = (a.c1 + a.c2) / CS;
    constexpr int spp = TapOffsets<P>::kSteps; // K steps per slice (the packed order's spp)
    static_assert(PD >= 2 && PD <= spp, "prefetch depth");
    const int lbase = ((wave * kHY) * kHZ + r) * P;
    // weights (L2-resident, the same for every block): a ring of PD K steps; step
    // st + PD - 1 is fetched when step st starts
    u32x4 bw[PD][NTB];
    auto wload = [&](int ch, u32x4 (&w)[NTB]) {
#pragma unroll
        for (int t = 0; t < NTB; t++)
            w[t] = (t0 + t < a.ntile) ? a.w[((int64_t)(t0 + t) * a.nchunk + ch) * 64 + lane] : zero;
    };
    // halo of one channel slice, fetched into registers (wrapped periodically)
    u32x4 stg[NE];
    auto stage_load = [&](int sl) {
        const int cb = sl * CS;
        const bool one = cb < a.c1;
        const u16 *src = one ? a.in1 : a.in2;
        const int cs = one ? a.c1 : a.c2, c0 = one ? cb : cb - a.c1;
#pragma unroll
        for (int k = 0; k < NE; k++) {
            const int e = threadIdx.x + k * kNBlock;
            stg[k] = zero;
            if (e < kTile) {
                const int o = e % P, hv = e / P;
                const int hz = hv % kHZ, hy = (hv / kHZ) % kHY, hx = hv / (kHZ * kHY);
                const int gx = wrapn(x0 + hx - 1, n), gy = wrapn(y0 + hy - 1, n), gz = wrapn(z0 + hz - 1, n);
                stg[k] = *(const u32x4 *)(src + (((int64_t)gx * n + gy) * n + gz) * cs + c0 + o * 8);
            }
        }
    };
    for (int sl = 0; sl < nslice; sl++) {
        // every staging load of the slice is issued before the first LDS store
        stage_load(sl);
        static_for<PD - 1>([&](auto k) { wload(sl * spp + decltype(k)::value, bw[decltype(k)::value]); });
        __syncthreads(); // previous slice consumed
#pragma unroll
        for (int k = 0; k < NE; k++) {
            const int e = threadIdx.x + k * kNBlock;
            if (e < kTile) smem[e] = stg[k];
        }
        __syncthreads();
        // K steps unrolled: the halo offsets of the taps are compile-time constants
        // (one select by lane group per step)
        static_for<spp>([&](auto stc) {
            constexpr int st = decltype(stc)::value;
            if constexpr (st + PD - 1 < spp) wload(sl * spp + st + PD - 1, bw[(st + PD - 1) % PD]);
            const u32x4 *ap = smem + lbase + tap_offset<P, st>(g);
            u32x4 av[4];
#pragma unroll
            for (int q = 0; q < 4; q++) av[q] = ap[q * kHZ * P];
            if constexpr (4 * st + 3 >= 27 * P) { // last step: octets past the 27 taps
                if (4 * st + g >= 27 * P) {
#pragma unroll
                    for (int q = 0; q < 4; q++) av[q] = zero;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int t = 0; t < NTB; t++) acc[q][t] = mfma(av[q], bw[st % PD][t], acc[q][t]);
        });
    }
    // epilogue through LDS: every thread then writes whole channel octets
    float *os = (float *)smem;
#pragma unroll
    for (int t = 0; t < NTB; t++) {
        if ((t0 + t) * 16 >= a.cout) break;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int i = 0; i < 4; i++) os[(wave * 64 + q * 16 + 4 * g + i) * kOutRow + r] = acc[q][t][i];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int e = threadIdx.x + k * kNBlock; // 256 cells x 2 octets
            const int cell = e >> 1, o = e & 1;
            const int vx = cell >> 6, vy = (cell >> 4) & 3, vz = cell & 15;
            float f[8];
#pragma unroll
            for (int j = 0; j < 8; j++) f[j] = os[cell * kOutRow + o * 8 + j];
            const int64_t v = ((int64_t)(x0 + vx) * n + (y0 + vy)) * n + (z0 + vz);
            conv_store8(a, (t0 + t) * 16 + o * 8, v, f);
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
            const unsigned uv = (unsigned)v, un = (unsigned)n, t = uv / un; // n^3 < 2^32
            pz[j] = (int)(uv - t * un);
            py[j] = (int)(t % un);
            px[j] = (int)(t / un);
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

// Brick version (n a multiple of 16), ci tiles of 16 channels.  Per brick of
// 4 x 4 x 16 cells the block stages dy of its co tile transposed,
// dyT[co][cell], and the input halo transposed as three copies shifted by the
// z offset, hT[dz][ci][x][y][z'] = a(x, y, z' + dz) (z' = 0..15): every A and
// B operand of the MFMA (8 consecutive z cells of one channel) is then one
// aligned 16-byte LDS read.  Row strides are padded so that the 16 lanes of a
// read hit distinct banks.  Blocks take contiguous ranges of bricks.
constexpr int kDyStride = 256 + 8;          // u16 per co row of dyT
constexpr int kHtStride = kHX * kHY * 16 + 8; // u16 per ci plane of one hT copy

struct WgtBrick {
    WgtArgs a;
    int bricks_per_split;
};

__global__ void __launch_bounds__(kNBlock) k_conv3_wgrad_brick(WgtBrick wb)
{
    __shared__ __attribute__((aligned(16))) u16 dyT[16 * kDyStride];
    __shared__ __attribute__((aligned(16))) u16 hT[3 * 16 * kHtStride];
    const WgtArgs &a = wb.a;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n;
    const int nbz = n / 16, nby = n / 4;
    const int nbricks = nbz * nby * (n / 4);
    const int cotile = blockIdx.x, citile = blockIdx.y, split = blockIdx.z;
    const int cin = a.c1 + a.c2;
    // the ci tile's source: one input (tiles never straddle in1 / in2), octets present
    const int cb = citile * 16;
    const bool one = cb < a.c1;
    const u16 *src = one ? a.in1 : a.in2;
    const int cs = one ? a.c1 : a.c2, c0 = one ? cb : cb - a.c1;
    const int nci8 = min(2, (min(cin, cb + 16) - cb) / 8); // 1 or 2 octets of real channels
    const int nco8 = min(2, (a.cy - cotile * 16) / 8);
    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.0f;
    const int b0 = split * wb.bricks_per_split;
    const int b1 = min(nbricks, b0 + wb.bricks_per_split);
    for (int bi = b0; bi < b1; bi++) {
        const int bz = bi % nbz, by = (bi / nbz) % nby, bx = bi / (nbz * nby);
        const int x0 = bx * 4, y0 = by * 4, z0 = bz * 16;
        // staging: threads 0..143 build the three shifted halo copies for one
        // (x, y, z quad) from 6 consecutive halo cells; threads 144..207 the
        // transposed dy of one (x, y, z quad); every LDS write is 8 bytes
        // (4 consecutive z of one channel)
        const int tid = threadIdx.x;
        u32x4 ld[12];
        int kind = 0, ix = 0, iy = 0, iq = 0;
        if (tid < 144) {
            kind = 1;
            iq = tid & 3;
            iy = (tid >> 2) % kHY;
            ix = (tid >> 2) / kHY;
            const int gx = wrapn(x0 + ix - 1, n), gy = wrapn(y0 + iy - 1, n);
#pragma unroll
            for (int k = 0; k < 6; k++) {
                const int gz = wrapn(z0 + 4 * iq + k - 1, n);
                const int64_t v = ((int64_t)gx * n + gy) * n + gz;
#pragma unroll
                for (int o = 0; o < 2; o++)
                    ld[2 * k + o] = (o < nci8) ? *(const u32x4 *)(src + v * cs + c0 + o * 8) : u32x4{0u, 0u, 0u, 0u};
            }
        } else if (tid < 208) {
            kind = 2;
            const int t = tid - 144;
            iq = t & 3;
            iy = (t >> 2) & 3;
            ix = t >> 4;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int64_t v = ((int64_t)(x0 + ix) * n + (y0 + iy)) * n + (z0 + 4 * iq + k);
#pragma unroll
                for (int o = 0; o < 2; o++)
                    ld[2 * k + o] = (o < nco8) ? *(const u32x4 *)(a.dy + v * a.cy + cotile * 16 + o * 8)
                                               : u32x4{0u, 0u, 0u, 0u};
            }
        }
        __syncthreads(); // the previous brick's operands are consumed
        if (kind == 1) {
#pragma unroll
            for (int c = 0; c < 16; c++) {
                const int o = c >> 3, w = (c & 7) >> 1, hi = c & 1;
                uint32_t h[6];
#pragma unroll
                for (int k = 0; k < 6; k++) h[k] = hi ? (ld[2 * k + o][w] >> 16) : (ld[2 * k + o][w] & 0xffffu);
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    // copy d holds z' = hz - d: z' = 4 iq + k' reads halo cell 4 iq + k' + d
                    uint2 q;
                    q.x = h[d] | (h[d + 1] << 16);
                    q.y = h[d + 2] | (h[d + 3] << 16);
                    *(uint2 *)&hT[(d * 16 + c) * kHtStride + (ix * kHY + iy) * 16 + 4 * iq] = q;
                }
            }
        } else if (kind == 2) {
#pragma unroll
            for (int c = 0; c < 16; c++) {
                const int o = c >> 3, w = (c & 7) >> 1, hi = c & 1;
                const bool ok = cotile * 16 + c < a.cout;
                uint32_t h[4];
#pragma unroll
                for (int k = 0; k < 4; k++)
                    h[k] = ok ? (hi ? (ld[2 * k + o][w] >> 16) : (ld[2 * k + o][w] & 0xffffu)) : 0u;
                uint2 q;
                q.x = h[0] | (h[1] << 16);
                q.y = h[2] | (h[3] << 16);
                *(uint2 *)&dyT[c * kDyStride + (ix * 4 + iy) * 16 + 4 * iq] = q;
            }
        }
        __syncthreads();
        // wave: x row x0 + wave; K steps of 32 cells = rows (2s, 2s + 1) of y, all 16 z
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const int row = 2 * s + (g >> 1), zh = (g & 1) * 8;
            const u32x4 A = *(const u32x4 *)&dyT[r * kDyStride + (wave * 4 + row) * 16 + zh];
            if (citile == 0) {
                float h[8];
                unpack8(A, h);
#pragma unroll
                for (int j = 0; j < 8; j++) dbias += h[j];
            }
#pragma unroll
            for (int t = 0; t < 27; t++) {
                const int dx = t / 9, dy = (t / 3) % 3, dz = t % 3;
                const u32x4 B =
                    *(const u32x4 *)&hT[(dz * 16 + r) * kHtStride + ((wave + dx) * kHY + row + dy) * 16 + zh];
                acc[t] = mfma(A, B, acc[t]);
            }
        }
    }
    // reduce the waves in LDS (reusing hT) in a fixed order and write the partial
    float *red = (float *)hT; // 16*16*27 + 16 floats fit in hT
    dbias += __shfl_xor(dbias, 16, 64);
    dbias += __shfl_xor(dbias, 32, 64);
    for (int w = 0; w < kNBlock / 64; w++) {
        __syncthreads();
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
    }
    __syncthreads();
    const int64_t ldco = (int64_t)a.cit * 16 * 27;
    float *dst = a.part + (int64_t)split * a.cot * 16 * ldco;
    for (int e = threadIdx.x; e < 16 * 16 * 27; e += kNBlock) {
        const int rco = e / (16 * 27), rem = e - rco * 16 * 27;
        dst[(int64_t)(cotile * 16 + rco) * ldco + (int64_t)citile * 16 * 27 + rem] = red[e];
    }
    if (citile == 0 && threadIdx.x < 16)
        a.partb[(int64_t)split * a.cot * 16 + cotile * 16 + threadIdx.x] = red[16 * 16 * 27 + threadIdx.x];
}

// grad[(co*cin + ci)*27 + t] (+)= sum_s part[s][co][ci][t]; gradb[co] (+)= sum_s partb[s][co].
// A block reduces 16 values with 16 threads each (thread k sums splits
// k, k + 16, ...); the 16 sums are added in a fixed order.
__global__ void __launch_bounds__(kNBlock) k_wgrad_reduce(const float *part, const float *partb, int nsplit,
                                                         int cot, int cit, int cout, int cin, float *grad,
                                                         float *gradb, int accumulate)
{
    __shared__ float sh[16][17];
    const int el = threadIdx.x & 15, k = threadIdx.x >> 4;
    const int64_t nw = (int64_t)cout * cin * 27;
    const int64_t e = (int64_t)blockIdx.x * 16 + el;
    const int64_t per = (int64_t)cot * 16 * cit * 16 * 27;
    float s = 0.0f;
    if (e < nw) {
        const int co = (int)(e / ((int64_t)cin * 27));
        const int rem = (int)(e - (int64_t)co * cin * 27);
        const int ci = rem / 27, t = rem - ci * 27;
        const int64_t off = ((int64_t)co * cit * 16 + ci) * 27 + t;
        for (int q = k; q < nsplit; q += 16) s += part[q * per + off];
    } else if (e < nw + cout) {
        const int co = (int)(e - nw);
        for (int q = k; q < nsplit; q += 16) s += partb[(int64_t)q * cot * 16 + co];
    }
    sh[el][k] = s;
    __syncthreads();
    if (k == 0 && e < nw + cout) {
        float t = 0.0f;
        for (int q = 0; q < 16; q++) t += sh[el][q];
        if (e < nw)
            grad[e] = accumulate ? grad[e] + t : t;
        else
            gradb[e - nw] = accumulate ? gradb[e - nw] + t : t;
    }
}

// ---- weight packing -------------------------------------------------------------------
//
// Forward pack of a layer W[co][ci][27] (cin_real real input channels):
// element (tile, chunk, lane) holds the 8 weights W[tile*16 + lane%16][c0 + j][tap]
// of the octet (tap, c0) that KOrder assigns to (chunk, lane/16), zero where
// the channel or the octet does not exist.  The transposed pack (backward
// data) does the same for W'[ci][co][26 - tap], i.e. the layer with inputs and
// outputs exchanged and the taps mirrored.
__global__ void __launch_bounds__(kNBlock) k_pack_weights(const float *W, int cin_real, int cout, KOrder ko,
                                                         int nchunk, int ntile, int transposed, u32x4 *out)
{
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    const int64_t total = (int64_t)ntile * nchunk * 64;
    if (e >= total) return;
    const int lane = (int)(e % 64);
    const int64_t tc = e / 64;
    const int chunk = (int)(tc % nchunk), tile = (int)(tc / nchunk);
    const int col = tile * 16 + lane % 16; // output channel of the (possibly transposed) layer
    float f[8];
#pragma unroll
    for (int j = 0; j < 8; j++) f[j] = 0.0f;
    int tap, c0;
    if (ko.at(chunk, lane / 16, tap, c0)) {
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = c0 + j; // input channel of the (possibly transposed) layer
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
// coarse I and 1/4 of coarse I-1 (a = 0) or I+1 (a = 1).  One thread per
// (coarse cell, octet) fetches the 3 x 3 x 3 coarse neighbourhood once and
// writes the octet of all 8 children; each child sums its 8 terms in the order
// (own, neighbour) per axis, x outermost.
__global__ void __launch_bounds__(kNBlock) k_up(const u16 *z, int C, int nc, int act, u16 *out)
{
    const int oc = C / 8;
    const int64_t Vc = (int64_t)nc * nc * nc;
    const int64_t e = (int64_t)blockIdx.x * kNBlock + threadIdx.x;
    if (e >= Vc * oc) return;
    const int o = (int)(e % oc);
    const int64_t v = e / oc;
    const int K = (int)(v % nc), J = (int)((v / nc) % nc), I = (int)(v / ((int64_t)nc * nc));
    int xi[3], yj[3], zk[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        xi[d] = wrapn(I + d - 1, nc);
        yj[d] = wrapn(J + d - 1, nc);
        zk[d] = wrapn(K + d - 1, nc);
    }
    u32x4 nb[3][3][3];
#pragma unroll
    for (int dx = 0; dx < 3; dx++)
#pragma unroll
        for (int dy = 0; dy < 3; dy++)
#pragma unroll
            for (int dz = 0; dz < 3; dz++) {
                const int64_t vc = ((int64_t)xi[dx] * nc + yj[dy]) * nc + zk[dz];
                u32x4 w = *(const u32x4 *)(z + vc * C + 8 * o);
                nb[dx][dy][dz] = act ? silu8(w) : w;
            }
    const float wt[2] = {0.75f, 0.25f};
    const int nf = 2 * nc;
#pragma unroll
    for (int ca = 0; ca < 2; ca++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int cc = 0; cc < 2; cc++) {
                float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < 2; b++)
#pragma unroll
                        for (int c = 0; c < 2; c++) {
                            // own cell (index 1) or the neighbour on the child's side
                            const int dx = a ? (ca ? 2 : 0) : 1, dy = b ? (cb ? 2 : 0) : 1, dz = c ? (cc ? 2 : 0) : 1;
                            float f[8];
                            unpack8(nb[dx][dy][dz], f);
                            const float ww = wt[a] * wt[b] * wt[c];
#pragma unroll
                            for (int q = 0; q < 8; q++) s[q] += ww * f[q];
                        }
                const int64_t vf = ((int64_t)(2 * I + ca) * nf + (2 * J + cb)) * nf + (2 * K + cc);
                *(u32x4 *)(out + vf * C + 8 * o) = pack8(s);
            }
}

// The same interpolation with one thread per (fine cell, octet), each reading
// its 8 coarse cells (the same sums in the same order as k_up).
__global__ void __launch_bounds__(kNBlock) k_up_fine(const u16 *z, int C, int nc, int act, u16 *out)
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

// Block partial sums of v and v^2, v = x + y (y may be null), grid-stride:
// partials[block] and partials[gridDim.x + block]
__global__ void __launch_bounds__(kNBlock) k_moments(const double *x, const double *y, int64_t count,
                                                    double *partials)
{
    __shared__ double sh[2][kNBlock / 64];
    double s = 0.0, s2 = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kNBlock + threadIdx.x; q < count; q += (int64_t)gridDim.x * kNBlock) {
        const double v = y ? x[q] + y[q] : x[q];
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
