// grtnn.hip -- host runtime and C ABI of the warm-start network (grtnn.h).
//
// A context carves the caller's workspace into the packed BF16 weights of
// every convolution (forward and mirrored-transposed copies), the activations
// of every level (pre-activations only: consumers apply SiLU on load), and in
// training contexts the gradient buffers and the weight-gradient partials.
// Everything runs on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>

#include "grtnn.h"
#include "nn_kernels.hpp"
#include "mg_internal.h"

using namespace grtnn;

namespace {

constexpr int kMaxLayers = 15;      // 4 levels: 8 encoder + 6 decoder convolutions + head
constexpr int kWgradBlocks = 512;   // target grid of the weight-gradient kernel
constexpr int kMomentBlocks = 1024; // grid of the moments kernel

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
unsigned nblk(int64_t count) { return (unsigned)((count + kNBlock - 1) / kNBlock); }

struct Carver {
    char *base;
    size_t off = 0;
    void *take(size_t bytes)
    {
        off = align_up(off, 256);
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

struct Layer {
    int cin, cout;        // real channels
    int cin_pad, cout8;   // stored input channels; cout rounded up to 8
    int64_t w_off, b_off; // offsets in the parameter array
    int c1, c2;           // the input as a concatenation of two tensors (c2 = 0: one)
    KOrder ko, ko_t;      // K order of the forward / backward-data GEMM
    int nchunk, ntile;    // forward GEMM: K steps, N tiles
    int nchunk_t, ntile_t; // backward-data GEMM (0 tiles: not needed)
    u32x4 *wf, *wt;       // packed weights
    float *bias;          // FP32 copy of the biases
};

// Channel slice of the K order: the largest of 32, 16, 8 dividing both inputs.
int slice_width(int c1, int c2)
{
    for (int cs = 32; cs >= 8; cs /= 2)
        if (c1 % cs == 0 && c2 % cs == 0) return cs;
    return 8;
}

KOrder korder(int c1, int c2, int &nchunk)
{
    KOrder k;
    k.cs = slice_width(c1, c2);
    k.spp = ceil_div(27 * k.cs, 32);
    nchunk = (c1 + c2) / k.cs * k.spp;
    return k;
}

// A convolution cin -> cout whose input is stored as [c1 channels, c2 channels]
// (c1 + c2 = cin_pad >= cin).
void make_layer(Layer &ly, int cin, int cout, int c1, int c2, bool need_bwd_data, int64_t &off)
{
    ly.cin = cin;
    ly.cout = cout;
    ly.c1 = c1;
    ly.c2 = c2;
    ly.cin_pad = c1 + c2;
    ly.cout8 = (cout + 7) / 8 * 8;
    ly.w_off = off;
    off += (int64_t)27 * cin * cout;
    ly.b_off = off;
    off += cout;
    ly.ko = korder(c1, c2, ly.nchunk);
    ly.ntile = ceil_div(cout, 16);
    ly.ko_t = korder(ly.cout8, 0, ly.nchunk_t);
    ly.ntile_t = need_bwd_data ? ceil_div(cin, 16) : 0;
    ly.wf = ly.wt = nullptr;
    ly.bias = nullptr;
}

size_t packed_bytes(int ntile, int nchunk) { return (size_t)ntile * nchunk * 64 * sizeof(u32x4); }

// Split of the weight-gradient reduction over cells for one layer.
struct WSplit {
    int cot, cit, nsplit, steps, bricks;
};

bool brick_ok(int n) { return n >= 16 && n % 16 == 0; }

// Cells of one weight-gradient launch are split into nsplit ranges: 32-cell
// steps (general kernel) or 4 x 4 x 16 bricks (brick kernel, brick = true).
WSplit wsplit(int cin_pad, int cout, int n, bool brick)
{
    WSplit w;
    const int64_t V = (int64_t)n * n * n;
    w.cot = ceil_div(cout, 16);
    w.cit = ceil_div(cin_pad, 16);
    const int64_t units = brick ? V / 256 : (V + 31) / 32;
    int ns = ceil_div(kWgradBlocks, (int64_t)w.cot * w.cit);
    ns = std::max(1, std::min<int>(ns, brick ? (int)units : ceil_div(units, 4)));
    const int per = ceil_div(units, ns);
    w.nsplit = ceil_div(units, per);
    w.steps = brick ? 0 : per;
    w.bricks = brick ? per : 0;
    return w;
}

size_t wsplit_floats(const WSplit &w) { return (size_t)w.nsplit * w.cot * 16 * w.cit * 16 * 27; }

mg_status check_config(const nn_config *c)
{
    if (!c) return MG_ERR_INVALID;
    if (c->levels < 1 || c->levels > 4) return MG_ERR_INVALID;
    if (c->c_in < 1 || c->c_in > 8 || c->c_out < 1 || c->c_out > 16) return MG_ERR_INVALID;
    for (int l = 0; l < c->levels; l++)
        if (c->ch[l] < 16 || c->ch[l] > 128 || c->ch[l] % 16 != 0) return MG_ERR_INVALID;
    if (c->n < 2 || c->n > 1024) return MG_ERR_INVALID;
    const int f = 1 << (c->levels - 1);
    if (c->n % f != 0 || c->n / f < 2) return MG_ERR_INVALID;
    return MG_OK;
}

} // namespace

struct nn_ctx {
    nn_config cfg;
    bool training;
    hipStream_t s;
    int L, nlayers;
    int nl[4];
    int64_t V[4];
    Layer layer[kMaxLayers];
    int64_t nparams;
    // per level: pre-activations z* (training only) and activations a* of the
    // encoder convolutions (a, b), the decoder convolutions (da, db), the
    // pooled input pl and the upsampled decoder input upb
    u16 *za[4], *zb[4], *zda[4], *zdb[4];
    u16 *aa[4], *ab[4], *ada[4], *adb[4];
    u16 *pl[4], *upb[4];
    u16 *x;
    float *out;
    u16 *dzH, *dzA, *dzB;
    float *skipg[4], *upg, *pg;
    float *part, *partb;
    double *dpart;
    double *hpin;
    const u16 *last_in;
};

namespace {

int enc_layer(int l, int half) { return 2 * l + half; }
int dec_layer(const nn_ctx *c, int l, int half) { return 2 * c->L + 2 * (c->L - 2 - l) + half; }
int head_layer(const nn_ctx *c) { return 4 * c->L - 2; }

void plan(nn_ctx *c)
{
    const nn_config &g = c->cfg;
    c->L = g.levels;
    for (int l = 0; l < c->L; l++) {
        c->nl[l] = g.n >> l;
        c->V[l] = (int64_t)c->nl[l] * c->nl[l] * c->nl[l];
    }
    int64_t off = 0;
    int k = 0;
    for (int l = 0; l < c->L; l++) {
        const int cin = l == 0 ? g.c_in : g.ch[l - 1];
        make_layer(c->layer[k++], cin, g.ch[l], l == 0 ? 8 : cin, 0, l > 0, off);
        make_layer(c->layer[k++], g.ch[l], g.ch[l], g.ch[l], 0, true, off);
    }
    for (int l = c->L - 2; l >= 0; l--) {
        make_layer(c->layer[k++], g.ch[l] + g.ch[l + 1], g.ch[l], g.ch[l], g.ch[l + 1], true, off);
        make_layer(c->layer[k++], g.ch[l], g.ch[l], g.ch[l], 0, true, off);
    }
    make_layer(c->layer[k++], g.ch[0], g.c_out, g.ch[0], 0, true, off);
    c->nlayers = k;
    c->nparams = off;
}

void carve(nn_ctx *c, Carver &cv)
{
    const nn_config &g = c->cfg;
    const int L = c->L;
    for (int k = 0; k < c->nlayers; k++) {
        Layer &ly = c->layer[k];
        ly.wf = (u32x4 *)cv.take(packed_bytes(ly.ntile, ly.nchunk));
        ly.wt = ly.ntile_t ? (u32x4 *)cv.take(packed_bytes(ly.ntile_t, ly.nchunk_t)) : nullptr;
        ly.bias = (float *)cv.take((size_t)ly.cout * sizeof(float));
    }
    for (int l = 0; l < L; l++) {
        const size_t bytes = (size_t)c->V[l] * g.ch[l] * 2;
        const bool dec = l <= L - 2;
        c->aa[l] = (u16 *)cv.take(bytes);
        c->ab[l] = (u16 *)cv.take(bytes);
        c->za[l] = c->training ? (u16 *)cv.take(bytes) : nullptr;
        c->zb[l] = c->training ? (u16 *)cv.take(bytes) : nullptr;
        c->ada[l] = dec ? (u16 *)cv.take(bytes) : nullptr;
        c->adb[l] = dec ? (u16 *)cv.take(bytes) : nullptr;
        c->zda[l] = dec && c->training ? (u16 *)cv.take(bytes) : nullptr;
        c->zdb[l] = dec && c->training ? (u16 *)cv.take(bytes) : nullptr;
        c->pl[l] = l > 0 ? (u16 *)cv.take((size_t)c->V[l] * g.ch[l - 1] * 2) : nullptr;
        c->upb[l] = dec ? (u16 *)cv.take((size_t)c->V[l] * g.ch[l + 1] * 2) : nullptr;
    }
    c->x = (u16 *)cv.take((size_t)c->V[0] * 8 * 2);
    c->out = (float *)cv.take((size_t)c->V[0] * g.c_out * 4);
    const size_t nd = std::max<size_t>(2 * kMomentBlocks, nblk(c->V[0] * 8)) + 8;
    c->dpart = (double *)cv.take(nd * sizeof(double));
    if (!c->training) {
        c->dzH = c->dzA = c->dzB = nullptr;
        c->upg = c->pg = c->part = c->partb = nullptr;
        for (int l = 0; l < 4; l++) c->skipg[l] = nullptr;
        return;
    }
    size_t dz = 0, up = 0, pg = 0;
    for (int l = 0; l < L; l++) {
        dz = std::max(dz, (size_t)c->V[l] * g.ch[l]);
        if (l <= L - 2) up = std::max(up, (size_t)c->V[l] * g.ch[l + 1]);
        if (l >= 1) pg = std::max(pg, (size_t)c->V[l] * g.ch[l - 1]);
    }
    c->dzH = (u16 *)cv.take((size_t)c->V[0] * 8 * 2);
    c->dzA = (u16 *)cv.take(dz * 2);
    c->dzB = (u16 *)cv.take(dz * 2);
    for (int l = 0; l < 4; l++)
        c->skipg[l] = (l <= L - 2) ? (float *)cv.take((size_t)c->V[l] * g.ch[l] * 4) : nullptr;
    c->upg = up ? (float *)cv.take(up * 4) : nullptr;
    c->pg = pg ? (float *)cv.take(pg * 4) : nullptr;
    size_t pf = 0, pb = 0;
    for (int l = 0; l < L; l++) {
        // every layer of level l runs its weight gradient on V[l] cells
        for (int k = 0; k < c->nlayers; k++) {
            const Layer &ly = c->layer[k];
            for (int br = 0; br < 2; br++) {
                const WSplit w = wsplit(ly.cin_pad, ly.cout, c->nl[l], br == 1 && brick_ok(c->nl[l]));
                pf = std::max(pf, wsplit_floats(w));
                pb = std::max(pb, (size_t)w.nsplit * w.cot * 16);
            }
        }
    }
    c->part = (float *)cv.take(pf * 4);
    c->partb = (float *)cv.take(pb * 4);
}

// ---- launchers ----------------------------------------------------------------------

struct Out {
    int channels = 0, mode = kEpStoreBf16;
    void *ptr = nullptr;
    const u16 *zref = nullptr;
    u16 *zout = nullptr; // kEpSiluBf16: pre-activations (first destination only)
};



// Brick kernel launch: one block per 4 x 4 x 16 brick (n a multiple of 16).  Grids
// of fewer than 1024 blocks keep 7 K steps of weights in flight, larger ones 2.
template <int NTB, int PD>
void launch_conv_brick_pd(hipStream_t s, const ConvArgs &a, const dim3 &grid, int cs)
{
    if (cs == 32)
        hipLaunchKernelGGL((k_conv3_brick<NTB, 32, PD>), grid, dim3(kNBlock), 0, s, a);
    else if (cs == 16)
        hipLaunchKernelGGL((k_conv3_brick<NTB, 16, PD>), grid, dim3(kNBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_conv3_brick<NTB, 8, PD>), grid, dim3(kNBlock), 0, s, a);
}

template <int NTB>
void launch_conv_brick(hipStream_t s, const ConvArgs &a, int n, int cs, unsigned gy)
{
    const dim3 grid((unsigned)((int64_t)n * n * n / 256), gy);
    if constexpr (NTB == 1) {
        if ((int64_t)grid.x * gy < 1024) {
            launch_conv_brick_pd<1, 7>(s, a, grid, cs);
            return;
        }
    }
    launch_conv_brick_pd<NTB, 2>(s, a, grid, cs);
}

void launch_conv(hipStream_t s, const Layer &ly, bool transposed, int n, const u16 *in1, int c1, int act1,
                 const u16 *in2, int c2, int act2, const float *bias, Out o1, Out o2)
{
    ConvArgs a;
    a.in1 = in1;
    a.in2 = in2;
    a.c1 = c1;
    a.c2 = in2 ? c2 : 0;
    a.act1 = act1;
    a.act2 = act2;
    a.w = transposed ? ly.wt : ly.wf;
    a.bias = bias;
    a.n = n;
    a.ko = transposed ? ly.ko_t : ly.ko;
    a.nchunk = transposed ? ly.nchunk_t : ly.nchunk;
    a.ntile = transposed ? ly.ntile_t : ly.ntile;
    a.oc1 = o1.channels;
    a.oc2 = o2.channels;
    a.cout = o1.channels + o2.channels;
    a.mode1 = o1.mode;
    a.mode2 = o2.mode;
    a.out1 = o1.ptr;
    a.out2 = o2.ptr;
    a.zref1 = o1.zref;
    a.zref2 = o2.zref;
    a.zout1 = o1.zout;
    // the brick kernel reads activations as stored (no SiLU on load)
    const bool brick = brick_ok(n) && !act1 && !act2;
    // output tiles per block: all of them (the staged halo and every A operand
    // read once per block) unless the grid would then have fewer than ~4 blocks
    // per CU (32^3 and 16^3 levels: 128 and 16 bricks)
    int ntb = std::min(a.ntile, 4);
    if (brick) {
        const int64_t bricks = (int64_t)n * n * n / 256;
        while (ntb > 1 && bricks * ceil_div(a.ntile, ntb) < 1024) ntb--;
    }
    const unsigned gy = (unsigned)ceil_div(a.ntile, ntb);
    if (!brick) {
        const int64_t V = (int64_t)n * n * n;
        if (V <= 4096) {
            // small grids (the coarsest levels): one M tile and one N tile per wave, so
            // that the (cell, channel) tiles spread over many waves instead of 2 blocks
            const dim3 grid((unsigned)ceil_div(V, (int64_t)(kNBlock / 64) * 16), (unsigned)a.ntile);
            hipLaunchKernelGGL((k_conv3<1, 1>), grid, dim3(kNBlock), 0, s, a);
            return;
        }
        const dim3 grid((unsigned)ceil_div(V, (int64_t)(kNBlock / 64) * 16 * kRows), gy);
        switch (ntb) {
        case 1: hipLaunchKernelGGL(k_conv3<1>, grid, dim3(kNBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_conv3<2>, grid, dim3(kNBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_conv3<3>, grid, dim3(kNBlock), 0, s, a); break;
        default: hipLaunchKernelGGL(k_conv3<4>, grid, dim3(kNBlock), 0, s, a); break;
        }
        return;
    }
    switch (ntb) {
    case 1: launch_conv_brick<1>(s, a, n, a.ko.cs, gy); break;
    case 2: launch_conv_brick<2>(s, a, n, a.ko.cs, gy); break;
    case 3: launch_conv_brick<3>(s, a, n, a.ko.cs, gy); break;
    default: launch_conv_brick<4>(s, a, n, a.ko.cs, gy); break;
    }
}

// weight and bias gradients of layer ly (input [in1, in2], output gradient dy)
void launch_wgrad_to(hipStream_t s, const Layer &ly, int n, const u16 *in1, int c1, int act1, const u16 *in2,
                     int c2, int act2, const u16 *dy, int cy, float *part, float *partb, float *gw, float *gb,
                     int accumulate)
{
    const bool brick = brick_ok(n) && !act1 && !act2;
    const WSplit w = wsplit(ly.cin_pad, ly.cout, n, brick);
    WgtArgs a;
    a.in1 = in1;
    a.in2 = in2;
    a.c1 = c1;
    a.c2 = in2 ? c2 : 0;
    a.act1 = act1;
    a.act2 = act2;
    a.dy = dy;
    a.cy = cy;
    a.cout = ly.cout;
    a.n = n;
    a.steps_per_split = w.steps;
    a.cot = w.cot;
    a.cit = w.cit;
    a.part = part;
    a.partb = partb;
    if (brick) {
        WgtBrick wb;
        wb.a = a;
        wb.a.cit = w.cit;
        wb.bricks_per_split = w.bricks;
        hipLaunchKernelGGL(k_conv3_wgrad_brick, dim3(w.cot, w.cit, w.nsplit), dim3(kNBlock), 0, s, wb);
    } else {
        hipLaunchKernelGGL(k_conv3_wgrad, dim3(w.cot, w.cit, w.nsplit), dim3(kNBlock), 0, s, a);
    }
    const int64_t nw = (int64_t)ly.cout * ly.cin * 27;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(ceil_div(nw + ly.cout, 16)), dim3(kNBlock), 0, s, (const float *)part,
                       (const float *)partb, w.nsplit, w.cot, w.cit, ly.cout, ly.cin, gw, gb, accumulate);
}

void launch_wgrad(hipStream_t s, const Layer &ly, int n, const u16 *in1, int c1, int act1, const u16 *in2, int c2,
                  int act2, const u16 *dy, int cy, float *part, float *partb, float *grad, int accumulate)
{
    launch_wgrad_to(s, ly, n, in1, c1, act1, in2, c2, act2, dy, cy, part, partb, grad + ly.w_off, grad + ly.b_off,
                    accumulate);
}

void pack_layer(hipStream_t s, const Layer &ly, const float *params)
{
    const float *W = params + ly.w_off;
    const int64_t nf = (int64_t)ly.ntile * ly.nchunk * 64;
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(nf)), dim3(kNBlock), 0, s, W, ly.cin, ly.cout, ly.ko, ly.nchunk,
                       ly.ntile, 0, ly.wf);
    if (ly.ntile_t) {
        const int64_t nt = (int64_t)ly.ntile_t * ly.nchunk_t * 64;
        hipLaunchKernelGGL(k_pack_weights, dim3(nblk(nt)), dim3(kNBlock), 0, s, W, ly.cin, ly.cout, ly.ko_t,
                           ly.nchunk_t, ly.ntile_t, 1, ly.wt);
    }
    if (ly.bias)
        (void)hipMemcpyAsync(ly.bias, params + ly.b_off, (size_t)ly.cout * sizeof(float), hipMemcpyDeviceToDevice,
                             s);
}

mg_status hip_ok() { return hipPeekAtLastError() == hipSuccess ? MG_OK : MG_ERR_HIP; }

Norm8 make_norm(const nn_norm *nm)
{
    Norm8 o;
    for (int q = 0; q < 4; q++) {
        o.in_mean[q] = (float)nm->in_mean[q];
        o.in_inv[q] = (float)(1.0 / nm->in_std[q]);
        o.out_mean[q] = (float)nm->out_mean[q];
        o.out_std[q] = (float)nm->out_std[q];
    }
    return o;
}

bool norm_ok(const nn_norm *nm)
{
    if (!nm) return false;
    for (int q = 0; q < 4; q++)
        if (!(nm->in_std[q] > 0.0) || !(nm->out_std[q] > 0.0) || !std::isfinite(nm->in_mean[q]) ||
            !std::isfinite(nm->out_mean[q]) || !std::isfinite(nm->in_std[q]) || !std::isfinite(nm->out_std[q]))
            return false;
    return true;
}

// Output descriptor of a forward convolution: SiLU activations (+ pre-activations)
Out act_out(int channels, u16 *a, u16 *z)
{
    Out o;
    o.channels = channels;
    o.mode = kEpSiluBf16;
    o.ptr = a;
    o.zout = z;
    return o;
}

void forward(nn_ctx *c, const u16 *in, float *out)
{
    const nn_config &g = c->cfg;
    const int L = c->L;
    hipStream_t s = c->s;
    const Out none;
    c->last_in = in;
    for (int l = 0; l < L; l++) {
        const int n = c->nl[l];
        const Layer &la = c->layer[enc_layer(l, 0)], &lb = c->layer[enc_layer(l, 1)];
        if (l == 0) {
            launch_conv(s, la, false, n, in, 8, 0, nullptr, 0, 0, la.bias, act_out(g.ch[0], c->aa[0], c->za[0]),
                        none);
        } else {
            const int64_t e = c->V[l] * (g.ch[l - 1] / 8);
            hipLaunchKernelGGL(k_pool, dim3(nblk(e)), dim3(kNBlock), 0, s, (const u16 *)c->ab[l - 1], g.ch[l - 1], n,
                               0, c->pl[l]);
            launch_conv(s, la, false, n, c->pl[l], g.ch[l - 1], 0, nullptr, 0, 0, la.bias,
                        act_out(g.ch[l], c->aa[l], c->za[l]), none);
        }
        launch_conv(s, lb, false, n, c->aa[l], g.ch[l], 0, nullptr, 0, 0, lb.bias,
                    act_out(g.ch[l], c->ab[l], c->zb[l]), none);
    }
    for (int l = L - 2; l >= 0; l--) {
        const int n = c->nl[l];
        const u16 *src = (l == L - 2) ? c->ab[L - 1] : c->adb[l + 1];
        // one thread per fine cell and octet where one per coarse cell would leave the chip idle
        const int64_t ec = c->V[l + 1] * (g.ch[l + 1] / 8);
        if (ec >= 65536)
            hipLaunchKernelGGL(k_up, dim3(nblk(ec)), dim3(kNBlock), 0, s, src, g.ch[l + 1], c->nl[l + 1], 0,
                               c->upb[l]);
        else
            hipLaunchKernelGGL(k_up_fine, dim3(nblk(8 * ec)), dim3(kNBlock), 0, s, src, g.ch[l + 1], c->nl[l + 1],
                               0, c->upb[l]);
        const Layer &da = c->layer[dec_layer(c, l, 0)], &db = c->layer[dec_layer(c, l, 1)];
        launch_conv(s, da, false, n, c->ab[l], g.ch[l], 0, c->upb[l], g.ch[l + 1], 0, da.bias,
                    act_out(g.ch[l], c->ada[l], c->zda[l]), none);
        launch_conv(s, db, false, n, c->ada[l], g.ch[l], 0, nullptr, 0, 0, db.bias,
                    act_out(g.ch[l], c->adb[l], c->zdb[l]), none);
    }
    const u16 *top = L >= 2 ? c->adb[0] : c->ab[0];
    Out oh;
    oh.channels = g.c_out;
    oh.mode = kEpStoreF32;
    oh.ptr = out;
    const Layer &lh = c->layer[head_layer(c)];
    launch_conv(s, lh, false, c->nl[0], top, g.ch[0], 0, nullptr, 0, 0, lh.bias, oh, none);
}

} // namespace

extern "C" {

mg_status nn_param_count(const nn_config *cfg, int64_t *count)
{
    if (!count) return MG_ERR_INVALID;
    mg_status st = check_config(cfg);
    if (st != MG_OK) return st;
    nn_ctx tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    tmp.cfg = *cfg;
    plan(&tmp);
    *count = tmp.nparams;
    return MG_OK;
}

mg_status nn_workspace_size(const nn_config *cfg, int32_t training, size_t *bytes)
{
    if (!bytes || (training != 0 && training != 1)) return MG_ERR_INVALID;
    mg_status st = check_config(cfg);
    if (st != MG_OK) return st;
    nn_ctx tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    tmp.cfg = *cfg;
    tmp.training = training != 0;
    plan(&tmp);
    Carver cv{nullptr};
    carve(&tmp, cv);
    *bytes = align_up(cv.off, 256);
    return MG_OK;
}

} // extern "C"

namespace {

Out dsilu_out(int channels, u16 *dz, const u16 *z)
{
    Out o;
    o.channels = channels;
    o.mode = kEpDsiluBf16;
    o.ptr = dz;
    o.zref = z;
    return o;
}

Out f32_out(int channels, float *p)
{
    Out o;
    o.channels = channels;
    o.mode = kEpStoreF32;
    o.ptr = p;
    return o;
}

// Backward pass for the loss gradient in dzH.  Weight gradients read the stored
// activations; the SiLU derivative reads the stored pre-activations.
void backward(nn_ctx *c, float *grad)
{
    const nn_config &g = c->cfg;
    const int L = c->L;
    hipStream_t s = c->s;
    const Out none;
    const u16 *top_a = L >= 2 ? c->adb[0] : c->ab[0];
    const u16 *top_z = L >= 2 ? c->zdb[0] : c->zb[0];
    {
        const Layer &lh = c->layer[head_layer(c)];
        launch_wgrad(s, lh, c->nl[0], top_a, g.ch[0], 0, nullptr, 0, 0, c->dzH, 8, c->part, c->partb, grad, 1);
        launch_conv(s, lh, true, c->nl[0], c->dzH, lh.cout8, 0, nullptr, 0, 0, nullptr,
                    dsilu_out(g.ch[0], c->dzB, top_z), none);
    }
    // decoder, from the top level down; dzB holds the gradient of the level's output
    for (int l = 0; l <= L - 2; l++) {
        const int n = c->nl[l];
        const Layer &da = c->layer[dec_layer(c, l, 0)], &db = c->layer[dec_layer(c, l, 1)];
        launch_wgrad(s, db, n, c->ada[l], g.ch[l], 0, nullptr, 0, 0, c->dzB, g.ch[l], c->part, c->partb, grad, 1);
        launch_conv(s, db, true, n, c->dzB, g.ch[l], 0, nullptr, 0, 0, nullptr, dsilu_out(g.ch[l], c->dzA, c->zda[l]),
                    none);
        launch_wgrad(s, da, n, c->ab[l], g.ch[l], 0, c->upb[l], g.ch[l + 1], 0, c->dzA, g.ch[l], c->part, c->partb,
                     grad, 1);
        launch_conv(s, da, true, n, c->dzA, g.ch[l], 0, nullptr, 0, 0, nullptr, f32_out(g.ch[l], c->skipg[l]),
                    f32_out(g.ch[l + 1], c->upg));
        const u16 *zref = (l + 1 == L - 1) ? c->zb[L - 1] : c->zdb[l + 1];
        const int64_t e = c->V[l + 1] * g.ch[l + 1];
        hipLaunchKernelGGL(k_up_adjoint_dsilu, dim3(nblk(e)), dim3(kNBlock), 0, s, (const float *)c->upg,
                           g.ch[l + 1], c->nl[l + 1], zref, c->dzB);
    }
    // encoder, from the bottom level up; dzB holds the gradient of e_l
    for (int l = L - 1; l >= 0; l--) {
        const int n = c->nl[l];
        const Layer &la = c->layer[enc_layer(l, 0)], &lb = c->layer[enc_layer(l, 1)];
        launch_wgrad(s, lb, n, c->aa[l], g.ch[l], 0, nullptr, 0, 0, c->dzB, g.ch[l], c->part, c->partb, grad, 1);
        launch_conv(s, lb, true, n, c->dzB, g.ch[l], 0, nullptr, 0, 0, nullptr, dsilu_out(g.ch[l], c->dzA, c->za[l]),
                    none);
        if (l == 0) {
            launch_wgrad(s, la, n, c->last_in, 8, 0, nullptr, 0, 0, c->dzA, g.ch[0], c->part, c->partb, grad, 1);
            break;
        }
        launch_wgrad(s, la, n, c->pl[l], g.ch[l - 1], 0, nullptr, 0, 0, c->dzA, g.ch[l], c->part, c->partb, grad,
                     1);
        launch_conv(s, la, true, n, c->dzA, g.ch[l], 0, nullptr, 0, 0, nullptr, f32_out(g.ch[l - 1], c->pg), none);
        const int64_t e = c->V[l - 1] * g.ch[l - 1];
        hipLaunchKernelGGL(k_pool_adjoint_dsilu, dim3(nblk(e)), dim3(kNBlock), 0, s, (const float *)c->pg,
                           (const float *)c->skipg[l - 1], g.ch[l - 1], n, (const u16 *)c->zb[l - 1], c->dzB);
    }
}

mg_status sync_status(hipStream_t s)
{
    if (hipPeekAtLastError() != hipSuccess) return MG_ERR_HIP;
    return hipStreamSynchronize(s) == hipSuccess ? MG_OK : MG_ERR_HIP;
}

bool aligned16(const void *p) { return ((uintptr_t)p % 16) == 0; }

} // namespace

extern "C" {

mg_status nn_setup(const nn_config *cfg, int32_t training, void *d_workspace, size_t bytes, void *stream,
                   nn_ctx **out)
{
    if (!out) return MG_ERR_INVALID;
    *out = nullptr;
    size_t need = 0;
    mg_status st = nn_workspace_size(cfg, training, &need);
    if (st != MG_OK) return st;
    if (!d_workspace || bytes < need || ((uintptr_t)d_workspace % 256) != 0) return MG_ERR_WORKSPACE;
    nn_ctx *c = new (std::nothrow) nn_ctx;
    if (!c) return MG_ERR_INVALID;
    std::memset(c, 0, sizeof(*c));
    c->cfg = *cfg;
    c->training = training != 0;
    c->s = (hipStream_t)stream;
    plan(c);
    Carver cv{(char *)d_workspace};
    carve(c, cv);
    if (hipHostMalloc((void **)&c->hpin, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return MG_ERR_HIP;
    }
    *out = c;
    return MG_OK;
}

void nn_destroy(nn_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    if (c->hpin) (void)hipHostFree(c->hpin);
    delete c;
}

mg_status nn_load_params(nn_ctx *c, const float *d_params)
{
    if (!c || !d_params) return MG_ERR_INVALID;
    for (int k = 0; k < c->nlayers; k++) pack_layer(c->s, c->layer[k], d_params);
    return hip_ok();
}

mg_status nn_forward(nn_ctx *c, const uint16_t *d_in, float *d_out)
{
    if (!c || !d_in || !d_out || !aligned16(d_in)) return MG_ERR_INVALID;
    forward(c, d_in, d_out);
    return hip_ok();
}

mg_status nn_mse(nn_ctx *c, const float *d_out, const uint16_t *d_target, double *h_loss)
{
    if (!c || !d_out || !d_target || !h_loss || !c->training) return MG_ERR_INVALID;
    const int64_t V = c->V[0];
    const unsigned nb = nblk(V * 8);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kNBlock), 0, c->s, d_out, d_target, c->cfg.c_out, V, c->dzH,
                       c->dpart);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kNBlock), 0, c->s, (const double *)c->dpart, (int64_t)nb,
                       c->dpart + nb);
    if (hipMemcpyAsync(c->hpin, c->dpart + nb, sizeof(double), hipMemcpyDeviceToHost, c->s) != hipSuccess)
        return MG_ERR_HIP;
    mg_status st = sync_status(c->s);
    if (st != MG_OK) return st;
    *h_loss = c->hpin[0] / ((double)V * c->cfg.c_out);
    return MG_OK;
}

mg_status nn_backward(nn_ctx *c, float *d_grad)
{
    if (!c || !d_grad || !c->training || !c->last_in) return MG_ERR_INVALID;
    backward(c, d_grad);
    return hip_ok();
}

mg_status nn_adam_step(nn_ctx *c, float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step,
                       double lr, double beta1, double beta2, double eps, double grad_scale)
{
    if (!c || !d_params || !d_grad || !d_m || !d_v || step < 1 || !(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
        !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0) || !std::isfinite(grad_scale))
        return MG_ERR_INVALID;
    const double c1 = 1.0 - std::pow(beta1, step), c2 = 1.0 - std::pow(beta2, step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(c->nparams)), dim3(kNBlock), 0, c->s, d_params, d_grad, d_m, d_v,
                       c->nparams, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1, (float)c2,
                       (float)grad_scale);
    return nn_load_params(c, d_params);
}

mg_status nn_pack_input(nn_ctx *c, const double *d_rho5, const double *d_rho1, const double *d_S,
                        const nn_norm *norm, uint16_t *d_in)
{
    if (!c || !d_rho5 || !d_rho1 || !d_S || !d_in || !norm_ok(norm) || !aligned16(d_in)) return MG_ERR_INVALID;
    const int64_t V = c->V[0];
    hipLaunchKernelGGL(k_pack_input, dim3(nblk(V)), dim3(kNBlock), 0, c->s, d_rho5, d_rho1, d_S, V, make_norm(norm),
                       d_in);
    return hip_ok();
}

mg_status nn_pack_target(nn_ctx *c, const double *d_u, const double *d_W, const nn_norm *norm, uint16_t *d_target)
{
    if (!c || !d_u || !d_W || !d_target || !norm_ok(norm) || ((uintptr_t)d_target % 8) != 0 || c->cfg.c_out != 4)
        return MG_ERR_INVALID;
    const int64_t V = c->V[0];
    hipLaunchKernelGGL(k_pack_target, dim3(nblk(V)), dim3(kNBlock), 0, c->s, d_u, d_W, V, make_norm(norm), d_target);
    return hip_ok();
}

mg_status nn_unpack_output(nn_ctx *c, const float *d_out, const nn_norm *norm, double *d_u, double *d_W)
{
    if (!c || !d_out || !d_u || !d_W || !norm_ok(norm) || c->cfg.c_out != 4) return MG_ERR_INVALID;
    const int64_t V = c->V[0];
    hipLaunchKernelGGL(k_unpack_output, dim3(nblk(V)), dim3(kNBlock), 0, c->s, d_out, V, make_norm(norm), d_u, d_W);
    return hip_ok();
}

mg_status nn_moments(nn_ctx *c, const double *d_x, const double *d_y, int64_t count, double h_out[2])
{
    if (!c || !d_x || count < 0 || !h_out) return MG_ERR_INVALID;
    const int B = kMomentBlocks;
    hipLaunchKernelGGL(k_moments, dim3(B), dim3(kNBlock), 0, c->s, d_x, d_y, count, c->dpart);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kNBlock), 0, c->s, (const double *)c->dpart, (int64_t)B,
                       c->dpart + 2 * B);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kNBlock), 0, c->s, (const double *)(c->dpart + B), (int64_t)B,
                       c->dpart + 2 * B + 1);
    if (hipMemcpyAsync(c->hpin, c->dpart + 2 * B, 2 * sizeof(double), hipMemcpyDeviceToHost, c->s) != hipSuccess)
        return MG_ERR_HIP;
    mg_status st = sync_status(c->s);
    if (st != MG_OK) return st;
    h_out[0] = c->hpin[0];
    h_out[1] = c->hpin[1];
    return MG_OK;
}

} // extern "C"

namespace {

// keep_ratio: the prediction is kept when, after its check iteration, the worse of
// rms H and rms M is below keep_ratio times that of the zero state.
mg_status warm_start(nn_ctx *c, mg_ctx *solver, const double *d_rho5, const double *d_rho1, const double *d_S,
                     const nn_norm *norm, double *d_u, double *d_W, double keep_ratio, int32_t *h_used,
                     double h_norms[4])
{
    if (!c || !solver || !d_rho5 || !d_rho1 || !d_S || !d_u || !d_W || !h_used || !norm_ok(norm) ||
        c->cfg.c_in != 4 || c->cfg.c_out != 4)
        return MG_ERR_INVALID;
    // the prediction is written into the solver's arrays and checked by its own
    // iteration: both must describe the same periodic grid, the solver must
    // update W and psi (not CTTK, where psi is data), and both must order their work on the same stream (the check
    // iteration then follows the unpacked prediction)
    const grtmg::SolverShape sh = grtmg::solver_shape(solver);
    if (sh.n != c->cfg.n || sh.bc != MG_BC_PERIODIC || !sh.momentum || sh.cttk || sh.user_stream != (void *)c->s)
        return MG_ERR_INVALID;
    const int64_t V = c->V[0];
    double zero[4], pred[4];
    // residual of the zero start (u = 0, W = 0) on the solver's stream, while the
    // network runs on this one (the solver's calls are ordered after the work on
    // its caller stream; the prediction is written into u, W once it is done)
    mg_status st = grtmg::zero_norms_begin(solver, d_u, d_W);
    if (st != MG_OK) return st;
    st = nn_pack_input(c, d_rho5, d_rho1, d_S, norm, c->x);
    if (st == MG_OK) forward(c, c->x, c->out);
    const mg_status sz = grtmg::zero_norms_end(solver, zero);
    if (st != MG_OK) return st;
    if (sz != MG_OK) return sz;
    st = nn_unpack_output(c, c->out, norm, d_u, d_W);
    if (st != MG_OK) return st;
    // one outer iteration first: the smoother removes the BF16-level roughness
    // of the prediction at once, and the comparison is then about the smooth
    // error that decides the remaining iterations.  The solver runs it as its
    // own outer iteration (the captured graph the solve that follows replays)
    // and reports the norms after it; no tolerance can be met (tol 1e-300).
    mg_report rep;
    std::memset(&rep, 0, sizeof(rep));
    st = grtmg::check_iteration(solver, d_u, d_W, &rep);
    if (st != MG_OK && st != MG_ERR_NOT_CONVERGED && st != MG_ERR_DIVERGED) return st;
    pred[0] = rep.h_rms;
    pred[1] = rep.m_rms;
    pred[2] = rep.h_max;
    pred[3] = rep.m_max;
    if (st == MG_ERR_DIVERGED && std::isfinite(pred[0]) && std::isfinite(pred[1]))
        pred[0] = pred[1] = std::numeric_limits<double>::infinity(); // never kept
    const double wz = std::max(zero[0], zero[1]), wp = std::max(pred[0], pred[1]);
    const bool keep = std::isfinite(pred[0]) && std::isfinite(pred[1]) && wp < keep_ratio * wz;
    if (!keep) {
        grtmg::cancel_continue(solver);
        if (hipMemsetAsync(d_u, 0, V * sizeof(double), c->s) != hipSuccess ||
            hipMemsetAsync(d_W, 0, 3 * V * sizeof(double), c->s) != hipSuccess)
            return MG_ERR_HIP;
        st = sync_status(c->s);
        if (st != MG_OK) return st;
    }
    *h_used = keep ? 1 : 0;
    if (h_norms) {
        h_norms[0] = pred[0];
        h_norms[1] = pred[1];
        h_norms[2] = zero[0];
        h_norms[3] = zero[1];
    }
    return MG_OK;
}

} // namespace

extern "C" {

mg_status nn_warm_start(nn_ctx *c, mg_ctx *solver, const double *d_rho5, const double *d_rho1, const double *d_S,
                        const nn_norm *norm, double *d_u, double *d_W, int32_t *h_used, double h_norms[4])
{
    return warm_start(c, solver, d_rho5, d_rho1, d_S, norm, d_u, d_W, 1.0, h_used, h_norms);
}

mg_status nn_warm_start_ratio(nn_ctx *c, mg_ctx *solver, const double *d_rho5, const double *d_rho1,
                              const double *d_S, const nn_norm *norm, double *d_u, double *d_W, double keep_ratio,
                              int32_t *h_used, double h_norms[4])
{
    if (!(keep_ratio > 0.0 && keep_ratio <= 1.0)) return MG_ERR_INVALID;
    return warm_start(c, solver, d_rho5, d_rho1, d_S, norm, d_u, d_W, keep_ratio, h_used, h_norms);
}

// ---- single operations ------------------------------------------------------------------

namespace {

bool op_ok(int32_t n, int32_t cin, int32_t cout)
{
    return n >= 1 && n <= 512 && cin >= 8 && cin <= 256 && cin % 8 == 0 && cout >= 1 && cout <= 256;
}

Layer op_layer(int cin, int cout)
{
    Layer ly;
    int64_t off = 0;
    make_layer(ly, cin, cout, cin, 0, true, off);
    return ly;
}

struct OpScratch {
    size_t wf, wt, part, partb, total;
};

OpScratch op_scratch(int32_t cin, int32_t cout, int32_t n)
{
    const Layer ly = op_layer(cin, cout);
    size_t pf = 0, pb = 0;
    for (int br = 0; br < 2; br++) {
        const WSplit w = wsplit(ly.cin_pad, ly.cout, n, br == 1 && brick_ok(n));
        pf = std::max(pf, wsplit_floats(w));
        pb = std::max(pb, (size_t)w.nsplit * w.cot * 16);
    }
    OpScratch o;
    o.wf = 0;
    o.wt = align_up(packed_bytes(ly.ntile, ly.nchunk), 256);
    o.part = o.wt + align_up(packed_bytes(ly.ntile_t, ly.nchunk_t), 256);
    o.partb = o.part + align_up(pf * 4, 256);
    o.total = o.partb + align_up(pb * 4, 256);
    return o;
}

} // namespace

size_t nn_op_scratch_bytes(int32_t cin, int32_t cout, int32_t n)
{
    if (!op_ok(n, cin, cout)) return 0;
    return op_scratch(cin, cout, n).total;
}

mg_status nn_conv3_forward(int32_t n, int32_t cin, int32_t cout, const uint16_t *d_x, int32_t act, const float *d_w,
                           const float *d_b, float *d_y, void *d_scratch, size_t scratch_bytes, void *stream)
{
    if (!op_ok(n, cin, cout) || !d_x || !d_w || !d_y || !d_scratch || (act != 0 && act != 1) || !aligned16(d_x))
        return MG_ERR_INVALID;
    const OpScratch o = op_scratch(cin, cout, n);
    if (scratch_bytes < o.total || ((uintptr_t)d_scratch % 256) != 0) return MG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Layer ly = op_layer(cin, cout);
    ly.wf = (u32x4 *)((char *)d_scratch + o.wf);
    ly.wt = nullptr;
    ly.ntile_t = 0;
    const int64_t nf = (int64_t)ly.ntile * ly.nchunk * 64;
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(nf)), dim3(kNBlock), 0, s, d_w, cin, cout, ly.ko, ly.nchunk,
                       ly.ntile, 0, ly.wf);
    Out oy, none;
    oy.channels = cout;
    oy.mode = kEpStoreF32;
    oy.ptr = d_y;
    launch_conv(s, ly, false, n, d_x, cin, act, nullptr, 0, 0, d_b, oy, none);
    return hip_ok();
}

mg_status nn_conv3_backward_data(int32_t n, int32_t cin, int32_t cout, const uint16_t *d_dy, const float *d_w,
                                 float *d_dx, void *d_scratch, size_t scratch_bytes, void *stream)
{
    if (!op_ok(n, cin, cout) || !d_dy || !d_w || !d_dx || !d_scratch || !aligned16(d_dy)) return MG_ERR_INVALID;
    const OpScratch o = op_scratch(cin, cout, n);
    if (scratch_bytes < o.total || ((uintptr_t)d_scratch % 256) != 0) return MG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Layer ly = op_layer(cin, cout);
    ly.wt = (u32x4 *)((char *)d_scratch + o.wt);
    const int64_t nt = (int64_t)ly.ntile_t * ly.nchunk_t * 64;
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(nt)), dim3(kNBlock), 0, s, d_w, cin, cout, ly.ko_t, ly.nchunk_t,
                       ly.ntile_t, 1, ly.wt);
    Out ox, none;
    ox.channels = cin;
    ox.mode = kEpStoreF32;
    ox.ptr = d_dx;
    launch_conv(s, ly, true, n, d_dy, ly.cout8, 0, nullptr, 0, 0, nullptr, ox, none);
    return hip_ok();
}

mg_status nn_conv3_backward_weight(int32_t n, int32_t cin, int32_t cout, const uint16_t *d_x, int32_t act,
                                   const uint16_t *d_dy, float *d_dw, float *d_db, void *d_scratch,
                                   size_t scratch_bytes, void *stream)
{
    if (!op_ok(n, cin, cout) || !d_x || !d_dy || !d_dw || !d_db || !d_scratch || (act != 0 && act != 1))
        return MG_ERR_INVALID;
    const OpScratch o = op_scratch(cin, cout, n);
    if (scratch_bytes < o.total || ((uintptr_t)d_scratch % 256) != 0) return MG_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Layer ly = op_layer(cin, cout);
    float *part = (float *)((char *)d_scratch + o.part), *partb = (float *)((char *)d_scratch + o.partb);
    // the reduction overwrites dW (cout*cin*27) and db (cout)
    launch_wgrad_to(s, ly, n, d_x, cin, act, nullptr, 0, 0, d_dy, ly.cout8, part, partb, d_dw, d_db, 0);
    return hip_ok();
}

} // extern "C"
