// grtmg.hip -- host runtime and C ABI of the constraint multigrid.
//
// The runtime owns nothing on the device: mg_setup carves the caller's
// workspace into per-level buffers, the reduction partials, a few device
// scalars and the coarsest-level matrices.  Every kernel is enqueued on the
// caller's stream; the only host/device crossing per outer iteration is the
// copy of four norms (plus status flags) to pinned host memory.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>
#include <type_traits>

#include "grtmg.h"
#include "mg_kernels.hpp"
#include "mg_tiled.hpp"
#include "mg_cttk.hpp"
#include "mg_refine.hpp"
#include "mg_fourier.hpp"
#include "mg_internal.h"

using namespace grtmg;

namespace {

constexpr int kMaxLevels = 16;
constexpr int kMaxCoarsePsi = 1728; // coarsest psi unknowns (12^3)
constexpr int kMaxCoarseW = 1536;   // coarsest W unknowns (3 * 8^3)
constexpr int kSrcBlocks = 2048;    // grid of the source kernel (partials in scratch)

// device scalar slots
enum {
    S_NORM = 0,
    S_MEANS = 4,
    S_ACTIVE = 7,
    S_MEAND = 8,
    S_ITERS = 11,
    S_FLAG_PSI = 12,
    S_FLAG_W = 13,
    S_DIVERGED = 14,
    S_K2 = 15, // K^2 of a batch member
    S_AA = 16, // CTTK Anderson mixing: <dF, f>, <dF, dF>, steps taken, gamma
    S_COUNT = 20
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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

unsigned nblk(int64_t count) { return (unsigned)((count + kBlock - 1) / kBlock); }

// Calls f with a non-periodic boundary rule (Robin, reflective, extrapolating, zero) as a
// compile-time constant: f(std::integral_constant<int, kBc...>{}).
template <typename F>
void with_bc(int bc, F &&f)
{
    switch (bc) {
    case MG_BC_REFLECT: f(std::integral_constant<int, kBcReflect>{}); break;
    case MG_BC_EXTRAP: f(std::integral_constant<int, kBcExtrap>{}); break;
    case MG_BC_ZERO: f(std::integral_constant<int, kBcZero>{}); break;
    default: f(std::integral_constant<int, kBcRobin>{}); break;
    }
}

constexpr int kProbeMax = 4096;
// Brick depths along x of the tiled kernels: defaults and the candidates the
// autotuner times (per-cell arithmetic does not depend on the depth, so every
// candidate gives bitwise the same fields).  The FP64 W brick is limited by
// LDS (depth 2 uses 152 KB).
constexpr int kBrickPsi = 4;
constexpr int kBrickW = 2;
// marched columns of 64-cell rows (levels whose side is a multiple of 64 but
// not of 128): x planes per column of the W pass and of the W defect restriction
constexpr int kMarch64Pass = 1;
constexpr int kMarch64Defect = 2;
constexpr int kBrickR = 2;
constexpr int kCandPsi[] = {2, 4, 8};
// W pass depths: 1, 2, 4 are bricks staged whole, 8 and 16 columns marched plane by plane
constexpr int kCandW32[] = {2, 4, 8, 16};
constexpr int kCandW64[] = {1, 2, 8};
constexpr int kCandR[] = {2, 4, 8, 16}; // 8, 16: x-marched columns (periodic)
constexpr int kCandTail[] = {0, 1}; // V-cycle tail off / on

} // namespace

struct mg_ctx {
    mg_params p;
    hipStream_t user_s; // the caller's stream: every call is ordered after / before it by events
    hipStream_t s;      // internal stream (captured into the outer-iteration graph)
    // second stream of a single context with MG_FLAG_SAME_STATE: the psi step's branch
    // of the captured outer iteration (forked from and joined back into s by events)
    hipStream_t s2;
    hipEvent_t ev_fork, ev_join;
    bool capturing, forking; // inside capture_graph; the W step runs beside the psi step
    hipEvent_t ev_in, ev_out;
    hipEvent_t ev_norm[2];     // norm copies of consecutive iterations (pinned slots hpin[0 / S_COUNT ..])
    int L;
    bool f32;
    bool momentum;
    size_t esz;
    int n[kMaxLevels];
    int64_t cells[kMaxLevels];
    Geo geo[kMaxLevels];
    TileMap tile[kMaxLevels];  // brick map of the psi smoother per level (tx == 0: not tiled)
    TileMap tileW[kMaxLevels]; // brick map of the W smoother per level
    TileMap tileR;             // brick map of the finest-level residual
    int tail_psi, tail_W;      // first level of the workgroup-resident V-cycle tail (-1: not possible)
    int tail_psi_min, tail_W_min; // the highest level a tail can start from (its arrays fit in LDS)
    bool tail_psi_on, tail_W_on; // tail in use (chosen by mg_autotune / mg_set_tile; off by default)
    int fourier_W;               // level solved exactly by discrete Fourier modes in the W V-cycle (-1: none)
    bool fourier_W_on;           // in use (on by default; mg_autotune / mg_set_tile may turn it off)
    float2 *specZ;               // complex buffer of that solve on 32^3 and 64^3 levels (3 n^3)
    void *pd0[kMaxLevels], *pd1[kMaxLevels], *pr[kMaxLevels], *pc[kMaxLevels];
    void *wd0[kMaxLevels], *wd1[kMaxLevels], *wr[kMaxLevels];
    double *part;
    double *part_w; // the W step's partial sums while it runs beside the psi step
    double *scal;
    int m_psi, m_W;
    double *A_psi, *aug_psi, *inv_psi;
    double *A_W, *aug_W, *inv_W;
    double *hpin;
    const double *rho5, *rho1, *S, *f;
    const double *bg_psi0, *bg_A2; // optional background fields (mg_set_background), borrowed
    double K2;
    // CTTK (MG_FLAG_CTTK): psi is data, K follows from eq. Ham after every W step; the
    // residuals read the shifted rho5_eff and S_eff (rho5 and S point at them) made
    // from the caller's rho5_in and S_in, and Kf holds K of the last evaluated state
    bool cttk;
    const double *rho5_in, *S_in;
    double *rho5_eff, *S_eff, *Kf;
    double *aa_W, *aa_f; // Anderson mixing history of the CTTK solve: previous W and step (3 n^3 each)
    // mixing over mix_depth >= 2 steps: rings of difference pairs dG = dW + dF and dF
    // (mix_depth x 3 n^3 each) and its device state {pairs stored, next slot, steps, .., gamma_0 ..}
    void *aa_dG, *aa_dF; // in the working type T
    double *aa_st;
    int vc_psi, vc_W;
    // batch membership: streams borrowed from the batch, updates gated by the
    // instance's active flag, a convergence check after every evaluation
    bool batched, own_streams;
    double batch_tol;
    // grouped batch launches: gz members (member z's arrays zs bytes after this
    // context's) per launch; K^2 read per member from its scalar block
    int gz;
    long long zs;
    const double *K2p;
    // outer-iteration graph (keyed by the state pointers it was captured for)
    hipGraphExec_t gexec;
    const double *g_u, *g_W;
    // timing probe
    int probe_kernel, probe_level, probe_count;
    hipEvent_t *probe_ev; // 2 * kProbeMax events, created on first use
    // continuation: the state the last solve left in (cont_u, cont_W), whose
    // evaluation is still current in the workspace; cleared by every other call
    bool cont_valid;
    const double *cont_u, *cont_W;
    double cont_nr[4], cont_prev; // its norms; worst norm of the iteration before (< 0: none)
};

namespace {

// Both steps of an outer iteration from one state (MG_FLAG_SAME_STATE; CTTK has its own loop).
bool same_state(const mg_ctx *c)
{
    return (c->p.flags & MG_FLAG_SAME_STATE) && c->momentum && !(c->p.flags & MG_FLAG_CTTK);
}

mg_status validate(const mg_params *p)
{
    if (!p) return MG_ERR_INVALID;
    if (p->levels < 1 || p->levels > kMaxLevels) return MG_ERR_INVALID;
    if (p->n < 3 || p->n > 4096) return MG_ERR_INVALID;
    // cell indices are 32-bit (n^3 < 2^32, n <= 1625)
    if ((double)p->n * p->n * (double)p->n >= 4294967296.0) return MG_ERR_INVALID;
    if (p->bc < MG_BC_PERIODIC || p->bc > MG_BC_ZERO) return MG_ERR_INVALID;
    if (p->precision != MG_PREC_FP64 && p->precision != MG_PREC_FP32_IR) return MG_ERR_INVALID;
    // the finest level's first pre-smoothing pass comes with the residual: nu_pre >= 1
    if (p->nu_pre < 1 || p->nu_post < 1 || p->nu_pre > 16 || p->nu_post > 16) return MG_ERR_INVALID;
    if (p->nu_pre_W < 0 || p->nu_post_W < 0 || p->nu_pre_W > 16 || p->nu_post_W > 16) return MG_ERR_INVALID;
    if (p->mix_depth < 0 || p->mix_depth > kMixMax) return MG_ERR_INVALID;
    if (p->solve_momentum != 0 && p->solve_momentum != 1) return MG_ERR_INVALID;
    if (p->solve_momentum && p->bc != MG_BC_PERIODIC) return MG_ERR_INVALID;
    // the W kernels address one component with 32-bit byte offsets
    if (p->solve_momentum && (double)p->n * p->n * (double)p->n * sizeof(double) >= 4294967296.0)
        return MG_ERR_INVALID;
    if ((p->flags & ~(MG_FLAG_CONFORMAL_MATTER | MG_FLAG_EAGER | MG_FLAG_CTTK | MG_FLAG_CUBIC_PROLONG |
                      MG_FLAG_SAME_STATE)) != 0)
        return MG_ERR_INVALID;
    // CTTK: the coupled periodic solve with psi = 1 + u as data, K from eq. Ham
    if ((p->flags & MG_FLAG_CTTK) &&
        (!p->solve_momentum || p->bc != MG_BC_PERIODIC || p->K != 0.0 || p->puncture_mass != 0.0 ||
         (p->flags & MG_FLAG_CONFORMAL_MATTER)))
        return MG_ERR_INVALID;
    if (!(p->length > 0.0) || !std::isfinite(p->length)) return MG_ERR_INVALID;
    if (!std::isfinite(p->K) || !(p->puncture_mass >= 0.0) || !std::isfinite(p->puncture_mass))
        return MG_ERR_INVALID;
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(p->origin[a]) || !std::isfinite(p->puncture_pos[a])) return MG_ERR_INVALID;
    int n = p->n;
    for (int l = 0; l + 1 < p->levels; l++) {
        if (n % 2 != 0 || n < 6) return MG_ERR_INVALID;
        n /= 2;
    }
    if (n < 3) return MG_ERR_INVALID;
    const int64_t mc = (int64_t)n * n * n;
    if (mc > kMaxCoarsePsi) return MG_ERR_INVALID;
    if (p->solve_momentum && 3 * mc > kMaxCoarseW) return MG_ERR_INVALID;
    return MG_OK;
}

// The level of the W V-cycle solved exactly by discrete Fourier modes: the first one
// below the finest with 16, 32 or 64 cells per axis, in FP32 periodic contexts with
// momentum; -1 if none.
int spectral_level(const mg_ctx *c)
{
    if (!c->momentum || !c->f32 || c->p.bc != MG_BC_PERIODIC) return -1;
    for (int l = 1; l < c->L; l++)
        if (c->n[l] == 16 || c->n[l] == 32 || c->n[l] == 64) return l;
    return -1;
}

// Lay out (or measure, when base is null) every device buffer of a context.
void carve(mg_ctx *c, Carver &cv)
{
    const mg_params &p = c->p;
    int n = p.n;
    for (int l = 0; l < c->L; l++) {
        const int64_t m = (int64_t)n * n * n;
        c->n[l] = n;
        c->cells[l] = m;
        c->pd0[l] = cv.take(m * c->esz);
        c->pd1[l] = cv.take(m * c->esz);
        c->pr[l] = cv.take(m * c->esz);
        c->pc[l] = cv.take(m * c->esz);
        if (c->momentum) {
            c->wd0[l] = cv.take(3 * m * c->esz);
            c->wd1[l] = cv.take(3 * m * c->esz);
            c->wr[l] = cv.take(3 * m * c->esz);
        } else {
            c->wd0[l] = c->wd1[l] = c->wr[l] = nullptr;
        }
        n /= 2;
    }
    const int ls = spectral_level(c);
    c->specZ = ls >= 0 && c->n[ls] > kFourierN ? (float2 *)cv.take(3 * c->cells[ls] * sizeof(float2)) : nullptr;
    const int64_t nb = nblk(c->cells[0]);
    // 4 partials per block of the finest level, and room for one block of the Anderson sums
    c->part = (double *)cv.take((size_t)std::max<int64_t>(nb * 4, kMixState) * sizeof(double));
    c->part_w = (p.flags & MG_FLAG_SAME_STATE) && c->momentum
                    ? (double *)cv.take((size_t)sum_blocks(c->cells[0]) * 3 * sizeof(double))
                    : nullptr;
    if (p.flags & MG_FLAG_CTTK) {
        const size_t m0 = (size_t)c->cells[0] * sizeof(double);
        c->rho5_eff = (double *)cv.take(m0);
        c->S_eff = (double *)cv.take(3 * m0);
        c->Kf = (double *)cv.take(m0);
        c->aa_W = (double *)cv.take(3 * m0);
        c->aa_f = (double *)cv.take(3 * m0);
        if (p.mix_depth >= 2) {
            // in the working type: FP32 rings in FP32 contexts
            c->aa_dG = cv.take((size_t)p.mix_depth * 3 * c->cells[0] * c->esz);
            c->aa_dF = cv.take((size_t)p.mix_depth * 3 * c->cells[0] * c->esz);
            c->aa_st = (double *)cv.take(kMixState * sizeof(double));
        } else {
            c->aa_dG = c->aa_dF = c->aa_st = nullptr;
        }
    } else {
        c->rho5_eff = c->S_eff = c->Kf = c->aa_W = c->aa_f = nullptr;
        c->aa_dG = c->aa_dF = c->aa_st = nullptr;
    }
    c->scal = (double *)cv.take(S_COUNT * sizeof(double));
    c->m_psi = (int)c->cells[c->L - 1];
    const size_t mp = (size_t)c->m_psi;
    c->A_psi = (double *)cv.take(mp * mp * sizeof(double));
    c->aug_psi = (double *)cv.take(2 * mp * mp * sizeof(double));
    c->inv_psi = (double *)cv.take(mp * mp * sizeof(double));
    if (c->momentum) {
        c->m_W = 3 * c->m_psi;
        const size_t mw = (size_t)c->m_W;
        c->A_W = (double *)cv.take(mw * mw * sizeof(double));
        c->aug_W = (double *)cv.take(2 * mw * mw * sizeof(double));
        c->inv_W = (double *)cv.take(mw * mw * sizeof(double));
    } else {
        c->m_W = 0;
        c->A_W = c->aug_W = c->inv_W = nullptr;
    }
}

// Coarsest sizes solved by the register-resident Gauss-Jordan kernel (one block).
bool wave_solvable(int m) { return m == 8 || m == 27 || m == 64; }

TileMap tilemap_rt(int n, int tx)
{
    switch (tx) {
    case 1: return make_tilemap<1>(n);
    case 2: return make_tilemap<2>(n);
    case 4: return make_tilemap<4>(n);
    case 8: return make_tilemap<8>(n);
    case 16: return make_tilemap<16>(n);
    default: return TileMap{0, 0, 0, 0};
    }
}

// The tiled W pass addresses the three components with 32-bit byte offsets.
bool w_tileable(int n) { return 3.0 * n * n * (double)n * sizeof(double) < 4294967296.0; }

TileMap rtilemap_rt(int n, int tx)
{
    switch (tx) {
    case 1: return make_rtilemap<1>(n);
    case 2: return make_rtilemap<2>(n);
    case 4: return make_rtilemap<4>(n);
    case 8: return make_rmarchmap<8>(n);
    case 16: return make_rmarchmap<16>(n);
    default: return TileMap{0, 0, 0, 0};
    }
}

unsigned ntiles(const TileMap &t) { return (unsigned)(t.nx * t.ny * t.nz); }

void init_geo(mg_ctx *c)
{
    for (int l = 0; l < c->L; l++) {
        c->geo[l] = make_geo(c->n[l], c->p.bc, c->p.length, c->p.origin, c->p.puncture_pos);
        c->tile[l] = make_tilemap<kBrickPsi>(c->n[l]);
        c->tileW[l] = w_tileable(c->n[l]) ? make_tilemap<kBrickW>(c->n[l]) : TileMap{0, 0, 0, 0};
    }
    // finest residual: marched columns (periodic) when they still give two
    // workgroups per compute unit of a 256-CU device, else bricks
    c->tileR = make_rtilemap<kBrickR>(c->n[0]);
    if (c->p.bc == MG_BC_PERIODIC) {
        const TileMap r16 = make_rmarchmap<16>(c->n[0]), r8 = make_rmarchmap<8>(c->n[0]);
        if (r16.tx > 0 && ntiles(r16) >= 512)
            c->tileR = r16;
        else if (r8.tx > 0 && ntiles(r8) >= 512)
            c->tileR = r8;
    }
    // V-cycle tails: from the first level whose levels down to the coarsest fit
    // the tail's LDS arrays; at least one level above the coarsest, at most
    // kMaxTail levels, coarsest psi system solvable in registers.
    c->tail_psi = c->tail_W = -1;
    c->tail_psi_on = c->tail_W_on = false;
    const int cap_psi = c->p.bc != MG_BC_PERIODIC ? TailCap<float>::kPsiRobin
                        : c->f32                   ? TailCap<float>::kPsi
                                                   : TailCap<double>::kPsi;
    const int cap_W = c->f32 ? TailCap<float>::kW : TailCap<double>::kW;
    auto cells_from = [&](int l) {
        int64_t s = 0;
        for (int q = l; q < c->L; q++) s += c->cells[q];
        return s;
    };
    for (int l = 0; l + 1 < c->L; l++)
        if (cells_from(l) <= cap_psi && c->L - l <= kMaxTail && wave_solvable(c->m_psi)) {
            c->tail_psi = l;
            break;
        }
    if (c->momentum)
        for (int l = 0; l + 1 < c->L; l++)
            if (cells_from(l) <= cap_W && c->L - l <= kMaxTail && c->m_W <= 1536) {
                c->tail_W = l;
                break;
            }
    // the tails prolong trilinearly inside: none with cubic prolongation
    if (c->p.flags & MG_FLAG_CUBIC_PROLONG) c->tail_psi = c->tail_W = -1;
    c->tail_psi_min = c->tail_psi;
    c->tail_W_min = c->tail_W;
    // exact bottom of the W V-cycle
    c->fourier_W = spectral_level(c);
    c->fourier_W_on = c->fourier_W >= 0;
}

// Level l of the W V-cycle is solved by discrete Fourier modes (the float4 accesses
// need the members of a batch 16-byte apart).
bool fourier_at(const mg_ctx *c, int l) { return c->fourier_W_on && l == c->fourier_W && c->zs % 16 == 0; }


// Records an event pair around the launches in its scope when (kernel, level)
// matches the probe set by mg_probe.  A probe made with in_launch = true records
// no events itself: the single launch of its scope goes through probe_launch,
// which hands the pair to the dispatch, so that it spans the kernel alone.
struct Probe {
    mg_ctx *c;
    bool on, in_launch;
    Probe(mg_ctx *ctx, int kernel, int level, bool in_launch_ = false) : c(ctx), in_launch(in_launch_)
    {
        on = c->probe_ev && c->probe_kernel == kernel &&
             (c->probe_level < 0 || c->probe_level == level) && c->probe_count < kProbeMax;
        if (on && !in_launch) (void)hipEventRecord(c->probe_ev[2 * c->probe_count], c->s);
    }
    ~Probe()
    {
        if (on) {
            if (!in_launch) (void)hipEventRecord(c->probe_ev[2 * c->probe_count + 1], c->s);
            c->probe_count++;
        }
    }
};

template <typename F, typename... Args>
void probe_launch(const Probe &pr, F kernel, const dim3 &grid, const dim3 &blk, hipStream_t s, Args... args)
{
    if (pr.on && pr.in_launch)
        hipExtLaunchKernelGGL(kernel, grid, blk, 0, s, pr.c->probe_ev[2 * pr.c->probe_count],
                              pr.c->probe_ev[2 * pr.c->probe_count + 1], 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, blk, 0, s, args...);
}

template <typename T>
void fill(hipStream_t s, T *a, int64_t count, T v, int gz = 1, long long zs = 0)
{
    if (count > 0) hipLaunchKernelGGL(k_fill<T>, dim3(nblk(count), 1, gz), dim3(kBlock), 0, s, a, count, v, zs);
}

// Defect+restriction form: one thread per fine cell on grids of at most 32^3
// cells (latency-bound), one per coarse cell above (register reuse).
bool fine_threads(int n_fine) { return n_fine <= 32; }

// ---- coarsest level -----------------------------------------------------------------

void factor(hipStream_t s, double *A, double *aug, double *inv, int m, double *flag)
{
    hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(kGjThreads), 0, s, (const double *)A, aug, inv,
                       m, flag);
}


template <int BC, typename T>
void launch_coarse_wave(mg_ctx *c, int l, const T *r, T *x)
{
    const Geo &g = c->geo[l];
    const T *cf = (const T *)c->pc[l];
    double *flag = c->scal + S_FLAG_PSI;
    switch (c->m_psi) {
    case 8: hipLaunchKernelGGL((k_coarse_psi_block<BC, T, 8>), dim3(1, 1, c->gz), dim3(kGjWaves * kWave), 0, c->s, g, cf, r, x, flag); break;
    case 27: hipLaunchKernelGGL((k_coarse_psi_block<BC, T, 27>), dim3(1, 1, c->gz), dim3(kGjWaves * kWave), 0, c->s, g, cf, r, x, flag); break;
    default: hipLaunchKernelGGL((k_coarse_psi_block<BC, T, 64>), dim3(1, 1, c->gz), dim3(kGjWaves * kWave), 0, c->s, g, cf, r, x, flag); break;
    }
}

template <typename T>
void coarse_psi(mg_ctx *c, const T *r, T *x)
{
    const int l = c->L - 1;
    Probe pr(c, MG_PROBE_COARSE, l);
    const int m = c->m_psi;
    if (wave_solvable(m)) {
        if (c->p.bc == MG_BC_PERIODIC)
            launch_coarse_wave<kBcPeriodic, T>(c, l, r, x);
        else
            with_bc(c->p.bc, [&](auto bcx) {
                constexpr int BCX = decltype(bcx)::value;
                launch_coarse_wave<BCX, T>(c, l, r, x);
            });
        return;
    }
    if (m <= kKrylovMax) {
        // conjugate gradients (periodic) or BiCGSTAB (Robin) on one block; a system it
        // does not solve to 1e-12 raises the singular flag
        if (c->p.bc == MG_BC_PERIODIC)
            hipLaunchKernelGGL((k_coarse_psi_krylov<kBcPeriodic, T>), dim3(1, 1, c->gz), dim3(kGjWaves * kWave), 0, c->s,
                               c->geo[l], m, (const T *)c->pc[l], r, x, c->scal + S_FLAG_PSI);
        else
            with_bc(c->p.bc, [&](auto bcx) {
                constexpr int BCX = decltype(bcx)::value;
                hipLaunchKernelGGL((k_coarse_psi_krylov<BCX, T>), dim3(1, 1, c->gz), dim3(kGjWaves * kWave), 0, c->s,
                                   c->geo[l], m, (const T *)c->pc[l], r, x, c->scal + S_FLAG_PSI);
            });
        return;
    }
    fill<double>(c->s, c->A_psi, (int64_t)m * m, 0.0);
    if (c->p.bc == MG_BC_PERIODIC)
        hipLaunchKernelGGL((k_assemble_psi<kBcPeriodic, T>), dim3(nblk(m)), dim3(kBlock), 0, c->s,
                           c->geo[l], (const T *)c->pc[l], c->A_psi);
    else
        with_bc(c->p.bc, [&](auto bcx) {
            constexpr int BCX = decltype(bcx)::value;
            hipLaunchKernelGGL((k_assemble_psi<BCX, T>), dim3(nblk(m)), dim3(kBlock), 0, c->s,
                               c->geo[l], (const T *)c->pc[l], c->A_psi);
        });
    factor(c->s, c->A_psi, c->aug_psi, c->inv_psi, m, c->scal + S_FLAG_PSI);
    hipLaunchKernelGGL(k_coarse_apply<T>, dim3((m + kApplyRows - 1) / kApplyRows, 1, c->gz), dim3(kBlock),
                       m * sizeof(double), c->s, (const double *)c->inv_psi, m, r, x, 0, c->zs);
}

template <typename T>
void coarse_W(mg_ctx *c, const T *r, T *x)
{
    const int m = c->m_W;
    Probe pr(c, MG_PROBE_COARSE, c->L - 1);
    hipLaunchKernelGGL(k_coarse_apply<T>, dim3((m + kApplyRows - 1) / kApplyRows, 1, c->gz), dim3(kBlock),
                       m * sizeof(double), c->s, (const double *)c->inv_W, m, r, x, 3, c->zs);
}

// ---- psi V-cycle ----------------------------------------------------------------------

template <int BC, typename T>
void launch_psi_tiled(hipStream_t s, const Geo &g, const TileMap &tm, const T *in, T *out, const T *r, const T *cf,
                      int colour)
{
    const dim3 blk(kLanes, kTY), grid(ntiles(tm), 1, g.gz);
    switch (tm.tx) {
    case 2: hipLaunchKernelGGL((k_pass_psi_tiled<BC, T, 2>), grid, blk, 0, s, g, tm, in, out, r, cf, colour); break;
    case 8: hipLaunchKernelGGL((k_pass_psi_tiled<BC, T, 8>), grid, blk, 0, s, g, tm, in, out, r, cf, colour); break;
    default: hipLaunchKernelGGL((k_pass_psi_tiled<BC, T, 4>), grid, blk, 0, s, g, tm, in, out, r, cf, colour); break;
    }
}

template <typename T>
void pass_psi(mg_ctx *c, int l, const T *in, T *out, int colour)
{
    Probe pr(c, MG_PROBE_PASS_PSI, l);
    const Geo &g = c->geo[l];
    const unsigned nb = nblk(c->cells[l]);
    const TileMap &tm = c->tile[l];
    if (tm.tx > 0) {
        const T *r = (const T *)c->pr[l], *cf = (const T *)c->pc[l];
        if (c->p.bc == MG_BC_PERIODIC)
            launch_psi_tiled<kBcPeriodic, T>(c->s, g, tm, in, out, r, cf, colour);
        else
            with_bc(c->p.bc, [&](auto bcx) {
                constexpr int BCX = decltype(bcx)::value;
                launch_psi_tiled<BCX, T>(c->s, g, tm, in, out, r, cf, colour);
            });
        return;
    }
    if (c->p.bc == MG_BC_PERIODIC && c->n[l] % 2 == 0)
        hipLaunchKernelGGL(k_pass_psi_pairs<T>, dim3(nblk(c->cells[l] / 2), 1, c->gz), dim3(kBlock), 0, c->s, g, in, out,
                           (const T *)c->pr[l], (const T *)c->pc[l], colour);
    else if (c->p.bc == MG_BC_PERIODIC)
        hipLaunchKernelGGL((k_pass_psi<kBcPeriodic, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, g, in, out,
                           (const T *)c->pr[l], (const T *)c->pc[l], colour);
    else
        with_bc(c->p.bc, [&](auto bcx) {
            constexpr int BCX = decltype(bcx)::value;
            hipLaunchKernelGGL((k_pass_psi<BCX, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, g, in, out,
                               (const T *)c->pr[l], (const T *)c->pc[l], colour);
        });
}

template <typename T>
// first_done: the first colour pass from a zero correction was written into
// pd1 by the producer of this level's right-hand side.
void smooth_psi(mg_ctx *c, int l, int sweeps, bool first_done = false)
{
    for (int s = 0; s < sweeps; s++) {
        if (s > 0 || !first_done) pass_psi<T>(c, l, (const T *)c->pd0[l], (T *)c->pd1[l], 0);
        pass_psi<T>(c, l, (const T *)c->pd1[l], (T *)c->pd0[l], 1);
    }
}

template <typename T>
// d1 (may be null; needs cc): first colour pass of the coarse level from zero.
void defect_restrict_psi(mg_ctx *c, int l, const T *d, const T *r, const T *cf, T *rc, T *cc, T *d1 = nullptr)
{
    Probe pr(c, MG_PROBE_DEFECT_RESTRICT_PSI, l);
    const Geo &g = c->geo[l], &gc = c->geo[l + 1];
    if (!cc) d1 = nullptr;
    if (fine_threads(c->n[l])) {
        const unsigned nb = nblk(8 * c->cells[l + 1]);
        if (c->p.bc == MG_BC_PERIODIC)
            hipLaunchKernelGGL((k_defect_restrict_psi_fine<kBcPeriodic, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, g, d, r,
                               cf, rc, cc, d1, gc);
        else
            with_bc(c->p.bc, [&](auto bcx) {
                constexpr int BCX = decltype(bcx)::value;
                hipLaunchKernelGGL((k_defect_restrict_psi_fine<BCX, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, g, d, r,
                                   cf, rc, cc, d1, gc);
            });
    } else {
        const unsigned nb = nblk(c->cells[l + 1]);
        if (c->p.bc == MG_BC_PERIODIC)
            hipLaunchKernelGGL((k_defect_restrict_psi<kBcPeriodic, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, g, d, r, cf,
                               rc, cc, d1, gc);
        else
            with_bc(c->p.bc, [&](auto bcx) {
                constexpr int BCX = decltype(bcx)::value;
                hipLaunchKernelGGL((k_defect_restrict_psi<BCX, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, g, d, r, cf,
                                   rc, cc, d1, gc);
            });
    }
}

// d1 (may be null): first colour pass of the coarse level from zero.
template <typename T>
void defect_restrict_W(mg_ctx *c, int l, const T *d, const T *r, T *rc, T *d1 = nullptr)
{
    Probe pr(c, MG_PROBE_DEFECT_RESTRICT_W, l);
    const int n = c->n[l];
    const T idiag = (T)(1.0 / (-100.0 * c->geo[l + 1].inv12h2));
    const TileMap tm = w_tileable(n) ? make_marchmap<8, 128>(n) : TileMap{0, 0, 0, 0};
    const TileMap tm64 = w_tileable(n) ? make_marchmap<kMarch64Defect, 64>(n) : TileMap{0, 0, 0, 0};
    if (tm.tx > 0)
        hipLaunchKernelGGL((k_defect_restrict_W_march<T, 8, 128>), dim3(ntiles(tm), 1, c->gz), dim3(kLanes, kTY), 0, c->s,
                           c->geo[l], tm, d, r, rc, d1, idiag);
    else if (tm64.tx > 0)
        hipLaunchKernelGGL((k_defect_restrict_W_march<T, kMarch64Defect, 64>), dim3(ntiles(tm64), 1, c->gz),
                           dim3(kLanes, kTY), 0, c->s, c->geo[l], tm64, d, r, rc, d1, idiag);
    else if (fine_threads(n))
        hipLaunchKernelGGL(k_defect_restrict_W_quad<T>, dim3(nblk(32 * c->cells[l + 1]), 1, c->gz), dim3(kBlock), 0, c->s,
                           c->geo[l], d, r, rc, d1, idiag);
    else
        hipLaunchKernelGGL(k_defect_restrict_W<T>, dim3(nblk(c->cells[l + 1]), 1, c->gz), dim3(kBlock), 0, c->s, c->geo[l], d,
                           r, rc, d1, idiag);
}

template <typename T>
void prolong_add(mg_ctx *c, int lc, const T *coarse, T *fine, int ncomp)
{
    Probe pr(c, MG_PROBE_PROLONG, lc - 1);
    const Geo &gc = c->geo[lc];
    if (c->p.flags & MG_FLAG_CUBIC_PROLONG) {
        const int nc = c->n[lc];
        const bool staged = nc % kCubZ == 0 && nc % kCubY == 0 && nc % kCubX == 0;
        const unsigned nbk = staged ? (unsigned)((nc / kCubX) * (nc / kCubY) * (nc / kCubZ)) : nblk(c->cells[lc]);
        auto launch = [&](auto bcx) {
            constexpr int BCX = decltype(bcx)::value;
            if (staged)
                hipLaunchKernelGGL((k_prolong_cubic_add_staged<BCX, T>), dim3(nbk, 1, c->gz), dim3(kBlock), 0, c->s, gc,
                                   coarse, fine, ncomp);
            else
                hipLaunchKernelGGL((k_prolong_cubic_add<BCX, T>), dim3(nbk, 1, c->gz), dim3(kBlock), 0, c->s, gc,
                                   coarse, fine, ncomp);
        };
        if (c->p.bc == MG_BC_PERIODIC)
            launch(std::integral_constant<int, kBcPeriodic>{});
        else
            with_bc(c->p.bc, launch);
        return;
    }
    const unsigned nb = nblk(c->cells[lc - 1]);
    if (c->p.bc == MG_BC_PERIODIC) // one thread per fine z pair
        hipLaunchKernelGGL(k_prolong_add_pairs<T>, dim3(nblk(c->cells[lc - 1] / 2), 1, c->gz), dim3(kBlock), 0, c->s, gc,
                           coarse, fine, ncomp);
    else
        with_bc(c->p.bc, [&](auto bcx) {
            constexpr int BCX = decltype(bcx)::value;
            hipLaunchKernelGGL((k_prolong_add<BCX, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, gc, coarse,
                               fine, ncomp);
        });
}

// After the residual wrote the finest c: restrict c level by level and, when
// the coarsest system is too large for the register-resident solver, assemble and
// invert it.  All on the context's stream: the V-cycle kernels that follow
// stay on one queue of the graph.
// Without a V-cycle tail and with the coarsest psi system solved in registers,
// the coefficient c of each coarser level is restricted by the defect
// restriction that produces that level's right-hand side (the level is not
// smoothed before), so no separate sweep over the levels is needed.
// A tail restricts c below its own first level.
bool c_with_defect(const mg_ctx *c) { return wave_solvable(c->m_psi) || c->m_psi <= kKrylovMax; }

template <typename T>
void restrict_coefficients(mg_ctx *c)
{
    if (c_with_defect(c)) return; // each level's c comes with its defect restriction
    for (int l = 0; l + 1 < c->L; l++)
        hipLaunchKernelGGL(k_restrict<T>, dim3(nblk(c->cells[l + 1]), 1, c->gz), dim3(kBlock), 0, c->s, c->n[l],
                           (const T *)c->pc[l], (T *)c->pc[l + 1], c->zs);
    const int l = c->L - 1;
    const int m = c->m_psi;
    if (wave_solvable(m) || m <= kKrylovMax) return; // solved directly at the bottom of the V-cycle
    fill<double>(c->s, c->A_psi, (int64_t)m * m, 0.0);
    if (c->p.bc == MG_BC_PERIODIC)
        hipLaunchKernelGGL((k_assemble_psi<kBcPeriodic, T>), dim3(nblk(m)), dim3(kBlock), 0, c->s, c->geo[l],
                           (const T *)c->pc[l], c->A_psi);
    else
        with_bc(c->p.bc, [&](auto bcx) {
            constexpr int BCX = decltype(bcx)::value;
            hipLaunchKernelGGL((k_assemble_psi<BCX, T>), dim3(nblk(m)), dim3(kBlock), 0, c->s, c->geo[l],
                               (const T *)c->pc[l], c->A_psi);
        });
    factor(c->s, c->A_psi, c->aug_psi, c->inv_psi, m, c->scal + S_FLAG_PSI);
}

// Sweeps of the W V-cycle: the parameters' own while its bottom is exact, else the psi
// cycle's.
int nu_pre_W(const mg_ctx *c)
{
    return c->p.nu_pre_W > 0 && fourier_at(c, c->fourier_W) ? c->p.nu_pre_W : c->p.nu_pre;
}
int nu_post_W(const mg_ctx *c)
{
    return c->p.nu_post_W > 0 && fourier_at(c, c->fourier_W) ? c->p.nu_post_W : c->p.nu_post;
}

template <typename T>
TailArgs<T> tail_args(mg_ctx *c, int l0, bool W)
{
    TailArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.nl = c->L - l0;
    a.nu_pre = c->p.nu_pre; // a W tail runs only below a multigrid bottom
    a.nu_post = c->p.nu_post;
    for (int q = 0; q < a.nl; q++) a.geo[q] = c->geo[l0 + q];
    a.r0 = (const T *)(W ? c->wr[l0] : c->pr[l0]);
    a.c0 = W ? nullptr : (const T *)c->pc[l0];
    a.d0 = (T *)(W ? c->wd0[l0] : c->pd0[l0]);
    a.inv = c->inv_W;
    a.flag = c->scal + S_FLAG_PSI;
    return a;
}

template <typename T>
void tail_psi(mg_ctx *c)
{
    Probe pr(c, MG_PROBE_COARSE, c->L - 1);
    const TailArgs<T> a = tail_args<T>(c, c->tail_psi, false);
    const dim3 g1(1, 1, c->gz), blk(kTailThreads);
    if (c->p.bc == MG_BC_PERIODIC) {
        switch (c->m_psi) {
        case 8: hipLaunchKernelGGL((k_tail_psi<kBcPeriodic, T, 8>), g1, blk, 0, c->s, a); break;
        case 27: hipLaunchKernelGGL((k_tail_psi<kBcPeriodic, T, 27>), g1, blk, 0, c->s, a); break;
        default: hipLaunchKernelGGL((k_tail_psi<kBcPeriodic, T, 64>), g1, blk, 0, c->s, a); break;
        }
    } else {
        with_bc(c->p.bc, [&](auto bcx) {
            constexpr int BCX = decltype(bcx)::value;
            switch (c->m_psi) {
            case 8: hipLaunchKernelGGL((k_tail_psi<BCX, T, 8>), g1, blk, 0, c->s, a); break;
            case 27: hipLaunchKernelGGL((k_tail_psi<BCX, T, 27>), g1, blk, 0, c->s, a); break;
            default: hipLaunchKernelGGL((k_tail_psi<BCX, T, 64>), g1, blk, 0, c->s, a); break;
            }
        });
    }
}

// psi V-cycle on level l; the coefficients of levels > 0 and the coarsest
// inverse come from restrict_coefficients (and the tail kernel below its first level).
template <typename T>
// first_done: the producer of this level's right-hand side also wrote the
// first colour pass from a zero correction into pd1 (coarser levels, when c
// is restricted with the defect).
void vcycle_psi(mg_ctx *c, int l, bool first_done = false)
{
    if (c->tail_psi_on && l == c->tail_psi) {
        tail_psi<T>(c);
        return;
    }
    if (l == c->L - 1) {
        const int m = c->m_psi;
        if (wave_solvable(m) || m <= kKrylovMax) {
            coarse_psi<T>(c, (const T *)c->pr[l], (T *)c->pd0[l]);
            return;
        }
        Probe pr(c, MG_PROBE_COARSE, l);
        hipLaunchKernelGGL(k_coarse_apply<T>, dim3((m + kApplyRows - 1) / kApplyRows, 1, c->gz), dim3(kBlock),
                           m * sizeof(double), c->s, (const double *)c->inv_psi, m, (const T *)c->pr[l],
                           (T *)c->pd0[l], 0, c->zs);
        return;
    }
    if (!first_done) fill<T>(c->s, (T *)c->pd0[l], c->cells[l], T(0), c->gz, c->zs);
    smooth_psi<T>(c, l, c->p.nu_pre, first_done);
    // the next level's first pass comes with its defect when that level is
    // smoothed by grid launches (a tail starts from zero in LDS)
    const bool next_first = c_with_defect(c) && l + 2 < c->L && !(c->tail_psi_on && l + 1 == c->tail_psi);
    defect_restrict_psi<T>(c, l, (const T *)c->pd0[l], (const T *)c->pr[l], (const T *)c->pc[l],
                           (T *)c->pr[l + 1], c_with_defect(c) ? (T *)c->pc[l + 1] : nullptr,
                           next_first ? (T *)c->pd1[l + 1] : nullptr);
    vcycle_psi<T>(c, l + 1, next_first);
    prolong_add<T>(c, l + 1, (const T *)c->pd0[l + 1], (T *)c->pd0[l], 1);
    smooth_psi<T>(c, l, c->p.nu_post);
}

// ---- W V-cycle ------------------------------------------------------------------------

template <typename T>
void launch_W_tiled(const Probe &pr, hipStream_t s, const Geo &g, const TileMap &tm, const T *in, T *out, const T *r,
                    int colour)
{
    const dim3 blk(kLanes, kTY), grid(ntiles(tm), 1, g.gz);
    if (tm.tx == 8)
        probe_launch(pr, k_pass_W_march<T, 8, 128>, grid, blk, s, g, tm, in, out, r, colour);
    else if (tm.tx == 16)
        probe_launch(pr, k_pass_W_march<T, 16, 128>, grid, blk, s, g, tm, in, out, r, colour);
    else if (tm.tx == 1)
        probe_launch(pr, k_pass_W_tiled<T, 1>, grid, blk, s, g, tm, in, out, r, colour);
    else if (tm.tx == 4 && sizeof(T) == 4)
        probe_launch(pr, k_pass_W_tiled<float, 4>, grid, blk, s, g, tm, (const float *)in, (float *)out,
                     (const float *)r, colour);
    else
        probe_launch(pr, k_pass_W_tiled<T, 2>, grid, blk, s, g, tm, in, out, r, colour);
}

template <typename T>
void pass_W(mg_ctx *c, int l, const T *in, T *out, const T *r, int colour)
{
    // the roofline kernel: its timing events are taken by the dispatch itself
    Probe pr(c, MG_PROBE_PASS_W, l, true);
    const TileMap &tm = c->tileW[l];
    const TileMap tm64 =
        tm.tx == 0 && w_tileable(c->n[l]) ? make_marchmap<kMarch64Pass, 64>(c->n[l]) : TileMap{0, 0, 0, 0};
    if (tm.tx > 0)
        launch_W_tiled<T>(pr, c->s, c->geo[l], tm, in, out, r, colour);
    else if (tm64.tx > 0)
        probe_launch(pr, k_pass_W_march<T, kMarch64Pass, 64>, dim3(ntiles(tm64), 1, c->gz), dim3(kLanes, kTY), c->s,
                     c->geo[l], tm64, in, out, r, colour);
    else if (c->n[l] % 2 == 0 && c->n[l] <= 32)
        probe_launch(pr, k_pass_W_quad<T>, dim3(nblk(2 * c->cells[l]), 1, c->gz), dim3(kBlock), c->s, c->geo[l], in, out, r,
                     colour);
    else
        probe_launch(pr, k_pass_W<T>, dim3(nblk(c->cells[l]), 1, c->gz), dim3(kBlock), c->s, c->geo[l], in, out, r, colour);
}

template <typename T>
void smooth_W(mg_ctx *c, int l, int sweeps, bool first_done = false)
{
    for (int s = 0; s < sweeps; s++) {
        if (s > 0 || !first_done) pass_W<T>(c, l, (const T *)c->wd0[l], (T *)c->wd1[l], (const T *)c->wr[l], 0);
        pass_W<T>(c, l, (const T *)c->wd1[l], (T *)c->wd0[l], (const T *)c->wr[l], 1);
    }
}

template <typename T>
void fourier_W(mg_ctx *c, int l, const T *r, T *x)
{
    if constexpr (sizeof(T) == sizeof(float)) {
        Probe pr(c, MG_PROBE_COARSE, l);
        const Geo &g = c->geo[l];
        const float *rf = (const float *)r;
        float *xf = (float *)x;
        const int n = c->n[l];
        if (n == kFourierN) {
            hipLaunchKernelGGL(k_fourier_W, dim3(1, 1, c->gz), dim3(kFourierThreads), 0, c->s, g, rf, xf);
        } else if (n == 32) { // a quad of threads per line transform; x planes x components
            hipLaunchKernelGGL(k_spec_fwd<32>, dim3(32, 3, c->gz), dim3(4 * 32), 0, c->s, g, rf, c->specZ);
            hipLaunchKernelGGL(k_spec_solve<32>, dim3(32 * 32 / kSpecPencils, 1, c->gz), dim3(12 * kSpecPencils), 0,
                               c->s, g, c->specZ);
            hipLaunchKernelGGL(k_spec_inv<32>, dim3(32, 3, c->gz), dim3(4 * 32), 0, c->s, g, (const float2 *)c->specZ,
                               xf);
        } else {
            hipLaunchKernelGGL(k_spec_fwd<64>, dim3(64, 3, c->gz), dim3(4 * 64), 0, c->s, g, rf, c->specZ);
            hipLaunchKernelGGL(k_spec_solve<64>, dim3(64 * 64 / kSpecPencils, 1, c->gz), dim3(12 * kSpecPencils), 0,
                               c->s, g, c->specZ);
            hipLaunchKernelGGL(k_spec_inv<64>, dim3(64, 3, c->gz), dim3(4 * 64), 0, c->s, g, (const float2 *)c->specZ,
                               xf);
        }
    }
}

template <typename T>
void vcycle_W(mg_ctx *c, int l, bool first_done = false)
{
    if (fourier_at(c, l)) {
        fourier_W<T>(c, l, (const T *)c->wr[l], (T *)c->wd0[l]);
        return;
    }
    if (c->tail_W_on && l == c->tail_W) {
        Probe pr(c, MG_PROBE_COARSE, c->L - 1);
        hipLaunchKernelGGL(k_tail_W<T>, dim3(1, 1, c->gz), dim3(kTailThreads), 0, c->s, tail_args<T>(c, l, true));
        return;
    }
    if (l == c->L - 1) {
        coarse_W<T>(c, (const T *)c->wr[l], (T *)c->wd0[l]);
        return;
    }
    if (!first_done) fill<T>(c->s, (T *)c->wd0[l], 3 * c->cells[l], T(0), c->gz, c->zs);
    smooth_W<T>(c, l, nu_pre_W(c), first_done);
    // the next level is smoothed by grid launches (not the coarsest, not a tail)
    const bool next_first = l + 2 < c->L && !(c->tail_W_on && l + 1 == c->tail_W) && !fourier_at(c, l + 1);
    defect_restrict_W<T>(c, l, (const T *)c->wd0[l], (const T *)c->wr[l], (T *)c->wr[l + 1],
                         next_first ? (T *)c->wd1[l + 1] : nullptr);
    vcycle_W<T>(c, l + 1, next_first);
    prolong_add<T>(c, l + 1, (const T *)c->wd0[l + 1], (T *)c->wd0[l], 3);
    smooth_W<T>(c, l, nu_post_W(c));
}

// ---- residuals and outer steps ----------------------------------------------------------

bool source_mean_needed(const mg_ctx *c) { return c->S && c->p.bc == MG_BC_PERIODIC; }

// sums_ready: the psi update just wrote the partial sums at this state.
void source_mean(mg_ctx *c, const double *u, bool sums_ready = false)
{
    if (!source_mean_needed(c)) return;
    const Geo &g = c->geo[0];
    const int64_t nb = sum_blocks(c->cells[0]);
    if (c->p.bc == MG_BC_PERIODIC && !sums_ready)
        hipLaunchKernelGGL(k_source_sum<kBcPeriodic>, dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, g, u, c->S,
                           c->p.puncture_mass, (c->p.flags & MG_FLAG_CONFORMAL_MATTER) ? 1 : 0,
                           c->part);
    hipLaunchKernelGGL(k_reduce_final<3>, dim3(1, 1, c->gz), dim3(kBlock), 0, c->s, (const double *)c->part, nb,
                       0u, 1.0 / (double)c->cells[0], c->scal + S_MEANS, c->zs);
}

template <int BC, typename T, int TX>
void launch_residual_tx(hipStream_t s, const Geo &g, const TileMap &tm, const ResArgs &a, bool hasW)
{
    const dim3 blk(kLanes, kTY), grid(ntiles(tm), 1, g.gz);
    if (hasW)
        hipLaunchKernelGGL((k_residual_tiled<BC, T, TX, true>), grid, blk, 0, s, g, tm, a);
    else
        hipLaunchKernelGGL((k_residual_tiled<BC, T, TX, false>), grid, blk, 0, s, g, tm, a);
}

template <typename T, int LX>
void launch_residual_march(hipStream_t s, const Geo &g, const TileMap &tm, const ResArgs &a, bool hasW)
{
    const dim3 blk(kLanes, kTY), grid(ntiles(tm), 1, g.gz);
    if (hasW)
        hipLaunchKernelGGL((k_residual_march<T, LX, true>), grid, blk, 0, s, g, tm, a);
    else
        hipLaunchKernelGGL((k_residual_march<T, LX, false>), grid, blk, 0, s, g, tm, a);
}

// Depths 1, 2, 4 stage bricks; 8 and 16 march columns (periodic only).
template <int BC, typename T>
void launch_residual_tiled(hipStream_t s, const Geo &g, const TileMap &tm, const ResArgs &a, bool hasW)
{
    if (BC == kBcPeriodic && tm.tx == 8)
        launch_residual_march<T, 8>(s, g, tm, a, hasW);
    else if (BC == kBcPeriodic && tm.tx == 16)
        launch_residual_march<T, 16>(s, g, tm, a, hasW);
    else if (tm.tx == 1)
        launch_residual_tx<BC, T, 1>(s, g, tm, a, hasW);
    else if (tm.tx == 4)
        launch_residual_tx<BC, T, 4>(s, g, tm, a, hasW);
    else
        launch_residual_tx<BC, T, 2>(s, g, tm, a, hasW);
}

template <typename T>
// first: also write the finest level's first colour pass from a zero
// correction beside r (pd1) or rW (wd1), for the V-cycle that follows.
void residual(mg_ctx *c, const double *u, const double *W, bool want_M, double *H, double *M,
              double *cc, void *r, void *rc, void *rW, bool norms, bool first = false)
{
    ResArgs a;
    a.u = u;
    a.psi0f = c->bg_psi0;
    a.A2bg = c->bg_A2;
    a.K2p = c->K2p;
    a.W = W;
    a.rho5 = c->rho5;
    a.rho1 = c->rho1;
    a.S = c->S;
    a.f = c->f;
    a.meanS = c->scal + S_MEANS;
    a.K2 = c->K2;
    a.pmass = c->p.puncture_mass;
    a.H = H;
    a.M = M;
    a.c = cc;
    a.r = r;
    a.rc = rc;
    a.rW = rW;
    a.partials = norms ? c->part : nullptr;
    a.d1 = first && r && rc ? c->pd1[0] : nullptr;
    a.d1W = first && rW && want_M ? c->wd1[0] : nullptr;
    a.idiagW = 1.0 / (-100.0 * c->geo[0].inv12h2);
    a.want_M = want_M ? 1 : 0;
    a.conformal = (c->p.flags & MG_FLAG_CONFORMAL_MATTER) ? 1 : 0;
    int64_t nb = nblk(c->cells[0]);
    {
        Probe pr(c, MG_PROBE_RESIDUAL, 0);
        TileMap tm = c->tileR;
        // marched columns carry no background fields: bricks of depth 2 instead
        if (tm.tx >= 8 && (c->bg_psi0 || c->bg_A2)) tm = rtilemap_rt(c->n[0], 2);
        if (tm.tx > 0) {
            nb = ntiles(tm);
            if (c->p.bc == MG_BC_PERIODIC)
                launch_residual_tiled<kBcPeriodic, T>(c->s, c->geo[0], tm, a, W != nullptr);
            else
                with_bc(c->p.bc, [&](auto bcx) {
                    constexpr int BCX = decltype(bcx)::value;
                    launch_residual_tiled<BCX, T>(c->s, c->geo[0], tm, a, W != nullptr);
                });
        } else if (c->p.bc == MG_BC_PERIODIC)
            hipLaunchKernelGGL((k_residual<kBcPeriodic, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, c->geo[0], a);
        else
            with_bc(c->p.bc, [&](auto bcx) {
                constexpr int BCX = decltype(bcx)::value;
                hipLaunchKernelGGL((k_residual<BCX, T>), dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, c->geo[0], a);
            });
    }
    if (norms)
        hipLaunchKernelGGL(k_reduce_final<4>, dim3(1, 1, c->gz), dim3(kBlock), 0, c->s, (const double *)c->part, nb,
                           0xAu, 0.0, c->scal + S_NORM, c->zs);
}

// The CTTK update mixed over the last D >= 2 steps: the newest difference pair and the
// normal-equation sums in one pass, their reduction, gamma, the update.
template <typename T, int D>
void mix_ring(mg_ctx *c, double *W, int64_t m, unsigned db)
{
    constexpr int NV = mix_nv<D>();
    hipLaunchKernelGGL((k_aa_push_dots<T, D>), dim3(db), dim3(kBlock), 0, c->s, (const T *)c->wd0[0],
                       (const double *)(c->scal + S_MEAND), (const double *)W, (const double *)c->aa_W,
                       (const double *)c->aa_f, (T *)c->aa_dG, (T *)c->aa_dF, (const double *)c->aa_st, m, c->part);
    hipLaunchKernelGGL(k_reduce_final<NV>, dim3(1), dim3(kBlock), 0, c->s, (const double *)c->part, (int64_t)db, 0u,
                       0.0, c->aa_st + kMixRed, 0LL);
    hipLaunchKernelGGL(k_aa_solve<D>, dim3(1), dim3(64), 0, c->s, (const double *)(c->aa_st + kMixRed), c->aa_st);
    Probe pr(c, MG_PROBE_UPDATE, 0);
    hipLaunchKernelGGL((k_aa_update_ring<T, D>), dim3(nblk(3 * m)), dim3(kBlock), 0, c->s, W, (const T *)c->wd0[0],
                       (const double *)(c->scal + S_MEAND), c->aa_W, c->aa_f, (const T *)c->aa_dG,
                       (const double *)c->aa_st, m);
}

// mix: the CTTK solve's Anderson-mixed update in place of W += d - mean(d).
template <typename T>
void step_W(mg_ctx *c, const double *u, double *W, bool residual_done, bool mix = false)
{
    if (!residual_done) {
        source_mean(c, u);
        residual<T>(c, u, W, true, nullptr, nullptr, nullptr, nullptr, nullptr, c->wr[0], false, true);
    }
    // the residual (this step's or the evaluation's) wrote the first pass into wd1
    vcycle_W<T>(c, 0, true);
    const int64_t m = c->cells[0];
    const int64_t nb = nblk(m), sb = sum_blocks(m);
    double *part = c->forking ? c->part_w : c->part; // the psi update sums into part meanwhile
    hipLaunchKernelGGL(k_sum3<T>, dim3(sb, 1, c->gz), dim3(kBlock), 0, c->s, (const T *)c->wd0[0], m, part, c->zs);
    hipLaunchKernelGGL(k_reduce_final<3>, dim3(1, 1, c->gz), dim3(kBlock), 0, c->s, (const double *)part, sb, 0u,
                       1.0 / (double)m, c->scal + S_MEAND, c->zs);
    if (mix && c->aa_st) {
        // mix_nv(D) partials per block in c->part (4 per block of the finest level)
        const int D = c->p.mix_depth, nv = D + D * (D + 1) / 2;
        const unsigned db = std::max<unsigned>(
            1u, std::min<unsigned>(std::min<unsigned>(nblk(3 * m), kSrcBlocks), (unsigned)(4 * nb / nv)));
        switch (D) {
        case 2: mix_ring<T, 2>(c, W, m, db); break;
        case 3: mix_ring<T, 3>(c, W, m, db); break;
        case 4: mix_ring<T, 4>(c, W, m, db); break;
        case 5: mix_ring<T, 5>(c, W, m, db); break;
        default: mix_ring<T, 6>(c, W, m, db); break;
        }
    } else if (mix) {
        // two partials per block in c->part (4 per block of the finest level)
        const unsigned db = std::min<unsigned>(std::min<unsigned>(nblk(3 * m), kSrcBlocks), 2 * (unsigned)nb);
        hipLaunchKernelGGL(k_aa_dots<T>, dim3(db), dim3(kBlock), 0, c->s, (const T *)c->wd0[0],
                           (const double *)(c->scal + S_MEAND), (const double *)c->aa_f, m, c->part);
        hipLaunchKernelGGL(k_reduce_final<2>, dim3(1), dim3(kBlock), 0, c->s, (const double *)c->part, (int64_t)db,
                           0u, 0.0, c->scal + S_AA, 0LL);
        hipLaunchKernelGGL(k_aa_gamma, dim3(1), dim3(64), 0, c->s, c->scal + S_AA);
        Probe pr(c, MG_PROBE_UPDATE, 0);
        hipLaunchKernelGGL(k_aa_update<T>, dim3(nblk(3 * m)), dim3(kBlock), 0, c->s, W, (const T *)c->wd0[0],
                           (const double *)(c->scal + S_MEAND), c->aa_W, c->aa_f, (const double *)(c->scal + S_AA), m);
    } else {
        Probe pr(c, MG_PROBE_UPDATE, 0);
        hipLaunchKernelGGL(k_update_W<T>, dim3(nb, 1, c->gz), dim3(kBlock), 0, c->s, W, (const T *)c->wd0[0],
                           (const double *)(c->scal + S_MEAND), m,
                           c->batched ? (const double *)(c->scal + S_ACTIVE) : nullptr, c->zs);
    }
    c->vc_W++;
}

template <typename T>
void step_psi(mg_ctx *c, double *u, const double *W, bool residual_done)
{
    if (!residual_done)
        residual<T>(c, u, W, false, nullptr, nullptr, nullptr, c->pr[0], c->pc[0], nullptr, false, true);
    restrict_coefficients<T>(c);
    // the residual (this step's or the evaluation's) wrote the first pass into pd1
    vcycle_psi<T>(c, 0, true);
    const int64_t m = c->cells[0];
    {
        Probe pr(c, MG_PROBE_UPDATE, 0);
        const double *gate = c->batched ? (const double *)(c->scal + S_ACTIVE) : nullptr;
        if (source_mean_needed(c)) // the update also sums the periodic source of the next evaluation
            hipLaunchKernelGGL((k_update_u_source<kBcPeriodic, T>), dim3(sum_blocks(m), 1, c->gz), dim3(kBlock), 0, c->s,
                               c->geo[0], u, (const T *)c->pd0[0], gate, c->S, c->p.puncture_mass,
                               (c->p.flags & MG_FLAG_CONFORMAL_MATTER) ? 1 : 0, c->part);
        else
            hipLaunchKernelGGL(k_update_u<T>, dim3(nblk(m), 1, c->gz), dim3(kBlock), 0, c->s, u, (const T *)c->pd0[0], m,
                               gate, c->zs);
    }
    c->vc_psi++;
}

mg_status hip_status()
{
    return hipPeekAtLastError() == hipSuccess ? MG_OK : MG_ERR_HIP;
}

// Copy the device scalars to pinned memory and wait; converts sums to RMS.
mg_status fetch_norms(mg_ctx *c, double out[4], double *flag_psi)
{
    if (hipMemcpyAsync(c->hpin, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->s) !=
        hipSuccess)
        return MG_ERR_HIP;
    if (hipStreamSynchronize(c->s) != hipSuccess) return MG_ERR_HIP;
    const double inv = 1.0 / (double)c->cells[0];
    out[0] = std::sqrt(c->hpin[S_NORM + 0] * inv);
    out[1] = std::sqrt(c->hpin[S_NORM + 2] * inv);
    out[2] = c->hpin[S_NORM + 1];
    out[3] = c->hpin[S_NORM + 3];
    if (flag_psi) *flag_psi = c->hpin[S_FLAG_PSI];
    return MG_OK;
}

// Norms of an evaluation copied into pinned slot `slot` behind the work on the
// stream (post_norms), and read once that copy is done (read_norms), so that
// the host can wait for one iteration's norms while the next one runs.
mg_status post_norms(mg_ctx *c, int slot)
{
    if (hipMemcpyAsync(c->hpin + slot * S_COUNT, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                       c->s) != hipSuccess ||
        hipEventRecord(c->ev_norm[slot], c->s) != hipSuccess)
        return MG_ERR_HIP;
    return MG_OK;
}

mg_status read_norms(mg_ctx *c, int slot, double out[4], double *flag_psi)
{
    if (hipEventSynchronize(c->ev_norm[slot]) != hipSuccess) return MG_ERR_HIP;
    const double *h = c->hpin + slot * S_COUNT;
    const double inv = 1.0 / (double)c->cells[0];
    out[0] = std::sqrt(h[S_NORM + 0] * inv);
    out[1] = std::sqrt(h[S_NORM + 2] * inv);
    out[2] = h[S_NORM + 1];
    out[3] = h[S_NORM + 3];
    if (flag_psi) *flag_psi = h[S_FLAG_PSI];
    return MG_OK;
}

// CTTK: K of the state (u, W) from eq. Ham, K^2 = 12 H0 / psi^5 with H0 the
// Hamiltonian residual at K = 0 from the caller's rho5 (written into Kf first),
// then the shifted sources rho5_eff and S_eff the residuals read.
template <typename T>
void cttk_update(mg_ctx *c, const double *u, const double *W)
{
    const int64_t m = c->cells[0];
    const double *r5 = c->rho5;
    c->rho5 = c->rho5_in;
    residual<T>(c, u, W, false, c->Kf, nullptr, nullptr, nullptr, nullptr, nullptr, false);
    c->rho5 = r5;
    hipLaunchKernelGGL(k_cttk_K, dim3(nblk(m)), dim3(kBlock), 0, c->s, m, u, c->rho5_in, c->Kf, c->rho5_eff);
    hipLaunchKernelGGL(k_cttk_shift_S<kBcPeriodic>, dim3(nblk(m)), dim3(kBlock), 0, c->s, c->geo[0],
                       (const double *)c->Kf, c->S_in, c->S_eff);
}

// Evaluation of a state: norms (+ the residual the next update step uses);
// batch members also update their convergence flags.  CTTK: K and the shifted
// sources of the state first.
template <typename T>
void evaluate(mg_ctx *c, const double *u, const double *W, bool want_M, bool after_update = true,
              bool sums_ready = false)
{
    if (c->cttk) cttk_update<T>(c, u, W);
    source_mean(c, u, sums_ready);
    if (same_state(c)) // both steps' right-hand sides and first passes
        residual<T>(c, u, W, true, nullptr, nullptr, nullptr, c->pr[0], c->pc[0], c->wr[0], true, true);
    else if (c->momentum)
        residual<T>(c, u, W, true, nullptr, nullptr, nullptr, nullptr, nullptr, c->wr[0], true, true);
    else
        residual<T>(c, u, W, want_M, nullptr, nullptr, nullptr, c->pr[0], c->pc[0], nullptr, true, true);
    if (c->batched)
        hipLaunchKernelGGL(k_batch_check, dim3(1, 1, c->gz), dim3(64), 0, c->s, c->scal, (int)S_ACTIVE, (int)S_ITERS,
                           (int)S_DIVERGED, 1.0 / (double)c->cells[0], c->batch_tol, c->momentum ? 1 : 0,
                           after_update ? 1 : 0, c->zs);
}

// MG_FLAG_SAME_STATE: the W and psi steps from the right-hand sides the last
// evaluation formed at one state.  The psi step reads no W, so inside the capture of
// a single context it runs on the second stream as a graph branch beside the W step;
// the W step's partial sums then go to part_w (the psi update sums into part).
template <typename T>
void both_steps(mg_ctx *c, double *u, double *W)
{
    const bool fork = c->capturing && c->s2 && !c->batched && c->gz == 1;
    if (!fork) {
        step_W<T>(c, u, W, true);
        step_psi<T>(c, u, W, true);
        return;
    }
    (void)hipEventRecord(c->ev_fork, c->s);
    (void)hipStreamWaitEvent(c->s2, c->ev_fork, 0);
    std::swap(c->s, c->s2);
    step_psi<T>(c, u, W, true);
    std::swap(c->s, c->s2);
    c->forking = true;
    step_W<T>(c, u, W, true);
    c->forking = false;
    (void)hipEventRecord(c->ev_join, c->s2);
    (void)hipStreamWaitEvent(c->s, c->ev_join, 0);
}

// One outer step of mg_vcycle with MG_FLAG_SAME_STATE: both right-hand sides at the
// entry state, then both steps.
template <typename T>
void vcycle_same_state(mg_ctx *c, double *u, double *W)
{
    source_mean(c, u);
    residual<T>(c, u, W, true, nullptr, nullptr, nullptr, c->pr[0], c->pc[0], c->wr[0], false, true);
    step_W<T>(c, u, W, true);
    step_psi<T>(c, u, W, true);
}

// One outer update (W step, psi step) followed by the evaluation of the new state.
// CTTK: the W step alone (psi is data; the evaluation updates K).
template <typename T>
void outer_body(mg_ctx *c, double *u, double *W, bool want_M)
{
    if (c->cttk) {
        step_W<T>(c, u, W, true, true);
        evaluate<T>(c, u, W, want_M, true, false);
        return;
    }
    if (same_state(c)) {
        both_steps<T>(c, u, W);
    } else if (c->momentum) {
        step_W<T>(c, u, W, true);
        step_psi<T>(c, u, W, false);
    } else {
        step_psi<T>(c, u, W, true);
    }
    evaluate<T>(c, u, W, want_M, true, true); // the psi update summed the source
}

void drop_graph(mg_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_u = c->g_W = nullptr;
}

// Capture one outer_body for (u, W) on the context's own streams into a graph
// (the host-side V-cycle counters are left as they were).
template <typename T>
mg_status capture_graph(mg_ctx *c, double *u, double *W, bool want_M, hipGraph_t *out)
{
    *out = nullptr;
    if (hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal) != hipSuccess) return MG_ERR_HIP;
    const int vp = c->vc_psi, vw = c->vc_W;
    c->capturing = true;
    outer_body<T>(c, u, W, want_M);
    c->capturing = false;
    c->vc_psi = vp;
    c->vc_W = vw;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(c->s, &g) != hipSuccess || !g) return MG_ERR_HIP;
    *out = g;
    return MG_OK;
}

// Capture outer_body for (u, W) into an executable graph (reused while the
// state pointers stay the same).
template <typename T>
mg_status capture_body(mg_ctx *c, double *u, double *W, bool want_M)
{
    if (c->gexec && c->g_u == u && c->g_W == W) return MG_OK;
    drop_graph(c);
    hipGraph_t g = nullptr;
    mg_status st = capture_graph<T>(c, u, W, want_M, &g);
    if (st != MG_OK) return st;
    hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return MG_ERR_HIP;
    }
    c->g_u = u;
    c->g_W = W;
    return MG_OK;
}

// resume: (u, W) is the state the last solve on c left (c->cont_valid), whose
// evaluation is current in the workspace: it is not evaluated again, and the
// lookahead can start from the first iteration.  first_ahead: the first
// iteration is enqueued before the starting state's norms are read (for callers
// whose tolerance that state cannot meet).
template <typename T>
mg_status solve(mg_ctx *c, double *u, double *W, double tol, int max_outer, mg_report *rep, bool resume = false,
                bool first_ahead = false)
{
    auto t0 = std::chrono::steady_clock::now();
    c->vc_psi = c->vc_W = 0;
    mg_status st = MG_ERR_NOT_CONVERGED;
    double nr[4] = {0, 0, 0, 0}, first = -1.0;
    int it = 0, hist_len = 0, launched = 0;
    const bool mom = c->momentum;
    const bool want_M = mom || (c->S != nullptr && W != nullptr);
    // graphs replay fixed launch parameters; the probe needs eager launches
    const bool graph = !(c->p.flags & MG_FLAG_EAGER) && c->probe_kernel == MG_PROBE_NONE;
    // Lookahead: iteration it + 1 is enqueued before iteration it's norms are
    // read (the host round trip then overlaps the GPU work) when the
    // contraction of the last two iterations puts iteration it at least
    // kAheadMargin times above tol, so it cannot be the last one.  With one read
    // iteration only, the state must lie kFirstAhead times above tol (no outer
    // iteration contracts by that much: the first ones contract by 15-30x; the
    // coarse solve of a full-multigrid start begins ~4000x above its tolerance).
    constexpr double kAheadMargin = 10.0, kFirstAhead = 1e3;
    double w1 = -1.0, w2 = -1.0; // worst norm after the last and the one-before-last read iteration
    double last_worst = -1.0;      // worst norm of the last read iteration
    double resumed[4] = {0, 0, 0, 0};
    if (resume) {
        std::memcpy(resumed, c->cont_nr, sizeof(resumed));
        w1 = c->cont_prev;
    }
    c->cont_valid = false;
    fill<double>(c->s, c->scal + S_FLAG_PSI, 2, 0.0, c->gz, c->zs);
    if (c->cttk) fill<double>(c->s, c->scal + S_AA, 4, 0.0); // the mixing restarts with every solve
    if (c->aa_st) fill<double>(c->s, c->aa_st, kMixState, 0.0);
    if (!resume) {
        evaluate<T>(c, u, W, want_M);
        if (post_norms(c, 0) != MG_OK) return MG_ERR_HIP;
    }
    auto launch_next = [&]() -> mg_status {
        if (graph) {
            mg_status gs = capture_body<T>(c, u, W, want_M);
            if (gs != MG_OK) return gs;
            if (hipGraphLaunch(c->gexec, c->s) != hipSuccess) return MG_ERR_HIP;
            if (!c->cttk) c->vc_psi++;
            if (mom) c->vc_W++;
        } else {
            outer_body<T>(c, u, W, want_M);
        }
        launched++;
        return post_norms(c, launched & 1);
    };
    auto record = [&]() {
        if (rep && rep->history && hist_len < rep->history_cap) {
            std::memcpy(rep->history + 4 * hist_len, nr, sizeof(nr));
            hist_len++;
        }
    };
    for (;; it++) {
        if (graph && launched == it && it < max_outer &&
            ((w1 > 0.0 && w2 > 0.0 && w1 < w2 && w1 * (w1 / w2) > kAheadMargin * tol) ||
             (w1 > 0.0 && w2 < 0.0 && w1 > kFirstAhead * tol) || (it == 0 && first_ahead))) {
            mg_status ls = launch_next();
            if (ls != MG_OK) return ls;
        }
        double flag = 0.0;
        if (hip_status() != MG_OK) return MG_ERR_HIP;
        if (resume && it == 0) {
            std::memcpy(nr, resumed, sizeof(nr));
        } else {
            mg_status fs = read_norms(c, it & 1, nr, &flag);
            if (fs != MG_OK) return fs;
        }
        record();
        const double worst = mom ? std::fmax(nr[0], nr[1]) : nr[0];
        last_worst = worst;
        if (flag != 0.0) {
            st = MG_ERR_SINGULAR;
            break;
        }
        if (!std::isfinite(nr[0]) || !std::isfinite(nr[1])) {
            st = MG_ERR_DIVERGED;
            break;
        }
        if (first < 0.0) first = worst;
        if (nr[0] <= tol && (!mom || nr[1] <= tol)) {
            st = MG_OK;
            break;
        }
        if (worst > 1e6 * std::fmax(first, tol)) {
            st = MG_ERR_DIVERGED;
            break;
        }
        if (it >= max_outer) {
            st = MG_ERR_NOT_CONVERGED;
            break;
        }
        if (launched == it) {
            mg_status ls = launch_next();
            if (ls != MG_OK) return ls;
        }
        w2 = w1;
        w1 = worst;
    }
    double prev_worst = w1; // worst norm of the iteration before the final state
    if (launched > it) {
        // a lookahead iteration ran past the stop: report the state it left
        prev_worst = last_worst;
        double flag = 0.0;
        mg_status fs = read_norms(c, launched & 1, nr, &flag);
        if (fs != MG_OK) return fs;
        record();
        it = launched;
        if (flag != 0.0)
            st = MG_ERR_SINGULAR;
        else if (!std::isfinite(nr[0]) || !std::isfinite(nr[1]))
            st = MG_ERR_DIVERGED;
        else if (st == MG_OK && !(nr[0] <= tol && (!mom || nr[1] <= tol)))
            st = MG_ERR_NOT_CONVERGED;
    }
    if ((st == MG_OK || st == MG_ERR_NOT_CONVERGED) && !c->batched) {
        c->cont_valid = true;
        c->cont_u = u;
        c->cont_W = W;
        std::memcpy(c->cont_nr, nr, sizeof(nr));
        c->cont_prev = prev_worst;
    }
    auto t1 = std::chrono::steady_clock::now();
    if (rep) {
        rep->outer_iters = it;
        rep->vcycles_psi = c->vc_psi;
        rep->vcycles_W = c->vc_W;
        rep->status = st;
        rep->h_rms = nr[0];
        rep->m_rms = nr[1];
        rep->h_max = nr[2];
        rep->m_max = nr[3];
        rep->seconds = std::chrono::duration<double>(t1 - t0).count();
        rep->history_len = hist_len;
    }
    return st;
}

// Order the internal streams after the caller's stream (enter) and the
// caller's stream after the internal main stream (leave).
void enter(mg_ctx *c)
{
    (void)hipEventRecord(c->ev_in, c->user_s);
    (void)hipStreamWaitEvent(c->s, c->ev_in, 0);
}

void leave(mg_ctx *c)
{
    (void)hipEventRecord(c->ev_out, c->s);
    (void)hipStreamWaitEvent(c->user_s, c->ev_out, 0);
}

void release(mg_ctx *c)
{
    drop_graph(c);
    if (c->s) (void)hipStreamSynchronize(c->s);
    hipEvent_t *evs[] = {&c->ev_in, &c->ev_out, &c->ev_norm[0], &c->ev_norm[1], &c->ev_fork, &c->ev_join};
    for (hipEvent_t *e : evs)
        if (*e) (void)hipEventDestroy(*e);
    if (c->own_streams && c->s) (void)hipStreamDestroy(c->s);
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->hpin) (void)hipHostFree(c->hpin);
    if (c->probe_ev) {
        for (int q = 0; q < 2 * kProbeMax; q++) (void)hipEventDestroy(c->probe_ev[q]);
        delete[] c->probe_ev;
    }
    delete c;
}

// Create the context's events, and its stream unless it is borrowed (already
// set: batch members).
mg_status create_streams(mg_ctx *c)
{
    if (!c->s) {
        c->own_streams = true;
        if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess) return MG_ERR_HIP;
    }
    hipEvent_t *evs[] = {&c->ev_in, &c->ev_out, &c->ev_norm[0], &c->ev_norm[1]};
    for (hipEvent_t *e : evs)
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return MG_ERR_HIP;
    if (c->own_streams && same_state(c)) {
        if (hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
            return MG_ERR_HIP;
    }
    return MG_OK;
}

template <typename T>
mg_status kernel_op(mg_ctx *c, int op, int l, int arg, const void *in, void *out, const void *r,
                    const void *cf)
{
    if (l < 0 || l >= c->L) return MG_ERR_INVALID;
    const bool coarsest = (l == c->L - 1);
    switch (op) {
    case MG_OP_PASS_PSI: {
        if (!in || !out || !r || !cf || (arg != 0 && arg != 1) || coarsest) return MG_ERR_INVALID;
        // the pass reads r and c from the context's level buffers: stage the caller's
        if (hipMemcpyAsync(c->pr[l], r, c->cells[l] * sizeof(T), hipMemcpyDeviceToDevice, c->s) != hipSuccess ||
            hipMemcpyAsync(c->pc[l], cf, c->cells[l] * sizeof(T), hipMemcpyDeviceToDevice, c->s) != hipSuccess)
            return MG_ERR_HIP;
        pass_psi<T>(c, l, (const T *)in, (T *)out, arg);
        break;
    }
    case MG_OP_PASS_W:
        if (!in || !out || !r || (arg != 0 && arg != 1) || c->p.bc != MG_BC_PERIODIC || coarsest)
            return MG_ERR_INVALID;
        pass_W<T>(c, l, (const T *)in, (T *)out, (const T *)r, arg);
        break;
    case MG_OP_DEFECT_RESTRICT_PSI:
        if (!in || !out || !r || !cf || coarsest) return MG_ERR_INVALID;
        defect_restrict_psi<T>(c, l, (const T *)in, (const T *)r, (const T *)cf, (T *)out, nullptr);
        break;
    case MG_OP_DEFECT_RESTRICT_W:
        if (!in || !out || !r || coarsest || c->p.bc != MG_BC_PERIODIC) return MG_ERR_INVALID;
        defect_restrict_W<T>(c, l, (const T *)in, (const T *)r, (T *)out);
        break;
    case MG_OP_PROLONG_ADD:
        if (!in || !out || coarsest || (arg != 1 && arg != 3)) return MG_ERR_INVALID;
        prolong_add<T>(c, l + 1, (const T *)in, (T *)out, arg);
        break;
    case MG_OP_COARSE_PSI: {
        if (!in || !out || !cf || !coarsest) return MG_ERR_INVALID;
        // the coarse coefficient lives in the context: copy the caller's first
        if (hipMemcpyAsync(c->pc[l], cf, c->cells[l] * sizeof(T), hipMemcpyDeviceToDevice, c->s) !=
            hipSuccess)
            return MG_ERR_HIP;
        coarse_psi<T>(c, (const T *)in, (T *)out);
        break;
    }
    case MG_OP_COARSE_W:
        if (!in || !out || !coarsest || !c->momentum) return MG_ERR_INVALID;
        coarse_W<T>(c, (const T *)in, (T *)out);
        break;
    case MG_OP_FOURIER_W:
        if (!in || !out || l != c->fourier_W || ((uintptr_t)in | (uintptr_t)out) % 16 != 0) return MG_ERR_INVALID;
        fourier_W<T>(c, l, (const T *)in, (T *)out);
        break;
    default:
        return MG_ERR_INVALID;
    }
    return hip_status();
}

// ---- autotuning of the brick depths ----------------------------------------------------

const int *tune_candidates(const mg_ctx *c, int family, int &count)
{
    switch (family) {
    case MG_TUNE_PASS_PSI: count = 3; return kCandPsi;
    case MG_TUNE_PASS_W:
        if (c->f32) {
            count = 4;
            return kCandW32;
        }
        count = 3;
        return kCandW64;
    case MG_TUNE_RESIDUAL: count = 4; return kCandR;
    case MG_TUNE_TAIL_PSI:
    case MG_TUNE_TAIL_W: count = 2; return kCandTail;
    default: count = 0; return nullptr;
    }
}

// The brick map of (family, level) for depth tx (tx == 0 in the map: not tileable).
TileMap tune_map(const mg_ctx *c, int family, int level, int tx)
{
    if (family == MG_TUNE_RESIDUAL)
        return level == 0 && (tx < 8 || c->p.bc == MG_BC_PERIODIC) ? rtilemap_rt(c->n[0], tx) : TileMap{0, 0, 0, 0};
    if (family == MG_TUNE_PASS_W && (!c->momentum || !w_tileable(c->n[level]))) return TileMap{0, 0, 0, 0};
    return tilemap_rt(c->n[level], tx);
}

TileMap &tune_slot(mg_ctx *c, int family, int level)
{
    if (family == MG_TUNE_PASS_PSI) return c->tile[level];
    if (family == MG_TUNE_PASS_W) return c->tileW[level];
    return c->tileR;
}

// Times every candidate depth of every tileable (family, level) with HIP events
// around `reps` launches on the state's own data (residuals of (u, W), zero
// corrections), keeps the fastest, and drops the captured graph.
template <typename T>
mg_status autotune(mg_ctx *c, const double *u, const double *W, int reps, mg_tune *out, int cap, int *count)
{
    const int probe = c->probe_kernel;
    c->probe_kernel = MG_PROBE_NONE;
    const bool wantM = c->momentum || (c->S != nullptr && W != nullptr);
    if (c->cttk) cttk_update<T>(c, u, W);
    source_mean(c, u);
    residual<T>(c, u, W, false, nullptr, nullptr, nullptr, c->pr[0], c->pc[0], nullptr, false);
    restrict_coefficients<T>(c);
    for (int l = 0; l < c->L; l++) {
        fill<T>(c->s, (T *)c->pd0[l], c->cells[l], T(0));
        if (l > 0) fill<T>(c->s, (T *)c->pr[l], c->cells[l], T(0));
    }
    if (c->momentum) {
        residual<T>(c, u, W, true, nullptr, nullptr, nullptr, nullptr, nullptr, c->wr[0], false);
        for (int l = 0; l < c->L; l++) {
            fill<T>(c->s, (T *)c->wd0[l], 3 * c->cells[l], T(0));
            if (l > 0) fill<T>(c->s, (T *)c->wr[l], 3 * c->cells[l], T(0));
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        c->probe_kernel = probe;
        return MG_ERR_HIP;
    }
    mg_status st = MG_OK;
    int k = 0;
    // V-cycle tails: one whole V-cycle (with the coefficient restriction it needs)
    // timed with the tail off and on
    // (the exact W bottom first: while it is on, the W tail below it never runs)
    // A tail is timed off and starting at every level from the highest that fits down to
    // the one above the coarsest; the entry reports the fastest start as its level.
    for (int family : {MG_TUNE_FOURIER_W, MG_TUNE_TAIL_PSI, MG_TUNE_TAIL_W}) {
        if (st != MG_OK) break;
        const bool tail = family != MG_TUNE_FOURIER_W;
        const int first = family == MG_TUNE_TAIL_PSI ? c->tail_psi_min
                          : family == MG_TUNE_TAIL_W ? c->tail_W_min
                                                     : c->fourier_W;
        if (first < 0) continue;
        bool &on = family == MG_TUNE_TAIL_PSI ? c->tail_psi_on : family == MG_TUNE_TAIL_W ? c->tail_W_on : c->fourier_W_on;
        int &start = family == MG_TUNE_TAIL_PSI ? c->tail_psi : family == MG_TUNE_TAIL_W ? c->tail_W : c->fourier_W;
        mg_tune e;
        std::memset(&e, 0, sizeof(e));
        e.family = family;
        e.level = start;
        e.ncand = 2;
        e.us[1] = 1e300;
        double best = 1e300;
        bool best_on = on;
        int best_start = start;
        const int last = tail ? c->L - 2 : first;
        for (int q = 0; q < 2 + (last - first) && st == MG_OK; q++) {
            const int cq = q == 0 ? 0 : 1;
            e.cand[cq] = kCandTail[cq];
            on = cq != 0;
            if (q > 0) start = first + (q - 1);
            auto cycle = [&]() {
                if (family == MG_TUNE_TAIL_PSI) {
                    restrict_coefficients<T>(c);
                    vcycle_psi<T>(c, 0);
                } else {
                    vcycle_W<T>(c, 0);
                }
            };
            cycle();
            float ms = 0.0f;
            if (hipEventRecord(e0, c->s) != hipSuccess) st = MG_ERR_HIP;
            for (int r = 0; r < reps && st == MG_OK; r++) cycle();
            if (st == MG_OK && (hipEventRecord(e1, c->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = MG_ERR_HIP;
            if (st != MG_OK) break;
            const double us = 1e3 * ms / reps;
            if (q == 0 || us < e.us[1]) {
                e.us[cq] = us;
                if (q > 0) e.level = start;
            }
            if (us < best) {
                best = us;
                best_on = on;
                best_start = start;
                e.chosen = kCandTail[cq];
            }
        }
        on = best_on;
        start = best_start;
        if (!best_on && tail) start = first;
        if (best_on) e.level = best_start;
        if (out && k < cap) out[k] = e;
        k++;
    }
    for (int family = MG_TUNE_PASS_PSI; family <= MG_TUNE_RESIDUAL && st == MG_OK; family++) {
        int nc = 0;
        const int *cand = tune_candidates(c, family, nc);
        const int nlev = family == MG_TUNE_RESIDUAL ? 1 : c->L;
        for (int l = 0; l < nlev && st == MG_OK; l++) {
            if (tune_map(c, family, l, cand[0]).tx == 0) continue;
            mg_tune e;
            std::memset(&e, 0, sizeof(e));
            e.family = family;
            e.level = l;
            e.ncand = nc;
            double best = 1e300;
            TileMap bestmap = tune_slot(c, family, l);
            for (int q = 0; q < nc; q++) {
                e.cand[q] = cand[q];
                const TileMap tm = tune_map(c, family, l, cand[q]);
                e.us[q] = -1.0;
                if (tm.tx == 0) continue;
                tune_slot(c, family, l) = tm;
                auto launch = [&](int r) {
                    if (family == MG_TUNE_PASS_PSI)
                        pass_psi<T>(c, l, (const T *)c->pd0[l], (T *)c->pd1[l], r & 1);
                    else if (family == MG_TUNE_PASS_W)
                        pass_W<T>(c, l, (const T *)c->wd0[l], (T *)c->wd1[l], (const T *)c->wr[l], r & 1);
                    else if (c->momentum)
                        residual<T>(c, u, W, true, nullptr, nullptr, nullptr, nullptr, nullptr, c->wr[0], true);
                    else
                        residual<T>(c, u, W, wantM, nullptr, nullptr, nullptr, c->pr[0], c->pc[0], nullptr, true);
                };
                for (int r = 0; r < 2; r++) launch(r);
                float ms = 0.0f;
                if (hipEventRecord(e0, c->s) != hipSuccess) st = MG_ERR_HIP;
                for (int r = 0; r < reps && st == MG_OK; r++) launch(r);
                if (st == MG_OK && (hipEventRecord(e1, c->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    st = MG_ERR_HIP;
                if (st != MG_OK) break;
                e.us[q] = 1e3 * ms / reps;
                if (e.us[q] < best) {
                    best = e.us[q];
                    bestmap = tm;
                    e.chosen = cand[q];
                }
            }
            tune_slot(c, family, l) = bestmap;
            if (out && k < cap) out[k] = e;
            k++;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->probe_kernel = probe;
    drop_graph(c);
    if (count) *count = k;
    if (st == MG_OK) st = hip_status();
    return st;
}

} // namespace

// ======================================================================================
// C ABI
// ======================================================================================

extern "C" {

mg_status mg_workspace_size(const mg_params *p, size_t *bytes)
{
    if (!bytes) return MG_ERR_INVALID;
    mg_status st = validate(p);
    if (st != MG_OK) return st;
    mg_ctx tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    tmp.p = *p;
    tmp.L = p->levels;
    tmp.f32 = p->precision == MG_PREC_FP32_IR;
    tmp.esz = tmp.f32 ? sizeof(float) : sizeof(double);
    tmp.momentum = p->solve_momentum != 0;
    Carver cv{nullptr};
    carve(&tmp, cv);
    *bytes = align_up(cv.off, 256);
    return MG_OK;
}

} // extern "C"

namespace {

// Create a context on a caller-provided workspace.  s_main: a stream borrowed
// from a batch, or null to create the context's own.
mg_status ctx_create(const mg_params *p, void *d_workspace, size_t bytes, hipStream_t user_s,
                     const double *d_rho5, const double *d_rho1, const double *d_S, const double *d_f,
                     hipStream_t s_main, mg_ctx **out)
{
    *out = nullptr;
    mg_status st = validate(p);
    if (st != MG_OK) return st;
    if (!d_rho5 || !d_rho1) return MG_ERR_INVALID;
    if (p->solve_momentum && !d_S) return MG_ERR_INVALID;
    size_t need = 0;
    mg_workspace_size(p, &need);
    if (!d_workspace || bytes < need || ((uintptr_t)d_workspace % 256) != 0) return MG_ERR_WORKSPACE;
    mg_ctx *c = new (std::nothrow) mg_ctx;
    if (!c) return MG_ERR_INVALID;
    std::memset(c, 0, sizeof(*c));
    c->p = *p;
    c->user_s = user_s;
    c->s = s_main;
    c->L = p->levels;
    c->f32 = p->precision == MG_PREC_FP32_IR;
    c->esz = c->f32 ? sizeof(float) : sizeof(double);
    c->momentum = p->solve_momentum != 0;
    c->rho5 = d_rho5;
    c->rho1 = d_rho1;
    c->S = d_S;
    c->f = d_f;
    c->bg_psi0 = nullptr;
    c->bg_A2 = nullptr;
    c->K2 = p->K * p->K;
    c->gz = 1;
    c->zs = 0;
    c->K2p = nullptr;
    Carver cv{(char *)d_workspace};
    carve(c, cv);
    c->cttk = (p->flags & MG_FLAG_CTTK) != 0;
    if (c->cttk) {
        c->rho5_in = d_rho5;
        c->S_in = d_S;
        c->rho5 = c->rho5_eff;
        c->S = c->S_eff;
    }
    init_geo(c);
    if (create_streams(c) != MG_OK ||
        hipHostMalloc((void **)&c->hpin, 2 * S_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        release(c);
        return MG_ERR_HIP;
    }
    enter(c);
    fill<double>(c->s, c->scal, S_COUNT, 0.0);
    if (c->momentum) {
        const int m = c->m_W;
        fill<double>(c->s, c->A_W, (int64_t)m * m, 0.0);
        hipLaunchKernelGGL(k_assemble_W, dim3(nblk(m)), dim3(kBlock), 0, c->s, c->geo[c->L - 1], c->A_W);
        factor(c->s, c->A_W, c->aug_W, c->inv_W, m, c->scal + S_FLAG_W);
        if (hipMemcpyAsync(c->hpin, c->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, c->s) !=
                hipSuccess ||
            hipStreamSynchronize(c->s) != hipSuccess) {
            release(c);
            return MG_ERR_HIP;
        }
        if (c->hpin[S_FLAG_W] != 0.0) {
            release(c);
            return MG_ERR_SINGULAR;
        }
    }
    if (hip_status() != MG_OK) {
        release(c);
        return MG_ERR_HIP;
    }
    leave(c);
    *out = c;
    return MG_OK;
}

} // namespace

// ---- batches ---------------------------------------------------------------------------

constexpr int kBatchLanes = 4; // concurrent branches (stream pairs) of a batch

// A batch.  Members with the same parameters (all but K) form a group; the members
// of a group own equal workspace regions placed region_g bytes apart, each region
// holding the member's context workspace and its own copies of the sources and of
// the state, so that one launch with gridDim.z = group size runs a kernel for the
// whole group (MG_BATCH_GROUPS, through a group context whose launches span the
// group) and the member contexts run it member by member (MG_BATCH_GRAPH,
// MG_BATCH_LANES).
struct mg_batch {
    int count, ngroups;
    mg_ctx **ctx;    // member contexts
    mg_ctx **gctx;   // per group: a context over member 0's region spanning the group (or member 0's own)
    bool *gown;      // gctx[g] is a context of its own (group of more than one member)
    int *gfirst;     // members of group g: order[gfirst[g] .. gfirst[g + 1])
    int *order;      // region order -> member index
    int *slot;       // member index -> block of scal_all
    int *gof;        // member index -> group
    size_t *gstride; // per group: bytes between consecutive members' regions
    double **cu, **cW, **c5, **c1, **cS; // per member: device copies in its region
    bool *hasW;      // per member: the caller passes W
    hipStream_t user_s, s;
    hipStream_t lane_s[kBatchLanes];
    hipEvent_t ev_in, ev_out, ev_root;
    hipEvent_t *ev_join;
    double *scal_all; // device: count x S_COUNT, the members' scalar blocks gathered after each iteration
    double *hpin;     // pinned copy of scal_all
    hipGraphExec_t gexec; // the whole batch as one graph (launch mode MG_BATCH_GRAPH)
    bool captured_members, captured_groups;
    double g_tol;
    // launch mode: requested (MG_BATCH_AUTO tunes on the first solve), in use,
    // and the wall time of the tuning iteration in each mode
    int mode_req, mode;
    double ms_mode[3]; // graph, lanes, groups
};

namespace {

// Parameters that must agree within a group (everything but K).
bool same_group(const mg_params &a, const mg_params &b)
{
    mg_params x = a, y = b;
    x.K = y.K = 0.0;
    // the fields only: the struct's tail padding holds whatever the caller left there
    return std::memcmp(&x, &y, offsetof(mg_params, mix_depth) + sizeof(x.mix_depth)) == 0;
}

// A group runs as one launch per kernel only if every kernel of its path takes the
// member stride: the coarsest psi system must be solved by the Krylov kernels.
bool groupable(const mg_params &p)
{
    const int nc = p.n >> (p.levels - 1);
    return nc * nc * nc <= kKrylovMax;
}

struct BatchPlan {
    int ngroups;
    std::vector<int> gfirst, order, gof;
    std::vector<size_t> gbase, gstride;
    size_t total;
};

size_t member_region(const mg_params &p)
{
    size_t wb = 0;
    mg_workspace_size(&p, &wb);
    const size_t m = (size_t)p.n * p.n * p.n * sizeof(double);
    // workspace, rho5, rho1, S (3), u, W (3)
    return align_up(wb, 256) + 2 * align_up(m, 256) + align_up(3 * m, 256) + align_up(m, 256) + align_up(3 * m, 256);
}

BatchPlan batch_plan(const mg_params *p, int count)
{
    BatchPlan pl;
    pl.gof.assign(count, -1);
    for (int i = 0; i < count; i++) {
        if (pl.gof[i] >= 0) continue;
        const int g = (int)pl.gfirst.size();
        pl.gfirst.push_back((int)pl.order.size());
        pl.gof[i] = g;
        pl.order.push_back(i);
        if (!groupable(p[i])) continue;
        for (int j = i + 1; j < count; j++)
            if (pl.gof[j] < 0 && same_group(p[i], p[j])) {
                pl.gof[j] = g;
                pl.order.push_back(j);
            }
    }
    pl.ngroups = (int)pl.gfirst.size();
    pl.gfirst.push_back(count);
    size_t off = align_up((size_t)count * S_COUNT * sizeof(double), 256);
    for (int g = 0; g < pl.ngroups; g++) {
        const size_t r = align_up(member_region(p[pl.order[pl.gfirst[g]]]), 256);
        pl.gbase.push_back(off);
        pl.gstride.push_back(r);
        off += r * (size_t)(pl.gfirst[g + 1] - pl.gfirst[g]);
    }
    pl.total = off;
    return pl;
}

void batch_release(mg_batch *b)
{
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->s) (void)hipStreamSynchronize(b->s);
    if (b->gctx && b->gown)
        for (int g = 0; g < b->ngroups; g++)
            if (b->gctx[g] && b->gown[g]) release(b->gctx[g]);
    if (b->ctx)
        for (int i = 0; i < b->count; i++)
            if (b->ctx[i]) release(b->ctx[i]);
    for (int q = 0; q < kBatchLanes; q++)
        if (b->lane_s[q]) (void)hipStreamDestroy(b->lane_s[q]);
    if (b->ev_join) {
        for (int i = 0; i < b->count; i++)
            if (b->ev_join[i]) (void)hipEventDestroy(b->ev_join[i]);
        delete[] b->ev_join;
    }
    hipEvent_t evs[] = {b->ev_in, b->ev_out, b->ev_root};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    if (b->s) (void)hipStreamDestroy(b->s);
    if (b->hpin) (void)hipHostFree(b->hpin);
    delete[] b->ctx;
    delete[] b->gctx;
    delete[] b->gown;
    delete[] b->gfirst;
    delete[] b->order;
    delete[] b->slot;
    delete[] b->gof;
    delete[] b->gstride;
    delete[] b->cu;
    delete[] b->cW;
    delete[] b->c5;
    delete[] b->c1;
    delete[] b->cS;
    delete[] b->hasW;
    delete b;
}

// Fork every member from the batch stream, run fn(member) on its lane, join.
template <typename F>
void batch_fork_join(mg_batch *b, F fn)
{
    (void)hipEventRecord(b->ev_root, b->s);
    for (int i = 0; i < b->count; i++) {
        mg_ctx *c = b->ctx[i];
        (void)hipStreamWaitEvent(c->s, b->ev_root, 0);
        fn(i, c);
        (void)hipEventRecord(b->ev_join[i], c->s);
        (void)hipStreamWaitEvent(b->s, b->ev_join[i], 0);
    }
}

// The same for the groups, on their lanes.
template <typename F>
void group_fork_join(mg_batch *b, F fn)
{
    (void)hipEventRecord(b->ev_root, b->s);
    for (int g = 0; g < b->ngroups; g++) {
        mg_ctx *c = b->gctx[g];
        (void)hipStreamWaitEvent(c->s, b->ev_root, 0);
        fn(g, c);
        (void)hipEventRecord(b->ev_join[g], c->s);
        (void)hipStreamWaitEvent(b->s, b->ev_join[g], 0);
    }
}

double *member_W(const mg_batch *b, int i) { return b->hasW[i] ? b->cW[i] : nullptr; }
bool want_M_of(const mg_batch *b, int i) { return b->ctx[i]->momentum || (b->ctx[i]->S && b->hasW[i]); }

// Capture every member's outer iteration on the member's stream: each member
// keeps its own executable graph (launch mode MG_BATCH_LANES) and the batch
// graph holds them all as independent children (MG_BATCH_GRAPH).  The state
// arrays are the members' own copies, so the graphs stay valid for every solve.
template <typename T>
mg_status batch_capture_members(mg_batch *b)
{
    const int n = b->count;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    hipGraph_t parent = nullptr;
    if (hipGraphCreate(&parent, 0) != hipSuccess) return MG_ERR_HIP;
    mg_status st = MG_OK;
    for (int i = 0; i < n && st == MG_OK; i++) {
        mg_ctx *c = b->ctx[i];
        drop_graph(c);
        hipGraph_t g = nullptr;
        st = capture_graph<T>(c, b->cu[i], member_W(b, i), want_M_of(b, i), &g);
        if (st != MG_OK) break;
        hipGraphNode_t node = nullptr;
        if (hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
            c->gexec = nullptr;
            st = MG_ERR_HIP;
        } else if (hipGraphAddChildGraphNode(&node, parent, nullptr, 0, g) != hipSuccess) {
            st = MG_ERR_HIP;
        }
        c->g_u = b->cu[i];
        c->g_W = member_W(b, i);
        (void)hipGraphDestroy(g);
    }
    if (st == MG_OK && hipGraphInstantiate(&b->gexec, parent, nullptr, nullptr, 0) != hipSuccess) {
        b->gexec = nullptr;
        st = MG_ERR_HIP;
    }
    (void)hipGraphDestroy(parent);
    if (st == MG_OK) b->captured_members = true;
    return st;
}

// Capture every group's outer iteration on its group context: one launch per kernel
// for all members of the group (MG_BATCH_GROUPS).
template <typename T>
mg_status batch_capture_groups(mg_batch *b)
{
    for (int g = 0; g < b->ngroups; g++) {
        mg_ctx *c = b->gctx[g];
        const int i = b->order[b->gfirst[g]];
        drop_graph(c);
        hipGraph_t gr = nullptr;
        mg_status st = capture_graph<T>(c, b->cu[i], member_W(b, i), want_M_of(b, i), &gr);
        if (st != MG_OK) return st;
        const bool ok = hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0) == hipSuccess;
        (void)hipGraphDestroy(gr);
        if (!ok) {
            c->gexec = nullptr;
            return MG_ERR_HIP;
        }
        c->g_u = b->cu[i];
        c->g_W = member_W(b, i);
    }
    b->captured_groups = true;
    return MG_OK;
}

// Group g has an active member (host copy of the gathered scalars).
bool group_active(const mg_batch *b, int g)
{
    for (int q = b->gfirst[g]; q < b->gfirst[g + 1]; q++)
        if (b->hpin[b->slot[b->order[q]] * S_COUNT + S_ACTIVE] != 0.0) return true;
    return false;
}

// One outer iteration of the batch in launch mode `mode`: the batch graph on the
// batch stream, every still-active member's graph on the lane streams (members
// spread round-robin over kBatchLanes streams), or every still-active group's
// graph on its lane; joined on the batch stream.
mg_status batch_launch(mg_batch *b, int mode)
{
    if (mode == MG_BATCH_GRAPH) return hipGraphLaunch(b->gexec, b->s) == hipSuccess ? MG_OK : MG_ERR_HIP;
    const int lanes = std::min(kBatchLanes, mode == MG_BATCH_GROUPS ? b->ngroups : b->count);
    if (hipEventRecord(b->ev_root, b->s) != hipSuccess) return MG_ERR_HIP;
    for (int q = 0; q < lanes; q++)
        if (hipStreamWaitEvent(b->lane_s[q], b->ev_root, 0) != hipSuccess) return MG_ERR_HIP;
    if (mode == MG_BATCH_GROUPS) {
        for (int g = 0; g < b->ngroups; g++) {
            if (!group_active(b, g)) continue; // every member converged or diverged
            if (hipGraphLaunch(b->gctx[g]->gexec, b->gctx[g]->s) != hipSuccess) return MG_ERR_HIP;
        }
    } else {
        for (int i = 0; i < b->count; i++) {
            if (b->hpin[b->slot[i] * S_COUNT + S_ACTIVE] == 0.0) continue; // nothing to do
            if (hipGraphLaunch(b->ctx[i]->gexec, b->ctx[i]->s) != hipSuccess) return MG_ERR_HIP;
        }
    }
    for (int q = 0; q < lanes; q++) {
        if (hipEventRecord(b->ev_join[q], b->lane_s[q]) != hipSuccess ||
            hipStreamWaitEvent(b->s, b->ev_join[q], 0) != hipSuccess)
            return MG_ERR_HIP;
    }
    return MG_OK;
}

// Every member's scalar block into scal_all (block slot[i]) and to the host.
mg_status batch_read(mg_batch *b)
{
    for (int g = 0; g < b->ngroups; g++) {
        const int k = b->gfirst[g + 1] - b->gfirst[g];
        mg_ctx *c0 = b->ctx[b->order[b->gfirst[g]]];
        hipLaunchKernelGGL(k_gather_scal, dim3(1, 1, k), dim3(64), 0, b->s, (const double *)c0->scal,
                           (long long)b->gstride[g], (int)S_COUNT, b->scal_all + (size_t)b->gfirst[g] * S_COUNT);
    }
    if (hipMemcpyAsync(b->hpin, b->scal_all, (size_t)b->count * S_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                       b->s) != hipSuccess ||
        hipStreamSynchronize(b->s) != hipSuccess)
        return MG_ERR_HIP;
    return MG_OK;
}

template <typename T>
mg_status batch_solve(mg_batch *b, double *const *u, double *const *W, double tol, int max_outer, mg_report *reps)
{
    auto t0 = std::chrono::steady_clock::now();
    const int n = b->count;
    // the callers' states into the members' copies
    for (int i = 0; i < n; i++) {
        const int64_t m = b->ctx[i]->cells[0];
        if (hipMemcpyAsync(b->cu[i], u[i], m * sizeof(double), hipMemcpyDeviceToDevice, b->s) != hipSuccess)
            return MG_ERR_HIP;
        if (b->hasW[i] &&
            hipMemcpyAsync(b->cW[i], W[i], 3 * m * sizeof(double), hipMemcpyDeviceToDevice, b->s) != hipSuccess)
            return MG_ERR_HIP;
    }
    if (b->g_tol != tol) {
        for (int i = 0; i < n; i++) b->ctx[i]->batch_tol = tol;
        for (int g = 0; g < b->ngroups; g++) b->gctx[g]->batch_tol = tol;
        b->captured_members = b->captured_groups = false; // the check kernel carries tol
        b->g_tol = tol;
    }
    // reset the flags and evaluate every member (eager, group launches)
    group_fork_join(b, [&](int g, mg_ctx *c) {
        const int i = b->order[b->gfirst[g]];
        fill<double>(c->s, c->scal + S_FLAG_PSI, 2, 0.0, c->gz, c->zs);
        fill<double>(c->s, c->scal + S_ITERS, 1, 0.0, c->gz, c->zs);
        fill<double>(c->s, c->scal + S_DIVERGED, 1, 0.0, c->gz, c->zs);
        fill<double>(c->s, c->scal + S_ACTIVE, 1, 1.0, c->gz, c->zs);
        evaluate<T>(c, b->cu[i], member_W(b, i), want_M_of(b, i), false);
    });
    int it = 0;
    for (;; it++) {
        mg_status rs = batch_read(b);
        if (rs != MG_OK) return rs;
        int active = 0;
        for (int i = 0; i < n; i++) active += b->hpin[b->slot[i] * S_COUNT + S_ACTIVE] != 0.0;
        if (active == 0 || it >= max_outer) break;
        // launch-mode tuning: one timed outer iteration in each mode (every mode runs
        // the same kernels on the same arrays, so the results do not change)
        int mode = b->mode;
        const bool tune = b->mode_req == MG_BATCH_AUTO && b->mode == MG_BATCH_AUTO;
        if (tune) mode = b->ms_mode[0] < 0.0 ? MG_BATCH_GRAPH : b->ms_mode[1] < 0.0 ? MG_BATCH_LANES : MG_BATCH_GROUPS;
        if ((mode == MG_BATCH_GRAPH || mode == MG_BATCH_LANES) && !b->captured_members) {
            mg_status cs = batch_capture_members<T>(b);
            if (cs != MG_OK) return cs;
        }
        if (mode == MG_BATCH_GROUPS && !b->captured_groups) {
            mg_status cs = batch_capture_groups<T>(b);
            if (cs != MG_OK) return cs;
        }
        if (tune && hipStreamSynchronize(b->s) != hipSuccess) return MG_ERR_HIP;
        const auto l0 = std::chrono::steady_clock::now();
        mg_status ls = batch_launch(b, mode);
        if (ls != MG_OK) return ls;
        if (tune) {
            if (hipStreamSynchronize(b->s) != hipSuccess) return MG_ERR_HIP;
            b->ms_mode[mode - 1] =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - l0).count();
            if (mode == MG_BATCH_GROUPS) {
                int best = MG_BATCH_GRAPH;
                for (int q = MG_BATCH_LANES; q <= MG_BATCH_GROUPS; q++)
                    if (b->ms_mode[q - 1] < b->ms_mode[best - 1]) best = q;
                b->mode = best;
            }
        }
    }
    // the members' states back to the callers' arrays
    for (int i = 0; i < n; i++) {
        const int64_t m = b->ctx[i]->cells[0];
        if (hipMemcpyAsync(u[i], b->cu[i], m * sizeof(double), hipMemcpyDeviceToDevice, b->s) != hipSuccess)
            return MG_ERR_HIP;
        if (b->hasW[i] &&
            hipMemcpyAsync(W[i], b->cW[i], 3 * m * sizeof(double), hipMemcpyDeviceToDevice, b->s) != hipSuccess)
            return MG_ERR_HIP;
    }
    if (hipStreamSynchronize(b->s) != hipSuccess) return MG_ERR_HIP;
    auto t1 = std::chrono::steady_clock::now();
    mg_status worst = MG_OK;
    for (int i = 0; i < n; i++) {
        const double *h = b->hpin + (size_t)b->slot[i] * S_COUNT;
        const double inv = 1.0 / (double)b->ctx[i]->cells[0];
        mg_status st = h[S_ACTIVE] != 0.0 ? MG_ERR_NOT_CONVERGED : MG_OK;
        if (h[S_DIVERGED] != 0.0) st = MG_ERR_DIVERGED;
        if (h[S_FLAG_PSI] != 0.0) st = MG_ERR_SINGULAR;
        if (st != MG_OK && worst == MG_OK) worst = st;
        if (reps) {
            mg_report &r = reps[i];
            r.outer_iters = (int)h[S_ITERS];
            r.vcycles_psi = r.outer_iters;
            r.vcycles_W = b->ctx[i]->momentum ? r.outer_iters : 0;
            r.status = st;
            r.h_rms = std::sqrt(h[S_NORM + 0] * inv);
            r.m_rms = std::sqrt(h[S_NORM + 2] * inv);
            r.h_max = h[S_NORM + 1];
            r.m_max = h[S_NORM + 3];
            r.seconds = std::chrono::duration<double>(t1 - t0).count();
            r.history_len = 0;
        }
    }
    (void)it;
    return worst;
}

// ---------------------------------------------------------------------------------------
// Scalar-field sources (rho5, rho1, S_a of a field given by Fourier modes) and, on
// request, the grid mean of rho5 + rho1 and the constant K with K^2 = 24 pi <rho>, the
// value that makes the uniform part of the Hamiltonian constraint vanish at psi = 1.
// ---------------------------------------------------------------------------------------

mg_status check_sources_args(const mg_params *p, int n_phi, const double *h_phi_modes, int n_pi,
                             const double *h_pi_modes, double mass, const double *d_rho5,
                             const double *d_rho1, const double *d_S)
{
    if (!p || p->n < 1 || p->n > 4096 || !(p->length > 0.0)) return MG_ERR_INVALID;
    if (n_phi < 0 || n_phi > kMaxModes || n_pi < 0 || n_pi > kMaxModes) return MG_ERR_INVALID;
    if ((n_phi && !h_phi_modes) || (n_pi && !h_pi_modes)) return MG_ERR_INVALID;
    if (!d_rho5 || !d_rho1 || !d_S || !std::isfinite(mass)) return MG_ERR_INVALID;
    for (int q = 0; q < 5 * n_phi; q++)
        if (!std::isfinite(h_phi_modes[q])) return MG_ERR_INVALID;
    for (int q = 0; q < 5 * n_pi; q++)
        if (!std::isfinite(h_pi_modes[q])) return MG_ERR_INVALID;
    return MG_OK;
}

// Partials of the mean reduction: one per block of the source kernel, then the
// reduced mean at index kSrcBlocks.
constexpr size_t kSourcesScratchNeed = (size_t)(kSrcBlocks + 1) * sizeof(double);
static_assert(kSourcesScratchNeed <= MG_SOURCES_SCRATCH_BYTES, "source scratch");
static_assert(kSourcesScratchNeed <= MG_SOURCES_STATIC_SCRATCH_BYTES, "static source scratch");

// Arguments already checked by check_sources_args; scratch_d may be NULL when neither
// the mean nor K is requested.
mg_status scalar_sources(const mg_params *p, int n_phi, const double *h_phi_modes, int n_pi,
                         const double *h_pi_modes, double mass, double *d_rho5, double *d_rho1, double *d_S,
                         double *scratch_d, double *h_mean_rho, double *h_K, hipStream_t s)
{
    ModeTable t;
    std::memset(&t, 0, sizeof(t));
    t.nphi = n_phi;
    t.npi = n_pi;
    for (int q = 0; q < n_phi; q++)
        for (int e = 0; e < 5; e++) t.phi[q][e] = h_phi_modes[5 * q + e];
    for (int q = 0; q < n_pi; q++)
        for (int e = 0; e < 5; e++) t.pi[q][e] = h_pi_modes[5 * q + e];
    const Geo g = make_geo(p->n, p->bc, p->length, p->origin, p->puncture_pos);
    const int64_t m = (int64_t)p->n * p->n * p->n;
    const unsigned nb = std::min<unsigned>(nblk(m), kSrcBlocks);
    const bool want_mean = h_mean_rho || h_K;
    double *part = want_mean ? scratch_d : nullptr;
    hipLaunchKernelGGL(k_sources_modes, dim3(nb), dim3(kBlock), 0, s, g, p->length, t, mass, d_rho5,
                       d_rho1, d_S, part);
    if (want_mean) {
        double *res = scratch_d + kSrcBlocks;
        hipLaunchKernelGGL(k_reduce_final<1>, dim3(1), dim3(kBlock), 0, s, (const double *)part,
                           (int64_t)nb, 0u, 1.0 / (double)m, res, 0LL);
        double mean = 0.0;
        if (hipMemcpyAsync(&mean, res, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            return MG_ERR_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return MG_ERR_HIP;
        if (h_mean_rho) *h_mean_rho = mean;
        if (h_K) *h_K = std::sqrt(24.0 * M_PI * std::max(mean, 0.0));
    }
    return hip_status();
}

// Scratch of the allocation-free variant: a file-scope device array, one copy per
// GPU for the life of the process.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); it uses the device
// address looked up once per device with that device current.
static __device__ __align__(256) double scratch[MG_SOURCES_STATIC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices];

mg_status static_scratch_for(hipStream_t s, double **out)
{
    int dev = -1;
    if (s) {
        if (hipStreamGetDevice(s, &dev) != hipSuccess) return MG_ERR_HIP;
    } else if (hipGetDevice(&dev) != hipSuccess) {
        return MG_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return MG_ERR_INVALID;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return MG_ERR_HIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return MG_ERR_HIP;
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev && hipSetDevice(cur) != hipSuccess) return MG_ERR_HIP;
        if (e != hipSuccess || !ptr) return MG_ERR_HIP;
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MG_OK;
}

} // namespace

extern "C" {

mg_status mg_setup(const mg_params *p, void *d_workspace, size_t bytes, void *stream,
                   const double *d_rho5, const double *d_rho1, const double *d_S, const double *d_f,
                   mg_ctx **out)
{
    if (!out) return MG_ERR_INVALID;
    return ctx_create(p, d_workspace, bytes, (hipStream_t)stream, d_rho5, d_rho1, d_S, d_f, nullptr, out);
}

mg_status mg_batch_workspace_size(const mg_params *p, int32_t count, size_t *bytes)
{
    if (!p || !bytes || count < 1 || count > 4096) return MG_ERR_INVALID;
    for (int i = 0; i < count; i++) {
        mg_status st = validate(&p[i]);
        if (st != MG_OK) return st;
        if (p[i].precision != p[0].precision) return MG_ERR_INVALID;
    }
    *bytes = batch_plan(p, count).total;
    return MG_OK;
}

mg_status mg_setup_batch(const mg_params *p, int32_t count, void *d_workspace, size_t bytes, void *stream,
                         const double *const *d_rho5, const double *const *d_rho1, const double *const *d_S,
                         mg_batch **out)
{
    if (!out) return MG_ERR_INVALID;
    *out = nullptr;
    size_t need = 0;
    mg_status st = mg_batch_workspace_size(p, count, &need);
    if (st != MG_OK) return st;
    if (!d_rho5 || !d_rho1) return MG_ERR_INVALID;
    for (int i = 0; i < count; i++) {
        if (!d_rho5[i] || !d_rho1[i] || (p[i].flags & MG_FLAG_CTTK)) return MG_ERR_INVALID;
        if (p[i].solve_momentum && (!d_S || !d_S[i])) return MG_ERR_INVALID;
    }
    if (!d_workspace || bytes < need || ((uintptr_t)d_workspace % 256) != 0) return MG_ERR_WORKSPACE;
    const BatchPlan pl = batch_plan(p, count);
    mg_batch *b = new (std::nothrow) mg_batch;
    if (!b) return MG_ERR_INVALID;
    std::memset(b, 0, sizeof(*b));
    b->count = count;
    b->ngroups = pl.ngroups;
    b->user_s = (hipStream_t)stream;
    b->mode_req = b->mode = MG_BATCH_AUTO;
    b->ms_mode[0] = b->ms_mode[1] = b->ms_mode[2] = -1.0;
    b->g_tol = -1.0;
    b->ctx = new (std::nothrow) mg_ctx *[count]();
    b->gctx = new (std::nothrow) mg_ctx *[pl.ngroups]();
    b->gown = new (std::nothrow) bool[pl.ngroups]();
    b->gfirst = new (std::nothrow) int[pl.ngroups + 1]();
    b->order = new (std::nothrow) int[count]();
    b->slot = new (std::nothrow) int[count]();
    b->gof = new (std::nothrow) int[count]();
    b->gstride = new (std::nothrow) size_t[pl.ngroups]();
    b->cu = new (std::nothrow) double *[count]();
    b->cW = new (std::nothrow) double *[count]();
    b->c5 = new (std::nothrow) double *[count]();
    b->c1 = new (std::nothrow) double *[count]();
    b->cS = new (std::nothrow) double *[count]();
    b->hasW = new (std::nothrow) bool[count]();
    b->ev_join = new (std::nothrow) hipEvent_t[count]();
    if (!b->ctx || !b->gctx || !b->gown || !b->gfirst || !b->order || !b->slot || !b->gof || !b->gstride || !b->cu ||
        !b->cW || !b->c5 || !b->c1 || !b->cS || !b->hasW || !b->ev_join) {
        batch_release(b);
        return MG_ERR_INVALID;
    }
    for (int g = 0; g <= pl.ngroups; g++) b->gfirst[g] = pl.gfirst[g];
    for (int q = 0; q < count; q++) {
        b->order[q] = pl.order[q];
        b->slot[pl.order[q]] = q;
        b->gof[q] = pl.gof[q];
    }
    for (int g = 0; g < pl.ngroups; g++) b->gstride[g] = pl.gstride[g];
    bool ok = hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking) == hipSuccess;
    for (int q = 0; q < kBatchLanes && ok; q++)
        ok = hipStreamCreateWithFlags(&b->lane_s[q], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&b->ev_root, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < count && ok; i++)
        ok = hipEventCreateWithFlags(&b->ev_join[i], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&b->hpin, (size_t)count * S_COUNT * sizeof(double), hipHostMallocDefault) ==
                   hipSuccess;
    if (!ok) {
        batch_release(b);
        return MG_ERR_HIP;
    }
    b->scal_all = (double *)d_workspace;
    // members run after the work already on the caller's stream
    (void)hipEventRecord(b->ev_in, b->user_s);
    for (int q = 0; q < kBatchLanes; q++) (void)hipStreamWaitEvent(b->lane_s[q], b->ev_in, 0);
    for (int g = 0; g < pl.ngroups && st == MG_OK; g++) {
        hipStream_t ls = b->lane_s[g % kBatchLanes];
        for (int q = pl.gfirst[g]; q < pl.gfirst[g + 1] && st == MG_OK; q++) {
            const int i = pl.order[q];
            size_t wb = 0;
            mg_workspace_size(&p[i], &wb);
            const size_t m = (size_t)p[i].n * p[i].n * p[i].n * sizeof(double);
            char *r = (char *)d_workspace + pl.gbase[g] + (size_t)(q - pl.gfirst[g]) * pl.gstride[g];
            char *cp = r + align_up(wb, 256);
            b->c5[i] = (double *)cp;
            b->c1[i] = (double *)(cp + align_up(m, 256));
            b->cS[i] = (double *)(cp + 2 * align_up(m, 256));
            b->cu[i] = (double *)(cp + 2 * align_up(m, 256) + align_up(3 * m, 256));
            b->cW[i] = (double *)(cp + 3 * align_up(m, 256) + align_up(3 * m, 256));
            const bool hasS = d_S && d_S[i];
            if (hipMemcpyAsync(b->c5[i], d_rho5[i], m, hipMemcpyDeviceToDevice, ls) != hipSuccess ||
                hipMemcpyAsync(b->c1[i], d_rho1[i], m, hipMemcpyDeviceToDevice, ls) != hipSuccess ||
                (hasS && hipMemcpyAsync(b->cS[i], d_S[i], 3 * m, hipMemcpyDeviceToDevice, ls) != hipSuccess)) {
                st = MG_ERR_HIP;
                break;
            }
            st = ctx_create(&p[i], r, wb, ls, b->c5[i], b->c1[i], hasS ? b->cS[i] : nullptr, nullptr, ls, &b->ctx[i]);
            if (st != MG_OK) break;
            mg_ctx *c = b->ctx[i];
            c->batched = true;
            c->user_s = b->s;
            c->K2p = c->scal + S_K2;
        }
        if (st != MG_OK) break;
        // the group's context: member 0's region, launches spanning the group
        const int k = pl.gfirst[g + 1] - pl.gfirst[g];
        const int i0 = pl.order[pl.gfirst[g]];
        if (k == 1) {
            b->gctx[g] = b->ctx[i0];
            continue;
        }
        size_t wb = 0;
        mg_workspace_size(&p[i0], &wb);
        char *r0 = (char *)d_workspace + pl.gbase[g];
        st = ctx_create(&p[i0], r0, wb, ls, b->c5[i0], b->c1[i0], b->ctx[i0]->S, nullptr, ls, &b->gctx[g]);
        if (st != MG_OK) break;
        b->gown[g] = true;
        mg_ctx *gc = b->gctx[g];
        gc->batched = true;
        gc->user_s = b->s;
        gc->K2p = gc->scal + S_K2;
        gc->gz = k;
        gc->zs = (long long)pl.gstride[g];
        for (int l = 0; l < gc->L; l++) {
            gc->geo[l].gz = k;
            gc->geo[l].zs = gc->zs;
        }
    }
    // K^2 of every member into its scalar block (after every context's set-up)
    for (int i = 0; i < count && st == MG_OK; i++) {
        mg_ctx *c = b->ctx[i];
        fill<double>(c->s, c->scal + S_K2, 1, p[i].K * p[i].K);
    }
    for (int q = 0; q < kBatchLanes; q++) (void)hipStreamSynchronize(b->lane_s[q]);
    if (st == MG_OK && hip_status() != MG_OK) st = MG_ERR_HIP;
    if (st != MG_OK) {
        batch_release(b);
        return st;
    }
    *out = b;
    return MG_OK;
}

mg_status mg_solve_batch(mg_batch *b, double *const *d_u, double *const *d_W, double tol, int32_t max_outer,
                         mg_report *reps)
{
    if (!b || !d_u || !(tol > 0.0) || max_outer < 0) return MG_ERR_INVALID;
    for (int i = 0; i < b->count; i++) {
        if (!d_u[i]) return MG_ERR_INVALID;
        if (b->ctx[i]->momentum && (!d_W || !d_W[i])) return MG_ERR_INVALID;
    }
    // W given or not must agree within a group (one launch serves all of them)
    for (int g = 0; g < b->ngroups; g++)
        for (int q = b->gfirst[g]; q < b->gfirst[g + 1]; q++) {
            const int i = b->order[q], i0 = b->order[b->gfirst[g]];
            if ((d_W && d_W[i]) != (d_W && d_W[i0])) return MG_ERR_INVALID;
        }
    bool changed = false;
    for (int i = 0; i < b->count; i++) {
        const bool h = d_W && d_W[i];
        changed = changed || h != b->hasW[i];
        b->hasW[i] = h;
    }
    if (changed) b->captured_members = b->captured_groups = false;
    (void)hipEventRecord(b->ev_in, b->user_s);
    (void)hipStreamWaitEvent(b->s, b->ev_in, 0);
    double *const *W = d_W;
    double **Wn = nullptr;
    if (!d_W) {
        Wn = new (std::nothrow) double *[b->count]();
        if (!Wn) return MG_ERR_INVALID;
        W = Wn;
    }
    mg_status st = b->ctx[0]->f32 ? batch_solve<float>(b, d_u, W, tol, max_outer, reps)
                                  : batch_solve<double>(b, d_u, W, tol, max_outer, reps);
    delete[] Wn;
    (void)hipEventRecord(b->ev_out, b->s);
    (void)hipStreamWaitEvent(b->user_s, b->ev_out, 0);
    return st;
}

void mg_destroy_batch(mg_batch *b) { batch_release(b); }

mg_status mg_batch_launch_mode(mg_batch *b, int32_t request, int32_t *chosen, double h_ms[3])
{
    if (!b || request < -1 || request > MG_BATCH_GROUPS) return MG_ERR_INVALID;
    if (request >= 0) {
        b->mode_req = request;
        b->mode = request;
        if (request == MG_BATCH_AUTO) b->ms_mode[0] = b->ms_mode[1] = b->ms_mode[2] = -1.0;
    }
    if (chosen) *chosen = b->mode;
    if (h_ms)
        for (int q = 0; q < 3; q++) h_ms[q] = b->ms_mode[q];
    return MG_OK;
}

mg_status mg_batch_groups(mg_batch *b, int32_t *h_ngroups, int32_t *h_group_of)
{
    if (!b) return MG_ERR_INVALID;
    if (h_ngroups) *h_ngroups = b->ngroups;
    if (h_group_of)
        for (int i = 0; i < b->count; i++) h_group_of[i] = b->gof[i];
    return MG_OK;
}

mg_status mg_vcycle(mg_ctx *c, int32_t eq, double *d_u, double *d_W)
{
    if (!c || !d_u || eq < 1 || eq > 3) return MG_ERR_INVALID;
    if ((eq & MG_EQ_W) && (!c->momentum || !d_W)) return MG_ERR_INVALID;
    if (c->cttk && eq != MG_EQ_W) return MG_ERR_INVALID; // psi is data
    c->cont_valid = false;
    enter(c);
    if (eq == MG_EQ_BOTH && same_state(c)) {
        if (c->f32)
            vcycle_same_state<float>(c, d_u, d_W);
        else
            vcycle_same_state<double>(c, d_u, d_W);
    } else if (c->f32) {
        if (c->cttk) cttk_update<float>(c, d_u, d_W); // the W step reads this state's shifted sources
        if (eq & MG_EQ_W) step_W<float>(c, d_u, d_W, false);
        if (eq & MG_EQ_PSI) step_psi<float>(c, d_u, d_W, false);
    } else {
        if (c->cttk) cttk_update<double>(c, d_u, d_W);
        if (eq & MG_EQ_W) step_W<double>(c, d_u, d_W, false);
        if (eq & MG_EQ_PSI) step_psi<double>(c, d_u, d_W, false);
    }
    leave(c);
    return hip_status();
}

mg_status mg_solve_constraints(mg_ctx *c, double *d_u, double *d_W, double tol, int32_t max_outer,
                               mg_report *rep)
{
    if (!c || !d_u || !(tol > 0.0) || max_outer < 0) return MG_ERR_INVALID;
    if (c->momentum && !d_W) return MG_ERR_INVALID;
    if (rep && rep->history && rep->history_cap < 0) return MG_ERR_INVALID;
    c->cont_valid = false;
    enter(c);
    mg_status st = c->f32 ? solve<float>(c, d_u, d_W, tol, max_outer, rep)
                          : solve<double>(c, d_u, d_W, tol, max_outer, rep);
    leave(c);
    return st;
}

mg_status mg_solve_constraints_continue(mg_ctx *c, double *d_u, double *d_W, double tol, int32_t max_outer,
                                        mg_report *rep)
{
    if (!c || !d_u || !(tol > 0.0) || max_outer < 0) return MG_ERR_INVALID;
    if (c->momentum && !d_W) return MG_ERR_INVALID;
    if (rep && rep->history && rep->history_cap < 0) return MG_ERR_INVALID;
    if (!c->cont_valid || c->cont_u != d_u || c->cont_W != d_W) return MG_ERR_INVALID;
    enter(c);
    mg_status st = c->f32 ? solve<float>(c, d_u, d_W, tol, max_outer, rep, true)
                          : solve<double>(c, d_u, d_W, tol, max_outer, rep, true);
    leave(c);
    return st;
}

mg_status mg_residual_norm(mg_ctx *c, const double *d_u, const double *d_W, double out[4])
{
    if (!c || !d_u || !out) return MG_ERR_INVALID;
    const bool want_M = c->S != nullptr;
    if (c->cttk && !d_W) return MG_ERR_INVALID;
    c->cont_valid = false;
    enter(c);
    if (c->cttk) {
        if (c->f32)
            cttk_update<float>(c, d_u, d_W);
        else
            cttk_update<double>(c, d_u, d_W);
    }
    source_mean(c, d_u);
    if (c->f32)
        residual<float>(c, d_u, d_W, want_M, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true);
    else
        residual<double>(c, d_u, d_W, want_M, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true);
    if (hip_status() != MG_OK) return MG_ERR_HIP;
    mg_status st = fetch_norms(c, out, nullptr);
    leave(c);
    return st;
}

mg_status mg_residual_fields(mg_ctx *c, const double *d_u, const double *d_W, double *d_H, double *d_M,
                             double *d_c)
{
    if (!c || !d_u) return MG_ERR_INVALID;
    const bool want_M = d_M != nullptr;
    if (want_M && !c->S) return MG_ERR_INVALID;
    if (c->cttk && !d_W) return MG_ERR_INVALID;
    c->cont_valid = false;
    enter(c);
    if (c->cttk) cttk_update<double>(c, d_u, d_W);
    source_mean(c, d_u);
    residual<double>(c, d_u, d_W, want_M, d_H, d_M, d_c, nullptr, nullptr, nullptr, false);
    leave(c);
    return hip_status();
}

mg_status mg_cttk_trace(mg_ctx *c, const double *d_u, const double *d_W, double *d_K)
{
    if (!c || !c->cttk || !d_u || !d_W || !d_K) return MG_ERR_INVALID;
    c->cont_valid = false;
    enter(c);
    if (c->f32)
        cttk_update<float>(c, d_u, d_W);
    else
        cttk_update<double>(c, d_u, d_W);
    const bool ok = hipMemcpyAsync(d_K, c->Kf, (size_t)c->cells[0] * sizeof(double), hipMemcpyDeviceToDevice,
                                   c->s) == hipSuccess;
    leave(c);
    return ok ? hip_status() : MG_ERR_HIP;
}

mg_status mg_cttk_hybrid_sources(const mg_params *p, double *d_rho5, const double *d_rho1, double *d_S,
                                 double *d_K, void *d_scratch, size_t scratch_bytes, double *h_K0, void *stream)
{
    if (!p || p->n < 4 || p->n > 4096 || !(p->length > 0.0) || p->bc != MG_BC_PERIODIC) return MG_ERR_INVALID;
    if (!d_rho5 || !d_rho1 || !d_S || !d_K) return MG_ERR_INVALID;
    if (!d_scratch || scratch_bytes < kSourcesScratchNeed || ((uintptr_t)d_scratch % 256) != 0)
        return MG_ERR_WORKSPACE;
    const hipStream_t s = (hipStream_t)stream;
    const Geo g = make_geo(p->n, p->bc, p->length, p->origin, p->puncture_pos);
    const int64_t m = (int64_t)p->n * p->n * p->n;
    const unsigned nb = std::min<unsigned>(nblk(m), kSrcBlocks);
    double *part = (double *)d_scratch, *mean = part + kSrcBlocks;
    hipLaunchKernelGGL(k_sum_field, dim3(nb), dim3(kBlock), 0, s, d_rho1, m, part);
    hipLaunchKernelGGL(k_reduce_final<1>, dim3(1), dim3(kBlock), 0, s, (const double *)part, (int64_t)nb, 0u,
                       1.0 / (double)m, mean, 0LL);
    hipLaunchKernelGGL(k_cttk_hybrid_K, dim3(nblk(m)), dim3(kBlock), 0, s, m, (const double *)mean, d_rho5, d_K);
    hipLaunchKernelGGL(k_cttk_shift_S<kBcPeriodic>, dim3(nblk(m)), dim3(kBlock), 0, s, g, (const double *)d_K,
                       (const double *)d_S, d_S);
    if (h_K0) {
        double mv = 0.0;
        if (hipMemcpyAsync(&mv, mean, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return MG_ERR_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return MG_ERR_HIP;
        *h_K0 = std::sqrt(24.0 * M_PI * mv);
    }
    return hip_status();
}

mg_status mg_set_background(mg_ctx *c, const double *d_psi0, const double *d_A2)
{
    if (!c || c->batched || c->momentum) return MG_ERR_INVALID;
    if (d_psi0 && c->p.puncture_mass != 0.0) return MG_ERR_INVALID;
    c->bg_psi0 = d_psi0;
    c->bg_A2 = d_A2;
    c->cont_valid = false;
    drop_graph(c); // the captured residual launches carry the old pointers
    return MG_OK;
}

mg_status mg_bowen_york_sources(const mg_params *p, int32_t count, const double *h_table, double *d_psi0,
                                double *d_A2, void *stream)
{
    if (!p || p->n < 1 || p->n > 4096 || !(p->length > 0.0) || !d_psi0 || !d_A2) return MG_ERR_INVALID;
    if (count < 0 || count > kMaxPunctures || (count > 0 && !h_table)) return MG_ERR_INVALID;
    PunctureTable pt;
    std::memset(&pt, 0, sizeof(pt));
    pt.count = count;
    for (int q = 0; q < count; q++)
        for (int e = 0; e < 10; e++) {
            if (!std::isfinite(h_table[10 * q + e])) return MG_ERR_INVALID;
            pt.t[q][e] = h_table[10 * q + e];
        }
    const Geo g = make_geo(p->n, p->bc, p->length, p->origin, p->puncture_pos);
    const int64_t m = (int64_t)p->n * p->n * p->n;
    hipLaunchKernelGGL(k_bowen_york, dim3(nblk(m)), dim3(kBlock), 0, (hipStream_t)stream, g, pt, d_psi0, d_A2);
    return hip_status();
}

void mg_destroy(mg_ctx *c)
{
    if (!c) return;
    release(c);
}

mg_status mg_probe(mg_ctx *c, int32_t kernel, int32_t level)
{
    if (!c || kernel < MG_PROBE_NONE || kernel > MG_PROBE_UPDATE || level < -1 || level >= c->L)
        return MG_ERR_INVALID;
    if (kernel != MG_PROBE_NONE && !c->probe_ev) {
        c->probe_ev = new (std::nothrow) hipEvent_t[2 * kProbeMax];
        if (!c->probe_ev) return MG_ERR_INVALID;
        for (int q = 0; q < 2 * kProbeMax; q++)
            if (hipEventCreate(&c->probe_ev[q]) != hipSuccess) {
                for (int r = 0; r < q; r++) (void)hipEventDestroy(c->probe_ev[r]);
                delete[] c->probe_ev;
                c->probe_ev = nullptr;
                return MG_ERR_HIP;
            }
    }
    c->probe_kernel = kernel;
    c->probe_level = level;
    c->probe_count = 0;
    return MG_OK;
}

mg_status mg_probe_result(mg_ctx *c, int32_t *launches, double *total_ms)
{
    if (!c || !launches || !total_ms) return MG_ERR_INVALID;
    *launches = 0;
    *total_ms = 0.0;
    if (!c->probe_ev || c->probe_count == 0) return MG_OK;
    if (hipStreamSynchronize(c->s) != hipSuccess) return MG_ERR_HIP;
    double sum = 0.0;
    for (int q = 0; q < c->probe_count; q++) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->probe_ev[2 * q], c->probe_ev[2 * q + 1]) != hipSuccess)
            return MG_ERR_HIP;
        sum += ms;
    }
    *launches = c->probe_count;
    *total_ms = sum;
    c->probe_count = 0;
    return MG_OK;
}

const char *mg_status_str(mg_status s)
{
    switch (s) {
    case MG_OK: return "ok";
    case MG_ERR_INVALID: return "invalid argument";
    case MG_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case MG_ERR_HIP: return "HIP runtime error";
    case MG_ERR_NOT_CONVERGED: return "not converged within max_outer";
    case MG_ERR_DIVERGED: return "diverged (non-finite or exploding norm)";
    case MG_ERR_SINGULAR: return "singular coarsest-level matrix";
    }
    return "unknown status";
}

mg_status mg_scalar_field_sources(const mg_params *p, int32_t n_phi, const double *h_phi_modes,
                                  int32_t n_pi, const double *h_pi_modes, double mass, double *d_rho5,
                                  double *d_rho1, double *d_S, void *d_scratch, size_t scratch_bytes,
                                  double *h_mean_rho, double *h_K, void *stream)
{
    const mg_status st = check_sources_args(p, n_phi, h_phi_modes, n_pi, h_pi_modes, mass, d_rho5, d_rho1, d_S);
    if (st != MG_OK) return st;
    const bool want_mean = h_mean_rho || h_K;
    if (want_mean && (!d_scratch || scratch_bytes < MG_SOURCES_SCRATCH_BYTES ||
                      ((uintptr_t)d_scratch % 256) != 0))
        return MG_ERR_WORKSPACE;
    return scalar_sources(p, n_phi, h_phi_modes, n_pi, h_pi_modes, mass, d_rho5, d_rho1, d_S,
                          (double *)d_scratch, h_mean_rho, h_K, (hipStream_t)stream);
}

mg_status mg_scalar_field_sources_static(const mg_params *p, int32_t n_phi, const double *h_phi_modes,
                                         int32_t n_pi, const double *h_pi_modes, double mass,
                                         double *d_rho5, double *d_rho1, double *d_S, double *h_mean_rho,
                                         double *h_K, void *stream)
{
    const mg_status st = check_sources_args(p, n_phi, h_phi_modes, n_pi, h_pi_modes, mass, d_rho5, d_rho1, d_S);
    if (st != MG_OK) return st;
    double *scr = nullptr;
    if (h_mean_rho || h_K) {
        const int64_t m = (int64_t)p->n * p->n * p->n;
        const size_t need = ((size_t)std::min<unsigned>(nblk(m), kSrcBlocks) + 1) * sizeof(double);
        if (need > MG_SOURCES_STATIC_SCRATCH_BYTES) return MG_ERR_WORKSPACE;
        const mg_status ss = static_scratch_for((hipStream_t)stream, &scr);
        if (ss != MG_OK) return ss;
    }
    return scalar_sources(p, n_phi, h_phi_modes, n_pi, h_pi_modes, mass, d_rho5, d_rho1, d_S, scr, h_mean_rho,
                          h_K, (hipStream_t)stream);
}

mg_status mg_shell_field_sources(const mg_params *p, double amp, double r0, double width2, double mass,
                                 double *d_rho5, double *d_rho1, double *d_S, void *stream)
{
    if (!p || p->n < 1 || p->n > 4096 || !(p->length > 0.0) || !(width2 > 0.0)) return MG_ERR_INVALID;
    if (!d_rho5 || !d_rho1 || !d_S) return MG_ERR_INVALID;
    const Geo g = make_geo(p->n, p->bc, p->length, p->origin, p->puncture_pos);
    const int64_t m = (int64_t)p->n * p->n * p->n;
    hipLaunchKernelGGL(k_sources_shell, dim3(nblk(m)), dim3(kBlock), 0, (hipStream_t)stream, g, amp, r0,
                       width2, mass, d_rho5, d_rho1, d_S);
    return hip_status();
}

// ---- static mesh refinement by nested boxes ---------------------------------------------

} // extern "C"

namespace {

constexpr int kMaxRefineLevels = 8;

// Geometry of a box over its parent (corner at parent cell b0 on every axis, m parent
// cells per axis, 2m box cells): both psi-only, the box under the zero rule, a margin
// of 3 parent cells, matching spacing, origin and physics.
mg_status refine_check(const mg_params &pb, const mg_params &px, int b0)
{
    if (validate(&pb) != MG_OK || validate(&px) != MG_OK) return MG_ERR_INVALID;
    if (pb.solve_momentum || px.solve_momentum || px.bc != MG_BC_ZERO) return MG_ERR_INVALID;
    if ((pb.flags | px.flags) & MG_FLAG_CTTK) return MG_ERR_INVALID;
    if ((pb.flags & MG_FLAG_CONFORMAL_MATTER) != (px.flags & MG_FLAG_CONFORMAL_MATTER)) return MG_ERR_INVALID;
    if (px.n % 2 != 0) return MG_ERR_INVALID;
    const int m = px.n / 2;
    if (b0 < 3 || b0 + m + 3 > pb.n) return MG_ERR_INVALID;
    const double h = pb.length / pb.n, tol = 1e-12 * pb.length;
    if (std::fabs(px.length - m * h) > tol) return MG_ERR_INVALID;
    for (int a = 0; a < 3; a++)
        if (std::fabs(px.origin[a] - (pb.origin[a] + b0 * h)) > tol || px.puncture_pos[a] != pb.puncture_pos[a])
            return MG_ERR_INVALID;
    if (px.K != pb.K || px.puncture_mass != pb.puncture_mass) return MG_ERR_INVALID;
    return MG_OK;
}

mg_status refine_check_all(int L, const mg_params *const *p, const int32_t *b0)
{
    if (L < 2 || L > kMaxRefineLevels || !p || !b0) return MG_ERR_INVALID;
    for (int k = 0; k < L; k++)
        if (!p[k]) return MG_ERR_INVALID;
    if (p[0]->bc == MG_BC_ZERO) return MG_ERR_INVALID;
    for (int k = 1; k < L; k++) {
        const mg_status st = refine_check(*p[k - 1], *p[k], b0[k]);
        if (st != MG_OK) return st;
    }
    return MG_OK;
}

// Workspace: per level its residual field, the old values (all but the finest) and
// the FAS forcing of intermediate levels, then the norm partials and result.
struct RefineWork {
    double *H[kMaxRefineLevels], *old[kMaxRefineLevels], *tau[kMaxRefineLevels];
    double *part, *res;
    size_t bytes;
};

RefineWork refine_layout(int L, const mg_params *const *p, char *base)
{
    Carver cv{base};
    RefineWork w;
    std::memset(&w, 0, sizeof(w));
    for (int k = 0; k < L; k++) {
        const size_t bytes = (size_t)p[k]->n * p[k]->n * p[k]->n * sizeof(double);
        w.H[k] = (double *)cv.take(bytes);
        if (k + 1 < L) w.old[k] = (double *)cv.take(bytes);
        if (k > 0 && k + 1 < L) w.tau[k] = (double *)cv.take(bytes);
    }
    w.part = (double *)cv.take(2 * (size_t)L * kSrcBlocks * sizeof(double));
    w.res = (double *)cv.take(2 * sizeof(double));
    w.bytes = align_up(cv.off, 256);
    return w;
}

// One Newton-multigrid step of eq. Ham on a context, on its own stream (ordered
// after and before the caller's stream).
void psi_step(mg_ctx *c, double *u)
{
    enter(c);
    if (c->f32)
        step_psi<float>(c, u, nullptr, false);
    else
        step_psi<double>(c, u, nullptr, false);
    leave(c);
}

// H_h of a context at u (its forcing included) into H.
void residual_field(mg_ctx *c, const double *u, double *H)
{
    enter(c);
    residual<double>(c, u, nullptr, false, H, nullptr, nullptr, nullptr, nullptr, nullptr, false);
    leave(c);
}

mg_status refine_solve(int L, mg_ctx *const *c, const int32_t *b0, double *const *u, void *d_work, size_t work_bytes,
                       double tol, int max_outer, int nu_box, int nu_base, mg_report *rep)
{
    if (L < 2 || L > kMaxRefineLevels || !c || !b0 || !u || !(tol > 0.0) || max_outer < 0 || nu_box < 1 ||
        nu_base < 1)
        return MG_ERR_INVALID;
    if (rep && rep->history && rep->history_cap < 0) return MG_ERR_INVALID;
    const mg_params *p[kMaxRefineLevels];
    for (int k = 0; k < L; k++) {
        if (!c[k] || !u[k] || c[k]->batched || !c[k]->f || c[k]->user_s != c[0]->user_s || c[k]->bg_psi0 ||
            c[k]->bg_A2)
            return MG_ERR_INVALID;
        for (int q = 0; q < k; q++)
            if (c[q] == c[k] || u[q] == u[k]) return MG_ERR_INVALID;
        p[k] = &c[k]->p;
    }
    if (refine_check_all(L, p, b0) != MG_OK) return MG_ERR_INVALID;
    const RefineWork w = refine_layout(L, p, (char *)d_work);
    if (!d_work || work_bytes < w.bytes || ((uintptr_t)d_work % 256) != 0) return MG_ERR_WORKSPACE;
    auto t0 = std::chrono::steady_clock::now();
    const hipStream_t s = c[0]->user_s;
    BoxGeo bx[kMaxRefineLevels]; // bx[k]: level k as the box of level k - 1
    int64_t cells[kMaxRefineLevels];
    double *f[kMaxRefineLevels], vol[kMaxRefineLevels];
    for (int k = 0; k < L; k++) {
        c[k]->cont_valid = false;
        c[k]->vc_psi = 0;
        cells[k] = (int64_t)p[k]->n * p[k]->n * p[k]->n;
        f[k] = const_cast<double *>(c[k]->f);
        const double h = p[k]->length / p[k]->n;
        vol[k] = h * h * h;
        bx[k] = k ? BoxGeo{p[k - 1]->n, b0[k], p[k]->n / 2} : BoxGeo{0, 0, 0};
    }
    const double total = p[0]->length * p[0]->length * p[0]->length;
    // a parent's cells under box k take their children's average
    auto to_parent = [&](int k) {
        hipLaunchKernelGGL(k_box_restrict, dim3(nblk((int64_t)bx[k].m * bx[k].m * bx[k].m)), dim3(kBlock), 0, s, bx[k],
                           (const double *)u[k], u[k - 1]);
    };
    // the forcing of level k: interface ghosts from its parent (+ its FAS forcing);
    // the base level: its FAS forcing or zero
    auto forcing = [&](int k, const double *tau) {
        if (k > 0)
            hipLaunchKernelGGL(k_box_ghost_forcing, dim3(nblk(cells[k])), dim3(kBlock), 0, s, bx[k],
                               c[k]->geo[0].inv12h2, (const double *)u[k - 1], tau, f[k]);
        else
            fill<double>(s, f[0], cells[0], 0.0);
    };
    const unsigned nbn = kSrcBlocks;
    mg_status st = MG_ERR_NOT_CONVERGED;
    double nr[4] = {0, 0, 0, 0}, first = -1.0;
    int it = 0, hist = 0;
    for (;; it++) {
        // composite norm of the synchronised state
        for (int k = L - 1; k > 0; k--) to_parent(k);
        for (int k = 0; k < L; k++) {
            forcing(k, nullptr);
            residual_field(c[k], u[k], w.H[k]);
            const BoxGeo child = k + 1 < L ? bx[k + 1] : BoxGeo{0, 0, 0};
            const unsigned nb = std::min<unsigned>(nblk(cells[k]), nbn);
            fill<double>(s, w.part + 2 * (size_t)k * nbn, 2 * (int64_t)nbn, 0.0);
            hipLaunchKernelGGL(k_level_norm, dim3(nb), dim3(kBlock), 0, s, p[k]->n, child, vol[k],
                               (const double *)w.H[k], w.part + 2 * (size_t)k * nbn);
        }
        hipLaunchKernelGGL(k_reduce_final<2>, dim3(1), dim3(kBlock), 0, s, (const double *)w.part,
                           (int64_t)L * nbn, 0x2u, 0.0, w.res, 0LL);
        if (hipMemcpyAsync(c[0]->hpin, w.res, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MG_ERR_HIP;
        nr[0] = std::sqrt(c[0]->hpin[0] / total);
        nr[2] = c[0]->hpin[1];
        if (rep && rep->history && hist < rep->history_cap) {
            std::memcpy(rep->history + 4 * hist, nr, sizeof(nr));
            hist++;
        }
        if (!std::isfinite(nr[0]) || !std::isfinite(nr[2])) {
            st = MG_ERR_DIVERGED;
            break;
        }
        if (first < 0.0) first = nr[0];
        if (nr[0] <= tol) {
            st = MG_OK;
            break;
        }
        if (nr[0] > 1e6 * std::fmax(first, tol)) {
            st = MG_ERR_DIVERGED;
            break;
        }
        if (it >= max_outer) {
            st = MG_ERR_NOT_CONVERGED;
            break;
        }
        // down the levels: box steps, then the FAS forcing of the parent
        for (int k = L - 1; k > 0; k--) {
            const double *tau_k = k + 1 < L ? w.tau[k] : nullptr;
            for (int q = 0; q < nu_box; q++) {
                to_parent(k);
                forcing(k, tau_k);
                psi_step(c[k], u[k]);
            }
            to_parent(k);
            forcing(k, tau_k);
            residual_field(c[k], u[k], w.H[k]);
            forcing(k - 1, nullptr);
            residual_field(c[k - 1], u[k - 1], w.H[k - 1]);
            double *dst = k - 1 > 0 ? w.tau[k - 1] : f[0];
            hipLaunchKernelGGL(k_box_tau, dim3(nblk(cells[k - 1])), dim3(kBlock), 0, s, bx[k], (const double *)w.H[k],
                               (const double *)w.H[k - 1], dst);
            if (hipMemcpyAsync(w.old[k - 1], u[k - 1], cells[k - 1] * sizeof(double), hipMemcpyDeviceToDevice, s) !=
                hipSuccess)
                return MG_ERR_HIP;
        }
        // the base grid with its FAS forcing (f[0] holds tau)
        for (int q = 0; q < nu_base; q++) psi_step(c[0], u[0]);
        // up the levels: every box adds the cubic interpolation of its parent's change
        for (int k = 1; k < L; k++)
            hipLaunchKernelGGL(k_box_correct, dim3(nblk((int64_t)bx[k].m * bx[k].m * bx[k].m)), dim3(kBlock), 0, s,
                               bx[k], (const double *)u[k - 1], (const double *)w.old[k - 1], u[k]);
        if (hip_status() != MG_OK) return MG_ERR_HIP;
    }
    // the parents' cells under every box end as their children's average
    for (int k = L - 1; k > 0; k--) to_parent(k);
    if (hip_status() != MG_OK) return MG_ERR_HIP;
    auto t1 = std::chrono::steady_clock::now();
    if (rep) {
        int vc = 0;
        for (int k = 0; k < L; k++) vc += c[k]->vc_psi;
        rep->outer_iters = it;
        rep->vcycles_psi = vc;
        rep->vcycles_W = 0;
        rep->status = st;
        rep->h_rms = nr[0];
        rep->m_rms = 0.0;
        rep->h_max = nr[2];
        rep->m_max = 0.0;
        rep->seconds = std::chrono::duration<double>(t1 - t0).count();
        rep->history_len = hist;
    }
    return st;
}

} // namespace

extern "C" {

mg_status mg_refine_workspace_size(const mg_params *base, const mg_params *box, int32_t b0, size_t *bytes)
{
    const mg_params *p[2] = {base, box};
    const int32_t off[2] = {0, b0};
    return mg_refine_nested_workspace_size(2, p, off, bytes);
}

mg_status mg_refine_nested_workspace_size(int32_t levels, const mg_params *const *p, const int32_t *b0, size_t *bytes)
{
    if (!bytes) return MG_ERR_INVALID;
    const mg_status st = refine_check_all(levels, p, b0);
    if (st != MG_OK) return st;
    *bytes = refine_layout(levels, p, nullptr).bytes;
    return MG_OK;
}

mg_status mg_refine_solve(mg_ctx *cb, mg_ctx *cx, int32_t b0, double *d_uc, double *d_uf, void *d_work,
                          size_t work_bytes, double tol, int32_t max_outer, int32_t nu_box, int32_t nu_base,
                          mg_report *rep)
{
    mg_ctx *c[2] = {cb, cx};
    const int32_t off[2] = {0, b0};
    double *u[2] = {d_uc, d_uf};
    return refine_solve(2, c, off, u, d_work, work_bytes, tol, max_outer, nu_box, nu_base, rep);
}

mg_status mg_refine_solve_nested(int32_t levels, mg_ctx *const *ctx, const int32_t *b0, double *const *d_u,
                                 void *d_work, size_t work_bytes, double tol, int32_t max_outer, int32_t nu_box,
                                 int32_t nu_base, mg_report *rep)
{
    return refine_solve(levels, ctx, b0, d_u, d_work, work_bytes, tol, max_outer, nu_box, nu_base, rep);
}

mg_status mg_interp_cubic(const mg_params *pc, const double *d_coarse, double *d_fine, void *stream)
{
    if (!pc || pc->n < 2 || pc->n > 2048 || !(pc->length > 0.0) || !d_coarse || !d_fine)
        return MG_ERR_INVALID;
    if (pc->bc < MG_BC_PERIODIC || pc->bc > MG_BC_ZERO) return MG_ERR_INVALID;
    const Geo gc = make_geo(pc->n, pc->bc, pc->length, pc->origin, pc->puncture_pos);
    const int64_t mf = 8 * (int64_t)pc->n * pc->n * pc->n;
    if (pc->bc == MG_BC_PERIODIC)
        hipLaunchKernelGGL(k_interp_cubic<kBcPeriodic>, dim3(nblk(mf / 8)), dim3(kBlock), 0, (hipStream_t)stream,
                           gc, d_coarse, d_fine);
    else
        with_bc(pc->bc, [&](auto bcx) {
            constexpr int BCX = decltype(bcx)::value;
            hipLaunchKernelGGL(k_interp_cubic<BCX>, dim3(nblk(mf / 8)), dim3(kBlock), 0, (hipStream_t)stream, gc,
                               d_coarse, d_fine);
        });
    return hip_status();
}

mg_status mg_fmg_start(mg_ctx *cc, mg_ctx *cf, double *d_uc, double *d_Wc, double tol_c, int32_t max_outer,
                       double *d_uf, double *d_Wf, mg_report *rep_c)
{
    if (!cc || !cf || !d_uc || !d_uf || !(tol_c > 0.0) || max_outer < 0) return MG_ERR_INVALID;
    cc->cont_valid = cf->cont_valid = false;
    const mg_params &a = cc->p, &b = cf->p;
    if (b.n != 2 * a.n || a.bc != b.bc || a.length != b.length || cc->momentum != cf->momentum) return MG_ERR_INVALID;
    if (cc->cttk || cf->cttk) return MG_ERR_INVALID; // CTTK: psi is data, not interpolated
    for (int q = 0; q < 3; q++)
        if (a.origin[q] != b.origin[q] || a.puncture_pos[q] != b.puncture_pos[q]) return MG_ERR_INVALID;
    if (cf->momentum && (!d_Wc || !d_Wf)) return MG_ERR_INVALID;
    const mg_status st = mg_solve_constraints(cc, d_uc, d_Wc, tol_c, max_outer, rep_c);
    if (st != MG_OK && st != MG_ERR_NOT_CONVERGED) return st;
    // the fine context's stream waits for the caller's stream (after the coarse solve)
    enter(cf);
    const Geo gc = make_geo(a.n, a.bc, a.length, a.origin, a.puncture_pos);
    const int64_t mc = (int64_t)a.n * a.n * a.n, mf = 8 * mc;
    const int ncomp = (cf->momentum || (d_Wc && d_Wf)) ? 4 : 1;
    for (int q = 0; q < ncomp; q++) {
        const double *src = q == 0 ? d_uc : d_Wc + (q - 1) * mc;
        double *dst = q == 0 ? d_uf : d_Wf + (q - 1) * mf;
        if (a.bc == MG_BC_PERIODIC)
            hipLaunchKernelGGL(k_interp_cubic<kBcPeriodic>, dim3(nblk(mf / 8)), dim3(kBlock), 0, cf->s, gc, src, dst);
        else
            with_bc(a.bc, [&](auto bcx) {
                constexpr int BCX = decltype(bcx)::value;
                hipLaunchKernelGGL(k_interp_cubic<BCX>, dim3(nblk(mf / 8)), dim3(kBlock), 0, cf->s, gc, src, dst);
            });
    }
    leave(cf);
    if (hip_status() != MG_OK) return MG_ERR_HIP;
    return st;
}

mg_status mg_autotune(mg_ctx *c, const double *d_u, const double *d_W, int32_t reps, mg_tune *h_out, int32_t cap,
                      int32_t *h_count)
{
    if (!c || !d_u || reps < 1 || reps > 1000 || cap < 0 || (cap > 0 && !h_out)) return MG_ERR_INVALID;
    if (c->momentum && !d_W) return MG_ERR_INVALID;
    c->cont_valid = false;
    enter(c);
    int k = 0;
    mg_status st = c->f32 ? autotune<float>(c, d_u, d_W, reps, h_out, cap, &k)
                          : autotune<double>(c, d_u, d_W, reps, h_out, cap, &k);
    leave(c);
    if (h_count) *h_count = k;
    return st;
}

mg_status mg_set_tile(mg_ctx *c, int32_t family, int32_t level, int32_t tx)
{
    if (!c || level < 0 || level >= c->L) return MG_ERR_INVALID;
    c->cont_valid = false;
    if (family == MG_TUNE_FOURIER_W) {
        if (c->fourier_W < 0 || level != c->fourier_W || (tx != 0 && tx != 1)) return MG_ERR_INVALID;
        c->fourier_W_on = tx != 0;
        drop_graph(c);
        return MG_OK;
    }
    if (family == MG_TUNE_TAIL_PSI || family == MG_TUNE_TAIL_W) {
        // a tail may start at any level from the highest that fits down to the one above the coarsest
        const int first = family == MG_TUNE_TAIL_PSI ? c->tail_psi_min : c->tail_W_min;
        if (first < 0 || level < first || level > c->L - 2 || (tx != 0 && tx != 1)) return MG_ERR_INVALID;
        (family == MG_TUNE_TAIL_PSI ? c->tail_psi : c->tail_W) = tx != 0 ? level : first;
        (family == MG_TUNE_TAIL_PSI ? c->tail_psi_on : c->tail_W_on) = tx != 0;
        drop_graph(c);
        return MG_OK;
    }
    int nc = 0;
    const int *cand = tune_candidates(c, family, nc);
    bool ok = false;
    for (int q = 0; q < nc; q++) ok = ok || cand[q] == tx;
    if (!ok) return MG_ERR_INVALID;
    const TileMap tm = tune_map(c, family, level, tx);
    if (tm.tx == 0) return MG_ERR_INVALID;
    tune_slot(c, family, level) = tm;
    drop_graph(c);
    return MG_OK;
}

mg_status mg_kernel_op(mg_ctx *c, int32_t op, int32_t level, int32_t arg, const void *d_in, void *d_out,
                       const void *d_r, const void *d_c)
{
    if (!c) return MG_ERR_INVALID;
    c->cont_valid = false;
    enter(c);
    mg_status st = c->f32 ? kernel_op<float>(c, op, level, arg, d_in, d_out, d_r, d_c)
                          : kernel_op<double>(c, op, level, arg, d_in, d_out, d_r, d_c);
    leave(c);
    return st;
}

} // extern "C"

namespace grtmg {

SolverShape solver_shape(const mg_ctx *c)
{
    SolverShape sh;
    sh.n = c->p.n;
    sh.bc = c->p.bc;
    sh.momentum = c->momentum;
    sh.cttk = c->cttk;
    sh.user_stream = (void *)c->user_s;
    return sh;
}

mg_status zero_norms_begin(mg_ctx *c, double *d_u, double *d_W)
{
    if (!c || !d_u || (c->S && !d_W)) return MG_ERR_INVALID;
    const bool want_M = c->S != nullptr;
    const int64_t m = c->cells[0];
    c->cont_valid = false;
    enter(c);
    if (hipMemsetAsync(d_u, 0, m * sizeof(double), c->s) != hipSuccess ||
        (d_W && hipMemsetAsync(d_W, 0, 3 * m * sizeof(double), c->s) != hipSuccess)) {
        leave(c);
        return MG_ERR_HIP;
    }
    source_mean(c, d_u);
    if (c->f32)
        residual<float>(c, d_u, d_W, want_M, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true);
    else
        residual<double>(c, d_u, d_W, want_M, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, true);
    mg_status st = hip_status();
    if (st == MG_OK) st = post_norms(c, 0);
    if (st != MG_OK) leave(c);
    return st;
}

void cancel_continue(mg_ctx *c)
{
    if (c) c->cont_valid = false;
}

mg_status check_iteration(mg_ctx *c, double *d_u, double *d_W, mg_report *rep)
{
    if (!c || !d_u || (c->momentum && !d_W)) return MG_ERR_INVALID;
    c->cont_valid = false;
    enter(c);
    constexpr double kNever = 1e-300;
    mg_status st = c->f32 ? solve<float>(c, d_u, d_W, kNever, 1, rep, false, true)
                          : solve<double>(c, d_u, d_W, kNever, 1, rep, false, true);
    leave(c);
    return st;
}

mg_status zero_norms_end(mg_ctx *c, double out[4])
{
    if (!c || !out) return MG_ERR_INVALID;
    mg_status st = read_norms(c, 0, out, nullptr);
    leave(c);
    return st;
}

} // namespace grtmg
