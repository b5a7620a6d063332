/*
 * grtmg.h -- C ABI of the MI355X multigrid solver for the initial-data
 * constraints of numerical relativity.
 *
 * The problem is the pair of constraint equations of the paper's Summary:
 * the Hamiltonian constraint (eq. Ham) and the momentum constraint (eq. Mom),
 * with the matter projections rho and S_i of a scalar field, solved in
 * conformal transverse-traceless (CTT) form for the conformal factor psi and
 * the vector potential W_i of the longitudinal extrinsic curvature.  The
 * solver is geometric multigrid (Key features: "Fast", a multigrid method
 * over a hierarchy of discretisations) and reports the constraint norms at
 * every iteration (Key features: "Diagnostics").
 *
 * Discrete system solved (cell-centred N^3 grid, h = L/N, 4th-order central
 * differences D_a, D_aa, D_ab = D_a D_b; psi = psi0 + u):
 *   H_h = L_h u + 2 pi rho5 psi^5 + 2 pi rho1 psi - (K^2/12) psi^5
 *         + (1/8) A2 psi^-7 + f                                   -> 0
 *   M_h = Delta_L,h W - (8 pi psi^6 S - mean(8 pi psi^6 S))       -> 0
 * with Abar_ab = D_a W_b + D_b W_a - (2/3) delta_ab D_c W_c, A2 = Abar_ab Abar_ab,
 * (Delta_L W)_a = sum_b D_bb W_a + (1/3)(D_aa W_a + sum_{b!=a} D_ab W_b),
 * rho = rho5 + psi^-4 rho1 (rho5 = Pi^2/2 + V(phi), rho1 = |d phi|^2/2),
 * S_a = -Pi d_a phi, constant K; psi0 = 1, or 1 + M/(2r) with a puncture.
 * The mean of the momentum source is removed on periodic grids.
 *
 * Conventions for every call:
 *  - Arrays are structure-of-arrays, cell-centred, z fastest:
 *    element (i,j,k) of an N^3 field is at (i*N + j)*N + k; a 3-vector field
 *    stores its x, y, z components as three consecutive N^3 blocks.
 *  - Names starting with d_ are device pointers, h_ host pointers.
 *  - The caller owns every array and the workspace; the library never
 *    allocates device memory and only carves the workspace it is given.  It
 *    owns the host-side mg_ctx until mg_destroy, plus a few bytes of pinned
 *    host memory per context for the norms.
 *  - Source arrays passed to mg_setup are borrowed and must outlive the ctx.
 *  - All work is ordered on the HIP stream given at setup (a hipStream_t
 *    passed as void*; NULL means the default stream): each call waits for
 *    the work already on that stream and that stream waits for the call's
 *    work.  Internally a context runs on a stream of its own (created at
 *    setup with default priority), whose outer-iteration body is captured
 *    once into a hipGraph and replayed; a context with MG_FLAG_SAME_STATE
 *    and the momentum equation creates a second one (default priority) for
 *    the psi branch of that graph, forked from and joined back into the
 *    first within every iteration.  Calls that return host scalars (norms,
 *    reports) wait for the context's own work only.
 *  - No call throws.  Arguments are validated before any HIP call; a non-OK
 *    status leaves device arrays untouched unless stated otherwise.
 */
#ifndef GRTMG_H
#define GRTMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mg_status {
    MG_OK = 0,
    MG_ERR_INVALID = 1,       /* bad argument (checked before any HIP call)        */
    MG_ERR_WORKSPACE = 2,     /* workspace missing, too small or misaligned        */
    MG_ERR_HIP = 3,           /* a HIP runtime call failed                         */
    MG_ERR_NOT_CONVERGED = 4, /* max_outer updates done without reaching tol        */
    MG_ERR_DIVERGED = 5,      /* non-finite or exploding constraint norm            */
    MG_ERR_SINGULAR = 6       /* coarsest-level matrix could not be factorised      */
} mg_status;

enum { MG_BC_PERIODIC = 0, MG_BC_ROBIN = 1, MG_BC_REFLECT = 2, MG_BC_EXTRAP = 3, MG_BC_ZERO = 4 };
enum { MG_PREC_FP64 = 0, MG_PREC_FP32_IR = 1 };
enum { MG_EQ_PSI = 1, MG_EQ_W = 2, MG_EQ_BOTH = 3 };
enum {
    MG_FLAG_CONFORMAL_MATTER = 1,
    MG_FLAG_EAGER = 2,
    MG_FLAG_CTTK = 4,
    MG_FLAG_CUBIC_PROLONG = 8,
    MG_FLAG_SAME_STATE = 16
};

/*
 * Problem and solver parameters.
 *  n              cells per axis (n^3 < 2^32, i.e. n <= 1625); every level but
 *                 the coarsest must have n_l even and n_l >= 6, the coarsest
 *                 n >> (levels-1) >= 3.
 *  levels         number of multigrid levels (1..16).
 *  bc             boundary rule for every field on every level, applied as two
 *                 ghost layers (Key features, "Boundary conditions": periodic,
 *                 reflective and extrapolating; the Robin rule serves isolated
 *                 black holes):
 *                 MG_BC_PERIODIC: wrap.  MG_BC_ROBIN: ghost a(g) = a(b)|x_b|/|x_g|,
 *                 b = grid cell nearest g, radii from puncture_pos.
 *                 MG_BC_REFLECT: mirror image across the face (a(-1) = a(0),
 *                 a(-2) = a(1); even parity).  MG_BC_EXTRAP: zeroth-order
 *                 extrapolation along the face normal (a(-1) = a(-2) = a(0)).
 *                 MG_BC_ZERO: homogeneous ghosts (a(-1) = a(-2) = 0), the rule of a
 *                 refined box whose interface values enter through the forcing f
 *                 (see mg_refine_solve).
 *                 The momentum equation is supported on periodic grids only.
 *  precision      MG_PREC_FP64: every kernel in FP64.  MG_PREC_FP32_IR: V-cycle
 *                 interior (smoothers, transfers, defects) in FP32 inside FP64
 *                 iterative refinement; residual, update and coarsest solve FP64.
 *  nu_pre/nu_post red-black sweeps before/after the coarse correction (>= 1).
 *  solve_momentum 0: W frozen at the caller's values; 1: coupled solve
 *                 (n^3 * 8 bytes below 4 GiB, i.e. n <= 812).
 *  flags          bit MG_FLAG_CONFORMAL_MATTER: the matter arrays are the
 *                 conformally rescaled free data rho_bar = psi^8 rho (taken as
 *                 rho5 + rho1) and S_bar = psi^6 S; H_h then carries
 *                 2 pi rho_bar psi^-3 and M_h the source 8 pi S_bar (the
 *                 textbook CTT rescaling that keeps dH_h/dpsi negative).
 *                 bit MG_FLAG_EAGER: launch every kernel from the host instead
 *                 of replaying the captured outer-iteration graph (results are
 *                 identical; for measurement and tests).
 *                 bit MG_FLAG_CTTK: the CTTK method (Key features, "Methods";
 *                 read from eqs. Ham and Mom with a spatially varying K): psi =
 *                 1 + u is free data that no call changes, and eq. Ham is solved
 *                 for the trace instead, K^2 = 12 H0 / psi^5 with H0 = H_h at
 *                 K = 0 (the caller's rho5, rho1 and f).  Every evaluation of a
 *                 state (u, W) first forms that K and the shifted sources
 *                 rho5 - K^2/(24 pi) and S + D K/(12 pi) (the -(2/3) psi^6 d_a K of
 *                 eq. Mom), so H_h vanishes up to rounding and M_h carries the
 *                 trace term; an outer iteration is the W step alone.  Where
 *                 K^2 < 0 (a psi whose Laplacian outweighs the energy density)
 *                 K is NaN and a solve ends with MG_ERR_DIVERGED.  Requires
 *                 solve_momentum = 1, periodic boundaries, K = 0, no puncture and
 *                 no conformal matter; not in batches, mg_fmg_start or
 *                 nn_warm_start (MG_ERR_INVALID).  The workspace grows by
 *                 5 n^3 doubles.
 *                 bit MG_FLAG_CUBIC_PROLONG: the V-cycles prolong corrections with
 *                 the 4-point cubic of mg_interp_cubic (weights (-5, 35, 105, -7)/128
 *                 and mirror per axis, ghosts by the boundary rule) instead of
 *                 trilinearly; no V-cycle tails (MG_TUNE_TAIL_* unavailable).
 *                 bit MG_FLAG_SAME_STATE: with solve_momentum = 1 (not CTTK), both
 *                 steps of an outer iteration (mg_vcycle with MG_EQ_BOTH, every
 *                 iteration of a solve) linearise eqs. Mom and Ham at the same
 *                 state: the psi step no longer sees the W update of its own
 *                 iteration.  One finest residual launch per iteration then
 *                 forms both steps' right-hand sides, and inside the captured
 *                 iteration of a single (not batched) context the two V-cycles
 *                 run as concurrent graph branches.  The fixed point is the same
 *                 discrete solution; the contraction per iteration can be
 *                 slightly lower.  No effect without the momentum equation.
 *                 Other bits must be 0.
 *  length, origin box side L and corner of the box (cell centres at
 *                 origin + (i + 1/2) L/n).
 *  K              constant trace of the extrinsic curvature.
 *  puncture_mass  0: psi0 = 1; > 0: psi0 = 1 + M / (2 |x - puncture_pos|).
 *  nu_pre_W/nu_post_W  sweeps of the W V-cycle while its bottom is exact (see
 *                 MG_TUNE_FOURIER_W; 0: nu_pre / nu_post; else 1 .. 16).  Its coarse
 *                 correction is then exact, and one post-sweep can do what two do
 *                 above a multigrid bottom.  Without the exact bottom the W cycle
 *                 uses nu_pre / nu_post.
 *  mix_depth      MG_FLAG_CTTK solves: steps the Anderson mixing of the W fixed
 *                 point combines (0 or 1: the one-step secant form; 2 .. 6: least
 *                 squares over the newest mix_depth difference pairs, with a ridge of
 *                 1e-12 of the largest Gram diagonal entry; the workspace grows by
 *                 2 mix_depth 3 n^3 values of the working precision).  Ignored
 *                 without MG_FLAG_CTTK.
 */
typedef struct mg_params {
    int32_t n, levels, bc, precision, nu_pre, nu_post, solve_momentum, flags;
    double length;
    double origin[3];
    double K;
    double puncture_mass;
    double puncture_pos[3];
    int32_t nu_pre_W, nu_post_W;
    int32_t mix_depth;
} mg_params;

/* Per-solve report.  history (host, caller-owned, may be NULL) receives
 * 4 doubles per recorded iteration: rms H, rms |M|, max |H|, max |M|. */
typedef struct mg_report {
    int32_t outer_iters, vcycles_psi, vcycles_W, status;
    double h_rms, m_rms, h_max, m_max;
    double seconds;
    double *history;
    int32_t history_cap, history_len;
} mg_report;

typedef struct mg_ctx mg_ctx;

/* Bytes of device workspace mg_setup needs for these parameters.  Host only. */
mg_status mg_workspace_size(const mg_params *p, size_t *bytes);

/*
 * Create a context for the discrete constraint system above (Summary: eq. Ham
 * and eq. Mom with the matter projections rho and S_i as sources; the free data
 * are the flat conformal metric, K and the matter fields).
 * d_workspace: caller-owned device buffer of at least
 * mg_workspace_size bytes, 256-byte aligned.  d_rho5, d_rho1: n^3 FP64 each;
 * d_S: 3 n^3 FP64 (may be NULL when solve_momentum is 0 and no momentum
 * norm is wanted); d_f: n^3 FP64 forcing added to H_h, or NULL.  The coarse
 * operator of the momentum equation is factorised here (enqueued on stream).
 */
mg_status mg_setup(const mg_params *p, void *d_workspace, size_t bytes, void *stream,
                   const double *d_rho5, const double *d_rho1, const double *d_S,
                   const double *d_f, mg_ctx **out);

/*
 * One outer multigrid step (Key features, "Fast": one multigrid V-cycle over
 * the hierarchy of discretisations per equation, eq. Mom for W and the Newton
 * linearisation of eq. Ham for psi) at the current state (d_u: n^3, d_W: 3 n^3, FP64,
 * updated in place).  eq = MG_EQ_W: r = -M_h(u, W), one W V-cycle, W += dW -
 * mean(dW).  eq = MG_EQ_PSI: r = -H_h(u, W), c = dH_h/dpsi, one psi V-cycle,
 * u += d.  eq = MG_EQ_BOTH: the W step then the psi step (one Newton outer
 * iteration).  Enqueued only (does not synchronise).
 */
mg_status mg_vcycle(mg_ctx *ctx, int32_t eq, double *d_u, double *d_W);

/*
 * Newton-multigrid solve of eqs. Ham and Mom (Summary; Key features, "Fast",
 * with the constraint norms of every iteration recorded as in Key features,
 * "Diagnostics") from the initial guess in (d_u, d_W) until
 * rms(H_h) <= tol and (if solve_momentum) rms(|M_h|) <= tol, or max_outer
 * outer updates.  Returns MG_OK, MG_ERR_NOT_CONVERGED or MG_ERR_DIVERGED;
 * rep (may be NULL) is filled in every case, and (u, W) hold the last finite
 * iterate.  Synchronises the stream once per outer iteration.
 */
mg_status mg_solve_constraints(mg_ctx *ctx, double *d_u, double *d_W, double tol,
                               int32_t max_outer, mg_report *rep);

/*
 * Continues the last mg_solve_constraints (or mg_solve_constraints_continue)
 * call on this context from the state it left in the same d_u, d_W: that
 * state's evaluation, still held in the workspace, is not repeated, and the
 * host round trips overlap the GPU work from the first iteration on.  Valid
 * only while no other call has been made on the context and the arrays have
 * not been changed since (the caller's guarantee for the arrays; nn_warm_start
 * leaves a continuable state when it keeps its prediction); otherwise, or after
 * a call that ended in any status but MG_OK or MG_ERR_NOT_CONVERGED, returns
 * MG_ERR_INVALID.  Iteration counts and norms as mg_solve_constraints (the
 * resumed state counts as iteration 0).  A runtime addition, not in the paper.
 */
mg_status mg_solve_constraints_continue(mg_ctx *ctx, double *d_u, double *d_W, double tol,
                                        int32_t max_outer, mg_report *rep);

/* Constraint norms (Key features, "Diagnostics": the Hamiltonian and momentum
 * constraint errors of eqs. Ham and Mom reduced to norms over the grid) at
 * (d_u, d_W): out[4] (host) = rms H_h, rms |M_h|, max |H_h|, max |M_h| (the
 * momentum entries are 0 when d_S was NULL).  Synchronises. */
mg_status mg_residual_norm(mg_ctx *ctx, const double *d_u, const double *d_W, double out[4]);

/* The residual fields themselves: d_H (n^3), d_M (3 n^3), d_c (n^3, dH_h/dpsi),
 * FP64; any may be NULL.  Enqueued only. */
mg_status mg_residual_fields(mg_ctx *ctx, const double *d_u, const double *d_W, double *d_H,
                             double *d_M, double *d_c);

/*
 * Background fields of a psi-only context (solve_momentum = 0), borrowed, FP64 on
 * the finest grid (n^3 each, either may be NULL to clear it):
 *  d_psi0  replaces psi0 = 1 + M/(2r) in psi = psi0 + u (several punctures;
 *          puncture_mass must then be 0; puncture_pos stays the centre of the
 *          Robin rule);
 *  d_A2    Abar_ij Abar_ij of an analytic traceless extrinsic curvature, added to
 *          the A2 of W in H_h and in c (cross terms with W are not formed, so W is
 *          meant to be zero: the Bowen-York data below solve the momentum
 *          constraint themselves).
 * Key features, "Flexibility": binary black holes with boosted and/or spinning
 * punctures.  MG_ERR_INVALID for a momentum or batch context, or with
 * puncture_mass != 0 and d_psi0 given.  Takes effect for the next call.
 */
mg_status mg_set_background(mg_ctx *ctx, const double *d_psi0, const double *d_A2);

/*
 * Bowen-York puncture data (Key features, "Flexibility"; the momentum constraint,
 * Summary eq. Mom, with K = 0 and no matter, solved analytically): h_table holds
 * 10 doubles per puncture (mass m, centre C[3], momentum P[3], spin S[3]; up to 8
 * punctures, all finite).  With n = (x - C)/r and r = |x - C| the traceless
 * extrinsic curvature is the sum over punctures of
 *   (3/(2 r^2)) [P_i n_j + P_j n_i - (delta_ij - n_i n_j) P.n]
 *   + (3/r^3) [(S x n)_i n_j + (S x n)_j n_i];
 * writes d_psi0 = 1 + sum m/(2r) and d_A2 = Abar_ij Abar_ij at the cell centres of
 * the grid of p (n, length, origin), FP64 n^3 each.  Enqueued only.
 */
mg_status mg_bowen_york_sources(const mg_params *p, int32_t count, const double *h_table, double *d_psi0,
                                double *d_A2, void *stream);

/*
 * CTTK trace (Key features, "Methods"; a context set up with MG_FLAG_CTTK): writes
 * d_K (n^3 FP64) = K of the state (d_u, d_W) from eq. Ham, K^2 = 12 H0 / psi^5, the
 * trace a solve of that state used.  MG_ERR_INVALID for other contexts.  Enqueued
 * only.
 */
mg_status mg_cttk_trace(mg_ctx *ctx, const double *d_u, const double *d_W, double *d_K);

/*
 * CTTK-Hybrid sources (Key features, "Methods"; read from eqs. Ham and Mom with a
 * spatially varying K): the psi-independent energy density rho5 is carried by a
 * local trace, the gradient energy by psi as in CTT with a constant trace K0:
 *   K^2(x) = 24 pi (rho5(x) + <rho1>),  K0^2 = 24 pi <rho1>.
 * Transforms the CTT sources in place into those of an ordinary mg_setup context
 * with trace K0 (p->K = *h_K0): d_rho5 -> 0 and d_S -> d_S + D K / (12 pi) (the
 * -(2/3) psi^6 d_a K of eq. Mom; D the fourth-order first derivative), and writes
 * d_K = K(x) (all FP64 n^3, d_S 3 n^3).  Periodic grids only (p: n 4..4096,
 * length, origin).  d_scratch: caller-owned device scratch, 256-byte aligned, of at
 * least MG_SOURCES_SCRATCH_BYTES for the mean of rho1 (MG_ERR_WORKSPACE otherwise).
 * If h_K0 is not NULL, K0 is returned there and the call synchronises the stream.
 * The solution (u, W) with K(x) then satisfies eqs. Ham and Mom as written.
 */
mg_status mg_cttk_hybrid_sources(const mg_params *p, double *d_rho5, const double *d_rho1, double *d_S,
                                 double *d_K, void *d_scratch, size_t scratch_bytes, double *h_K0, void *stream);

/*
 * Two-level static mesh refinement of eq. Ham (Key features, "Adaptive Mesh
 * Refinement": a block-structured hierarchy of refined boxes, here one static box;
 * "Fast": multigrid over the hierarchy).  The composite grid is the base context
 * cb's grid (n_c^3 cells of spacing h) and the box context cx's grid: 2m cells per
 * axis of spacing h/2 covering the m^3 base cells from base cell (b0, b0, b0) on,
 * set up with boundary rule MG_BC_ZERO, length m h and origin = base origin + b0 h
 * (same K, puncture, conformal-matter flag; both psi-only, not CTTK, not in a
 * batch, no background fields; margin b0 >= 3 and b0 + m + 3 <= n_c).  Both
 * contexts must have been set up with a forcing array d_f, which this call
 * overwrites, and with the same caller stream.
 * Composite equations: H_h of the box with its two ghost layers taken from the base
 * grid by the cubic of mg_interp_cubic (the box solves them under the zero rule with
 * the ghost taps as its forcing), H_h of the base cells the box does not cover, and
 * base values under the box equal to the average of their 8 children.
 * Iteration (a two-level FAS cycle, Brandt's multi-level adaptive technique): base
 * cells under the box take their children's average; nu_box Newton-multigrid steps
 * of the box; the base forcing tau = R H_f - H_c(R u_f) on covered cells (0
 * elsewhere); nu_base steps of the base grid; the box adds the cubic interpolation
 * of the base grid's change.  Stops when the composite norm
 * sqrt((sum_box H^2 (h/2)^3 + sum_uncovered H^2 h^3) / L^3) <= tol, or after
 * max_outer iterations.  d_uc (n_c^3) and d_uf ((2m)^3) hold the initial guess and
 * the result (u of psi = psi0 + u on each grid; on return the base cells under the
 * box hold their children's average).  d_work: caller-owned device workspace,
 * 256-byte aligned, of mg_refine_workspace_size bytes.  rep (may be NULL): iterations,
 * status, h_rms / h_max = composite rms and max |H| (m_* = 0), history of
 * (rms, 0, max, 0).  Synchronises once per iteration.  Returns MG_OK,
 * MG_ERR_NOT_CONVERGED, MG_ERR_DIVERGED, MG_ERR_INVALID or MG_ERR_WORKSPACE.
 */
mg_status mg_refine_workspace_size(const mg_params *base, const mg_params *box, int32_t b0, size_t *bytes);
mg_status mg_refine_solve(mg_ctx *cb, mg_ctx *cx, int32_t b0, double *d_uc, double *d_uf, void *d_work,
                          size_t work_bytes, double tol, int32_t max_outer, int32_t nu_box, int32_t nu_base,
                          mg_report *rep);

/*
 * Nested boxes (the same reading, 2..8 levels): ctx[0] is the base context, ctx[k]
 * (k >= 1) a box over m_k^3 cells of ctx[k-1] from its cell (b0[k], b0[k], b0[k]) on
 * (b0[0] unused), each with the requirements mg_refine_solve states for a box and its
 * base (zero rule, margin of 3 parent cells, matching spacing, origin and physics,
 * forcing arrays that are overwritten, one caller stream); d_u[k] holds u of level k.
 * A cell under a finer box holds the average of its children; every box's ghosts come
 * from its parent.  One iteration: from the finest level down to level 1, nu_box steps
 * of the level (interface-ghost forcing formed before each, plus the FAS forcing it
 * received from the box inside it), then the FAS forcing of its parent,
 * tau = R (H of the level, its own FAS forcing included) - H_parent(R u) on the cells
 * under it; nu_base steps of the base grid; from level 1 up, every box adds the cubic
 * interpolation of its parent's change.  The composite norm sums every level over the
 * cells no finer box covers.  Two levels give mg_refine_solve.  Workspace:
 * mg_refine_nested_workspace_size (p[k]: the levels' parameters).
 */
mg_status mg_refine_nested_workspace_size(int32_t levels, const mg_params *const *p, const int32_t *b0,
                                          size_t *bytes);
mg_status mg_refine_solve_nested(int32_t levels, mg_ctx *const *ctx, const int32_t *b0, double *const *d_u,
                                 void *d_work, size_t work_bytes, double tol, int32_t max_outer, int32_t nu_box,
                                 int32_t nu_base, mg_report *rep);

void mg_destroy(mg_ctx *ctx);
const char *mg_status_str(mg_status s);

/*
 * Matter sources of a scalar field given as Fourier modes (Summary: rho and
 * S_i as the projections of the stress-energy onto the slice normal; Key
 * features: scalar-field matter with analytic initial data).
 * h_phi_modes, h_pi_modes: host tables of 5 doubles per mode (kx, ky, kz,
 * amplitude, phase); field = sum amp cos(2 pi k.x / L + phase); up to 32 modes
 * each, every entry finite.  V(phi) = mass^2 phi^2 / 2.  Writes d_rho5 =
 * Pi^2/2 + V, d_rho1 = |d phi|^2/2, d_S = -Pi d phi (3 n^3), all FP64.
 * If h_mean_rho is not NULL the grid mean <rho> of rho5 + rho1 is returned
 * there; if h_K is not NULL, the constant trace K = sqrt(24 pi <rho>), for which
 * the uniform part of the Hamiltonian constraint (eq. Ham with psi = 1,
 * Abar = 0: (2/3) K^2 = 16 pi <rho>) vanishes.  Either output synchronises the
 * stream and needs a caller-owned device scratch d_scratch, 256-byte aligned,
 * of at least MG_SOURCES_SCRATCH_BYTES (otherwise d_scratch may be NULL).
 * Uses p->n (1..4096), p->length and p->origin only.  MG_ERR_INVALID before
 * any HIP call on bad arguments, MG_ERR_WORKSPACE on a missing or small scratch.
 */
#define MG_SOURCES_SCRATCH_BYTES 32768
mg_status mg_scalar_field_sources(const mg_params *p, int32_t n_phi, const double *h_phi_modes,
                                  int32_t n_pi, const double *h_pi_modes, double mass,
                                  double *d_rho5, double *d_rho1, double *d_S,
                                  void *d_scratch, size_t scratch_bytes, double *h_mean_rho,
                                  double *h_K, void *stream);

/*
 * Allocation-free variant of mg_scalar_field_sources, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and the same results,
 * bit for bit, with the reduction scratch taken from a device array inside the
 * library instead of a d_scratch argument.  That array holds
 * MG_SOURCES_STATIC_SCRATCH_BYTES on every GPU the library runs on (its address
 * is looked up once per device, on the first call that wants the mean or K,
 * and the array lives until the process ends); the reduction needs 2049
 * doubles whatever n, so every accepted n (1..4096) fits, and a call whose need
 * exceeded the array would return MG_ERR_WORKSPACE before any launch.  The
 * call itself makes no hipMalloc, hipFree or other allocating call.  All calls
 * on one GPU share the array: calls that overlap in time on one GPU (from
 * several host threads or on several streams) race and must be serialised by
 * the caller.  Nothing in the array needs clearing: every call writes each
 * value it reads.  Arguments, outputs and errors as mg_scalar_field_sources;
 * the device is the stream's (the current device for a NULL stream).
 */
#define MG_SOURCES_STATIC_SCRATCH_BYTES 32768
mg_status mg_scalar_field_sources_static(const mg_params *p, int32_t n_phi, const double *h_phi_modes,
                                         int32_t n_pi, const double *h_pi_modes, double mass,
                                         double *d_rho5, double *d_rho1, double *d_S,
                                         double *h_mean_rho, double *h_K, void *stream);

/*
 * Scalar shell around the puncture: phi = amp exp(-(r - r0)^2 / width2) Y_11
 * with the real dipole harmonic Y_11 = sqrt(3/(4 pi)) x/r about puncture_pos,
 * Pi = 0.  Writes d_rho5 = mass^2 phi^2/2, d_rho1 = |d phi|^2/2, d_S = 0.
 */
mg_status mg_shell_field_sources(const mg_params *p, double amp, double r0, double width2,
                                 double mass, double *d_rho5, double *d_rho1, double *d_S,
                                 void *stream);

/*
 * Fourth-order (four-point cubic Lagrange, weights (-5, 35, 105, -7)/128 and
 * mirror) interpolation of an FP64 field from the coarse grid described by
 * *pc (n = coarse cells) to the grid with 2n cells per axis: d_fine = Q d_coarse.
 * Used to start a fine solve from a coarse one.
 */
mg_status mg_interp_cubic(const mg_params *pc, const double *d_coarse, double *d_fine,
                          void *stream);

/*
 * Full-multigrid start of a fine solve from the coarse problem: solves the
 * coarse context cc (grid n/2 of the same box and boundary rule, sources
 * evaluated on that grid) from (d_uc, d_Wc) to tol_c with mg_solve_constraints
 * (rep_c may be NULL), then interpolates u and, when both W arrays are given,
 * every W component to the fine grid of cf with the cubic of mg_interp_cubic
 * (d_uf: (2n)^3, d_Wf: 3 (2n)^3).  The fine arrays are written also when the
 * coarse solve stops at max_outer (status MG_ERR_NOT_CONVERGED); other
 * failures leave them untouched.  Both contexts must use the same stream.
 */
mg_status mg_fmg_start(mg_ctx *cc, mg_ctx *cf, double *d_uc, double *d_Wc, double tol_c,
                       int32_t max_outer, double *d_uf, double *d_Wf, mg_report *rep_c);

/*
 * Autotuning of the tiled kernels' brick depth (the x extent of the LDS brick
 * of the finest-level smoothers and residual; other levels are not tiled).
 * For every tileable (family, level) of the context, mg_autotune times each
 * candidate depth with HIP events around `reps` launches on the context's own
 * data (the residuals of the state (d_u, d_W), zero corrections; the state is
 * not changed), keeps the fastest in the context and drops the captured
 * outer-iteration graph.  The candidates compute every cell with the same
 * arithmetic, so the solution does not depend on the choice.  h_out (cap
 * entries, may be NULL with cap 0) receives one mg_tune per tuned (family,
 * level); *h_count (may be NULL) the number of entries.  Waits for the
 * stream.  mg_set_tile applies a stored choice (a candidate of the family;
 * MG_ERR_INVALID otherwise).  Candidates: psi pass {2, 4, 8}; W pass {2, 4, 8,
 * 16} (FP32) or {1, 2, 8} (FP64), where depths up to 4 stage a whole brick and
 * 8 and 16 march a column of that many x planes through a ring of staged
 * planes; residual {2, 4, 8, 16}, where 2 and 4 stage bricks and 8 and 16
 * (periodic only) march columns of that many x planes.
 * Two further families choose how the coarse levels of each V-cycle run: as
 * separate grid launches (0, the default) or as one workgroup-resident "tail"
 * kernel per V-cycle (1) that runs every level from its first one down to the
 * coarsest and back, phase by phase with block barriers, on arrays held in
 * LDS (same per-cell arithmetic; the restriction sums group the 8 children
 * differently, so results agree to rounding).  The tail starts at the first
 * level from which the cells of all levels down to the coarsest sum to at
 * most 4680 (psi, FP32, periodic) or 1971 (psi otherwise; W), spanning at
 * most 4 levels (e.g. 16^3 for psi and 8^3 for W, FP32 periodic), or from any
 * level below it down to the one above the coarsest.  Their `level` is the tail's
 * first level: mg_autotune times one whole V-cycle with the tail off and starting
 * at each such level and reports the fastest start (chosen 1) or the fastest
 * start tried (chosen 0, the tail off); mg_set_tile(family, level, 1) starts the
 * tail at `level`, (family, level, 0) turns it off.
 * MG_TUNE_FOURIER_W (FP32 periodic contexts with momentum whose levels include a
 * 16^3 one below the finest; `level` is that level): the W V-cycle solves that
 * level exactly by discrete Fourier modes in one workgroup (1, the default) or
 * runs it and the levels below as multigrid (0).  The exact solve changes the
 * V-cycle (it is an exact coarse correction), not the equations: solutions agree
 * to the solve tolerance.
 */
enum {
    MG_TUNE_PASS_PSI = 1,
    MG_TUNE_PASS_W = 2,
    MG_TUNE_RESIDUAL = 3,
    MG_TUNE_TAIL_PSI = 4,
    MG_TUNE_TAIL_W = 5,
    MG_TUNE_FOURIER_W = 6
};
typedef struct mg_tune {
    int32_t family, level, chosen, ncand;
    int32_t cand[4];
    double us[4]; /* mean microseconds per launch, -1 if the candidate does not fit */
} mg_tune;
mg_status mg_autotune(mg_ctx *ctx, const double *d_u, const double *d_W, int32_t reps, mg_tune *h_out,
                      int32_t cap, int32_t *h_count);
mg_status mg_set_tile(mg_ctx *ctx, int32_t family, int32_t level, int32_t tx);

/*
 * Single-kernel entry points on one level of a context, for diagnostics and
 * kernel-level parity checks.  Arrays are in the context's V-cycle type
 * (double for MG_PREC_FP64, float for MG_PREC_FP32_IR), on level `level`
 * (n_l = n >> level cells per axis).
 *  MG_OP_PASS_PSI   out = colour pass (colour = arg) of (L_h + c) d = r, in = d
 *  MG_OP_PASS_W     out = colour pass of Delta_L,h d = r (3 components)
 *  MG_OP_DEFECT_RESTRICT_PSI  out (coarse) = average of 8 children of r - (L_h + c) in
 *  MG_OP_DEFECT_RESTRICT_W    the same for Delta_L,h (3 components)
 *  MG_OP_PROLONG_ADD out (level l) += trilinear interpolation of in (level l+1),
 *                   arg = number of components
 *  MG_OP_COARSE_PSI out = (L_h + c)^-1 r on the coarsest level (r = in)
 *  MG_OP_COARSE_W   out = mean-free Delta_L,h^-1 (r - mean r) on the coarsest level
 *  MG_OP_FOURIER_W  out = mean-free Delta_L,h^-1 (r - mean r) on a 16^3 level of an FP32
 *                   periodic context, by discrete Fourier modes (r = in; in and out
 *                   16-byte aligned): the exact bottom of the W V-cycle
 * Unused pointers may be NULL.  Enqueued only.
 */
enum {
    MG_OP_PASS_PSI = 1,
    MG_OP_PASS_W = 2,
    MG_OP_DEFECT_RESTRICT_PSI = 3,
    MG_OP_DEFECT_RESTRICT_W = 4,
    MG_OP_PROLONG_ADD = 5,
    MG_OP_COARSE_PSI = 6,
    MG_OP_COARSE_W = 7,
    MG_OP_FOURIER_W = 8
};
mg_status mg_kernel_op(mg_ctx *ctx, int32_t op, int32_t level, int32_t arg, const void *d_in,
                       void *d_out, const void *d_r, const void *d_c);

/*
 * Batches of independent instances (a parameter scan of uneven grid sizes; Key
 * features: parameter studies of cosmological spacetimes).  Members whose
 * parameters agree in everything but K form a group (a size class of the scan).
 * All members are carved from one caller-owned workspace: every member owns a
 * region holding its context workspace and its own copies of the sources and of
 * the state (u, W), and the regions of a group are equally spaced, so that one
 * kernel launch covers the whole group (the member index is the block index
 * along z; every array address moves by the region stride).  A member that has
 * converged (or diverged) keeps its state: its update kernels are gated by a
 * device-side flag set by a check kernel after each evaluation.
 *  p: host array of count parameter sets (same precision for all; momentum
 *     members need periodic boundaries as for mg_setup).
 *  d_rho5, d_rho1, d_S: host arrays of count device pointers (n_i^3, n_i^3,
 *     3 n_i^3 FP64); d_S may be NULL when no member solves the momentum
 *     equation.  The sources are copied into the workspace at set-up.
 *  mg_solve_batch: d_u, d_W host arrays of device pointers (d_W may be NULL
 *     when no member solves the momentum equation; W given or not must agree
 *     within a group); the states are copied in before and out after the solve.
 *     reps (may be NULL) gets count reports (no per-iteration history).  Returns
 *     MG_OK when every member converged, else the first non-OK member status.
 *     Synchronises once per outer iteration (one copy of every member's norms).
 *  mg_batch_groups: the number of groups and (h_group_of, count entries, may be
 *     NULL) each member's group.
 */
typedef struct mg_batch mg_batch;
enum { MG_BATCH_AUTO = 0, MG_BATCH_GRAPH = 1, MG_BATCH_LANES = 2, MG_BATCH_GROUPS = 3 };
mg_status mg_batch_workspace_size(const mg_params *p, int32_t count, size_t *bytes);
mg_status mg_setup_batch(const mg_params *p, int32_t count, void *d_workspace, size_t bytes, void *stream,
                         const double *const *d_rho5, const double *const *d_rho1,
                         const double *const *d_S, mg_batch **out);
mg_status mg_solve_batch(mg_batch *b, double *const *d_u, double *const *d_W, double tol, int32_t max_outer,
                         mg_report *reps);
void mg_destroy_batch(mg_batch *b);
mg_status mg_batch_groups(mg_batch *b, int32_t *h_ngroups, int32_t *h_group_of);

/*
 * Launch mode of a batch's outer iterations (the autotuned choice of the
 * batched execution).  MG_BATCH_GROUPS: every group with an active member runs
 * its captured outer iteration, one launch per kernel for the whole group (its
 * converged members with their updates gated off), the groups concurrently on
 * four streams.  MG_BATCH_GRAPH: one batch graph of every member's own outer
 * iteration.  MG_BATCH_LANES: every still-active member's own graph, spread
 * over four streams.  MG_BATCH_AUTO (the default): the first solve times one
 * outer iteration in each mode (wall clock, launch to completion) and keeps the
 * fastest; every mode runs the same kernels on the same arrays, so results are
 * identical in every mode.  request = -1 only queries.  *chosen (may be NULL):
 * the mode in use (MG_BATCH_AUTO until tuned); h_ms (may be NULL): the tuning
 * times in ms (graph, lanes, groups; -1 if not measured).
 */
mg_status mg_batch_launch_mode(mg_batch *b, int32_t request, int32_t *chosen, double h_ms[3]);

/*
 * Kernel timing probe (measurement support).  mg_probe(ctx, kernel, level)
 * starts recording a HIP event pair around every later launch of one kernel
 * family on one level (kernel = MG_PROBE_*, level = multigrid level, or -1
 * for all levels); kernel = MG_PROBE_NONE stops recording.  Up to 4096
 * launches are recorded; later ones are not.  mg_probe_result synchronises
 * the stream and returns the number of recorded launches and the summed
 * event-to-event time in milliseconds, then clears the record.  Events are
 * created on the first mg_probe call and released by mg_destroy.
 */
enum {
    MG_PROBE_NONE = 0,
    MG_PROBE_PASS_PSI = 1,
    MG_PROBE_PASS_W = 2,
    MG_PROBE_RESIDUAL = 3,
    MG_PROBE_DEFECT_RESTRICT_PSI = 4,
    MG_PROBE_DEFECT_RESTRICT_W = 5,
    MG_PROBE_PROLONG = 6,
    MG_PROBE_COARSE = 7,
    MG_PROBE_UPDATE = 8
};
mg_status mg_probe(mg_ctx *ctx, int32_t kernel, int32_t level);
mg_status mg_probe_result(mg_ctx *ctx, int32_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* GRTMG_H */
