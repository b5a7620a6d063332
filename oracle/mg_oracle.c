/*
 * mg_oracle.c -- CPU FP64 oracle for the multigrid solve of the initial-data
 * constraints (Hamiltonian constraint eq. (Ham) and momentum constraint
 * eq. (Mom) of the paper's Summary, in conformal transverse-traceless form).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or helper with the GPU library; it is a plain, slow, loop-per-operation
 * restatement of the discrete system and of the multigrid algorithm.
 *
 * Continuum problem (Summary, eqs. Ham and Mom; CTT reading of the methods the
 * paper names in its Summary): conformally flat metric gamma_ij = psi^4 delta_ij,
 * constant trace K, traceless extrinsic curvature A_ij = psi^-2 Abar_ij with
 * Abar_ij = d_i W_j + d_j W_i - (2/3) delta_ij d_k W_k.  Then, in conformal form,
 *
 *   H   = lap psi + 2 pi rho5 psi^5 + 2 pi rho1 psi - (K^2/12) psi^5
 *         + (1/8) Abar_ab Abar_ab psi^-7                          = 0
 *   M_a = lap W_a + (1/3) d_a d_b W_b - 8 pi psi^6 S_a               = 0
 *
 * where the scalar-field energy density rho = rho5 + psi^-4 rho1 (rho5 =
 * Pi^2/2 + V(phi), rho1 = |d phi|^2 / 2) and S_a = -Pi d_a phi are the matter
 * projections of the Summary.
 *
 * Discrete system (cell-centred N^3 grid, h = L/N, index (i*N + j)*N + k):
 *   D_a  f = [f(-2) - 8 f(-1) + 8 f(+1) - f(+2)] / (12 h)
 *   D_aa f = [-f(-2) + 16 f(-1) - 30 f(0) + 16 f(+1) - f(+2)] / (12 h^2)
 *   D_ab   = D_a D_b (a != b)
 *   psi = psi0 + u,  psi0 = 1 + M/(2 r) (puncture) or 1
 *   H_h = L_h u + 2 pi rho5 psi^5 + 2 pi rho1 psi - (K^2/12) psi^5 + A2 psi^-7 / 8 + f
 *   c   = dH_h/dpsi = 10 pi rho5 psi^4 + 2 pi rho1 - (5 K^2/12) psi^4 - (7/8) A2 psi^-8
 *   M_h = Delta_L,h W - (8 pi psi^6 S - mean(8 pi psi^6 S))   (periodic: mean removed)
 * The analytic Laplacian of psi0 = 1 + M/(2r) vanishes away from the puncture
 * and is not added.
 *
 * Conformally rescaled matter (flags bit 0; the textbook CTT choice of free
 * data rho_bar = psi^8 rho, S_bar_a = psi^6 S_a, which keeps dH/dpsi negative):
 * with rho_bar = rho5 + rho1,
 *   H_h = L_h u + 2 pi rho_bar psi^-3 - (K^2/12) psi^5 + A2 psi^-7 / 8 + f
 *   c   = -6 pi rho_bar psi^-4 - (5 K^2/12) psi^4 - (7/8) A2 psi^-8
 *   M_h = Delta_L,h W - (8 pi S - mean(8 pi S))
 *
 * Methods with a spatially varying K (Key features, "Methods": CTTK and
 * CTTK-Hybrid): the readings and their shifted sources are stated with
 * orc_cttk_hybrid_sources / orc_cttk_update below.
 *
 * Boundary conditions (Key features, "Boundary conditions": extrapolating,
 * reflective and periodic; the 1/r Robin rule serves the isolated black hole):
 * periodic wrap; Robin: a ghost value a(g) = a(b) |x_b| / |x_g| with b the grid
 * cell nearest to g (coordinates clamped into the grid), radii measured from
 * the puncture position; reflective: the mirror image of the grid across the
 * boundary face (even parity); extrapolating: zeroth-order extrapolation along
 * the face normal (each ghost takes the value of the grid cell next to the face);
 * zero: homogeneous ghosts (every ghost is 0), the rule of a refined box whose
 * interface ghosts enter as a forcing (see oracle/refine.py).
 *
 * Multigrid (Key features, "Fast": errors reduced across a hierarchy of
 * discretisations): V(nu_pre, nu_post) cycles with double-buffered red-black
 * Gauss-Seidel (colour (i+j+k) mod 2, red first; every value read by a colour
 * pass is the value before that pass), defect restriction by the average of
 * the 8 children, rediscretised coarse operators, exact dense LU with partial
 * pivoting on the coarsest level, trilinear cell-centred prolongation (or, with
 * flags bit 1, the 4-point cubic of the FMG start for the corrections too).  The
 * outer loop is a segregated inexact Newton iteration: W cycle, W update,
 * re-linearise, psi cycle, psi update; the constraint norms are recorded at
 * every iteration (Key features, "Diagnostics").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OBC_PERIODIC 0
#define OBC_ROBIN 1
#define OBC_REFLECT 2
#define OBC_EXTRAP 3
#define OBC_ZERO 4
#define OMAXLEV 16

/* flags bit 0: conformally rescaled matter (see orc_residuals); bit 1: corrections
 * prolonged by the 4-point cubic of orc_interp_cubic instead of trilinearly; bit 2:
 * the W and psi steps of an outer iteration both linearise at the state the
 * iteration starts from (the psi step reads W from before the W update) instead of
 * the psi step following the W update.  The paper does not say how the two
 * equations are coupled between multigrid solves; either order has the discrete
 * solution as its fixed point. */
#define OFLAG_CONFORMAL_MATTER 1
#define OFLAG_CUBIC_PROLONG 2
#define OFLAG_SAME_STATE 4

typedef struct {
    int32_t n, levels, bc, nu_pre, nu_post, solve_momentum, flags, mix_depth;
    double length, origin[3], K, puncture_mass, puncture_pos[3];
    /* optional fields on the finest grid (NULL: not used): psi0 replacing
     * 1 + M/(2r) (several punctures), and Abar_ij Abar_ij of an analytic
     * traceless extrinsic curvature added to the one of W (Bowen-York data,
     * with W = 0) */
    const double *bg_psi0, *bg_A2;
} orc_params;

typedef struct {
    int n, bc;
    double h, org[3], ctr[3];
} geom;

static const double W1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};     /* / (12 h)   */
static const double W2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0}; /* / (12 h^2) */

static long idx3(int n, int i, int j, int k) { return ((long)i * n + j) * n + k; }
static long cells(int n) { return (long)n * n * n; }

static int wrapi(int i, int n)
{
    i %= n;
    if (i < 0) i += n;
    return i;
}

static int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

static geom make_geom(const orc_params *p, int n)
{
    geom g;
    g.n = n;
    g.bc = p->bc;
    g.h = p->length / n;
    for (int a = 0; a < 3; a++) {
        g.org[a] = p->origin[a];
        g.ctr[a] = p->puncture_pos[a];
    }
    return g;
}

static void cell_pos(const geom *g, int i, int j, int k, double x[3])
{
    x[0] = g->org[0] + (i + 0.5) * g->h - g->ctr[0];
    x[1] = g->org[1] + (j + 0.5) * g->h - g->ctr[1];
    x[2] = g->org[2] + (k + 0.5) * g->h - g->ctr[2];
}

static double cell_radius(const geom *g, int i, int j, int k)
{
    double x[3];
    cell_pos(g, i, j, k, x);
    return sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
}

static int inside(int n, int i, int j, int k)
{
    return i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n;
}

/* Reflective and extrapolating rules, one axis at a time: the value at index i
 * (possibly outside 0..n-1) as a grid value idx[0] with weight w[0]; returns
 * the number of terms (kept general for rules that combine several cells).
 *   reflective:    the mirror image across the boundary face (-1 -> 0, -2 -> 1,
 *                  n -> n-1, n+1 -> n-2), weight 1 (even parity);
 *   extrapolating: zeroth-order extrapolation along the face normal, every
 *                  ghost layer taking the value of the grid cell next to the
 *                  face (-1, -2 -> 0; n, n+1 -> n-1).
 * A cell outside along several axes applies the rule of each axis in turn. */
static int axis_terms(int bc, int n, int i, int idx[2], double w[2])
{
    if (i >= 0 && i < n) {
        idx[0] = i;
    } else if (bc == OBC_REFLECT) {
        idx[0] = i < 0 ? -1 - i : 2 * n - 1 - i;
    } else {
        idx[0] = i < 0 ? 0 : n - 1;
    }
    w[0] = 1.0;
    return 1;
}

/* Field value at cell (i,j,k), which may lie outside the grid (boundary rule). */
static double at(const geom *g, const double *a, int i, int j, int k)
{
    int n = g->n;
    if (g->bc == OBC_PERIODIC)
        return a[idx3(n, wrapi(i, n), wrapi(j, n), wrapi(k, n))];
    if (inside(n, i, j, k)) return a[idx3(n, i, j, k)];
    if (g->bc == OBC_ZERO) return 0.0; /* homogeneous ghosts (the interface of a refined box) */
    if (g->bc == OBC_REFLECT || g->bc == OBC_EXTRAP) {
        int I[2], J[2], K[2];
        double wi[2], wj[2], wk[2], s = 0.0;
        int ni = axis_terms(g->bc, n, i, I, wi), nj = axis_terms(g->bc, n, j, J, wj),
            nk = axis_terms(g->bc, n, k, K, wk);
        for (int x = 0; x < ni; x++)
            for (int y = 0; y < nj; y++)
                for (int z = 0; z < nk; z++) s += wi[x] * wj[y] * wk[z] * a[idx3(n, I[x], J[y], K[z])];
        return s;
    }
    int bi = clampi(i, n), bj = clampi(j, n), bk = clampi(k, n);
    return a[idx3(n, bi, bj, bk)] * cell_radius(g, bi, bj, bk) / cell_radius(g, i, j, k);
}

/* Weight with which the value fetched at (i+di, j+dj, k+dk) depends on the
 * value stored at (i,j,k) itself. */
static double self_weight(const geom *g, int i, int j, int k, int di, int dj, int dk)
{
    int n = g->n, ii = i + di, jj = j + dj, kk = k + dk;
    if (g->bc == OBC_PERIODIC)
        return (wrapi(ii, n) == i && wrapi(jj, n) == j && wrapi(kk, n) == k) ? 1.0 : 0.0;
    if (inside(n, ii, jj, kk)) return (di == 0 && dj == 0 && dk == 0) ? 1.0 : 0.0;
    if (g->bc == OBC_ZERO) return 0.0;
    if (g->bc == OBC_REFLECT || g->bc == OBC_EXTRAP) {
        int I[2], J[2], K[2];
        double wi[2], wj[2], wk[2], s = 0.0;
        int ni = axis_terms(g->bc, n, ii, I, wi), nj = axis_terms(g->bc, n, jj, J, wj),
            nk = axis_terms(g->bc, n, kk, K, wk);
        for (int x = 0; x < ni; x++)
            for (int y = 0; y < nj; y++)
                for (int z = 0; z < nk; z++)
                    if (I[x] == i && J[y] == j && K[z] == k) s += wi[x] * wj[y] * wk[z];
        return s;
    }
    int bi = clampi(ii, n), bj = clampi(jj, n), bk = clampi(kk, n);
    if (bi != i || bj != j || bk != k) return 0.0;
    return cell_radius(g, bi, bj, bk) / cell_radius(g, ii, jj, kk);
}

static void unit(int axis, int d, int o[3])
{
    o[0] = o[1] = o[2] = 0;
    o[axis] = d;
}

/* ---- stencils ------------------------------------------------------------ */

static double D1(const geom *g, const double *a, int i, int j, int k, int axis)
{
    double s = 0.0;
    for (int d = -2; d <= 2; d++) {
        int o[3];
        unit(axis, d, o);
        s += W1[d + 2] * at(g, a, i + o[0], j + o[1], k + o[2]);
    }
    return s / (12.0 * g->h);
}

static double D2(const geom *g, const double *a, int i, int j, int k, int axis)
{
    double s = 0.0;
    for (int d = -2; d <= 2; d++) {
        int o[3];
        unit(axis, d, o);
        s += W2[d + 2] * at(g, a, i + o[0], j + o[1], k + o[2]);
    }
    return s / (12.0 * g->h * g->h);
}

/* D_p D_q with p != q: product of two first-derivative stencils. */
static double Dmix(const geom *g, const double *a, int i, int j, int k, int p, int q)
{
    double s = 0.0;
    for (int d = -2; d <= 2; d++)
        for (int e = -2; e <= 2; e++) {
            int o[3] = {0, 0, 0};
            o[p] += d;
            o[q] += e;
            s += W1[d + 2] * W1[e + 2] * at(g, a, i + o[0], j + o[1], k + o[2]);
        }
    return s / (144.0 * g->h * g->h);
}

static double lap(const geom *g, const double *a, int i, int j, int k)
{
    return D2(g, a, i, j, k, 0) + D2(g, a, i, j, k, 1) + D2(g, a, i, j, k, 2);
}

/* (Delta_L W)_a = sum_b D_bb W_a + (1/3) [D_aa W_a + sum_{b != a} D_ab W_b] */
static double deltaL(const geom *g, const double *W, int i, int j, int k, int a)
{
    long m = cells(g->n);
    const double *Wa = W + a * m;
    double s = lap(g, Wa, i, j, k);
    double t = D2(g, Wa, i, j, k, a);
    for (int b = 0; b < 3; b++)
        if (b != a) t += Dmix(g, W + b * m, i, j, k, a, b);
    return s + t / 3.0;
}

/* Diagonal entry of the discrete Laplacian at (i,j,k), boundary rule included. */
static double lap_diag(const geom *g, int i, int j, int k)
{
    double s = 0.0;
    for (int axis = 0; axis < 3; axis++)
        for (int d = -2; d <= 2; d++) {
            int o[3];
            unit(axis, d, o);
            s += W2[d + 2] * self_weight(g, i, j, k, o[0], o[1], o[2]);
        }
    return s / (12.0 * g->h * g->h);
}

/* Diagonal entry of component a of Delta_L,h (periodic grids). */
static double deltaL_diag(const geom *g, int i, int j, int k, int a)
{
    double s = lap_diag(g, i, j, k);
    double t = 0.0;
    for (int d = -2; d <= 2; d++) {
        int o[3];
        unit(a, d, o);
        t += W2[d + 2] * self_weight(g, i, j, k, o[0], o[1], o[2]);
    }
    t /= 12.0 * g->h * g->h;
    /* the mixed taps D_ab W_b act on other components: no diagonal part */
    return s + t / 3.0;
}

static double psi0_at(const orc_params *p, const geom *g, int i, int j, int k)
{
    if (p->bg_psi0) return p->bg_psi0[idx3(g->n, i, j, k)];
    if (p->puncture_mass > 0.0) return 1.0 + p->puncture_mass / (2.0 * cell_radius(g, i, j, k));
    return 1.0;
}

/* ---- residuals ----------------------------------------------------------- */

/* Abar_ab Abar_ab from the first derivatives dW[a][b] = D_a W_b. */
static double a2_from_grad(double dW[3][3])
{
    double div = dW[0][0] + dW[1][1] + dW[2][2];
    double s = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double A = dW[a][b] + dW[b][a] - (a == b ? 2.0 * div / 3.0 : 0.0);
            s += A * A;
        }
    return s;
}

static double A2_at(const geom *g, const double *W, int i, int j, int k)
{
    long m = cells(g->n);
    double dW[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) dW[a][b] = D1(g, W + b * m, i, j, k, a);
    return a2_from_grad(dW);
}

/*
 * Hamiltonian residual H_h, Newton coefficient c, and mean-free momentum
 * residual M_h (3 components, SoA) at the state (u, W).  Any output may be
 * NULL; W, S and f may be NULL (taken as zero).
 */
void orc_residuals(const orc_params *p, const double *u, const double *W, const double *rho5,
                   const double *rho1, const double *S, const double *f, double *H, double *M,
                   double *c)
{
    const int n = p->n;
    const long m = cells(n);
    geom g = make_geom(p, n);
    const double pi = M_PI, K2 = p->K * p->K;
    double *Wz = NULL;
    if (!W) {
        Wz = (double *)calloc(3 * m, sizeof(double));
        W = Wz;
    }
    if (H || c) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++)
                for (int k = 0; k < n; k++) {
                    long q = idx3(n, i, j, k);
                    double psi = psi0_at(p, &g, i, j, k) + u[q];
                    double A2 = A2_at(&g, W, i, j, k) + (p->bg_A2 ? p->bg_A2[q] : 0.0);
                    double psi4 = pow(psi, 4), psi5 = pow(psi, 5);
                    double matter, dmatter; /* matter term of H and its psi-derivative */
                    if (p->flags & OFLAG_CONFORMAL_MATTER) {
                        double rbar = rho5[q] + rho1[q];
                        matter = 2.0 * pi * rbar * pow(psi, -3);
                        dmatter = -6.0 * pi * rbar * pow(psi, -4);
                    } else {
                        matter = 2.0 * pi * rho5[q] * psi5 + 2.0 * pi * rho1[q] * psi;
                        dmatter = 10.0 * pi * rho5[q] * psi4 + 2.0 * pi * rho1[q];
                    }
                    if (H) {
                        double v = lap(&g, u, i, j, k) + matter - (K2 / 12.0) * psi5 +
                                   0.125 * A2 * pow(psi, -7);
                        if (f) v += f[q];
                        H[q] = v;
                    }
                    if (c)
                        c[q] = dmatter - (5.0 * K2 / 12.0) * psi4 - 0.875 * A2 * pow(psi, -8);
                }
    }
    if (M) {
        double *src = (double *)malloc(3 * m * sizeof(double));
        double mean[3] = {0.0, 0.0, 0.0};
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++)
                for (int k = 0; k < n; k++) {
                    long q = idx3(n, i, j, k);
                    double psi = psi0_at(p, &g, i, j, k) + u[q];
                    double w6 = (p->flags & OFLAG_CONFORMAL_MATTER) ? 1.0 : pow(psi, 6);
                    for (int a = 0; a < 3; a++)
                        src[a * m + q] = S ? 8.0 * pi * w6 * S[a * m + q] : 0.0;
                }
        if (p->bc == OBC_PERIODIC) {
            for (int a = 0; a < 3; a++) {
                double s = 0.0;
                for (long q = 0; q < m; q++) s += src[a * m + q];
                mean[a] = s / (double)m;
            }
        }
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++)
                for (int k = 0; k < n; k++) {
                    long q = idx3(n, i, j, k);
                    for (int a = 0; a < 3; a++)
                        M[a * m + q] = deltaL(&g, W, i, j, k, a) - (src[a * m + q] - mean[a]);
                }
        free(src);
    }
    free(Wz);
}

/* RMS and max of H and of |M| (vector norm per cell).  M may be NULL. */
void orc_norms(int n, const double *H, const double *M, double out[4])
{
    long m = cells(n);
    double sh = 0.0, sm = 0.0, mh = 0.0, mm = 0.0;
    for (long q = 0; q < m; q++) {
        double hv = H[q];
        sh += hv * hv;
        mh = fmax(mh, fabs(hv));
        if (M) {
            double v2 = M[q] * M[q] + M[m + q] * M[m + q] + M[2 * m + q] * M[2 * m + q];
            sm += v2;
            mm = fmax(mm, sqrt(v2));
        }
    }
    out[0] = sqrt(sh / (double)m);
    out[1] = sqrt(sm / (double)m);
    out[2] = mh;
    out[3] = mm;
}

/* ---- whole-field operators (exported for the pins) ----------------------- */

void orc_apply_lap(const orc_params *p, int n, const double *a, double *out)
{
    geom g = make_geom(p, n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) out[idx3(n, i, j, k)] = lap(&g, a, i, j, k);
}

void orc_apply_d1(const orc_params *p, int n, const double *a, int axis, double *out)
{
    geom g = make_geom(p, n);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) out[idx3(n, i, j, k)] = D1(&g, a, i, j, k, axis);
}

void orc_apply_deltaL(const orc_params *p, int n, const double *W, double *out)
{
    geom g = make_geom(p, n);
    long m = cells(n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                for (int a = 0; a < 3; a++) out[a * m + idx3(n, i, j, k)] = deltaL(&g, W, i, j, k, a);
}

/* ---- smoothers (double-buffered red-black Gauss-Seidel) ------------------ */

/* One colour pass on (L_h + c) d = r: cells of the given colour get
 * d + (r - (L_h + c) d) / diag, all others are copied; reads only `in`. */
void orc_pass_psi(const orc_params *p, int n, const double *in, double *out, const double *r,
                  const double *c, int colour)
{
    geom g = make_geom(p, n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long q = idx3(n, i, j, k);
                if (((i + j + k) & 1) != colour) {
                    out[q] = in[q];
                    continue;
                }
                double Ad = lap(&g, in, i, j, k) + c[q] * in[q];
                double diag = lap_diag(&g, i, j, k) + c[q];
                out[q] = in[q] + (r[q] - Ad) / diag;
            }
}

/* One colour pass on Delta_L,h d = r for the three components together. */
void orc_pass_W(const orc_params *p, int n, const double *in, double *out, const double *r,
                int colour)
{
    geom g = make_geom(p, n);
    long m = cells(n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long q = idx3(n, i, j, k);
                for (int a = 0; a < 3; a++) {
                    if (((i + j + k) & 1) != colour) {
                        out[a * m + q] = in[a * m + q];
                        continue;
                    }
                    double Ad = deltaL(&g, in, i, j, k, a);
                    double diag = deltaL_diag(&g, i, j, k, a);
                    out[a * m + q] = in[a * m + q] + (r[a * m + q] - Ad) / diag;
                }
            }
}

/* ---- transfers ----------------------------------------------------------- */

/* coarse = average of the 8 children (nf = fine cells per axis). */
void orc_restrict(int nf, const double *fine, double *coarse)
{
    int nc = nf / 2;
#pragma omp parallel for schedule(static)
    for (int I = 0; I < nc; I++)
        for (int J = 0; J < nc; J++)
            for (int K = 0; K < nc; K++) {
                double s = 0.0;
                for (int di = 0; di < 2; di++)
                    for (int dj = 0; dj < 2; dj++)
                        for (int dk = 0; dk < 2; dk++)
                            s += fine[idx3(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
                coarse[idx3(nc, I, J, K)] = s / 8.0;
            }
}

/* Neighbour coarse index and 1D weights for a fine index: the fine centre
 * sits a quarter coarse spacing from its parent's centre. */
static void lin_taps(int i, int *I0, int *I1)
{
    int I = i / 2;
    *I0 = I;
    *I1 = (i % 2 == 0) ? I - 1 : I + 1;
}

void orc_interp_cubic(const orc_params *p, int nc, const double *coarse, double *fine);

/* fine += trilinear interpolation of coarse (cell-centred, weights 3/4, 1/4), or, with
 * OFLAG_CUBIC_PROLONG, fine += the 4-point cubic interpolation of coarse. */
void orc_prolong_add(const orc_params *p, int nc, const double *coarse, double *fine)
{
    int nf = 2 * nc;
    if (p->flags & OFLAG_CUBIC_PROLONG) {
        long mf = (long)nf * nf * nf;
        double *q = (double *)malloc(mf * sizeof(double));
        orc_interp_cubic(p, nc, coarse, q);
        for (long i = 0; i < mf; i++) fine[i] += q[i];
        free(q);
        return;
    }
    geom gc = make_geom(p, nc);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nf; i++)
        for (int j = 0; j < nf; j++)
            for (int k = 0; k < nf; k++) {
                int Ii[2], Jj[2], Kk[2];
                lin_taps(i, &Ii[0], &Ii[1]);
                lin_taps(j, &Jj[0], &Jj[1]);
                lin_taps(k, &Kk[0], &Kk[1]);
                const double w[2] = {0.75, 0.25};
                double s = 0.0;
                for (int a = 0; a < 2; a++)
                    for (int b = 0; b < 2; b++)
                        for (int e = 0; e < 2; e++)
                            s += w[a] * w[b] * w[e] * at(&gc, coarse, Ii[a], Jj[b], Kk[e]);
                fine[idx3(nf, i, j, k)] += s;
            }
}

/* Four-point cubic Lagrange interpolation (fourth-order accurate) from the
 * coarse grid to every fine cell; fine = Q coarse. */
void orc_interp_cubic(const orc_params *p, int nc, const double *coarse, double *fine)
{
    int nf = 2 * nc;
    geom gc = make_geom(p, nc);
    /* Lagrange weights at offset -1/4 (even fine index) from nodes I-2..I+1 and
     * at +1/4 (odd fine index) from nodes I-1..I+2, in coarse spacings. */
    double wl[2][4];
    const double t[2] = {-0.25, 0.25};
    for (int s = 0; s < 2; s++) {
        int base = (s == 0) ? -2 : -1;
        for (int a = 0; a < 4; a++) {
            double num = 1.0, den = 1.0;
            for (int b = 0; b < 4; b++) {
                if (b == a) continue;
                num *= t[s] - (double)(base + b);
                den *= (double)(base + a) - (double)(base + b);
            }
            wl[s][a] = num / den;
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nf; i++)
        for (int j = 0; j < nf; j++)
            for (int k = 0; k < nf; k++) {
                int pi_ = i % 2, pj = j % 2, pk = k % 2;
                int bi = i / 2 + (pi_ == 0 ? -2 : -1);
                int bj = j / 2 + (pj == 0 ? -2 : -1);
                int bk = k / 2 + (pk == 0 ? -2 : -1);
                double s = 0.0;
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++)
                        for (int e = 0; e < 4; e++)
                            s += wl[pi_][a] * wl[pj][b] * wl[pk][e] *
                                 at(&gc, coarse, bi + a, bj + b, bk + e);
                fine[idx3(nf, i, j, k)] = s;
            }
}

/* ---- coarsest-level dense solves ----------------------------------------- */

/* LU factorisation with partial pivoting, row-major m x m, in place. */
static int lu_factor(double *A, int *piv, int m)
{
    for (int k = 0; k < m; k++) {
        int pr = k;
        double best = fabs(A[(long)k * m + k]);
        for (int r = k + 1; r < m; r++)
            if (fabs(A[(long)r * m + k]) > best) {
                best = fabs(A[(long)r * m + k]);
                pr = r;
            }
        piv[k] = pr;
        if (best == 0.0) return -1;
        if (pr != k)
            for (int col = 0; col < m; col++) {
                double t = A[(long)k * m + col];
                A[(long)k * m + col] = A[(long)pr * m + col];
                A[(long)pr * m + col] = t;
            }
        for (int r = k + 1; r < m; r++) {
            double l = A[(long)r * m + k] / A[(long)k * m + k];
            A[(long)r * m + k] = l;
            for (int col = k + 1; col < m; col++) A[(long)r * m + col] -= l * A[(long)k * m + col];
        }
    }
    return 0;
}

static void lu_solve(const double *LU, const int *piv, int m, double *b)
{
    for (int k = 0; k < m; k++)
        if (piv[k] != k) {
            double t = b[k];
            b[k] = b[piv[k]];
            b[piv[k]] = t;
        }
    for (int r = 0; r < m; r++)
        for (int col = 0; col < r; col++) b[r] -= LU[(long)r * m + col] * b[col];
    for (int r = m - 1; r >= 0; r--) {
        for (int col = r + 1; col < m; col++) b[r] -= LU[(long)r * m + col] * b[col];
        b[r] /= LU[(long)r * m + r];
    }
}

/* Solve (L_h + c) x = r exactly on an n^3 grid by a dense LU whose columns are
 * the operator applied to unit vectors.  Returns 0 on success. */
int orc_coarse_solve_psi(const orc_params *p, int n, const double *c, const double *r, double *x)
{
    geom g = make_geom(p, n);
    long m = cells(n);
    double *A = (double *)malloc(m * m * sizeof(double));
    double *e = (double *)calloc(m, sizeof(double));
    int *piv = (int *)malloc(m * sizeof(int));
    for (long col = 0; col < m; col++) {
        e[col] = 1.0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++)
                for (int k = 0; k < n; k++) {
                    long row = idx3(n, i, j, k);
                    A[row * m + col] = lap(&g, e, i, j, k) + c[row] * e[row];
                }
        e[col] = 0.0;
    }
    int rc = lu_factor(A, piv, (int)m);
    if (rc == 0) {
        memcpy(x, r, m * sizeof(double));
        lu_solve(A, piv, (int)m, x);
    }
    free(A);
    free(e);
    free(piv);
    return rc;
}

/* Solve Delta_L,h x = r on a periodic n^3 grid: the right-hand side's mean is
 * removed per component, and the constant null vectors are fixed by adding
 * -(1/(N h^2)) to every entry that couples two cells of the same component,
 * which makes the mean of each solution component zero. */
int orc_coarse_solve_W(const orc_params *p, int n, const double *r, double *x)
{
    geom g = make_geom(p, n);
    long cn = cells(n), m = 3 * cn;
    double *A = (double *)malloc(m * m * sizeof(double));
    double *e = (double *)calloc(m, sizeof(double));
    int *piv = (int *)malloc(m * sizeof(int));
    for (long col = 0; col < m; col++) {
        e[col] = 1.0;
        for (int a = 0; a < 3; a++)
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++)
                    for (int k = 0; k < n; k++) {
                        long row = a * cn + idx3(n, i, j, k);
                        A[row * m + col] = deltaL(&g, e, i, j, k, a);
                    }
        e[col] = 0.0;
    }
    double reg = 1.0 / ((double)cn * g.h * g.h);
    for (long row = 0; row < m; row++)
        for (long col = 0; col < m; col++)
            if (row / cn == col / cn) A[row * m + col] -= reg;
    for (int a = 0; a < 3; a++) {
        double s = 0.0;
        for (long q = 0; q < cn; q++) s += r[a * cn + q];
        for (long q = 0; q < cn; q++) x[a * cn + q] = r[a * cn + q] - s / (double)cn;
    }
    int rc = lu_factor(A, piv, (int)m);
    if (rc == 0) lu_solve(A, piv, (int)m, x);
    free(A);
    free(e);
    free(piv);
    return rc;
}

/* ---- V-cycles ------------------------------------------------------------ */

typedef struct {
    orc_params p;
    int L;
    int n[OMAXLEV];
    double *d[OMAXLEV], *t[OMAXLEV], *r[OMAXLEV], *c[OMAXLEV], *def[OMAXLEV];
} hier;

static void hier_init(hier *H, const orc_params *p, int comps)
{
    memset(H, 0, sizeof(*H));
    H->p = *p;
    H->L = p->levels;
    int n = p->n;
    for (int l = 0; l < H->L; l++) {
        long m = cells(n) * comps;
        H->n[l] = n;
        H->d[l] = (double *)calloc(m, sizeof(double));
        H->t[l] = (double *)calloc(m, sizeof(double));
        H->r[l] = (double *)calloc(m, sizeof(double));
        H->def[l] = (double *)calloc(m, sizeof(double));
        H->c[l] = (double *)calloc(cells(n), sizeof(double));
        n /= 2;
    }
}

static void hier_free(hier *H)
{
    for (int l = 0; l < H->L; l++) {
        free(H->d[l]);
        free(H->t[l]);
        free(H->r[l]);
        free(H->def[l]);
        free(H->c[l]);
    }
}

/* One V-cycle for (L_h + c) d = r on level l (d starts at zero). */
static int vcycle_psi(hier *H, int l)
{
    const orc_params *p = &H->p;
    int n = H->n[l];
    long m = cells(n);
    if (l == H->L - 1) return orc_coarse_solve_psi(p, n, H->c[l], H->r[l], H->d[l]);
    memset(H->d[l], 0, m * sizeof(double));
    for (int s = 0; s < p->nu_pre; s++)
        for (int col = 0; col < 2; col++) {
            orc_pass_psi(p, n, H->d[l], H->t[l], H->r[l], H->c[l], col);
            memcpy(H->d[l], H->t[l], m * sizeof(double));
        }
    /* defect d = r - (L_h + c) d, restricted */
    orc_apply_lap(p, n, H->d[l], H->def[l]);
    for (long q = 0; q < m; q++) H->def[l][q] = H->r[l][q] - (H->def[l][q] + H->c[l][q] * H->d[l][q]);
    orc_restrict(n, H->def[l], H->r[l + 1]);
    int rc = vcycle_psi(H, l + 1);
    if (rc) return rc;
    orc_prolong_add(p, n / 2, H->d[l + 1], H->d[l]);
    for (int s = 0; s < p->nu_post; s++)
        for (int col = 0; col < 2; col++) {
            orc_pass_psi(p, n, H->d[l], H->t[l], H->r[l], H->c[l], col);
            memcpy(H->d[l], H->t[l], m * sizeof(double));
        }
    return 0;
}

static int vcycle_W(hier *H, int l)
{
    const orc_params *p = &H->p;
    int n = H->n[l];
    long cn = cells(n), m = 3 * cn;
    if (l == H->L - 1) return orc_coarse_solve_W(p, n, H->r[l], H->d[l]);
    memset(H->d[l], 0, m * sizeof(double));
    for (int s = 0; s < p->nu_pre; s++)
        for (int col = 0; col < 2; col++) {
            orc_pass_W(p, n, H->d[l], H->t[l], H->r[l], col);
            memcpy(H->d[l], H->t[l], m * sizeof(double));
        }
    orc_apply_deltaL(p, n, H->d[l], H->def[l]);
    for (long q = 0; q < m; q++) H->def[l][q] = H->r[l][q] - H->def[l][q];
    for (int a = 0; a < 3; a++) orc_restrict(n, H->def[l] + a * cn, H->r[l + 1] + a * (cn / 8));
    int rc = vcycle_W(H, l + 1);
    if (rc) return rc;
    for (int a = 0; a < 3; a++) orc_prolong_add(p, n / 2, H->d[l + 1] + a * (cn / 8), H->d[l] + a * cn);
    for (int s = 0; s < p->nu_post; s++)
        for (int col = 0; col < 2; col++) {
            orc_pass_W(p, n, H->d[l], H->t[l], H->r[l], col);
            memcpy(H->d[l], H->t[l], m * sizeof(double));
        }
    return 0;
}

/* One psi V-cycle for a given right-hand side and coefficient (exported for
 * operator-level parity): d = V(r, c). */
int orc_vcycle_psi(const orc_params *p, const double *c, const double *r, double *d)
{
    hier H;
    hier_init(&H, p, 1);
    long m = cells(p->n);
    memcpy(H.r[0], r, m * sizeof(double));
    memcpy(H.c[0], c, m * sizeof(double));
    for (int l = 0; l + 1 < H.L; l++) orc_restrict(H.n[l], H.c[l], H.c[l + 1]);
    int rc = vcycle_psi(&H, 0);
    memcpy(d, H.d[0], m * sizeof(double));
    hier_free(&H);
    return rc;
}

int orc_vcycle_W(const orc_params *p, const double *r, double *d)
{
    hier H;
    hier_init(&H, p, 3);
    long m = 3 * cells(p->n);
    memcpy(H.r[0], r, m * sizeof(double));
    int rc = vcycle_W(&H, 0);
    memcpy(d, H.d[0], m * sizeof(double));
    hier_free(&H);
    return rc;
}

/* ---- outer Newton iteration ---------------------------------------------- */

typedef struct {
    const double *rho5, *rho1, *S, *f;
} sources;

/* W step: r_W = -M_h(u, W); one W V-cycle; W += dW - mean(dW). */
static int step_W(hier *HW, const orc_params *p, const double *u, double *W, const sources *s)
{
    long cn = cells(p->n);
    orc_residuals(p, u, W, s->rho5, s->rho1, s->S, s->f, NULL, HW->r[0], NULL);
    for (long q = 0; q < 3 * cn; q++) HW->r[0][q] = -HW->r[0][q];
    int rc = vcycle_W(HW, 0);
    if (rc) return rc;
    for (int a = 0; a < 3; a++) {
        double mean = 0.0;
        for (long q = 0; q < cn; q++) mean += HW->d[0][a * cn + q];
        mean /= (double)cn;
        for (long q = 0; q < cn; q++) W[a * cn + q] += HW->d[0][a * cn + q] - mean;
    }
    return 0;
}

/* psi step: r = -H_h(u, W), c = dH_h/dpsi; one psi V-cycle; u += d. */
static int step_psi(hier *HP, const orc_params *p, double *u, const double *W, const sources *s)
{
    long m = cells(p->n);
    orc_residuals(p, u, W, s->rho5, s->rho1, s->S, s->f, HP->r[0], NULL, HP->c[0]);
    for (long q = 0; q < m; q++) HP->r[0][q] = -HP->r[0][q];
    for (int l = 0; l + 1 < HP->L; l++) orc_restrict(HP->n[l], HP->c[l], HP->c[l + 1]);
    int rc = vcycle_psi(HP, 0);
    if (rc) return rc;
    for (long q = 0; q < m; q++) u[q] += HP->d[0][q];
    return 0;
}

/* One outer step for eq = 1 (psi), 2 (W) or 3 (W then psi; with OFLAG_SAME_STATE the
 * psi step reads the W the step started from). */
int orc_step(const orc_params *p, int eq, double *u, double *W, const double *rho5,
             const double *rho1, const double *S, const double *f)
{
    sources s = {rho5, rho1, S, f};
    int rc = 0;
    double *W_start = NULL;
    if (eq == 3 && (p->flags & OFLAG_SAME_STATE)) {
        W_start = (double *)malloc(3 * cells(p->n) * sizeof(double));
        memcpy(W_start, W, 3 * cells(p->n) * sizeof(double));
    }
    if (eq & 2) {
        hier HW;
        hier_init(&HW, p, 3);
        rc = step_W(&HW, p, u, W, &s);
        hier_free(&HW);
    }
    if (!rc && (eq & 1)) {
        hier HP;
        hier_init(&HP, p, 1);
        rc = step_psi(&HP, p, u, W_start ? W_start : W, &s);
        hier_free(&HP);
    }
    free(W_start);
    return rc;
}

/*
 * Newton-multigrid solve.  hist receives 4 doubles per recorded iteration
 * (h_rms, m_rms, h_max, m_max), at most hist_cap entries.  Returns 0 when
 * converged, 4 when max_outer updates did not reach tol, 5 on a non-finite
 * norm, 1 on a singular coarse matrix.  *iters = number of outer updates.
 */
int orc_solve(const orc_params *p, double *u, double *W, const double *rho5, const double *rho1,
              const double *S, const double *f, double tol, int max_outer, double *hist,
              int hist_cap, int *iters, double out_norms[4])
{
    sources s = {rho5, rho1, S, f};
    long m = cells(p->n);
    double *H = (double *)malloc(m * sizeof(double));
    double *M = (double *)malloc(3 * m * sizeof(double));
    hier HP, HW;
    hier_init(&HP, p, 1);
    if (p->solve_momentum) hier_init(&HW, p, 3);
    int status = 4, it = 0;
    for (;; it++) {
        double nr[4];
        orc_residuals(p, u, W, rho5, rho1, S, f, H, p->solve_momentum ? M : NULL, NULL);
        orc_norms(p->n, H, p->solve_momentum ? M : NULL, nr);
        if (hist && it < hist_cap) memcpy(hist + 4 * it, nr, sizeof(nr));
        if (out_norms) memcpy(out_norms, nr, sizeof(nr));
        if (!isfinite(nr[0]) || !isfinite(nr[1])) {
            status = 5;
            break;
        }
        if (nr[0] <= tol && (!p->solve_momentum || nr[1] <= tol)) {
            status = 0;
            break;
        }
        if (it >= max_outer) {
            status = 4;
            break;
        }
        int rc = 0;
        if (p->solve_momentum && (p->flags & OFLAG_SAME_STATE)) {
            memcpy(M, W, 3 * m * sizeof(double)); /* M is free until the next evaluation */
            rc = step_W(&HW, p, u, W, &s);
            if (!rc) rc = step_psi(&HP, p, u, M, &s);
        } else {
            if (p->solve_momentum) rc = step_W(&HW, p, u, W, &s);
            if (!rc) rc = step_psi(&HP, p, u, W, &s);
        }
        if (rc) {
            status = 1;
            break;
        }
    }
    if (iters) *iters = it;
    hier_free(&HP);
    if (p->solve_momentum) hier_free(&HW);
    free(H);
    free(M);
    return status;
}

/* ---- CTTK and CTTK-Hybrid (Summary and Key features, "Methods") -----------
 *
 * The two CTT variants the paper implements let the trace K vary in space; their
 * equations are given in the formalism the paper cites, not in the paper, so this
 * is a reading of eqs. Ham and Mom with a spatially varying K (conformally flat,
 * A_ij = psi^-2 Abar_ij, gamma^ij = psi^-4 delta_ij).  Eq. Mom then reads
 *   Delta_L W_a - (2/3) psi^6 d_a K - 8 pi psi^6 S_a = 0,
 * and eq. Ham keeps its -(K^2/12) psi^5 term, now with K = K(x).  Both new terms
 * carry the psi power of an existing matter term, so the CTT residuals take them
 * as shifted sources:
 *   S_a  -> S_a + D_a K / (12 pi)           (8 pi psi^6 times it gives both terms)
 *   rho5 -> rho5 - (K^2 - K0^2) / (24 pi)   (2 pi psi^5 times it, with constant K0)
 *
 * CTTK-Hybrid: K^2(x) = 24 pi (rho5(x) + <rho1>): the psi-independent energy density is
 * carried by K locally (so rho5 -> 0), the gradient energy by psi, solved as in CTT
 * with the constant trace K0, K0^2 = 24 pi <rho1>.  K is fixed before the solve.
 *
 * CTTK: psi is free data (u is left as given) and eq. Ham is solved for K:
 *   K^2 = 12 H0 / psi^5,   H0 = H_h at K = 0,
 * after every W step; with it H_h vanishes and rho5 -> rho5 - K^2 / (24 pi) (K0 = 0).
 * A negative K^2 has no real trace: K and the shifted rho5 are NaN there.
 */

/* CTTK-Hybrid: rho5 (in place) -> 0, S (in place) -> S + D K / (12 pi), K (out) the
 * field, *K0 = sqrt(24 pi <rho1>). */
void orc_cttk_hybrid_sources(const orc_params *p, double *rho5, const double *rho1, double *S, double *K,
                             double *K0)
{
    const int n = p->n;
    const long m = cells(n);
    geom g = make_geom(p, n);
    double mean1 = 0.0;
    for (long q = 0; q < m; q++) mean1 += rho1[q];
    mean1 /= (double)m;
    for (long q = 0; q < m; q++) {
        K[q] = sqrt(24.0 * M_PI * (rho5[q] + mean1));
        rho5[q] = 0.0;
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long q = idx3(n, i, j, k);
                for (int a = 0; a < 3; a++) S[a * m + q] += D1(&g, K, i, j, k, a) / (12.0 * M_PI);
            }
    *K0 = sqrt(24.0 * M_PI * mean1);
}

/* CTTK: K from eq. Ham at (u, W) (K^2 = 12 H0 / psi^5), and the shifted sources
 * rho5_eff = rho5 - K^2 / (24 pi), S_eff = S + D K / (12 pi).  p->K is not used. */
void orc_cttk_update(const orc_params *p, const double *u, const double *W, const double *rho5,
                     const double *rho1, const double *S, const double *f, double *rho5_eff, double *S_eff,
                     double *K)
{
    const int n = p->n;
    const long m = cells(n);
    geom g = make_geom(p, n);
    orc_params p0 = *p;
    p0.K = 0.0;
    orc_residuals(&p0, u, W, rho5, rho1, S, f, K, NULL, NULL); /* H0 into K */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long q = idx3(n, i, j, k);
                double psi = psi0_at(p, &g, i, j, k) + u[q];
                double K2 = 12.0 * K[q] / pow(psi, 5);
                if (!(K2 >= 0.0)) K2 = NAN;
                K[q] = sqrt(K2);
                rho5_eff[q] = rho5[q] - K2 / (24.0 * M_PI);
            }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                long q = idx3(n, i, j, k);
                for (int a = 0; a < 3; a++)
                    S_eff[a * m + q] = (S ? S[a * m + q] : 0.0) + D1(&g, K, i, j, k, a) / (12.0 * M_PI);
            }
}

/*
 * CTTK solve: u is data; W is solved.  Every iteration: K and the shifted sources
 * from (u, W), the norms of H_h and M_h with them (H_h vanishes up to rounding), the
 * convergence test, then one W step, W -> W + f.  The K-W coupling makes this a
 * fixed-point iteration whose contraction grows with resolution, so the steps are
 * combined by Anderson mixing over the last m = max(1, p->mix_depth) steps: with the
 * differences dF_j = f_{j+1} - f_j and dW_j = W_{j+1} - W_j of consecutive steps
 * (the newest m of them), gamma minimises |f - sum_j gamma_j dF_j| (its normal
 * equations), and
 *   W -> W + f - sum_j gamma_j (dW_j + dF_j).
 * With one stored pair this is the secant step gamma = <dF, f> / <dF, dF> (gamma = 0 on
 * the first iteration or when dF = 0).  With more, the normal equations carry a ridge of
 * 1e-12 of their largest diagonal entry and are solved by Gaussian elimination with
 * partial pivoting (gamma = 0 if that entry is 0).  K receives the trace of the final
 * state.  Status and outputs as orc_solve (p->solve_momentum must be 1).
 */
#define OMAXMIX 8

/* gamma of the Anderson step from its normal equations A gamma = b (n x n, symmetric):
 * one unknown, the secant quotient; more, a ridge of 1e-12 of the largest diagonal entry
 * and Gaussian elimination with partial pivoting.  gamma = 0 when A vanishes. */
static void mix_solve(double *A, double *b, int n, double *gam)
{
    if (n == 1) {
        gam[0] = A[0] > 0.0 ? b[0] / A[0] : 0.0;
        return;
    }
    double dmax = 0.0;
    for (int i = 0; i < n; i++) dmax = fmax(dmax, A[i * n + i]);
    if (!(dmax > 0.0)) return;
    for (int i = 0; i < n; i++) A[i * n + i] += 1e-12 * dmax;
    for (int k = 0; k < n; k++) {
        int piv = k;
        for (int i = k + 1; i < n; i++)
            if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < n; j++) {
                const double t = A[k * n + j];
                A[k * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            const double t = b[k];
            b[k] = b[piv];
            b[piv] = t;
        }
        for (int i = k + 1; i < n; i++) {
            const double l = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; j++) A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; i--) {
        double v = b[i];
        for (int j = i + 1; j < n; j++) v -= A[i * n + j] * gam[j];
        gam[i] = v / A[i * n + i];
    }
}

int orc_cttk_solve(const orc_params *p, const double *u, double *W, const double *rho5, const double *rho1,
                   const double *S, const double *f, double *K, double tol, int max_outer, double *hist,
                   int hist_cap, int *iters, double out_norms[4])
{
    const long m = cells(p->n);
    orc_params p0 = *p;
    p0.K = 0.0;
    double *r5 = (double *)malloc(m * sizeof(double));
    double *Se = (double *)malloc(3 * m * sizeof(double));
    double *H = (double *)malloc(m * sizeof(double));
    double *M = (double *)malloc(3 * m * sizeof(double));
    double *Wk = (double *)malloc(3 * m * sizeof(double));
    double *Wp = (double *)malloc(3 * m * sizeof(double));
    double *fp = (double *)malloc(3 * m * sizeof(double));
    const int depth = p->mix_depth > 1 ? p->mix_depth : 1;
    double *dWs = (double *)malloc((size_t)depth * 3 * m * sizeof(double));
    double *dFs = (double *)malloc((size_t)depth * 3 * m * sizeof(double));
    int count = 0, head = 0;
    sources s = {r5, rho1, Se, f};
    hier HW;
    hier_init(&HW, &p0, 3);
    int status = 4, it = 0;
    for (;; it++) {
        double nr[4];
        orc_cttk_update(&p0, u, W, rho5, rho1, S, f, r5, Se, K);
        orc_residuals(&p0, u, W, r5, rho1, Se, f, H, M, NULL);
        orc_norms(p0.n, H, M, nr);
        if (hist && it < hist_cap) memcpy(hist + 4 * it, nr, sizeof(nr));
        if (out_norms) memcpy(out_norms, nr, sizeof(nr));
        if (!isfinite(nr[0]) || !isfinite(nr[1])) {
            status = 5;
            break;
        }
        if (nr[0] <= tol && nr[1] <= tol) {
            status = 0;
            break;
        }
        if (it >= max_outer) {
            status = 4;
            break;
        }
        memcpy(Wk, W, 3 * m * sizeof(double));
        if (step_W(&HW, &p0, u, W, &s)) {
            status = 1;
            break;
        }
        /* W now holds W_k + f; Anderson mixing with the stored differences */
        if (it > 0) { /* the newest difference pair replaces the oldest */
            double *dWn = dWs + (long)head * 3 * m, *dFn = dFs + (long)head * 3 * m;
            for (long q = 0; q < 3 * m; q++) {
                dFn[q] = (W[q] - Wk[q]) - fp[q];
                dWn[q] = Wk[q] - Wp[q];
            }
            if (count < depth) count++;
            head = (head + 1) % depth;
        }
        double gam[OMAXMIX] = {0.0};
        if (count > 0) {
            double A[OMAXMIX * OMAXMIX], b[OMAXMIX];
            for (int i = 0; i < count; i++) {
                const double *Fi = dFs + (long)i * 3 * m;
                double bi = 0.0;
                for (long q = 0; q < 3 * m; q++) bi += Fi[q] * (W[q] - Wk[q]);
                b[i] = bi;
                for (int j = 0; j <= i; j++) {
                    const double *Fj = dFs + (long)j * 3 * m;
                    double a = 0.0;
                    for (long q = 0; q < 3 * m; q++) a += Fi[q] * Fj[q];
                    A[i * count + j] = A[j * count + i] = a;
                }
            }
            mix_solve(A, b, count, gam);
        }
        for (long q = 0; q < 3 * m; q++) {
            const double fk = W[q] - Wk[q];
            double corr = 0.0;
            for (int j = 0; j < count; j++) corr += gam[j] * (dWs[(long)j * 3 * m + q] + dFs[(long)j * 3 * m + q]);
            W[q] = Wk[q] + fk - corr;
            Wp[q] = Wk[q];
            fp[q] = fk;
        }
    }
    if (iters) *iters = it;
    hier_free(&HW);
    free(Wk);
    free(Wp);
    free(fp);
    free(dWs);
    free(dFs);
    free(r5);
    free(Se);
    free(H);
    free(M);
    return status;
}

/* ---- sources from the scalar field (matter projections, Summary) --------- */

/*
 * Fourier scalar field: phi = sum amp cos(2 pi k.x/L + phase), Pi likewise
 * (mode tables: kx, ky, kz, amp, phase per row), V(phi) = mass^2 phi^2 / 2.
 * rho5 = Pi^2/2 + V, rho1 = |d phi|^2 / 2, S_a = -Pi d_a phi (SoA).
 */
void orc_scalar_sources(const orc_params *p, int nphi, const double *phi_modes, int npi,
                        const double *pi_modes, double mass, double *rho5, double *rho1,
                        double *S)
{
    int n = p->n;
    long m = cells(n);
    geom g = make_geom(p, n);
    double tw = 2.0 * M_PI / p->length;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                double x[3] = {g.org[0] + (i + 0.5) * g.h, g.org[1] + (j + 0.5) * g.h,
                               g.org[2] + (k + 0.5) * g.h};
                double phi = 0.0, dphi[3] = {0.0, 0.0, 0.0}, Pi = 0.0;
                for (int q = 0; q < nphi; q++) {
                    const double *md = phi_modes + 5 * q;
                    double arg = tw * (md[0] * x[0] + md[1] * x[1] + md[2] * x[2]) + md[4];
                    phi += md[3] * cos(arg);
                    for (int a = 0; a < 3; a++) dphi[a] -= md[3] * tw * md[a] * sin(arg);
                }
                for (int q = 0; q < npi; q++) {
                    const double *md = pi_modes + 5 * q;
                    double arg = tw * (md[0] * x[0] + md[1] * x[1] + md[2] * x[2]) + md[4];
                    Pi += md[3] * cos(arg);
                }
                long c = idx3(n, i, j, k);
                rho5[c] = 0.5 * Pi * Pi + 0.5 * mass * mass * phi * phi;
                rho1[c] = 0.5 * (dphi[0] * dphi[0] + dphi[1] * dphi[1] + dphi[2] * dphi[2]);
                for (int a = 0; a < 3; a++) S[a * m + c] = -Pi * dphi[a];
            }
}

/*
 * Scalar shell around the puncture: phi = amp exp(-(r - r0)^2 / width2) Y_11,
 * Y_11 = sqrt(3 / (4 pi)) x / r (real dipole harmonic, x measured from the
 * puncture), Pi = 0.  rho5 = mass^2 phi^2 / 2, rho1 = |d phi|^2 / 2, S = 0.
 */
void orc_shell_sources(const orc_params *p, double amp, double r0, double width2, double mass,
                       double *rho5, double *rho1, double *S)
{
    int n = p->n;
    long m = cells(n);
    geom g = make_geom(p, n);
    const double ylm = sqrt(3.0 / (4.0 * M_PI));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                double x[3];
                cell_pos(&g, i, j, k, x);
                double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                double fr = amp * exp(-(r - r0) * (r - r0) / width2);
                double dfr = -2.0 * (r - r0) / width2 * fr;
                double phi = fr * ylm * x[0] / r;
                double dphi[3];
                for (int a = 0; a < 3; a++) {
                    /* d_a [f(r) x / r] = f'(r) (x_a / r)(x / r) + f(r) (delta_a0 / r - x x_a / r^3) */
                    dphi[a] = ylm * (dfr * (x[a] / r) * (x[0] / r) +
                                     fr * ((a == 0 ? 1.0 : 0.0) / r - x[0] * x[a] / (r * r * r)));
                }
                long c = idx3(n, i, j, k);
                rho5[c] = 0.5 * mass * mass * phi * phi;
                rho1[c] = 0.5 * (dphi[0] * dphi[0] + dphi[1] * dphi[1] + dphi[2] * dphi[2]);
                for (int a = 0; a < 3; a++) S[a * m + c] = 0.0;
            }
}

/*
 * Bowen-York data for punctures (Key features, "Flexibility": binary black holes
 * with boosted and/or spinning punctures; the momentum constraint with K = 0 and
 * no matter is solved analytically, leaving the Hamiltonian constraint for u).
 * tab: 10 doubles per puncture: mass m, centre C[3], momentum P[3], spin S[3].
 * With n = (x - C)/r, r = |x - C|, the traceless extrinsic curvature is the sum
 * over punctures of
 *   (3 / (2 r^2)) [P_i n_j + P_j n_i - (delta_ij - n_i n_j) P.n]
 *   + (3 / r^3) [(S x n)_i n_j + (S x n)_j n_i],
 * and psi0 = 1 + sum m / (2 r).
 * orc_bowen_york_tensor: the six components xx, xy, xz, yy, yz, zz at point x.
 * orc_bowen_york: psi0 and A2 = Abar_ij Abar_ij at every cell centre.
 */
void orc_bowen_york_tensor(int count, const double *tab, const double x[3], double out[6])
{
    double A[3][3] = {{0.0}};
    for (int q = 0; q < count; q++) {
        const double *t = tab + 10 * q;
        double d[3] = {x[0] - t[1], x[1] - t[2], x[2] - t[3]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double nv[3] = {d[0] / r, d[1] / r, d[2] / r};
        const double *P = t + 4, *S = t + 7;
        double pn = P[0] * nv[0] + P[1] * nv[1] + P[2] * nv[2];
        double sxn[3] = {S[1] * nv[2] - S[2] * nv[1], S[2] * nv[0] - S[0] * nv[2], S[0] * nv[1] - S[1] * nv[0]};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double boost = P[a] * nv[b] + P[b] * nv[a] - ((a == b ? 1.0 : 0.0) - nv[a] * nv[b]) * pn;
                double spin = sxn[a] * nv[b] + sxn[b] * nv[a];
                A[a][b] += 1.5 / (r * r) * boost + 3.0 / (r * r * r) * spin;
            }
    }
    out[0] = A[0][0];
    out[1] = A[0][1];
    out[2] = A[0][2];
    out[3] = A[1][1];
    out[4] = A[1][2];
    out[5] = A[2][2];
}

void orc_bowen_york(const orc_params *p, int count, const double *tab, double *psi0, double *A2)
{
    int n = p->n;
    geom g = make_geom(p, n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                double x[3], A[6];
                x[0] = g.org[0] + (i + 0.5) * g.h;
                x[1] = g.org[1] + (j + 0.5) * g.h;
                x[2] = g.org[2] + (k + 0.5) * g.h;
                orc_bowen_york_tensor(count, tab, x, A);
                long c = idx3(n, i, j, k);
                A2[c] = A[0] * A[0] + A[3] * A[3] + A[5] * A[5] + 2.0 * (A[1] * A[1] + A[2] * A[2] + A[4] * A[4]);
                double s = 1.0;
                for (int q = 0; q < count; q++) {
                    const double *t = tab + 10 * q;
                    double d0 = x[0] - t[1], d1 = x[1] - t[2], d2 = x[2] - t[3];
                    s += t[0] / (2.0 * sqrt(d0 * d0 + d1 * d1 + d2 * d2));
                }
                psi0[c] = s;
            }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
