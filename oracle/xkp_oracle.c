/*
 * xkp oracle: a plain, slow, FP64 CPU reference of the cross-matrix Krylov projection path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline load this library.  It shares no code, header or constant with the HIP library.
 *
 * Built with `gcc -O2 -ffp-contract=off` so that every product and sum is rounded as written.
 *
 * What each function follows (paper: Lau, Na, Wan, "Efficient Score Pre-computation for Diffusion
 * Models via Cross-Matrix Krylov Projection", arXiv 2511.17634):
 *   xo_coeffs / xo_rhs / xo_apply / xo_dense  -- Section 2.3, the five-point coefficients
 *       C_diag, C_north, C_south, C_east, C_west and b of the discretised system, the
 *       block-tridiagonal matrix form and the unknown ordering (y index fastest); the appendix
 *       ("Coefficient Definitions") restates the same coefficients.
 *   xo_lu_solve / xo_banded_solve  -- the direct LU solve the paper uses as its baseline
 *       (end of Section 2.3; Experiment 2, "SpSolve").
 *   xo_gmres  -- the Krylov solve of Section 3 (Krylov subspace K_a(A, r0)), as restarted GMRES:
 *       Arnoldi with modified Gram-Schmidt (one pass, or two: the second re-orthogonalises),
 *       Givens rotations on the Hessenberg matrix, restart on the true residual (Saad,
 *       Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 6.2, Alg. 6.9 and Section
 *       6.5.3).  The first cycle's orthonormal basis V and
 *       Hessenberg matrix are returned: that is the per-timestep seed basis V_a^n of Section 3,
 *       Phase 1.
 *   xo_project  -- Section 3, Phase 2: A_proj alpha = b_proj in the seed basis, x0 = V alpha.
 *   xo_accumulate  -- Krylov subspace expansion over an image cycle (Experiment 2: a new seed
 *       every 50 images, subspace dimension capped): the seeds' basis vectors, in order,
 *       orthogonalised against the vectors gathered so far and appended.
 *
 * Conventions: a grid is square (H == W, h = 1/H, Section 2.3 sets dx = dy = h); unknown
 * p = i*H + j with i the x (width) index and j the y (height) index; values outside the grid
 * are zero (zero padding).  Matrices are column-major unless stated.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Status codes (numeric values are part of the oracle's interface). */
#define XO_OK 0
#define XO_EINVAL 1
#define XO_ENOMEM 2
#define XO_ENOCONV 4
#define XO_ESINGULAR 5

/*
 * Planted-mistake switch for the pin-strength tests: 0 (the default) is the method as written.
 * 1: the sign of the linearised <grad m~, grad m> term is flipped in C_east/C_west/C_north/C_south.
 * 2: C_east and C_west are exchanged.
 * 3: h = 1/(H+1) instead of 1/H.
 * 4: the y-neighbour offset wraps across grid columns (the j boundary mask is dropped).
 * 5: the projected matrix is transposed (V^T A V read as its transpose).
 */
int xo_mutation = 0;

typedef struct {
    int H, W;
    double dt, g;
    const double *mt; /* lagged log-density m~, n values */
    const double *fx; /* drift x component, n values, or NULL for f = 0 */
    const double *fy; /* drift y component, n values, or NULL for f = 0 */
} xo_op;

typedef struct {
    int status, iters, restarts, basis_dim;
    double res_est, res_true;
} xo_info;

static double at(const double *a, int H, int W, int i, int j)
{
    if (a == NULL || i < 0 || i >= W || j < 0 || j >= H) return 0.0;
    return a[i * H + j];
}

static double grid_h(const xo_op *A)
{
    if (xo_mutation == 3) return 1.0 / (double)(A->H + 1);
    return 1.0 / (double)A->H;
}

/* Section 2.3: the five coefficients of row p = i*H + j. */
void xo_coeffs(const xo_op *A, double *cd, double *ce, double *cw, double *cn, double *cs)
{
    const int H = A->H, W = A->W;
    const double h = grid_h(A), g2 = A->g * A->g;
    const double sgn = (xo_mutation == 1) ? -1.0 : 1.0;
    for (int i = 0; i < W; ++i) {
        for (int j = 0; j < H; ++j) {
            const int p = i * H + j;
            const double dmx = at(A->mt, H, W, i + 1, j) - at(A->mt, H, W, i - 1, j);
            const double dmy = at(A->mt, H, W, i, j + 1) - at(A->mt, H, W, i, j - 1);
            const double fxp = at(A->fx, H, W, i, j);
            const double fyp = at(A->fy, H, W, i, j);
            double e, w;
            cd[p] = 1.0 / A->dt + 2.0 * g2 / (h * h);
            cn[p] = -g2 / (2.0 * h * h) + fyp / (2.0 * h) - sgn * g2 / (8.0 * h * h) * dmy;
            cs[p] = -g2 / (2.0 * h * h) - fyp / (2.0 * h) + sgn * g2 / (8.0 * h * h) * dmy;
            e = -g2 / (2.0 * h * h) + fxp / (2.0 * h) - sgn * g2 / (8.0 * h * h) * dmx;
            w = -g2 / (2.0 * h * h) - fxp / (2.0 * h) + sgn * g2 / (8.0 * h * h) * dmx;
            if (xo_mutation == 2) { double t = e; e = w; w = t; }
            ce[p] = e;
            cw[p] = w;
        }
    }
}

/* Section 2.3: b = m^{n-1}/dt - [(fx_{i+1,j} - fx_{i-1,j}) + (fy_{i,j+1} - fy_{i,j-1})]/(2h). */
void xo_rhs(const xo_op *A, const double *mprev, double *b)
{
    const int H = A->H, W = A->W;
    const double h = grid_h(A);
    for (int i = 0; i < W; ++i) {
        for (int j = 0; j < H; ++j) {
            const int p = i * H + j;
            const double div = (at(A->fx, H, W, i + 1, j) - at(A->fx, H, W, i - 1, j))
                             + (at(A->fy, H, W, i, j + 1) - at(A->fy, H, W, i, j - 1));
            b[p] = mprev[p] / A->dt - div / (2.0 * h);
        }
    }
}

/* y = A u, row by row: C_diag u_p + C_east u_{i+1,j} + C_west u_{i-1,j} + C_north u_{i,j+1}
 * + C_south u_{i,j-1}, neighbours outside the grid dropped (zero padding). */
void xo_apply(const xo_op *A, const double *u, double *y)
{
    const int H = A->H, W = A->W, n = H * W;
    double *c = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    double *cd = c, *ce = c + n, *cw = c + 2 * n, *cn = c + 3 * n, *cs = c + 4 * n;
    xo_coeffs(A, cd, ce, cw, cn, cs);
    for (int i = 0; i < W; ++i) {
        for (int j = 0; j < H; ++j) {
            const int p = i * H + j;
            double s = cd[p] * u[p];
            if (i + 1 < W) s += ce[p] * u[p + H];
            if (i >= 1) s += cw[p] * u[p - H];
            if (j + 1 < H || (xo_mutation == 4 && p + 1 < n)) s += cn[p] * u[p + 1];
            if (j >= 1 || (xo_mutation == 4 && p >= 1)) s += cs[p] * u[p - 1];
            y[p] = s;
        }
    }
    free(c);
}

/* The block-tridiagonal matrix of Section 2.3, dense, row-major: A[p*n + q]. */
void xo_dense(const xo_op *A, double *D)
{
    const int H = A->H, W = A->W, n = H * W;
    double *c = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    double *cd = c, *ce = c + n, *cw = c + 2 * n, *cn = c + 3 * n, *cs = c + 4 * n;
    xo_coeffs(A, cd, ce, cw, cn, cs);
    memset(D, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int i = 0; i < W; ++i) {
        for (int j = 0; j < H; ++j) {
            const int p = i * H + j;
            D[(size_t)p * n + p] = cd[p];
            if (i + 1 < W) D[(size_t)p * n + p + H] = ce[p];
            if (i >= 1) D[(size_t)p * n + p - H] = cw[p];
            if (j + 1 < H || (xo_mutation == 4 && p + 1 < n)) D[(size_t)p * n + p + 1] = cn[p];
            if (j >= 1 || (xo_mutation == 4 && p >= 1)) D[(size_t)p * n + p - 1] = cs[p];
        }
    }
    free(c);
}

/* Dense LU with partial pivoting; D is row-major n x n and is overwritten; the solution
 * overwrites b.  A pivot of magnitude <= 1e-13 * max|D| counts as zero: returns XO_ESINGULAR. */
int xo_lu_solve(int n, double *D, double *b)
{
    double amax = 0.0;
    for (long t = 0; t < (long)n * n; ++t) amax = fmax(amax, fabs(D[t]));
    if (amax == 0.0) return XO_ESINGULAR;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(D[(size_t)r * n + k]) > fabs(D[(size_t)piv * n + k])) piv = r;
        if (fabs(D[(size_t)piv * n + k]) <= 1e-13 * amax) return XO_ESINGULAR;
        if (piv != k) {
            for (int q = 0; q < n; ++q) {
                double t = D[(size_t)k * n + q];
                D[(size_t)k * n + q] = D[(size_t)piv * n + q];
                D[(size_t)piv * n + q] = t;
            }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            const double l = D[(size_t)r * n + k] / D[(size_t)k * n + k];
            D[(size_t)r * n + k] = 0.0;
            for (int q = k + 1; q < n; ++q) D[(size_t)r * n + q] -= l * D[(size_t)k * n + q];
            b[r] -= l * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int q = k + 1; q < n; ++q) s -= D[(size_t)k * n + q] * b[q];
        b[k] = s / D[(size_t)k * n + k];
    }
    return XO_OK;
}

/* Banded LU with partial pivoting for the stencil matrix: lower and upper bandwidth H; with row
 * exchanges the upper factor widens to 2H.  Row r stores columns r-H .. r+2H. */
int xo_banded_solve(const xo_op *A, const double *b, double *x)
{
    const int H = A->H, W = A->W, n = H * W;
    const int kl = H, ku = H, wd = 2 * kl + ku + 1;
    double *B = (double *)calloc((size_t)n * wd, sizeof(double));
    double *rhs = (double *)malloc(sizeof(double) * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    if (!B || !rhs || !c) { free(B); free(rhs); free(c); return XO_ENOMEM; }
    double *cd = c, *ce = c + n, *cw = c + 2 * n, *cn = c + 3 * n, *cs = c + 4 * n;
#define BND(r, q) B[(size_t)(r) * wd + ((q) - (r) + kl)]
    xo_coeffs(A, cd, ce, cw, cn, cs);
    for (int i = 0; i < W; ++i) {
        for (int j = 0; j < H; ++j) {
            const int p = i * H + j;
            BND(p, p) = cd[p];
            if (i + 1 < W) BND(p, p + H) = ce[p];
            if (i >= 1) BND(p, p - H) = cw[p];
            if (j + 1 < H) BND(p, p + 1) = cn[p];
            if (j >= 1) BND(p, p - 1) = cs[p];
        }
    }
    memcpy(rhs, b, sizeof(double) * (size_t)n);
    int status = XO_OK;
    for (int k = 0; k < n; ++k) {
        const int rlast = (k + kl < n - 1) ? k + kl : n - 1;
        const int qlast = (k + kl + ku < n - 1) ? k + kl + ku : n - 1;
        int piv = k;
        for (int r = k + 1; r <= rlast; ++r)
            if (fabs(BND(r, k)) > fabs(BND(piv, k))) piv = r;
        if (BND(piv, k) == 0.0) { status = XO_ESINGULAR; break; }
        if (piv != k) {
            for (int q = k; q <= qlast; ++q) {
                double t = BND(k, q); BND(k, q) = BND(piv, q); BND(piv, q) = t;
            }
            double t = rhs[k]; rhs[k] = rhs[piv]; rhs[piv] = t;
        }
        for (int r = k + 1; r <= rlast; ++r) {
            const double l = BND(r, k) / BND(k, k);
            if (l == 0.0) continue;
            BND(r, k) = 0.0;
            for (int q = k + 1; q <= qlast; ++q) BND(r, q) -= l * BND(k, q);
            rhs[r] -= l * rhs[k];
        }
    }
    if (status == XO_OK) {
        for (int k = n - 1; k >= 0; --k) {
            const int qlast = (k + kl + ku < n - 1) ? k + kl + ku : n - 1;
            double s = rhs[k];
            for (int q = k + 1; q <= qlast; ++q) s -= BND(k, q) * x[q];
            x[k] = s / BND(k, k);
        }
    }
#undef BND
    free(B); free(rhs); free(c);
    return status;
}

/* ---------------------------------------------------------------------------------------- */
/* Linear operator for GMRES: the stencil operator, or an explicit dense row-major matrix. */
typedef struct {
    int kind;            /* 0: stencil (op), 1: dense (dense, row-major n x n) */
    int n;
    const xo_op *op;
    const double *dense;
} xo_linop;

static void linop_apply(const xo_linop *L, const double *u, double *y)
{
    if (L->kind == 0) { xo_apply(L->op, u, y); return; }
    for (int p = 0; p < L->n; ++p) {
        double s = 0.0;
        for (int q = 0; q < L->n; ++q) s += L->dense[(size_t)p * L->n + q] * u[q];
        y[p] = s;
    }
}

static double dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int p = 0; p < n; ++p) s += a[p] * b[p];
    return s;
}

static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

double xo_residual_linop(const xo_linop *L, const double *b, const double *x)
{
    const int n = L->n;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    linop_apply(L, x, r);
    for (int p = 0; p < n; ++p) r[p] = b[p] - r[p];
    const double rn = nrm2(n, r), bn = nrm2(n, b);
    free(r);
    return bn > 0.0 ? rn / bn : rn;
}

/* ||b - A x||_2 / ||b||_2 for the stencil operator (||r||_2 when b = 0). */
double xo_residual(const xo_op *A, const double *b, const double *x)
{
    xo_linop L = {0, A->H * A->W, A, NULL};
    return xo_residual_linop(&L, b, x);
}

/*
 * Restarted GMRES(m) for A x = b; x holds x0 on entry and the result on exit.
 *   tol:          stop when ||b - A x||_2 <= tol ||b||_2 (true residual, checked at cycle end).
 *   max_restarts: number of restarts allowed after the first cycle (XO_ENOCONV beyond it).
 *   max_iters:    if > 0, caps the Arnoldi steps of each cycle below m (for exact-step tests).
 *   V1, H1:       if not NULL, receive the first cycle's basis V (n x (m+1), column-major,
 *                 ld n) and Hessenberg matrix (ld m+1, m columns, unrotated); info->basis_dim
 *                 is the number k of Arnoldi steps of that cycle.  Column k of V1 is the
 *                 normalised last Arnoldi vector, or zero after a breakdown.
 *   hist:         if not NULL, receives the Givens residual estimate after each step (up to
 *                 hist_cap values).
 *   passes:       modified Gram-Schmidt passes per Arnoldi step (1 or 2).
 * Arnoldi step j: w = A v_j; `passes` passes of modified Gram-Schmidt against v_0..v_j (Saad
 * Alg. 6.2; a second pass re-orthogonalises and adds to the same Hessenberg entries);
 * h_{j+1,j} = ||w||; breakdown when h_{j+1,j} <= 1e-14 ||A v_j||.
 */
int xo_gmres_linop(const xo_linop *L, const double *b, double *x, int m, int max_restarts,
                   double tol, int max_iters, int passes, double *V1, double *H1, xo_info *info,
                   double *hist, int hist_cap)
{
    const int n = L->n, ldh = m + 1;
    xo_info inf = {XO_OK, 0, 0, 0, 0.0, 0.0};
    const double bn = nrm2(n, b);
    if (V1) memset(V1, 0, sizeof(double) * (size_t)n * (m + 1));
    if (H1) memset(H1, 0, sizeof(double) * (size_t)ldh * m);
    if (bn == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        if (info) *info = inf;
        return XO_OK;
    }
    double *V = (double *)malloc(sizeof(double) * (size_t)n * (m + 1));
    double *Hb = (double *)malloc(sizeof(double) * (size_t)ldh * m);
    double *R = (double *)malloc(sizeof(double) * (size_t)ldh * m);
    double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
    double *gv = (double *)malloc(sizeof(double) * (m + 1)), *y = (double *)malloc(sizeof(double) * m);
    double *r = (double *)malloc(sizeof(double) * n), *w = (double *)malloc(sizeof(double) * n);
    int nh = 0, first = 1;

    linop_apply(L, x, r);
    for (int p = 0; p < n; ++p) r[p] = b[p] - r[p];
    double beta = nrm2(n, r);
    inf.res_true = beta / bn;
    inf.res_est = inf.res_true;
    if (beta <= tol * bn) goto done;

    for (;;) {
        for (int p = 0; p < n; ++p) V[p] = r[p] / beta;
        memset(gv, 0, sizeof(double) * (m + 1));
        memset(Hb, 0, sizeof(double) * (size_t)ldh * m);
        gv[0] = beta;
        int k = 0, steps = (max_iters > 0 && max_iters < m) ? max_iters : m;
        for (int j = 0; j < steps; ++j) {
            double *vj = V + (size_t)j * n, *hc = Hb + (size_t)j * ldh, *rc = R + (size_t)j * ldh;
            linop_apply(L, vj, w);
            inf.iters++;
            const double wn0 = nrm2(n, w);
            for (int pass = 0; pass < passes; ++pass) {
                for (int i = 0; i <= j; ++i) {
                    const double *vi = V + (size_t)i * n;
                    const double d = dot(n, w, vi);
                    hc[i] += d;
                    for (int p = 0; p < n; ++p) w[p] -= d * vi[p];
                }
            }
            const double hn = nrm2(n, w);
            hc[j + 1] = hn;
            const int breakdown = !(hn > 1e-14 * wn0);
            if (!breakdown)
                for (int p = 0; p < n; ++p) V[(size_t)(j + 1) * n + p] = w[p] / hn;
            else
                memset(V + (size_t)(j + 1) * n, 0, sizeof(double) * n);
            /* Givens: apply the previous rotations to column j, then make rotation j. */
            for (int i = 0; i <= j + 1; ++i) rc[i] = hc[i];
            for (int i = 0; i < j; ++i) {
                const double a = rc[i], c2 = rc[i + 1];
                rc[i] = cs[i] * a + sn[i] * c2;
                rc[i + 1] = -sn[i] * a + cs[i] * c2;
            }
            const double den = sqrt(rc[j] * rc[j] + rc[j + 1] * rc[j + 1]);
            cs[j] = rc[j] / den;
            sn[j] = rc[j + 1] / den;
            rc[j] = den;
            rc[j + 1] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            k = j + 1;
            inf.res_est = fabs(gv[j + 1]) / bn;
            if (hist && nh < hist_cap) hist[nh++] = inf.res_est;
            if (fabs(gv[j + 1]) <= tol * bn || breakdown) break;
        }
        /* y = R^{-1} g, x += V_k y */
        for (int i = k - 1; i >= 0; --i) {
            double s = gv[i];
            for (int c2 = i + 1; c2 < k; ++c2) s -= R[(size_t)c2 * ldh + i] * y[c2];
            y[i] = s / R[(size_t)i * ldh + i];
        }
        for (int i = 0; i < k; ++i)
            for (int p = 0; p < n; ++p) x[p] += y[i] * V[(size_t)i * n + p];
        if (first) {
            inf.basis_dim = k;
            if (V1) memcpy(V1, V, sizeof(double) * (size_t)n * (k + 1));
            if (H1)
                for (int c2 = 0; c2 < k; ++c2)
                    memcpy(H1 + (size_t)c2 * ldh, Hb + (size_t)c2 * ldh, sizeof(double) * ldh);
            first = 0;
        }
        linop_apply(L, x, r);
        for (int p = 0; p < n; ++p) r[p] = b[p] - r[p];
        beta = nrm2(n, r);
        inf.res_true = beta / bn;
        if (beta <= tol * bn) break;
        if (inf.restarts >= max_restarts || max_iters > 0) { inf.status = XO_ENOCONV; break; }
        inf.restarts++;
    }
done:
    if (info) *info = inf;
    free(V); free(Hb); free(R); free(cs); free(sn); free(gv); free(y); free(r); free(w);
    return inf.status;
}

int xo_gmres(const xo_op *A, const double *b, double *x, int m, int max_restarts, double tol,
             int max_iters, int passes, double *V1, double *H1, xo_info *info, double *hist,
             int hist_cap)
{
    xo_linop L = {0, A->H * A->W, A, NULL};
    return xo_gmres_linop(&L, b, x, m, max_restarts, tol, max_iters, passes, V1, H1, info, hist,
                          hist_cap);
}

int xo_gmres_dense(int n, const double *D, const double *b, double *x, int m, int max_restarts,
                   double tol, int max_iters, int passes, double *V1, double *H1, xo_info *info,
                   double *hist, int hist_cap)
{
    xo_linop L = {1, n, NULL, D};
    return xo_gmres_linop(&L, b, x, m, max_restarts, tol, max_iters, passes, V1, H1, info, hist,
                          hist_cap);
}

/* ---------------------------------------------------------------------------------------- */
/*
 * Section 3, Phase 2: project a target system A' x = b' onto the seed basis V_k and return
 * x0 = x_base + V_k alpha.
 *   mode 0 (target Galerkin): A_p = V_k^T (A' V_k), beta = V_k^T r_base, A_p alpha = beta.
 *   mode 1 (seed Galerkin):   A_p = H_k, the leading k x k block of the seed's Hessenberg matrix
 *                             (equal to V_k^T A_seed V_k by the Arnoldi relation) -- the matrix
 *                             the paper uses in place of the target's own.
 *   mode 2 (seed least squares): alpha minimises || V_{k+1}^T r_base - Hbar_k alpha ||_2.
 * r_base = b' - A' x_base (x_base NULL means zero).  V: n x (k+1), ld n; Hb: ld ldh.
 * Returns XO_ESINGULAR (and x0 = x_base, alpha = 0) when the k x k solve meets a zero pivot.
 */
int xo_project(const xo_op *At, const double *b, const double *x_base, int k, const double *V,
               const double *Hb, int ldh, int mode, double *x0, double *alpha)
{
    const int n = At->H * At->W;
    double *rb = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *Ap = (double *)malloc(sizeof(double) * (size_t)(k + 1) * (k + 1));
    double *z = (double *)malloc(sizeof(double) * (k + 1));
    int status = XO_OK;

    if (x_base) {
        xo_apply(At, x_base, w);
        for (int p = 0; p < n; ++p) rb[p] = b[p] - w[p];
    } else {
        memcpy(rb, b, sizeof(double) * n);
    }
    if (mode == 0) {
        for (int c = 0; c < k; ++c) {
            xo_apply(At, V + (size_t)c * n, w);
            for (int a = 0; a < k; ++a) {
                const double v = dot(n, V + (size_t)a * n, w);
                if (xo_mutation == 5) Ap[(size_t)c * k + a] = v; else Ap[(size_t)a * k + c] = v;
            }
        }
        for (int a = 0; a < k; ++a) z[a] = dot(n, V + (size_t)a * n, rb);
        status = xo_lu_solve(k, Ap, z);
    } else if (mode == 1) {
        for (int a = 0; a < k; ++a)
            for (int c = 0; c < k; ++c) Ap[(size_t)a * k + c] = Hb[(size_t)c * ldh + a];
        for (int a = 0; a < k; ++a) z[a] = dot(n, V + (size_t)a * n, rb);
        status = xo_lu_solve(k, Ap, z);
    } else if (mode == 2) {
        /* Givens QR of the (k+1) x k upper Hessenberg matrix, applied to z = V_{k+1}^T r_base. */
        for (int a = 0; a <= k; ++a) z[a] = dot(n, V + (size_t)a * n, rb);
        for (int a = 0; a <= k; ++a)
            for (int c = 0; c < k; ++c) Ap[(size_t)a * k + c] = Hb[(size_t)c * ldh + a];
        double amax = 0.0;
        for (int t = 0; t < (k + 1) * k; ++t) amax = fmax(amax, fabs(Ap[t]));
        for (int c = 0; c < k; ++c) {
            const double a0 = Ap[(size_t)c * k + c], a1 = Ap[(size_t)(c + 1) * k + c];
            const double den = sqrt(a0 * a0 + a1 * a1);
            if (den <= 1e-13 * amax) { status = XO_ESINGULAR; break; }
            const double cs = a0 / den, sn = a1 / den;
            for (int q = c; q < k; ++q) {
                const double u = Ap[(size_t)c * k + q], v = Ap[(size_t)(c + 1) * k + q];
                Ap[(size_t)c * k + q] = cs * u + sn * v;
                Ap[(size_t)(c + 1) * k + q] = -sn * u + cs * v;
            }
            const double u = z[c], v = z[c + 1];
            z[c] = cs * u + sn * v;
            z[c + 1] = -sn * u + cs * v;
        }
        if (status == XO_OK) {
            for (int a = k - 1; a >= 0; --a) {
                double s = z[a];
                for (int c = a + 1; c < k; ++c) s -= Ap[(size_t)a * k + c] * z[c];
                z[a] = s / Ap[(size_t)a * k + a];
            }
        }
    } else {
        status = XO_EINVAL;
    }
    for (int p = 0; p < n; ++p) x0[p] = x_base ? x_base[p] : 0.0;
    if (status == XO_OK) {
        for (int a = 0; a < k; ++a) {
            alpha[a] = z[a];
            for (int p = 0; p < n; ++p) x0[p] += z[a] * V[(size_t)a * n + p];
        }
    } else {
        for (int a = 0; a < k; ++a) alpha[a] = 0.0;
    }
    free(rb); free(w); free(Ap); free(z);
    return status;
}

/* ---------------------------------------------------------------------------------------- */
/*
 * Krylov subspace accumulation over an image cycle.  Sources s = 0..nsrc-1 in order; source s
 * holds ks[s] orthonormal columns (column-major, leading dimension n) at src[s].  Each source
 * column c = 0, 1, ... is made orthogonal to the columns gathered so far by two passes of
 * modified Gram-Schmidt (Saad Alg. 6.2, repeated); if the norm left exceeds 1e-8 the column is
 * normalised and appended.  At most per_source columns are appended from one source and cap in
 * total.  out: n x cap, column-major, ld n.  Returns the number of columns gathered.
 */
int xo_accumulate(int n, int nsrc, const double *const *src, const int *ks, int per_source,
                  int cap, double *out)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    int kd = 0;
    for (int s = 0; s < nsrc && kd < cap; ++s) {
        int taken = 0;
        for (int c = 0; c < ks[s] && taken < per_source && kd < cap; ++c) {
            memcpy(w, src[s] + (size_t)c * n, sizeof(double) * (size_t)n);
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i < kd; ++i) {
                    const double *vi = out + (size_t)i * n;
                    const double d = dot(n, w, vi);
                    for (int p = 0; p < n; ++p) w[p] -= d * vi[p];
                }
            const double nw = nrm2(n, w);
            if (nw > 1e-8) {
                for (int p = 0; p < n; ++p) out[(size_t)kd * n + p] = w[p] / nw;
                ++kd;
                ++taken;
            }
        }
    }
    free(w);
    return kd;
}
