/*
 * ORACLE — test infrastructure only.  A plain, slow, obviously correct FP64 CPU
 * implementation of the damped, smoothing-regularised LSQR solve.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code with the GPU library.
 *
 * Problem (the paper's eq. (6), Delta d = G Delta m, solved in the least-squares
 * sense; the paper names LSQR (Paige & Saunders 1982) among the solvers of its
 * "Solver for the Large-scale Linear System" section):
 *
 *     x* = argmin |G x - dt|^2 + w^2 |L x|^2 + lambda^2 |x|^2
 *
 * with the regularised operator written as three explicit row blocks
 *
 *     Abar = [ G ; w L ; lambda I ],   bbar = [ dt ; 0 ; 0 ],
 *
 * and an optional column scaling D (x = D y, A_D = Abar D).
 *
 * L is the 3-D 7-point Laplacian in index space on the (nx, ny, nz) grid whose
 * unknowns follow eq. (7) of the paper (depth fastest): unknown
 * p = (iy*nx + ix)*nz + iz.  Off-grid neighbours are dropped and the centre is
 * minus the number of in-grid neighbours, so L 1 = 0 and L is symmetric.
 *
 * LSQR here is Paige & Saunders' Golub-Kahan bidiagonalisation with one Givens
 * rotation per step (damping carried by the explicit lambda I block).  The
 * "implicit-damp" entry point eliminates lambda by an extra rotation instead,
 * as in Paige & Saunders' damped LSQR, for cross-checks only.
 *
 * Summation: every dot product and norm is a plain left-to-right sum; with
 * compensated != 0 the same sums use Neumaier's compensated summation, which
 * is how the oracle measures its own sensitivity to rounding order.
 *
 * Parallelism: rows of G are independent dot products, and so are columns of
 * G^T (computed from the oracle's own transpose, whose rows within a column are
 * ascending, i.e. the same order as a row-by-row scatter); threads split rows or
 * columns and never split a sum, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t m, n;
    int32_t nx, ny, nz;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
    double w;            /* smoothing weight */
    double damp;         /* lambda */
    const double *d;     /* column scale [n] or NULL (D = I) */
    int nthreads;
    int compensated;
    /* the oracle's own transpose of G */
    int64_t *ccol_ptr;
    int32_t *crow;
    double *cval;
} oracle_op;

/* ---------------------------------------------------------------- sums --- */
typedef struct { double s, c; } nsum;

static inline void nsum_add(nsum *a, double x, int comp)
{
    if (!comp) { a->s += x; return; }
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nsum_get(const nsum *a, int comp) { return comp ? a->s + a->c : a->s; }

static double norm2(const double *v, int64_t len, int comp)
{
    nsum a = {0.0, 0.0};
    for (int64_t i = 0; i < len; ++i) nsum_add(&a, v[i] * v[i], comp);
    return sqrt(nsum_get(&a, comp));
}

/* ------------------------------------------------------------ transpose --- */
int oracle_transpose(oracle_op *op)
{
    int64_t m = op->m, n = op->n, nnz = op->row_ptr[m];
    op->ccol_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    op->crow = (int32_t *)malloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
    op->cval = (double *)malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!op->ccol_ptr || !op->crow || !op->cval || !fill) { free(fill); return -1; }
    for (int64_t e = 0; e < nnz; ++e) op->ccol_ptr[op->col[e] + 1]++;
    for (int64_t j = 0; j < n; ++j) op->ccol_ptr[j + 1] += op->ccol_ptr[j];
    memcpy(fill, op->ccol_ptr, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = op->row_ptr[i]; e < op->row_ptr[i + 1]; ++e) {
            int64_t pos = fill[op->col[e]]++;
            op->crow[pos] = (int32_t)i;
            op->cval[pos] = op->val[e];
        }
    free(fill);
    return 0;
}

void oracle_free(oracle_op *op)
{
    free(op->ccol_ptr); free(op->crow); free(op->cval);
    op->ccol_ptr = NULL; op->crow = NULL; op->cval = NULL;
}

/* ------------------------------------------------------------ Laplacian --- */
/* y = L x on the (nx, ny, nz) grid, unknown p = (iy*nx + ix)*nz + iz. */
void oracle_laplacian(int32_t nx, int32_t ny, int32_t nz, const double *x, double *y, int nthreads)
{
    int64_t n = (int64_t)nx * ny * nz;
    #pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int64_t iz = p % nz, ixy = p / nz, ix = ixy % nx, iy = ixy / nx;
        double acc = 0.0;
        int deg = 0;
        /* neighbours in a fixed order: -x, +x, -y, +y, -z, +z */
        if (ix > 0)      { acc += x[p - nz]; ++deg; }
        if (ix < nx - 1) { acc += x[p + nz]; ++deg; }
        if (iy > 0)      { acc += x[p - (int64_t)nx * nz]; ++deg; }
        if (iy < ny - 1) { acc += x[p + (int64_t)nx * nz]; ++deg; }
        if (iz > 0)      { acc += x[p - 1]; ++deg; }
        if (iz < nz - 1) { acc += x[p + 1]; ++deg; }
        y[p] = acc - (double)deg * x[p];
    }
}

/* ------------------------------------------------------------- operator --- */
/* y[0:m] = G (D x), y[m:m+n] = w L (D x), y[m+n:m+2n] = lambda (D x).
 * ybar has m + 2n entries; scratch has n entries. */
void oracle_apply(const oracle_op *op, const double *x, double *ybar, double *scratch)
{
    int64_t m = op->m, n = op->n;
    const double *z = x;
    if (op->d) {
        for (int64_t j = 0; j < n; ++j) scratch[j] = op->d[j] * x[j];
        z = scratch;
    }
    int comp = op->compensated;
    #pragma omp parallel for num_threads(op->nthreads) schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        nsum a = {0.0, 0.0};
        for (int64_t e = op->row_ptr[i]; e < op->row_ptr[i + 1]; ++e)
            nsum_add(&a, op->val[e] * z[op->col[e]], comp);
        ybar[i] = nsum_get(&a, comp);
    }
    oracle_laplacian(op->nx, op->ny, op->nz, z, ybar + m, op->nthreads);
    for (int64_t j = 0; j < n; ++j) ybar[m + j] *= op->w;
    for (int64_t j = 0; j < n; ++j) ybar[m + n + j] = op->damp * z[j];
}

/* x = D (G^T yG + w L^T yL + lambda yD), with L^T = L.  scratch has n entries. */
void oracle_apply_t(const oracle_op *op, const double *ybar, double *x, double *scratch)
{
    int64_t m = op->m, n = op->n;
    int comp = op->compensated;
    oracle_laplacian(op->nx, op->ny, op->nz, ybar + m, scratch, op->nthreads);
    #pragma omp parallel for num_threads(op->nthreads) schedule(dynamic, 64)
    for (int64_t j = 0; j < n; ++j) {
        nsum a = {0.0, 0.0};
        for (int64_t e = op->ccol_ptr[j]; e < op->ccol_ptr[j + 1]; ++e)
            nsum_add(&a, op->cval[e] * ybar[op->crow[e]], comp);
        double g = nsum_get(&a, comp);
        double s = g + op->w * scratch[j] + op->damp * ybar[m + n + j];
        x[j] = op->d ? op->d[j] * s : s;
    }
}

/* ------------------------------------------------------------ Jacobi ------ */
/* d_j = 1 / |abar_j|, the norm of column j of the full operator:
 * sum_i g_ij^2 + w^2 sum_p L_pj^2 + lambda^2, where column j of L has the
 * centre -deg_j and deg_j ones. */
void oracle_jacobi(const oracle_op *op, double *d)
{
    int64_t n = op->n;
    for (int64_t j = 0; j < n; ++j) {
        int64_t iz = j % op->nz, ixy = j / op->nz, ix = ixy % op->nx, iy = ixy / op->nx;
        int deg = (ix > 0) + (ix < op->nx - 1) + (iy > 0) + (iy < op->ny - 1) + (iz > 0) + (iz < op->nz - 1);
        nsum a = {0.0, 0.0};
        for (int64_t e = op->ccol_ptr[j]; e < op->ccol_ptr[j + 1]; ++e)
            nsum_add(&a, op->cval[e] * op->cval[e], op->compensated);
        double lsq = (double)deg * (double)deg + (double)deg;
        double s = nsum_get(&a, op->compensated) + op->w * op->w * lsq + op->damp * op->damp;
        d[j] = 1.0 / sqrt(s);
    }
}

/* --------------------------------------------------------------- LSQR ----- */
/*
 * Explicit-block LSQR on A_D = Abar D.
 *   b      [m]   data right-hand side dt (bbar = [dt; 0; 0])
 *   iters        maximum number of iterations K (forward products)
 *   tol          stop when eta_k <= tol (tol <= 0: run K iterations)
 *   x      [n]   output: x = D y_k
 *   hist   [3*(K+1)] or NULL: row k = (phibar_{k+1}, psi_k, eta_k); row 0 is
 *                the start: (beta_1, alpha_1 beta_1, 1)
 *   info   [2]   output: istop, iterations done
 *   ucap, vcap   NULL or buffers of ncap*(m+2n) and ncap*n doubles receiving
 *                u_1..u_ncap and v_1..v_ncap (orthogonality tests)
 * Returns 0, or -3 when a scalar became non-finite, or -5 on allocation failure.
 *
 * istop: 0 bbar = 0 or Abar^T bbar = 0 (x = 0); 1 eta <= tol; 2 iteration
 * limit; 3 exact breakdown (alpha or beta = 0); 5 eta stagnated
 * (oracle_lsqr_ref only).
 */
static int lsqr_core(const oracle_op *op, const double *b, int iters, double tol, double *x,
                     double *hist, int32_t *info, double *ucap, double *vcap, int ncap,
                     double snap_tol, double *xsnap, int32_t *ksnap, int stall)
{
    int64_t m = op->m, n = op->n, mb = m + 2 * n;
    int comp = op->compensated;
    double *u = (double *)calloc((size_t)mb, sizeof(double));
    double *t = (double *)calloc((size_t)mb, sizeof(double));
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *q = (double *)calloc((size_t)n, sizeof(double));
    double *wv = (double *)calloc((size_t)n, sizeof(double));
    double *y = (double *)calloc((size_t)n, sizeof(double));
    double *sc = (double *)calloc((size_t)n, sizeof(double));
    double *dv = (double *)calloc((size_t)n, sizeof(double));
    int rc = 0;
    if (!u || !t || !v || !q || !wv || !y || !sc || !dv) { rc = -5; goto done; }
    info[0] = 0; info[1] = 0;
    for (int64_t j = 0; j < n; ++j) x[j] = 0.0;

    /* step 1: beta_1 u_1 = bbar */
    for (int64_t i = 0; i < m; ++i) u[i] = b[i];
    double beta = norm2(u, mb, comp);
    if (!isfinite(beta)) { rc = -3; goto done; }
    if (beta == 0.0) { if (hist) { hist[0] = 0.0; hist[1] = 0.0; hist[2] = 0.0; } goto done; }
    for (int64_t i = 0; i < mb; ++i) u[i] = u[i] / beta;

    /* step 2: alpha_1 v_1 = A_D^T u_1 */
    oracle_apply_t(op, u, q, sc);
    double alpha = norm2(q, n, comp);
    if (!isfinite(alpha)) { rc = -3; goto done; }
    if (alpha == 0.0) { if (hist) { hist[0] = beta; hist[1] = 0.0; hist[2] = 0.0; } goto done; }
    for (int64_t j = 0; j < n; ++j) v[j] = q[j] / alpha;
    for (int64_t j = 0; j < n; ++j) wv[j] = v[j];
    if (ucap && ncap > 0) memcpy(ucap, u, (size_t)mb * sizeof(double));
    if (vcap && ncap > 0) memcpy(vcap, v, (size_t)n * sizeof(double));
    double phibar = beta, rhobar = alpha;
    for (int64_t j = 0; j < n; ++j) dv[j] = op->d ? v[j] / op->d[j] : v[j];
    double arnorm0 = alpha * beta * norm2(dv, n, comp);     /* |Abar^T bbar| */
    if (hist) { hist[0] = phibar; hist[1] = alpha * beta; hist[2] = 1.0; }
    info[0] = 2;
    double eta_best = 1.0;
    int k_best = 0;

    for (int k = 1; k <= iters; ++k) {
        /* step 3.1: beta u = A_D v - alpha u */
        oracle_apply(op, v, t, sc);
        for (int64_t i = 0; i < mb; ++i) t[i] = t[i] - alpha * u[i];
        beta = norm2(t, mb, comp);
        if (!isfinite(beta)) { rc = -3; goto done; }
        if (beta > 0.0) {
            for (int64_t i = 0; i < mb; ++i) u[i] = t[i] / beta;
            /* step 3.2: alpha v = A_D^T u - beta v */
            oracle_apply_t(op, u, q, sc);
            for (int64_t j = 0; j < n; ++j) q[j] = q[j] - beta * v[j];
            alpha = norm2(q, n, comp);
            if (!isfinite(alpha)) { rc = -3; goto done; }
            if (alpha > 0.0) for (int64_t j = 0; j < n; ++j) v[j] = q[j] / alpha;
        } else {
            alpha = 0.0;
        }
        if (ucap && k < ncap) memcpy(ucap + (size_t)k * mb, u, (size_t)mb * sizeof(double));
        if (vcap && k < ncap) memcpy(vcap + (size_t)k * n, v, (size_t)n * sizeof(double));
        /* step 3.3: plane rotation */
        double rho = sqrt(rhobar * rhobar + beta * beta);
        double c = rhobar / rho;
        double s = beta / rho;
        double theta = s * alpha;
        rhobar = -c * alpha;
        double phi = c * phibar;
        phibar = s * phibar;
        /* step 3.4: update y and w */
        double t1 = phi / rho;
        double t2 = theta / rho;
        for (int64_t j = 0; j < n; ++j) y[j] = y[j] + t1 * wv[j];
        for (int64_t j = 0; j < n; ++j) wv[j] = v[j] - t2 * wv[j];
        /* step 3.5: estimates */
        double psi = phibar * alpha * fabs(c);
        for (int64_t j = 0; j < n; ++j) dv[j] = op->d ? v[j] / op->d[j] : v[j];
        double eta = psi * norm2(dv, n, comp) / arnorm0;
        if (hist) { hist[3 * k] = phibar; hist[3 * k + 1] = psi; hist[3 * k + 2] = eta; }
        info[1] = k;
        if (!isfinite(rho) || !isfinite(phi)) { rc = -3; goto done; }
        /* snapshot: the first iterate whose eta reaches snap_tol, as x = D y */
        if (xsnap && *ksnap < 0 && eta <= snap_tol) {
            for (int64_t j = 0; j < n; ++j) xsnap[j] = op->d ? op->d[j] * y[j] : y[j];
            *ksnap = k;
        }
        if (tol > 0.0 && eta <= tol) { info[0] = 1; break; }
        if (alpha == 0.0 || beta == 0.0) { info[0] = 3; break; }
        /* stagnation: no new smallest eta over the last `stall` iterations */
        if (eta < eta_best) { eta_best = eta; k_best = k; }
        if (stall > 0 && k - k_best >= stall) { info[0] = 5; break; }
    }
    /* step 4: x = D y */
    for (int64_t j = 0; j < n; ++j) x[j] = op->d ? op->d[j] * y[j] : y[j];
done:
    free(u); free(t); free(v); free(q); free(wv); free(y); free(sc); free(dv);
    return rc;
}

int oracle_lsqr(const oracle_op *op, const double *b, int iters, double tol, double *x,
                double *hist, int32_t *info, double *ucap, double *vcap, int ncap)
{
    return lsqr_core(op, b, iters, tol, x, hist, info, ucap, vcap, ncap, 0.0, NULL, NULL, 0);
}

/*
 * The same iteration, run towards a converged reference: besides stopping at
 * eta <= tol it keeps a copy of the first iterate with eta <= snap_tol
 * (xsnap [n], its iteration in *ksnap, -1 if never reached) and stops with
 * istop 5 when no new smallest eta has appeared for `stall` iterations
 * (0 = never).  The arithmetic is that of oracle_lsqr.
 */
int oracle_lsqr_ref(const oracle_op *op, const double *b, int iters, double tol, double *x,
                    double *hist, int32_t *info, double snap_tol, double *xsnap, int32_t *ksnap,
                    int stall)
{
    *ksnap = -1;
    return lsqr_core(op, b, iters, tol, x, hist, info, NULL, NULL, 0, snap_tol, xsnap, ksnap,
                     stall);
}

/*
 * Implicit-damp LSQR (test mode): operator [G; w L] (m + n rows), damp lambda
 * removed by an extra rotation each step.  No column scaling.  Generates the
 * same iterates as the explicit-block form in exact arithmetic, because
 * K_k(A^T A + lambda^2 I, A^T b) = K_k(A^T A, A^T b).
 */
int oracle_lsqr_implicit(const oracle_op *op, const double *b, int iters, double *x)
{
    int64_t m = op->m, n = op->n, mb = m + 2 * n;   /* last n rows kept at zero */
    int comp = op->compensated;
    oracle_op o2 = *op;
    o2.damp = 0.0;
    o2.d = NULL;
    double *u = (double *)calloc((size_t)mb, sizeof(double));
    double *t = (double *)calloc((size_t)mb, sizeof(double));
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *q = (double *)calloc((size_t)n, sizeof(double));
    double *wv = (double *)calloc((size_t)n, sizeof(double));
    double *sc = (double *)calloc((size_t)n, sizeof(double));
    int rc = 0;
    if (!u || !t || !v || !q || !wv || !sc) { rc = -5; goto done; }
    for (int64_t j = 0; j < n; ++j) x[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) u[i] = b[i];
    double beta = norm2(u, mb, comp);
    if (beta == 0.0) goto done;
    for (int64_t i = 0; i < mb; ++i) u[i] = u[i] / beta;
    oracle_apply_t(&o2, u, q, sc);
    double alpha = norm2(q, n, comp);
    if (alpha == 0.0) goto done;
    for (int64_t j = 0; j < n; ++j) v[j] = q[j] / alpha;
    for (int64_t j = 0; j < n; ++j) wv[j] = v[j];
    double phibar = beta, rhobar = alpha, lam = op->damp;
    for (int k = 1; k <= iters; ++k) {
        oracle_apply(&o2, v, t, sc);
        for (int64_t i = 0; i < mb; ++i) t[i] = t[i] - alpha * u[i];
        beta = norm2(t, mb, comp);
        if (beta > 0.0) {
            for (int64_t i = 0; i < mb; ++i) u[i] = t[i] / beta;
            oracle_apply_t(&o2, u, q, sc);
            for (int64_t j = 0; j < n; ++j) q[j] = q[j] - beta * v[j];
            alpha = norm2(q, n, comp);
            if (alpha > 0.0) for (int64_t j = 0; j < n; ++j) v[j] = q[j] / alpha;
        } else {
            alpha = 0.0;
        }
        /* eliminate the damping */
        double rhohat = sqrt(rhobar * rhobar + lam * lam);
        double chat = rhobar / rhohat;
        phibar = chat * phibar;
        /* plane rotation */
        double rho = sqrt(rhohat * rhohat + beta * beta);
        double c = rhohat / rho;
        double s = beta / rho;
        double theta = s * alpha;
        rhobar = -c * alpha;
        double phi = c * phibar;
        phibar = s * phibar;
        double t1 = phi / rho, t2 = theta / rho;
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + t1 * wv[j];
        for (int64_t j = 0; j < n; ++j) wv[j] = v[j] - t2 * wv[j];
        if (alpha == 0.0 || beta == 0.0) break;
    }
done:
    free(u); free(t); free(v); free(q); free(wv); free(sc);
    return rc;
}
