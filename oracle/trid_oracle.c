/*
 * trid_oracle.c -- the CPU oracle: plain, slow, obviously correct FP64 code.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  The HIP library never links,
 * includes or calls it, and it shares no code with the HIP library.
 *
 * What it computes (arxiv 2201.03950, "High Throughput Multidimensional
 * Tridiagonal Systems Solvers on FPGAs"):
 *   - the tridiagonal system of eqs. (1)-(2), a_i u_{i-1} + b_i u_i + c_i u_{i+1} = d_i,
 *     with a_0 = c_{N-1} = 0, solved by the Thomas algorithm (Alg. 1) per line;
 *   - the line systems of a multi-dimensional mesh (Section II-B): the lines
 *     of one axis of a column-major (x contiguous) mesh, batch outermost;
 *   - PCR (Alg. 2) and the tiled "modified Thomas" of eq. (7) as test-only
 *     cross-checks of the same solution;
 *   - the ADI heat-diffusion step of Alg. 3 (RHS from the explicit stencil, a
 *     solve along x, y and z, then u += d), read as the Douglas delta form;
 *   - the adjoint of the line solve and of one ADI step (not in the paper: the
 *     reverse-mode derivative of the same computation).
 *
 * Readings of the paper that this file fixes:
 *   R1 eq. (1) right-hand side is d_i;
 *   R2 Alg. 1 leaves u_{N-1} implicit: u_{N-1} = d*_{N-1};
 *   R3 c_{N-1} and a_0 are never read (treated as 0);
 *   R4 Alg. 2 normalises rows to b = 1 first, out-of-range neighbours
 *      contribute a = c = d = 0, and each level reads only the previous level;
 *   R5 Alg. 3's coefficients: a = c = -s, b = 1 + 2s, RHS d = 2 s L u with L the
 *      7-point (3D) / 5-point (2D) Laplacian with zero ghost values, s per point
 *      or constant;
 *   R6 sweep order x, then y, then z.
 *
 * Index convention: a mesh with dims[0..ndim) (dims[0] fastest) and `batch`
 * meshes; line (inner index i, outer index o) of axis `ax` starts at
 * o*n*inner + i and has element stride inner = prod(dims[0..ax)).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef long idx_t;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Line geometry of axis `ax`: number of lines, length, stride. */
static void line_geom(int ndim, const idx_t *dims, int ax, idx_t batch, idx_t *inner, idx_t *n,
                      idx_t *outer) {
    idx_t in = 1, out = batch;
    for (int k = 0; k < ax; ++k) in *= dims[k];
    for (int k = ax + 1; k < ndim; ++k) out *= dims[k];
    *inner = in;
    *n = dims[ax];
    *outer = out;
}

static idx_t mesh_points(int ndim, const idx_t *dims, idx_t batch) {
    idx_t p = batch;
    for (int k = 0; k < ndim; ++k) p *= dims[k];
    return p;
}

/* ---------------------------------------------------------------------------
 * Alg. 1 (Thomas) on one line: d is overwritten with the solution.
 * cs, ds: scratch of length n for c* and d*.
 * ------------------------------------------------------------------------- */
static void thomas_line(idx_t n, const double *a, const double *b, const double *c, double *d,
                        idx_t st, double *cs, double *ds) {
    /* first row: c*_0 = c_0 / b_0, d*_0 = d_0 / b_0 (a_0 never read) */
    double c0 = (n > 1) ? c[0] : 0.0;
    cs[0] = c0 / b[0];
    ds[0] = d[0] / b[0];
    for (idx_t i = 1; i < n; ++i) {
        double ai = a[i * st];
        double ci = (i < n - 1) ? c[i * st] : 0.0; /* c_{N-1} is treated as 0 */
        double r = 1.0 / (b[i * st] - ai * cs[i - 1]);
        ds[i] = r * (d[i * st] - ai * ds[i - 1]);
        cs[i] = r * ci;
    }
    /* back substitution: u_{N-1} = d*_{N-1}, then u_i = d*_i - c*_i u_{i+1} */
    d[(n - 1) * st] = ds[n - 1];
    for (idx_t i = n - 2; i >= 0; --i) d[i * st] = ds[i] - cs[i] * d[(i + 1) * st];
}

/* Same algorithm, every operation in binary32 (reference for the unrefined FP32 error). */
static void thomas_line_f32(idx_t n, const float *a, const float *b, const float *c, float *d,
                            idx_t st, float *cs, float *ds) {
    float c0 = (n > 1) ? c[0] : 0.0f;
    cs[0] = c0 / b[0];
    ds[0] = d[0] / b[0];
    for (idx_t i = 1; i < n; ++i) {
        float ai = a[i * st];
        float ci = (i < n - 1) ? c[i * st] : 0.0f;
        float r = 1.0f / (b[i * st] - ai * cs[i - 1]);
        ds[i] = r * (d[i * st] - ai * ds[i - 1]);
        cs[i] = r * ci;
    }
    d[(n - 1) * st] = ds[n - 1];
    for (idx_t i = n - 2; i >= 0; --i) d[i * st] = ds[i] - cs[i] * d[(i + 1) * st];
}

/* Solve every line of axis `ax` (Section II-B).  d in/out. */
int orc_gtsv(const double *a, const double *b, const double *c, double *d, int ndim,
             const idx_t *dims, int ax, idx_t batch) {
    if (ndim < 1 || ndim > 3 || ax < 0 || ax >= ndim || batch < 1) return 1;
    idx_t inner, n, outer;
    line_geom(ndim, dims, ax, batch, &inner, &n, &outer);
    if (n < 1) return 1;
    idx_t nlines = inner * outer;
#pragma omp parallel
    {
        double *cs = (double *)malloc(sizeof(double) * (size_t)n);
        double *ds = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (idx_t l = 0; l < nlines; ++l) {
            idx_t o = l / inner, i = l % inner;
            idx_t base = o * n * inner + i;
            thomas_line(n, a + base, b + base, c + base, d + base, inner, cs, ds);
        }
        free(cs);
        free(ds);
    }
    return 0;
}

int orc_gtsv_f32(const float *a, const float *b, const float *c, float *d, int ndim,
                 const idx_t *dims, int ax, idx_t batch) {
    if (ndim < 1 || ndim > 3 || ax < 0 || ax >= ndim || batch < 1) return 1;
    idx_t inner, n, outer;
    line_geom(ndim, dims, ax, batch, &inner, &n, &outer);
    if (n < 1) return 1;
    idx_t nlines = inner * outer;
#pragma omp parallel
    {
        float *cs = (float *)malloc(sizeof(float) * (size_t)n);
        float *ds = (float *)malloc(sizeof(float) * (size_t)n);
#pragma omp for schedule(static)
        for (idx_t l = 0; l < nlines; ++l) {
            idx_t o = l / inner, i = l % inner;
            idx_t base = o * n * inner + i;
            thomas_line_f32(n, a + base, b + base, c + base, d + base, inner, cs, ds);
        }
        free(cs);
        free(ds);
    }
    return 0;
}

/* Packed systems of different lengths: system k occupies [off[k], off[k+1]). */
int orc_gtsv_varlen(const double *a, const double *b, const double *c, double *d,
                    const idx_t *off, idx_t nsys) {
    idx_t nmax = 0;
    for (idx_t k = 0; k < nsys; ++k) {
        if (off[k + 1] - off[k] < 1) return 1;
        if (off[k + 1] - off[k] > nmax) nmax = off[k + 1] - off[k];
    }
#pragma omp parallel
    {
        double *cs = (double *)malloc(sizeof(double) * (size_t)(nmax > 0 ? nmax : 1));
        double *ds = (double *)malloc(sizeof(double) * (size_t)(nmax > 0 ? nmax : 1));
#pragma omp for schedule(dynamic, 16)
        for (idx_t k = 0; k < nsys; ++k) {
            idx_t s = off[k];
            thomas_line(off[k + 1] - s, a + s, b + s, c + s, d + s, 1, cs, ds);
        }
        free(cs);
        free(ds);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Alg. 2 (PCR) on one contiguous line, test-only.  On return d holds the
 * solution and a, c hold the level-P coefficients (exact zeros, by the method).
 * Rows are first normalised so that b = 1 (reading R4).
 * ------------------------------------------------------------------------- */
int orc_pcr_line(idx_t n, double *a, double *b, double *c, double *d) {
    if (n < 1) return 1;
    double *a2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *c2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *d2 = (double *)malloc(sizeof(double) * (size_t)n);
    a[0] = 0.0;
    c[n - 1] = 0.0;
    for (idx_t i = 0; i < n; ++i) {
        a[i] /= b[i];
        c[i] /= b[i];
        d[i] /= b[i];
        b[i] = 1.0;
    }
    int P = 0;
    while (((idx_t)1 << P) < n) ++P;
    for (int p = 1; p <= P; ++p) {
        idx_t s = (idx_t)1 << (p - 1);
        for (idx_t i = 0; i < n; ++i) {
            double am = (i - s >= 0) ? a[i - s] : 0.0, cm = (i - s >= 0) ? c[i - s] : 0.0;
            double dm = (i - s >= 0) ? d[i - s] : 0.0;
            double ap = (i + s < n) ? a[i + s] : 0.0, cp = (i + s < n) ? c[i + s] : 0.0;
            double dp = (i + s < n) ? d[i + s] : 0.0;
            double r = 1.0 / (1.0 - a[i] * cm - c[i] * ap);
            a2[i] = -r * (a[i] * am);
            c2[i] = -r * (c[i] * cp);
            d2[i] = r * (d[i] - a[i] * dm - c[i] * dp);
        }
        memcpy(a, a2, sizeof(double) * (size_t)n);
        memcpy(c, c2, sizeof(double) * (size_t)n);
        memcpy(d, d2, sizeof(double) * (size_t)n);
    }
    free(a2);
    free(c2);
    free(d2);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Tiled "modified Thomas" (eq. (7), Section III-B), test-only.  The line is cut
 * into tiles of m >= 3 rows (the last tile is padded with identity rows).  In
 * each tile every interior unknown is written in terms of the tile's first and
 * last unknowns; those 2*t unknowns form a tridiagonal reduced system, solved
 * here with Alg. 1, after which the interior unknowns are substituted back.
 * ------------------------------------------------------------------------- */
int orc_tiled_thomas_line(idx_t n, const double *a, const double *b, const double *c, double *d,
                          idx_t m) {
    if (n < 1 || m < 3) return 1;
    idx_t t = (n + m - 1) / m, np = t * m;
    double *A = (double *)calloc((size_t)np, sizeof(double));
    double *B = (double *)calloc((size_t)np, sizeof(double));
    double *C = (double *)calloc((size_t)np, sizeof(double));
    double *D = (double *)calloc((size_t)np, sizeof(double));
    double *ap = (double *)calloc((size_t)np, sizeof(double));
    double *cp = (double *)calloc((size_t)np, sizeof(double));
    double *dp = (double *)calloc((size_t)np, sizeof(double));
    idx_t nr = 2 * t;
    double *ra = (double *)calloc((size_t)nr, sizeof(double));
    double *rb = (double *)calloc((size_t)nr, sizeof(double));
    double *rc = (double *)calloc((size_t)nr, sizeof(double));
    double *rd = (double *)calloc((size_t)nr, sizeof(double));
    double *cs = (double *)calloc((size_t)nr, sizeof(double));
    double *ds = (double *)calloc((size_t)nr, sizeof(double));
    for (idx_t i = 0; i < np; ++i) { /* identity padding beyond the line */
        A[i] = (i < n && i > 0) ? a[i] : 0.0;
        B[i] = (i < n) ? b[i] : 1.0;
        C[i] = (i < n - 1) ? c[i] : 0.0;
        D[i] = (i < n) ? d[i] : 0.0;
    }
    for (idx_t p = 0; p < t; ++p) {
        idx_t o = p * m;
        /* forward: rows 1.. expressed as a'_k u_0 + u_k + c'_k u_{k+1} = d'_k */
        ap[o + 1] = A[o + 1] / B[o + 1];
        cp[o + 1] = C[o + 1] / B[o + 1];
        dp[o + 1] = D[o + 1] / B[o + 1];
        for (idx_t k = 2; k < m; ++k) {
            double r = 1.0 / (B[o + k] - A[o + k] * cp[o + k - 1]);
            ap[o + k] = -r * A[o + k] * ap[o + k - 1];
            cp[o + k] = r * C[o + k];
            dp[o + k] = r * (D[o + k] - A[o + k] * dp[o + k - 1]);
        }
        /* backward: rows m-3..1 expressed as a'_k u_0 + u_k + c'_k u_{m-1} = d'_k (eq. (7)) */
        for (idx_t k = m - 3; k >= 1; --k) {
            dp[o + k] = dp[o + k] - cp[o + k] * dp[o + k + 1];
            ap[o + k] = ap[o + k] - cp[o + k] * ap[o + k + 1];
            cp[o + k] = -cp[o + k] * cp[o + k + 1];
        }
        /* reduced rows: the tile's first row (after eliminating u_1) and last row */
        ra[2 * p] = A[o];
        rb[2 * p] = B[o] - C[o] * ap[o + 1];
        rc[2 * p] = -C[o] * cp[o + 1];
        rd[2 * p] = D[o] - C[o] * dp[o + 1];
        ra[2 * p + 1] = ap[o + m - 1];
        rb[2 * p + 1] = 1.0;
        rc[2 * p + 1] = cp[o + m - 1];
        rd[2 * p + 1] = dp[o + m - 1];
    }
    thomas_line(nr, ra, rb, rc, rd, 1, cs, ds);
    for (idx_t p = 0; p < t; ++p) {
        idx_t o = p * m;
        double u0 = rd[2 * p], ul = rd[2 * p + 1];
        for (idx_t k = 0; k < m; ++k) {
            idx_t g = o + k;
            double u = (k == 0) ? u0 : (k == m - 1) ? ul : dp[g] - ap[g] * u0 - cp[g] * ul;
            if (g < n) d[g] = u;
        }
    }
    free(A); free(B); free(C); free(D); free(ap); free(cp); free(dp);
    free(ra); free(rb); free(rc); free(rd); free(cs); free(ds);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Laplacian with zero ghost values: (L u)_p = sum of the 2*ndim neighbours
 * minus 2*ndim*u_p (7-point in 3D, 5-point in 2D).  L is symmetric.
 * ------------------------------------------------------------------------- */
int orc_laplacian(const double *u, double *out, int ndim, const idx_t *dims, idx_t batch) {
    if (ndim < 1 || ndim > 3 || batch < 1) return 1;
    idx_t n[3] = {1, 1, 1};
    for (int k = 0; k < ndim; ++k) n[k] = dims[k];
    idx_t sx = 1, sy = n[0], sz = n[0] * n[1], sm = n[0] * n[1] * n[2];
    idx_t total = sm * batch;
#pragma omp parallel for schedule(static)
    for (idx_t p = 0; p < total; ++p) {
        idx_t i = p % n[0], j = (p / sy) % n[1], k = (p / sz) % n[2];
        double acc = -2.0 * ndim * u[p];
        acc += (i > 0) ? u[p - sx] : 0.0;
        acc += (i < n[0] - 1) ? u[p + sx] : 0.0;
        if (ndim >= 2) {
            acc += (j > 0) ? u[p - sy] : 0.0;
            acc += (j < n[1] - 1) ? u[p + sy] : 0.0;
        }
        if (ndim >= 3) {
            acc += (k > 0) ? u[p - sz] : 0.0;
            acc += (k < n[2] - 1) ? u[p + sz] : 0.0;
        }
        out[p] = acc;
    }
    return 0;
}

/* Coefficient arrays of the implicit operator I - s*D2 along any axis:
 * a = c = -s, b = 1 + 2s (reading R5); s per point or the constant s0. */
static void implicit_coefs(const double *s, double s0, idx_t total, double *a, double *b,
                           double *c) {
    for (idx_t p = 0; p < total; ++p) {
        double sp = s ? s[p] : s0;
        a[p] = -sp;
        b[p] = 1.0 + 2.0 * sp;
        c[p] = -sp;
    }
}

/* Alg. 3: `nsteps` ADI steps in place on u (2D: x, y; 3D: x, y, z). */
int orc_adi_step(double *u, const double *s, double s0, int ndim, const idx_t *dims, idx_t batch,
                 int nsteps) {
    if (ndim < 2 || ndim > 3 || batch < 1 || nsteps < 0) return 1;
    idx_t total = mesh_points(ndim, dims, batch);
    double *a = (double *)malloc(sizeof(double) * (size_t)total);
    double *b = (double *)malloc(sizeof(double) * (size_t)total);
    double *c = (double *)malloc(sizeof(double) * (size_t)total);
    double *d = (double *)malloc(sizeof(double) * (size_t)total);
    implicit_coefs(s, s0, total, a, b, c);
    for (int it = 0; it < nsteps; ++it) {
        orc_laplacian(u, d, ndim, dims, batch); /* RHS: d = 2 s L u */
        for (idx_t p = 0; p < total; ++p) d[p] *= 2.0 * (s ? s[p] : s0);
        for (int ax = 0; ax < ndim; ++ax) orc_gtsv(a, b, c, d, ndim, dims, ax, batch);
        for (idx_t p = 0; p < total; ++p) u[p] += d[p];
    }
    free(a); free(b); free(c); free(d);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Adjoint of the line solve x = A^{-1} d.  On entry g = dL/dx; on return
 * g = dL/dd = lambda = A^{-T} g, and
 *   ga_i = -lambda_i x_{i-1} (0 at i = 0),  gb_i = -lambda_i x_i,
 *   gc_i = -lambda_i x_{i+1} (0 at i = N-1).
 * A^T is tridiagonal with sub-diagonal c_{i-1}, diagonal b_i and
 * super-diagonal a_{i+1}; it is solved with Alg. 1 like any other line.
 * ------------------------------------------------------------------------- */
int orc_gtsv_adjoint(const double *a, const double *b, const double *c, const double *x,
                     double *g, double *ga, double *gb, double *gc, int ndim, const idx_t *dims,
                     int ax, idx_t batch) {
    if (ndim < 1 || ndim > 3 || ax < 0 || ax >= ndim || batch < 1) return 1;
    idx_t inner, n, outer;
    line_geom(ndim, dims, ax, batch, &inner, &n, &outer);
    idx_t nlines = inner * outer;
#pragma omp parallel
    {
        double *ta = (double *)malloc(sizeof(double) * (size_t)n);
        double *tb = (double *)malloc(sizeof(double) * (size_t)n);
        double *tc = (double *)malloc(sizeof(double) * (size_t)n);
        double *cs = (double *)malloc(sizeof(double) * (size_t)n);
        double *ds = (double *)malloc(sizeof(double) * (size_t)n);
        double *td = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (idx_t l = 0; l < nlines; ++l) {
            idx_t o = l / inner, i0 = l % inner;
            idx_t base = o * n * inner + i0;
            /* gather the transposed rows of this line (contiguous copies) */
            for (idx_t i = 0; i < n; ++i) {
                ta[i] = (i > 0) ? c[base + (i - 1) * inner] : 0.0;
                tb[i] = b[base + i * inner];
                tc[i] = (i < n - 1) ? a[base + (i + 1) * inner] : 0.0;
                td[i] = g[base + i * inner];
            }
            thomas_line(n, ta, tb, tc, td, 1, cs, ds);
            for (idx_t i = 0; i < n; ++i) {
                idx_t q = base + i * inner;
                double lam = td[i];
                g[q] = lam;
                ga[q] = (i > 0) ? -lam * x[q - inner] : 0.0;
                gb[q] = -lam * x[q];
                gc[q] = (i < n - 1) ? -lam * x[q + inner] : 0.0;
            }
        }
        free(ta); free(tb); free(tc); free(cs); free(ds); free(td);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * One ADI step backwards.  Forward: u_{t+1} = u_t + Delta,
 *   Delta = Z^{-1} Y^{-1} X^{-1} r,  r = 2 s * (L u_t),
 * each operator with rows (-s, 1 + 2s, -s) along its axis.  Given the
 * checkpoint u_t and ubar = dL/du_{t+1}, this overwrites ubar with dL/du_t and
 * adds dL/ds of this step into sbar.  2D meshes use X and Y only.
 * ------------------------------------------------------------------------- */
int orc_adi_step_adjoint(const double *u, const double *s, double *ubar, double *sbar, int ndim,
                         const idx_t *dims, idx_t batch) {
    if (ndim < 2 || ndim > 3 || batch < 1 || !s) return 1;
    idx_t total = mesh_points(ndim, dims, batch);
    size_t bytes = sizeof(double) * (size_t)total;
    double *a = malloc(bytes), *b = malloc(bytes), *c = malloc(bytes);
    double *lu = malloc(bytes), *lam = malloc(bytes), *w = malloc(bytes);
    double *ga = malloc(bytes), *gb = malloc(bytes), *gc = malloc(bytes);
    double *xs[4]; /* xs[0] = r, xs[k+1] = solution after the axis-k solve */
    for (int k = 0; k <= ndim; ++k) xs[k] = malloc(bytes);
    implicit_coefs(s, 0.0, total, a, b, c);
    /* recompute the forward step from the checkpoint */
    orc_laplacian(u, lu, ndim, dims, batch);
    for (idx_t p = 0; p < total; ++p) xs[0][p] = 2.0 * s[p] * lu[p];
    for (int k = 0; k < ndim; ++k) {
        memcpy(xs[k + 1], xs[k], bytes);
        orc_gtsv(a, b, c, xs[k + 1], ndim, dims, k, batch);
    }
    /* u_{t+1} = u_t + Delta: both receive ubar */
    memcpy(lam, ubar, bytes);
    for (int k = ndim - 1; k >= 0; --k) {
        /* lam <- A_k^{-T} lam, coefficient gradients against that solve's output */
        orc_gtsv_adjoint(a, b, c, xs[k + 1], lam, ga, gb, gc, ndim, dims, k, batch);
        for (idx_t p = 0; p < total; ++p) sbar[p] += -ga[p] + 2.0 * gb[p] - gc[p];
    }
    /* lam is now rbar; r = 2 s (L u) */
    for (idx_t p = 0; p < total; ++p) {
        sbar[p] += 2.0 * lam[p] * lu[p];
        w[p] = 2.0 * s[p] * lam[p];
    }
    orc_laplacian(w, lu, ndim, dims, batch); /* L symmetric: dL/du_t += L^T (2 s rbar) */
    for (idx_t p = 0; p < total; ++p) ubar[p] += lu[p];
    free(a); free(b); free(c); free(lu); free(lam); free(w); free(ga); free(gb); free(gc);
    for (int k = 0; k <= ndim; ++k) free(xs[k]);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Synthetic stand-in for the SLV application's time loop (Alg. 4: explicit
 * predictor stencils alternating with x- and y-line solves).  The paper gives
 * the call structure but not the model's coefficient functions, so the PDE here
 * is a 2D convection-free model with a mixed derivative,
 *     u_t = F(u) = a u_xx + b u_yy + c u_xy   (unit spacing, zero ghosts),
 * with per-point a, b, c, integrated by the Hundsdorfer-Verwer ADI scheme
 * (Hundsdorfer & Verwer, Numerical Solution of Time-Dependent
 * Advection-Diffusion-Reaction Equations, 2003) with parameter theta.
 * F0 = c D_xy u (explicit only), F1 = a D_xx u, F2 = b D_yy u, with
 *   D_xx u = u(i-1,j) - 2u + u(i+1,j),  D_yy likewise along y,
 *   D_xy u = (u(i+1,j+1) - u(i+1,j-1) - u(i-1,j+1) + u(i-1,j-1)) / 4.
 * One step of size dt:
 *   Y0 = U + dt F(U)
 *   (I - theta dt A1) Y1 = Y0 - theta dt F1(U)
 *   (I - theta dt A2) Y2 = Y1 - theta dt F2(U)
 *   W0 = Y0 + dt/2 (F(Y2) - F(U))
 *   (I - theta dt A1) W1 = W0 - theta dt F1(Y2)
 *   (I - theta dt A2) W2 = W1 - theta dt F2(Y2)
 *   U <- W2
 * where A1 = a D_xx, A2 = b D_yy: rows (-s, 1 + 2s, -s) with s = theta dt a
 * (x lines) or theta dt b (y lines).
 * ------------------------------------------------------------------------- */
static void hv_operators(const double *u, const double *a, const double *b, const double *c,
                         idx_t nx, idx_t ny, idx_t batch, double *f0, double *f1, double *f2) {
    idx_t total = nx * ny * batch;
#pragma omp parallel for schedule(static)
    for (idx_t p = 0; p < total; ++p) {
        idx_t i = p % nx, j = (p / nx) % ny;
        double um = i > 0 ? u[p - 1] : 0.0, up = i < nx - 1 ? u[p + 1] : 0.0;
        double vm = j > 0 ? u[p - nx] : 0.0, vp = j < ny - 1 ? u[p + nx] : 0.0;
        double pp = (i < nx - 1 && j < ny - 1) ? u[p + 1 + nx] : 0.0;
        double pm = (i < nx - 1 && j > 0) ? u[p + 1 - nx] : 0.0;
        double mp = (i > 0 && j < ny - 1) ? u[p - 1 + nx] : 0.0;
        double mm = (i > 0 && j > 0) ? u[p - 1 - nx] : 0.0;
        f1[p] = a[p] * (um - 2.0 * u[p] + up);
        f2[p] = b[p] * (vm - 2.0 * u[p] + vp);
        f0[p] = c[p] * (pp - pm - mp + mm) / 4.0;
    }
}

int orc_hv_step(double *u, const double *a, const double *b, const double *c, double dt,
                double theta, const idx_t *dims, idx_t batch, int nsteps) {
    if (batch < 1 || nsteps < 0 || !dims || dims[0] < 1 || dims[1] < 1) return 1;
    idx_t nx = dims[0], ny = dims[1], total = nx * ny * batch;
    size_t bytes = sizeof(double) * (size_t)total;
    double *f0 = malloc(bytes), *f1 = malloc(bytes), *f2 = malloc(bytes);
    double *g0 = malloc(bytes), *g1 = malloc(bytes), *g2 = malloc(bytes);
    double *y0 = malloc(bytes), *y1 = malloc(bytes), *y2 = malloc(bytes), *w = malloc(bytes);
    double *xa = malloc(bytes), *xb = malloc(bytes), *xc = malloc(bytes);
    double *ya = malloc(bytes), *yb = malloc(bytes), *yc = malloc(bytes), *s = malloc(bytes);
    for (idx_t p = 0; p < total; ++p) s[p] = theta * dt * a[p];
    implicit_coefs(s, 0.0, total, xa, xb, xc);
    for (idx_t p = 0; p < total; ++p) s[p] = theta * dt * b[p];
    implicit_coefs(s, 0.0, total, ya, yb, yc);
    for (int it = 0; it < nsteps; ++it) {
        hv_operators(u, a, b, c, nx, ny, batch, f0, f1, f2);
        for (idx_t p = 0; p < total; ++p) {
            y0[p] = u[p] + dt * (f0[p] + f1[p] + f2[p]);
            y1[p] = y0[p] - theta * dt * f1[p];
        }
        orc_gtsv(xa, xb, xc, y1, 2, dims, 0, batch);
        for (idx_t p = 0; p < total; ++p) y2[p] = y1[p] - theta * dt * f2[p];
        orc_gtsv(ya, yb, yc, y2, 2, dims, 1, batch);
        hv_operators(y2, a, b, c, nx, ny, batch, g0, g1, g2);
        for (idx_t p = 0; p < total; ++p) {
            double w0 = y0[p] + 0.5 * dt * ((g0[p] + g1[p] + g2[p]) - (f0[p] + f1[p] + f2[p]));
            w[p] = w0 - theta * dt * g1[p];
        }
        orc_gtsv(xa, xb, xc, w, 2, dims, 0, batch);
        for (idx_t p = 0; p < total; ++p) u[p] = w[p] - theta * dt * g2[p];
        orc_gtsv(ya, yb, yc, u, 2, dims, 1, batch);
    }
    free(f0); free(f1); free(f2); free(g0); free(g1); free(g2);
    free(y0); free(y1); free(y2); free(w);
    free(xa); free(xb); free(xc); free(ya); free(yb); free(yc); free(s);
    return 0;
}
