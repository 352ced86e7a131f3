/*
 * oracle.c -- plain FP64 CPU reference for the time-stepped acoustic-wave
 * sweep.  TEST INFRASTRUCTURE ONLY: nothing in the product path links,
 * loads or calls this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header, table or
 * constant with the HIP library.
 *
 * Everything here is written for obviousness, not speed: no tiling, no
 * blocking, no fusion, one point at a time, double precision throughout.
 * OpenMP is used only over independent grid points (results do not depend on
 * the thread count).
 *
 * What is computed (the paper's evaluation chapter, AWE section, measures an
 * acoustic-wave operator but never prints its discretisation, so the scheme
 * below is the standard one for  m u_tt + damp u_t = lap u + q):
 *
 *   coefficients  c_j = 2(-1)^{j+1} (k!)^2 / (j^2 (k-j)! (k+j)!),  j=1..k,
 *                 c_0 = -2 sum_j c_j,  k = space_order/2  (central second
 *                 derivative of order 2k; k is the stencil radius, which the
 *                 paper's skewing section names as the minimum legal skew)
 *   Laplacian     (L u)_p = sum_a h_a^-2 [c_0 u_p + sum_j c_j (u_{p+j e_a} + u_{p-j e_a})]
 *                 with zero values outside the grid (Dirichlet ghosts), or
 *                 periodic wrap in the test-only periodic mode.
 *   damping       sigma_p = sigma_max * sum_a (d_a/nbl)^2, d_a = depth of the
 *                 point inside the absorbing layer along axis a (0 at the
 *                 layer's inner edge, nbl at the outer face); damp = m sigma,
 *                 eta = damp dt / 2.
 *   forward       u^{n+1} = [dt^2 (L u^n) + 2 m u^n - (m - eta) u^{n-1}
 *                            + dt^2 sum_s w_{s,p} q_s^n] / (m + eta)
 *                 receivers d_r^n = sum_p w_{r,p} u^{n+1}_p
 *   adjoint       mu^{nt} = mu^{nt+1} = 0, n = nt-1 .. 0:
 *                 mu^n = [dt^2 L mu^{n+1} + 2 m mu^{n+1} - (m - eta) mu^{n+2}
 *                         + sum_r w_{r,p} dd_r^n] / (m + eta)
 *                 source-side adjoint  g_q[n][s] = dt^2 sum_p w_{s,p} mu^n_p
 *   gradient of J = 1/2 sum_n |d^n - d_obs^n|^2 with respect to m:
 *                 form 1: -sum_{n=0}^{nt-1} mu^n ((1+st) u^{n+1} - 2 u^n + (1-st) u^{n-1})
 *                 form 2: -sum_{j=1}^{nt}   u^j ((1+st) mu^{j-1} - 2 mu^j + (1-st) mu^{j+1})
 *                 with st = sigma dt / 2 (the two agree by summation by parts
 *                 when u^0 = u^{-1} = 0).
 *   interpolation multilinear weights prod_a (1 - |xi_a - i_a|) over the 2^d
 *                 corners of the cell holding xi = x/h, i = floor(xi);
 *                 corners outside the grid are dropped.
 *
 * The paper's second workload, the Laplace operator family of its evaluation
 * chapter (first order in time, one time dependency), is never printed
 * either; it is read as explicit diffusion with a constant diffusivity a:
 *
 *   diffusion     u^{n+1} = u^n + dt a (L u^n)
 *                 with the same Laplacian, ghosts and coefficients as above.
 *
 * Layout: row-major [n0][n1][n2] (3D) or [n0][n1] (2D); the last axis has unit
 * stride.  Coordinates are in metres from grid node 0 along each axis.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;         /* 2 or 3 */
    int so;           /* space order, even, 2..16 */
    long n[3];        /* grid points per axis (axis ndim-1 has unit stride) */
    double h[3];      /* spacing per axis, metres */
    double dt;        /* time step, seconds */
    int nbl;          /* absorbing-layer width in points (0: no damping) */
    double sigma_max; /* damping profile maximum, 1/s */
    int periodic;     /* 1: periodic wrap instead of zero ghosts (tests only) */
} og_grid;

static long og_npts(const og_grid *g) {
    long n = 1;
    for (int a = 0; a < g->ndim; ++a) n *= g->n[a];
    return n;
}

/* Central second-derivative weights of order 2k (closed form above). */
int og_fd_coeffs(int so, double *c) {
    if (so < 2 || so > 16 || (so & 1)) return -1;
    int k = so / 2;
    double s = 0.0;
    for (int j = 1; j <= k; ++j) {
        /* (k!)^2 / ((k-j)! (k+j)!) = prod_{i=1..j} (k-i+1)/(k+i) */
        double r = 1.0;
        for (int i = 1; i <= j; ++i) r *= (double)(k - i + 1) / (double)(k + i);
        double cj = 2.0 * r / ((double)j * (double)j);
        if ((j & 1) == 0) cj = -cj;
        c[j] = cj;
        s += cj;
    }
    c[0] = -2.0 * s;
    return 0;
}

/* Value of u at index idx[] shifted by `off` along axis a; zero ghost or wrap. */
static double og_at(const og_grid *g, const double *u, const long *idx, int a, long off) {
    long i[3] = {idx[0], idx[1], idx[2]};
    i[a] += off;
    if (i[a] < 0 || i[a] >= g->n[a]) {
        if (!g->periodic) return 0.0;
        i[a] = ((i[a] % g->n[a]) + g->n[a]) % g->n[a];
    }
    long lin = 0;
    for (int b = 0; b < g->ndim; ++b) lin = lin * g->n[b] + i[b];
    return u[lin];
}

static void og_unravel(const og_grid *g, long p, long *idx) {
    idx[0] = idx[1] = idx[2] = 0;
    for (int b = g->ndim - 1; b >= 0; --b) {
        idx[b] = p % g->n[b];
        p /= g->n[b];
    }
}

/* out = L u over every grid point. */
int og_laplacian(const og_grid *g, const double *u, double *out) {
    double c[9];
    if (og_fd_coeffs(g->so, c)) return -1;
    int k = g->so / 2;
    long N = og_npts(g);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; ++p) {
        long idx[3];
        og_unravel(g, p, idx);
        double acc = 0.0;
        for (int a = 0; a < g->ndim; ++a) {
            double s = c[0] * u[p];
            for (int j = 1; j <= k; ++j)
                s += c[j] * (og_at(g, u, idx, a, j) + og_at(g, u, idx, a, -j));
            acc += s / (g->h[a] * g->h[a]);
        }
        out[p] = acc;
    }
    return 0;
}

/* sigma (1/s) at every point: sigma_max * sum_a (d_a / nbl)^2. */
int og_sigma(const og_grid *g, double *sig) {
    long N = og_npts(g);
    for (long p = 0; p < N; ++p) {
        long idx[3];
        og_unravel(g, p, idx);
        double s = 0.0;
        if (g->nbl > 0) {
            for (int a = 0; a < g->ndim; ++a) {
                long d = 0;
                if (idx[a] < g->nbl) d = g->nbl - idx[a];
                else if (idx[a] > g->n[a] - 1 - g->nbl) d = idx[a] - (g->n[a] - 1 - g->nbl);
                double f = (double)d / (double)g->nbl;
                s += f * f;
            }
            s *= g->sigma_max;
        }
        sig[p] = s;
    }
    return 0;
}

/* Interpolation corners of one point: up to 2^ndim (linear index, weight). */
static int og_corners(const og_grid *g, const double *x, long *lin, double *w) {
    long i0[3] = {0, 0, 0};
    double f[3] = {0, 0, 0};
    for (int a = 0; a < g->ndim; ++a) {
        double xi = x[a] / g->h[a];
        double fl = floor(xi);
        i0[a] = (long)fl;
        f[a] = xi - fl;
    }
    int nc = 0;
    for (int b = 0; b < (1 << g->ndim); ++b) {
        double wt = 1.0;
        long l = 0;
        int inside = 1;
        for (int a = 0; a < g->ndim; ++a) {
            int bit = (b >> (g->ndim - 1 - a)) & 1;
            long ia = i0[a] + bit;
            if (ia < 0 || ia >= g->n[a]) inside = 0;
            wt *= bit ? f[a] : (1.0 - f[a]);
            l = l * g->n[a] + ia;
        }
        if (!inside) continue;
        lin[nc] = l;
        w[nc] = wt;
        ++nc;
    }
    return nc;
}

/* Exposed for tests: the corners and weights of one coordinate. */
int og_interp_corners(const og_grid *g, const double *x, long *lin, double *w) {
    return og_corners(g, x, lin, w);
}

/* One leapfrog step:  out = [dt^2 (L cur) + 2 m cur - (m - eta) prev + f] / (m + eta),
 * where `f` is the injected forcing already in the bracket's units (may be NULL):
 * dt^2 sum_s w q for the forward sweep, sum_r w dd for the adjoint. */
static void og_step(const og_grid *g, const double *m, const double *sig,
                    const double *cur, const double *prev, const double *inj,
                    double *lap, double *out) {
    long N = og_npts(g);
    og_laplacian(g, cur, lap);
    double dt2 = g->dt * g->dt;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; ++p) {
        double eta = m[p] * sig[p] * g->dt / 2.0; /* damp dt / 2 with damp = m sigma */
        double f = inj ? inj[p] : 0.0;
        out[p] = (dt2 * lap[p] + 2.0 * m[p] * cur[p] - (m[p] - eta) * prev[p] + f) / (m[p] + eta);
    }
}

typedef struct {
    int n;        /* number of points */
    int *nc;      /* corners per point */
    long *lin;    /* [n][8] */
    double *w;    /* [n][8] */
} og_pts;

static int og_pts_make(const og_grid *g, int n, const double *xyz, og_pts *P) {
    P->n = n;
    P->nc = (int *)calloc(n > 0 ? n : 1, sizeof(int));
    P->lin = (long *)calloc((size_t)(n > 0 ? n : 1) * 8, sizeof(long));
    P->w = (double *)calloc((size_t)(n > 0 ? n : 1) * 8, sizeof(double));
    if (!P->nc || !P->lin || !P->w) return -1;
    for (int i = 0; i < n; ++i)
        P->nc[i] = og_corners(g, xyz + (size_t)i * g->ndim, P->lin + (size_t)i * 8, P->w + (size_t)i * 8);
    return 0;
}

static void og_pts_free(og_pts *P) {
    free(P->nc);
    free(P->lin);
    free(P->w);
}

/*
 * Forward modelling over nt steps.
 *   m         [N]            squared slowness (s^2/m^2)
 *   src_xyz   [nsrc][ndim]   source coordinates (m)
 *   wavelet   [nt][nsrc]     q_s^n
 *   rec_xyz   [nrec][ndim]
 *   rec       [nt][nrec]     out: d_r^n (may be NULL)
 *   u_init    [2][N]         (u^0, u^{-1}) or NULL for zeros
 *   u_final   [2][N]         out: (u^{nt}, u^{nt-1}) or NULL
 *   hist      [nt+2][N]      out: u^{-1}, u^0, ..., u^{nt} or NULL
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int og_forward(const og_grid *g, const double *m, int nt,
               int nsrc, const double *src_xyz, const double *wavelet,
               int nrec, const double *rec_xyz, double *rec,
               const double *u_init, double *u_final, double *hist) {
    if (g->ndim < 2 || g->ndim > 3 || nt < 0) return -1;
    long N = og_npts(g);
    double *sig = (double *)malloc(N * sizeof(double));
    double *a = (double *)calloc(N, sizeof(double)); /* u^{n-1} */
    double *b = (double *)calloc(N, sizeof(double)); /* u^n */
    double *c = (double *)calloc(N, sizeof(double)); /* u^{n+1} */
    double *lap = (double *)malloc(N * sizeof(double));
    double *inj = (double *)calloc(N, sizeof(double));
    og_pts S = {0, NULL, NULL, NULL}, R = {0, NULL, NULL, NULL};
    int rc = -1;
    if (!sig || !a || !b || !c || !lap || !inj) goto done;
    if (og_pts_make(g, nsrc, src_xyz, &S) || og_pts_make(g, nrec, rec_xyz, &R)) goto done;
    og_sigma(g, sig);
    if (u_init) {
        memcpy(b, u_init, N * sizeof(double));
        memcpy(a, u_init + N, N * sizeof(double));
    }
    if (hist) {
        memcpy(hist, a, N * sizeof(double));
        memcpy(hist + N, b, N * sizeof(double));
    }
    for (int n = 0; n < nt; ++n) {
        memset(inj, 0, N * sizeof(double));
        for (int s = 0; s < nsrc; ++s)
            for (int q = 0; q < S.nc[s]; ++q)
                inj[S.lin[(size_t)s * 8 + q]] += S.w[(size_t)s * 8 + q] * wavelet[(size_t)n * nsrc + s];
        for (long p = 0; p < N; ++p) inj[p] *= g->dt * g->dt;
        og_step(g, m, sig, b, a, inj, lap, c);
        if (rec) {
            for (int r = 0; r < nrec; ++r) {
                double d = 0.0;
                for (int q = 0; q < R.nc[r]; ++q)
                    d += R.w[(size_t)r * 8 + q] * c[R.lin[(size_t)r * 8 + q]];
                rec[(size_t)n * nrec + r] = d;
            }
        }
        if (hist) memcpy(hist + (size_t)(n + 2) * N, c, N * sizeof(double));
        double *t = a;
        a = b;
        b = c;
        c = t;
    }
    if (u_final) {
        memcpy(u_final, b, N * sizeof(double));
        memcpy(u_final + N, a, N * sizeof(double));
    }
    rc = 0;
done: /* every exit releases what was allocated */
    og_pts_free(&S);
    og_pts_free(&R);
    free(sig);
    free(a);
    free(b);
    free(c);
    free(lap);
    free(inj);
    return rc;
}

/*
 * Adjoint (time-reversed) sweep driven by receiver residuals, with the
 * gradient of J with respect to m and the source-side adjoint.
 *   resid     [nt][nrec]   dd_r^n
 *   hist      [nt+2][N]    forward history u^{-1} .. u^{nt} (needed for grad_m)
 *   grad_m    [N]          out or NULL
 *   grad_q    [nt][nsrc]   out or NULL
 *   form      1 or 2: which of the two equal gradient sums to evaluate
 *   mu_final  [2][N]       out: (mu^0, mu^1) or NULL
 */
int og_adjoint(const og_grid *g, const double *m, int nt,
               int nsrc, const double *src_xyz, int nrec, const double *rec_xyz,
               const double *resid, const double *hist,
               double *grad_m, double *grad_q, int form, double *mu_final) {
    if (g->ndim < 2 || g->ndim > 3 || nt < 0) return -1;
    if (grad_m && !hist) return -1;
    if (form != 1 && form != 2) return -1;
    long N = og_npts(g);
    double *sig = (double *)malloc(N * sizeof(double));
    double *a = (double *)calloc(N, sizeof(double)); /* mu^{n+2} */
    double *b = (double *)calloc(N, sizeof(double)); /* mu^{n+1} */
    double *c = (double *)calloc(N, sizeof(double)); /* mu^n */
    double *lap = (double *)malloc(N * sizeof(double));
    double *inj = (double *)calloc(N, sizeof(double));
    og_pts S = {0, NULL, NULL, NULL}, R = {0, NULL, NULL, NULL};
    int rc = -1;
    if (!sig || !a || !b || !c || !lap || !inj) goto done;
    if (og_pts_make(g, nsrc, src_xyz, &S) || og_pts_make(g, nrec, rec_xyz, &R)) goto done;
    og_sigma(g, sig);
    double dt2 = g->dt * g->dt;
    if (grad_m) memset(grad_m, 0, N * sizeof(double));
    for (int n = nt - 1; n >= 0; --n) {
        memset(inj, 0, N * sizeof(double));
        for (int r = 0; r < nrec; ++r)
            for (int q = 0; q < R.nc[r]; ++q)
                inj[R.lin[(size_t)r * 8 + q]] += R.w[(size_t)r * 8 + q] * resid[(size_t)n * nrec + r];
        og_step(g, m, sig, b, a, inj, lap, c);
        if (grad_q) {
            for (int s = 0; s < nsrc; ++s) {
                double v = 0.0;
                for (int q = 0; q < S.nc[s]; ++q)
                    v += S.w[(size_t)s * 8 + q] * c[S.lin[(size_t)s * 8 + q]];
                grad_q[(size_t)n * nsrc + s] = dt2 * v;
            }
        }
        if (grad_m) {
            double st_scale = g->dt / 2.0;
            if (form == 1) {
                /* term n: mu^n * ((1+st) u^{n+1} - 2 u^n + (1-st) u^{n-1}) */
                const double *up = hist + (size_t)(n + 2) * N;
                const double *u0 = hist + (size_t)(n + 1) * N;
                const double *um = hist + (size_t)n * N;
                for (long p = 0; p < N; ++p) {
                    double st = sig[p] * st_scale;
                    grad_m[p] -= c[p] * ((1.0 + st) * up[p] - 2.0 * u0[p] + (1.0 - st) * um[p]);
                }
            } else {
                /* term j = n+1: u^{n+1} * ((1+st) mu^n - 2 mu^{n+1} + (1-st) mu^{n+2}) */
                const double *uj = hist + (size_t)(n + 2) * N;
                for (long p = 0; p < N; ++p) {
                    double st = sig[p] * st_scale;
                    grad_m[p] -= uj[p] * ((1.0 + st) * c[p] - 2.0 * b[p] + (1.0 - st) * a[p]);
                }
            }
        }
        double *t = a;
        a = b;
        b = c;
        c = t;
    }
    if (mu_final) {
        memcpy(mu_final, b, N * sizeof(double));
        memcpy(mu_final + N, a, N * sizeof(double));
    }
    rc = 0;
done: /* every exit releases what was allocated */
    og_pts_free(&S);
    og_pts_free(&R);
    free(sig);
    free(a);
    free(b);
    free(c);
    free(lap);
    free(inj);
    return rc;
}

/* Explicit diffusion, the paper's Laplace-operator family: nt steps of
 * u <- u + dt * a * (L u) from u0, result in u_out (both N doubles). */
int og_diffuse(const og_grid *g, double a, int nt, const double *u0, double *u_out) {
    if (nt < 0) return -1;
    long N = og_npts(g);
    double *u = malloc(N * sizeof(double));
    double *lap = malloc(N * sizeof(double));
    if (!u || !lap) {
        free(u);
        free(lap);
        return -2;
    }
    memcpy(u, u0, N * sizeof(double));
    int rc = 0;
    for (int n = 0; n < nt && rc == 0; ++n) {
        rc = og_laplacian(g, u, lap);
        for (long p = 0; p < N; ++p) u[p] = u[p] + g->dt * a * lap[p];
    }
    memcpy(u_out, u, N * sizeof(double));
    free(u);
    free(lap);
    return rc;
}

/* The Laplace-operator family with a time dependence of two levels
 * (delta_t = 2; evaluation chapter, "Time-tiling with larger time
 * dependences", which names the Adams-Bashforth multi-step methods): the
 * two-step Adams-Bashforth rule applied to u' = a L u,
 *     u^{n+1} = u^n + dt a (3/2 L u^n - 1/2 L u^{n-1}),
 * started from u^{-1} = u^0 (so the first step is the forward Euler step).
 * nt steps from u0 into u_out (both N doubles). */
int og_diffuse_ab2(const og_grid *g, double a, int nt, const double *u0, double *u_out) {
    if (nt < 0) return -1;
    long N = og_npts(g);
    double *u = malloc(N * sizeof(double));
    double *lap_n = malloc(N * sizeof(double));   /* L u^n */
    double *lap_m = malloc(N * sizeof(double));   /* L u^{n-1} */
    int rc = 0;
    if (!u || !lap_n || !lap_m) {
        rc = -2;
        goto done;
    }
    memcpy(u, u0, N * sizeof(double));
    rc = og_laplacian(g, u, lap_m); /* u^{-1} = u^0 */
    for (int n = 0; n < nt && rc == 0; ++n) {
        rc = og_laplacian(g, u, lap_n);
        for (long p = 0; p < N; ++p) u[p] = u[p] + g->dt * a * (1.5 * lap_n[p] - 0.5 * lap_m[p]);
        double *t = lap_m;
        lap_m = lap_n;
        lap_n = t;
    }
    if (rc == 0) memcpy(u_out, u, N * sizeof(double));
done:
    free(u);
    free(lap_n);
    free(lap_m);
    return rc;
}
