/*
 * Reference oracle for the per-sample solve of the inexact MLMC method.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition that the GPU library is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant generator with the GPU
 * library, and the GPU library never calls it.
 *
 * Everything is IEEE double precision except the deliberately low-precision
 * factorisation inside the Algorithm 2.1 reference (ir_solve_f32), which
 * rounds the factor to single precision as the algorithm prescribes.
 *
 * Problem (Sec. 5.1, eq. of the model PDE): -div(a grad u) = f on D=(0,1)^2,
 * u = 0 on the boundary, with a lognormal coefficient a = exp(Z).  The
 * quantity of interest is the integral of u over D (Sec. 5.1).
 *
 * Readings where the paper leaves the discrete problem open (the paper uses
 * P1 finite elements on its own field; this oracle follows the vertex-centred
 * finite-volume discretisation and separable exponential KL field of the
 * workloads it checks):
 *   - grid: n cells per side, h = 1/n, nodes (ix, iy), 0 <= ix, iy <= n,
 *     node index p = iy*(n+1) + ix; unknowns are the (n-1)^2 interior nodes,
 *     ordered P = (iy-1)*(n-1) + (ix-1) (x fastest), half-bandwidth n-1.
 *   - coefficient is nodal; the coefficient of the edge between nodes p, q is
 *     the harmonic mean 2 a_p a_q / (a_p + a_q).
 *   - A_PP = sum of the four edge coefficients around P, A_PQ = -a_edge for an
 *     interior neighbour Q; b_P = h^2 f_P (finite-volume form).
 *   - Q = h^2 * sum_P u_P, which is the trapezoidal value of the integral of
 *     u over D because u vanishes on the boundary.
 *   - KL field: covariance sigma^2 exp(-|x1-y1|/lam) exp(-|x2-y2|/lam); the
 *     1D eigenpairs solve the transcendental equation
 *     (lam^2 w^2 - 1) sin w - 2 lam w cos w = 0, one root in each
 *     ((k-1) pi, k pi); mu_k = 2 lam / (1 + lam^2 w_k^2);
 *     phi_k(x) = (sin w x + lam w cos w x) / sqrt(nu_k) with nu_k the squared
 *     L2 norm of the numerator.  2D modes (i, j) are sorted by
 *     (-mu_i mu_j, i, j); the first K are kept;
 *     Phi[p, k] = sigma sqrt(mu_i mu_j) phi_i(x_p) phi_j(y_p).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Karhunen-Loeve basis of the separable exponential covariance        */
/* ------------------------------------------------------------------ */

static double kl_g(double w, double lam)
{
    return (lam * lam * w * w - 1.0) * sin(w) - 2.0 * lam * w * cos(w);
}

/* Roots w_1..w_M of the 1D eigen-equation by bisection on ((k-1)pi, k pi). */
int oracle_kl_roots(double lam, int M, double *w)
{
    for (int k = 1; k <= M; ++k) {
        double lo = (k - 1) * OR_PI, hi = k * OR_PI;
        if (k == 1) lo = 1e-300;
        double glo = kl_g(lo, lam), ghi = kl_g(hi, lam);
        if (k == 1) glo = -1.0; /* g(w) ~ -(1 + 2 lam) w for small w > 0 */
        if ((glo < 0) == (ghi < 0)) return -1;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            double gm = kl_g(mid, lam);
            if ((gm < 0) == (glo < 0)) { lo = mid; glo = gm; }
            else { hi = mid; }
        }
        w[k - 1] = 0.5 * (lo + hi);
    }
    return 0;
}

double oracle_kl_mu(double lam, double w) { return 2.0 * lam / (1.0 + lam * lam * w * w); }

double oracle_kl_nu(double lam, double w)
{
    return (0.5 - sin(2.0 * w) / (4.0 * w)) + lam * lam * w * w * (0.5 + sin(2.0 * w) / (4.0 * w)) +
           lam * (1.0 - cos(2.0 * w)) / 2.0;
}

double oracle_kl_phi1d(double lam, double w, double x)
{
    return (sin(w * x) + lam * w * cos(w * x)) / sqrt(oracle_kl_nu(lam, w));
}

typedef struct { double key; int i, j; } kl_mode;

static int kl_mode_cmp(const void *pa, const void *pb)
{
    const kl_mode *a = (const kl_mode *)pa, *b = (const kl_mode *)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

/* Selected 2D modes: mode_i[k], mode_j[k] are 1-based 1D indices (x, y). */
int oracle_kl_modes(double lam, int K, int M, int *mode_i, int *mode_j)
{
    double *w = (double *)malloc(sizeof(double) * M);
    if (oracle_kl_roots(lam, M, w)) { free(w); return -1; }
    kl_mode *all = (kl_mode *)malloc(sizeof(kl_mode) * M * M);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            all[i * M + j].key = -(oracle_kl_mu(lam, w[i]) * oracle_kl_mu(lam, w[j]));
            all[i * M + j].i = i + 1;
            all[i * M + j].j = j + 1;
        }
    qsort(all, (size_t)M * M, sizeof(kl_mode), kl_mode_cmp);
    int ok = 0;
    for (int k = 0; k < K; ++k) {
        mode_i[k] = all[k].i;
        mode_j[k] = all[k].j;
        if (all[k].i >= M || all[k].j >= M) ok = -2; /* too few roots */
    }
    free(all);
    free(w);
    return ok;
}

/* Phi[(n+1)^2 x K], row-major, on the nodes of the n x n grid. */
int oracle_kl_basis(int n, int K, double sigma2, double lam, double *Phi)
{
    const int M = 64;
    int *mi = (int *)malloc(sizeof(int) * K), *mj = (int *)malloc(sizeof(int) * K);
    double *w = (double *)malloc(sizeof(double) * M);
    int rc = oracle_kl_modes(lam, K, M, mi, mj);
    if (rc == 0) rc = oracle_kl_roots(lam, M, w);
    if (rc == 0) {
        double sigma = sqrt(sigma2);
        for (int iy = 0; iy <= n; ++iy)
            for (int ix = 0; ix <= n; ++ix) {
                double x = (double)ix / n, y = (double)iy / n;
                for (int k = 0; k < K; ++k) {
                    double wi = w[mi[k] - 1], wj = w[mj[k] - 1];
                    double amp = sigma * sqrt(oracle_kl_mu(lam, wi) * oracle_kl_mu(lam, wj));
                    Phi[((size_t)iy * (n + 1) + ix) * K + k] =
                        amp * oracle_kl_phi1d(lam, wi, x) * oracle_kl_phi1d(lam, wj, y);
                }
            }
    }
    free(mi); free(mj); free(w);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Field, assembly, banded Cholesky                                     */
/* ------------------------------------------------------------------ */

/* a[p] = exp(sum_k Phi[p,k] xi[k]) on all (n+1)^2 nodes. */
static void field(int n, int K, const double *Phi, const double *xi, double *a)
{
    int np = (n + 1) * (n + 1);
    for (int p = 0; p < np; ++p) {
        double z = 0.0;
        for (int k = 0; k < K; ++k) z += Phi[(size_t)p * K + k] * xi[k];
        a[p] = exp(z);
    }
}

static double hmean(double x, double y) { return 2.0 * x * y / (x + y); }

/* Discretisation of the edge coefficients (oracle_set_disc):
 * 0: vertex-centred finite volumes, the harmonic mean of the edge's end nodes;
 * 1: P1 finite elements (Sec. 3) on the mesh whose cells are cut along the
 *    diagonal (x,y)-(x+h,y+h), with the coefficient interpolated linearly.
 *    For a right triangle with legs h the element matrix couples the right
 *    angle's vertex with each acute vertex by -(mean of a over T)/2 and the
 *    two acute vertices by 0, so an axis edge, a leg of both its triangles,
 *    gets half the sum of their vertex means:
 *      edge (x,y)-(x+h,y):  its triangles' third vertices are (x+h,y+h) and (x,y-h);
 *      edge (x,y)-(x,y+h):  their third vertices are (x+h,y+h) and (x-h,y). */
static int g_disc = 0;
void oracle_set_disc(int d) { g_disc = d; }

/* a at node (ix, iy), 0 outside the node grid (only edges with both ends on
 * the boundary reach outside; they enter no equation). */
static double anode(int n, const double *a, int ix, int iy)
{
    return (ix < 0 || ix > n || iy < 0 || iy > n) ? 0.0 : a[iy * (n + 1) + ix];
}

/* Edge coefficients: aE[iy*n + ix] joins (ix,iy)-(ix+1,iy), ix<n, iy<=n;
 * aN[iy*(n+1) + ix] joins (ix,iy)-(ix,iy+1), iy<n, ix<=n. */
static void faces(int n, const double *a, double *aE, double *aN)
{
    for (int iy = 0; iy <= n; ++iy)
        for (int ix = 0; ix < n; ++ix) {
            double l = anode(n, a, ix, iy), r = anode(n, a, ix + 1, iy);
            double t1 = (l + r + anode(n, a, ix + 1, iy + 1)) / 3.0; /* triangle above */
            double t2 = (l + r + anode(n, a, ix, iy - 1)) / 3.0;     /* triangle below */
            aE[iy * n + ix] = g_disc ? 0.5 * (t1 + t2) : hmean(l, r);
        }
    for (int iy = 0; iy < n; ++iy)
        for (int ix = 0; ix <= n; ++ix) {
            double b = anode(n, a, ix, iy), t = anode(n, a, ix, iy + 1);
            double t1 = (b + t + anode(n, a, ix + 1, iy + 1)) / 3.0; /* triangle to the right */
            double t2 = (b + t + anode(n, a, ix - 1, iy)) / 3.0;     /* triangle to the left */
            aN[iy * (n + 1) + ix] = g_disc ? 0.5 * (t1 + t2) : hmean(b, t);
        }
}

/* Banded lower storage: Ab[P*(bw+1) + d] = A[P, P-d], d = 0..bw. */
static void assemble_band(int n, const double *aE, const double *aN, double *Ab)
{
    int m = n - 1, bw = m;
    memset(Ab, 0, sizeof(double) * (size_t)m * m * (bw + 1));
    for (int iy = 1; iy <= m; ++iy)
        for (int ix = 1; ix <= m; ++ix) {
            int P = (iy - 1) * m + (ix - 1);
            double w = aE[iy * n + ix - 1], e = aE[iy * n + ix];
            double s = aN[(iy - 1) * (n + 1) + ix], no = aN[iy * (n + 1) + ix];
            Ab[(size_t)P * (bw + 1)] = w + e + s + no;
            if (ix > 1) Ab[(size_t)P * (bw + 1) + 1] = -w;
            if (iy > 1) Ab[(size_t)P * (bw + 1) + bw] = -s;
        }
}

/* y = A x with the 5-point stencil (matrix-free, from the edge arrays). */
static void stencil_apply(int n, const double *aE, const double *aN, const double *x, double *y)
{
    int m = n - 1;
    for (int iy = 1; iy <= m; ++iy)
        for (int ix = 1; ix <= m; ++ix) {
            int P = (iy - 1) * m + (ix - 1);
            double w = aE[iy * n + ix - 1], e = aE[iy * n + ix];
            double s = aN[(iy - 1) * (n + 1) + ix], no = aN[iy * (n + 1) + ix];
            double v = (w + e + s + no) * x[P];
            if (ix > 1) v -= w * x[P - 1];
            if (ix < m) v -= e * x[P + 1];
            if (iy > 1) v -= s * x[P - m];
            if (iy < m) v -= no * x[P + m];
            y[P] = v;
        }
}

/* In-place Cholesky-Crout of the band matrix: Ab becomes L (same layout).
 * Returns -1 if a pivot is not positive. */
static int band_cholesky(int N, int bw, double *Ab)
{
#define L_(i, j) Ab[(size_t)(i) * (bw + 1) + ((i) - (j))]
    for (int j = 0; j < N; ++j) {
        int k0 = j - bw > 0 ? j - bw : 0;
        double s = L_(j, j);
        for (int k = k0; k < j; ++k) s -= L_(j, k) * L_(j, k);
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        L_(j, j) = ljj;
        int iend = j + bw < N - 1 ? j + bw : N - 1;
        for (int i = j + 1; i <= iend; ++i) {
            int ki = i - bw > 0 ? i - bw : 0;
            double t = L_(i, j);
            for (int k = ki; k < j; ++k) t -= L_(i, k) * L_(j, k);
            L_(i, j) = t / ljj;
        }
    }
    return 0;
#undef L_
}

/* Solve L L^T x = r (x may alias r). */
static void band_solve(int N, int bw, const double *Lb, const double *r, double *x)
{
    if (x != r) memcpy(x, r, sizeof(double) * N);
    for (int i = 0; i < N; ++i) {
        int k0 = i - bw > 0 ? i - bw : 0;
        double s = x[i];
        for (int k = k0; k < i; ++k) s -= Lb[(size_t)i * (bw + 1) + (i - k)] * x[k];
        x[i] = s / Lb[(size_t)i * (bw + 1)];
    }
    for (int i = N - 1; i >= 0; --i) {
        int k1 = i + bw < N - 1 ? i + bw : N - 1;
        double s = x[i];
        for (int k = i + 1; k <= k1; ++k) s -= Lb[(size_t)k * (bw + 1) + (k - i)] * x[k];
        x[i] = s / Lb[(size_t)i * (bw + 1)];
    }
}

/* Same two routines in single precision, for the u_f = single reference. */
static int band_cholesky_f32(int N, int bw, float *Ab)
{
#define L_(i, j) Ab[(size_t)(i) * (bw + 1) + ((i) - (j))]
    for (int j = 0; j < N; ++j) {
        int k0 = j - bw > 0 ? j - bw : 0;
        float s = L_(j, j);
        for (int k = k0; k < j; ++k) s -= L_(j, k) * L_(j, k);
        if (!(s > 0.0f)) return -1;
        float ljj = sqrtf(s);
        L_(j, j) = ljj;
        int iend = j + bw < N - 1 ? j + bw : N - 1;
        for (int i = j + 1; i <= iend; ++i) {
            int ki = i - bw > 0 ? i - bw : 0;
            float t = L_(i, j);
            for (int k = ki; k < j; ++k) t -= L_(i, k) * L_(j, k);
            L_(i, j) = t / ljj;
        }
    }
    return 0;
#undef L_
}

static void band_solve_f32(int N, int bw, const float *Lb, float *x)
{
    for (int i = 0; i < N; ++i) {
        int k0 = i - bw > 0 ? i - bw : 0;
        float s = x[i];
        for (int k = k0; k < i; ++k) s -= Lb[(size_t)i * (bw + 1) + (i - k)] * x[k];
        x[i] = s / Lb[(size_t)i * (bw + 1)];
    }
    for (int i = N - 1; i >= 0; --i) {
        int k1 = i + bw < N - 1 ? i + bw : N - 1;
        float s = x[i];
        for (int k = i + 1; k <= k1; ++k) s -= Lb[(size_t)k * (bw + 1) + (k - i)] * x[k];
        x[i] = s / Lb[(size_t)i * (bw + 1)];
    }
}

static double norm2(int N, const double *v)
{
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* ------------------------------------------------------------------ */
/* Public per-sample entry points                                       */
/* ------------------------------------------------------------------ */

/* Build a, edges, A (band) and b for one sample.  rhs_nodal (may be NULL)
 * gives f at the interior unknowns; otherwise f is the constant fconst. */
static void build_system(int n, int K, const double *Phi, const double *xi, const double *a_in,
                         double fconst, const double *rhs_nodal, double *a, double *aE, double *aN,
                         double *Ab, double *b)
{
    int m = n - 1, N = m * m;
    double h = 1.0 / n;
    if (a_in) memcpy(a, a_in, sizeof(double) * (n + 1) * (n + 1));
    else field(n, K, Phi, xi, a);
    faces(n, a, aE, aN);
    if (Ab) assemble_band(n, aE, aN, Ab);
    for (int P = 0; P < N; ++P) b[P] = h * h * (rhs_nodal ? rhs_nodal[P] : fconst);
}

/*
 * Exact discrete solve (FP64 banded Cholesky) of a batch of samples.
 * xi[S x K]; a_nodes (optional, [S x (n+1)^2]) overrides the KL field;
 * rhs_nodal (optional, [(n-1)^2]) overrides f.  Outputs: Q[S]; u (optional,
 * [S x (n-1)^2]).  Returns 0, or the 1-based index of a failing sample.
 */
int oracle_solve_batch(int n, int K, const double *Phi, int S, const double *xi,
                       const double *a_nodes, double fconst, const double *rhs_nodal, double *Q,
                       double *u)
{
    int m = n - 1, N = m * m, bw = m, np = (n + 1) * (n + 1);
    double h = 1.0 / n;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < S; ++s) {
        double *a = (double *)malloc(sizeof(double) * np);
        double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *Ab = (double *)malloc(sizeof(double) * (size_t)N * (bw + 1));
        double *b = (double *)malloc(sizeof(double) * N);
        build_system(n, K, Phi, xi ? xi + (size_t)s * K : NULL,
                     a_nodes ? a_nodes + (size_t)s * np : NULL, fconst, rhs_nodal, a, aE, aN, Ab, b);
        if (band_cholesky(N, bw, Ab)) {
#pragma omp critical
            fail = s + 1;
        } else {
            band_solve(N, bw, Ab, b, b);
            double q = 0.0;
            for (int P = 0; P < N; ++P) q += b[P];
            Q[s] = h * h * q;
            if (u) memcpy(u + (size_t)s * N, b, sizeof(double) * N);
        }
        free(a); free(aE); free(aN); free(Ab); free(b);
    }
    return fail;
}

/* Relative residual ||b - A x|| / ||b|| of given solutions (FP64). */
int oracle_relres_batch(int n, int K, const double *Phi, int S, const double *xi, double fconst,
                        const double *x, double *relres)
{
    int m = n - 1, N = m * m, np = (n + 1) * (n + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < S; ++s) {
        double *a = (double *)malloc(sizeof(double) * np);
        double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *b = (double *)malloc(sizeof(double) * N);
        double *r = (double *)malloc(sizeof(double) * N);
        build_system(n, K, Phi, xi + (size_t)s * K, NULL, fconst, NULL, a, aE, aN, NULL, b);
        stencil_apply(n, aE, aN, x + (size_t)s * N, r);
        for (int P = 0; P < N; ++P) r[P] = b[P] - r[P];
        relres[s] = norm2(N, r) / norm2(N, b);
        free(a); free(aE); free(aN); free(b); free(r);
    }
    return 0;
}

/*
 * Algorithm 2.1 (iterative refinement, Sec. 2.3) with u_f = u_s = single and
 * u = u_r = double: factorise in single, x0 by substitution in single stored
 * in double, then loop: residual in double, stop when ||r||/||b|| < delta
 * (strict), correction solve in single, update in double.  At most imax
 * corrections.  Outputs Q[S], trips[S] (corrections applied) and
 * relres[S] (final relative residual); returns the number of samples that
 * did not reach delta.
 */
int oracle_ir_f32_batch(int n, int K, const double *Phi, int S, const double *xi, double fconst,
                        double delta, int imax, double *Q, int *trips, double *relres)
{
    int m = n - 1, N = m * m, bw = m, np = (n + 1) * (n + 1);
    double h = 1.0 / n;
    int nfail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nfail)
    for (int s = 0; s < S; ++s) {
        double *a = (double *)malloc(sizeof(double) * np);
        double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *Ab = (double *)malloc(sizeof(double) * (size_t)N * (bw + 1));
        float *Lf = (float *)malloc(sizeof(float) * (size_t)N * (bw + 1));
        double *b = (double *)malloc(sizeof(double) * N);
        double *x = (double *)malloc(sizeof(double) * N);
        double *r = (double *)malloc(sizeof(double) * N);
        float *t = (float *)malloc(sizeof(float) * N);
        build_system(n, K, Phi, xi + (size_t)s * K, NULL, fconst, NULL, a, aE, aN, Ab, b);
        for (size_t e = 0; e < (size_t)N * (bw + 1); ++e) Lf[e] = (float)Ab[e];
        int it = 0;
        double rr = INFINITY;
        if (band_cholesky_f32(N, bw, Lf) == 0) {
            for (int P = 0; P < N; ++P) t[P] = (float)b[P];
            band_solve_f32(N, bw, Lf, t);
            for (int P = 0; P < N; ++P) x[P] = (double)t[P];
            double nb = norm2(N, b);
            for (;;) {
                stencil_apply(n, aE, aN, x, r);
                for (int P = 0; P < N; ++P) r[P] = b[P] - r[P];
                rr = norm2(N, r) / nb;
                if (rr < delta || it >= imax) break;
                for (int P = 0; P < N; ++P) t[P] = (float)r[P];
                band_solve_f32(N, bw, Lf, t);
                for (int P = 0; P < N; ++P) x[P] += (double)t[P];
                ++it;
            }
        }
        double q = 0.0;
        for (int P = 0; P < N; ++P) q += x[P];
        Q[s] = h * h * q;
        trips[s] = it;
        relres[s] = rr;
        if (!(rr < delta)) nfail += 1;
        free(a); free(aE); free(aN); free(Ab); free(Lf); free(b); free(x); free(r); free(t);
    }
    return nfail;
}

/*
 * Rounding to a binary floating-point format with p significand bits,
 * minimum normal exponent emin and largest finite value vmax, to nearest
 * with ties to even (the default rounding mode of nearbyint): every value is
 * a multiple of its binade's spacing 2^(e - p + 1), subnormals of 2^(emin -
 * p + 1); beyond vmax the result is infinite.  FP16: p = 11, emin = -14,
 * vmax = 65504; BF16: p = 8, emin = -126.
 */
static double round_fmt(double v, int p, int emin, double vmax)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    frexp(v, &e);
    int ex = e - 1 < emin ? emin : e - 1;
    double q = ldexp(1.0, ex - (p - 1));
    double r = nearbyint(v / q) * q;
    return fabs(r) > vmax ? copysign(INFINITY, v) : r;
}

typedef struct { int p, emin; double vmax; } lowp_fmt;
static const lowp_fmt LOWP_FMTS[3] = {{11, -14, 65504.0}, {8, -126, 3.3895313892515355e38},
                                      {24, -126, 3.4028234663852886e38}};
static double rnd(const lowp_fmt *f, double v) { return round_fmt(v, f->p, f->emin, f->vmax); }

/* v rounded to format fmt (0 FP16, 1 BF16, 2 FP32), for the tests. */
double oracle_round_lowp(double v, int fmt)
{
    return fmt >= 0 && fmt <= 2 ? rnd(&LOWP_FMTS[fmt], v) : NAN;
}

/* Band Cholesky-Crout and the two substitutions with every operation's
 * result rounded to the format (products, differences, square roots and
 * quotients separately: no fused operations), the simulation of a factor
 * computed in that precision. */
static int band_cholesky_lowp(const lowp_fmt *f, int N, int bw, double *Ab)
{
#define L_(i, j) Ab[(size_t)(i) * (bw + 1) + ((i) - (j))]
    for (int j = 0; j < N; ++j) {
        int k0 = j - bw > 0 ? j - bw : 0;
        double s = L_(j, j);
        for (int k = k0; k < j; ++k) s = rnd(f, s - rnd(f, L_(j, k) * L_(j, k)));
        if (!(s > 0.0) || !isfinite(s)) return -1;
        double ljj = rnd(f, sqrt(s));
        L_(j, j) = ljj;
        int iend = j + bw < N - 1 ? j + bw : N - 1;
        for (int i = j + 1; i <= iend; ++i) {
            int ki = i - bw > 0 ? i - bw : 0;
            double t = L_(i, j);
            for (int k = ki; k < j; ++k) t = rnd(f, t - rnd(f, L_(i, k) * L_(j, k)));
            L_(i, j) = rnd(f, t / ljj);
        }
    }
    return 0;
#undef L_
}

static void band_solve_lowp(const lowp_fmt *f, int N, int bw, const double *Lb, double *x)
{
    for (int i = 0; i < N; ++i) {
        int k0 = i - bw > 0 ? i - bw : 0;
        double s = x[i];
        for (int k = k0; k < i; ++k) s = rnd(f, s - rnd(f, Lb[(size_t)i * (bw + 1) + (i - k)] * x[k]));
        x[i] = rnd(f, s / Lb[(size_t)i * (bw + 1)]);
    }
    for (int i = N - 1; i >= 0; --i) {
        int k1 = i + bw < N - 1 ? i + bw : N - 1;
        double s = x[i];
        for (int k = i + 1; k <= k1; ++k) s = rnd(f, s - rnd(f, Lb[(size_t)k * (bw + 1) + (k - i)] * x[k]));
        x[i] = rnd(f, s / Lb[(size_t)i * (bw + 1)]);
    }
}

/*
 * Algorithm 2.1 with (u_f, u_s, u, u_r) = (x, x, d, d) for a low precision
 * x simulated by rounding every operation (fmt 0: FP16, 1: BF16, 2: FP32):
 * the system is scaled symmetrically to unit diagonal (S A S, S =
 * diag(A)^(-1/2), the scaling the paper recommends against overflow in low
 * precision), stored and factorised in x; x0 = S (SAS)^(-1) S b by
 * substitution in x; then residual in double, stop when ||r||/||b|| < delta
 * (strict), correction t = S (SAS)^(-1) S r in x, update in double.  At most
 * imax corrections.  trips[s] = corrections applied, or -1 when the
 * factorisation broke down (a pivot not positive or not finite).  Returns the
 * number of samples that did not reach delta.
 */
int oracle_ir_lowp_batch(int n, int K, const double *Phi, int S, const double *xi, double fconst, double delta,
                         int imax, int fmt, double *Q, int *trips, double *relres)
{
    if (fmt < 0 || fmt > 2) return -1;
    const lowp_fmt *f = &LOWP_FMTS[fmt];
    int m = n - 1, N = m * m, bw = m, np = (n + 1) * (n + 1);
    double h = 1.0 / n;
    int nfail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nfail)
    for (int s = 0; s < S; ++s) {
        double *a = (double *)malloc(sizeof(double) * np);
        double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *Ab = (double *)malloc(sizeof(double) * (size_t)N * (bw + 1));
        double *b = (double *)malloc(sizeof(double) * N);
        double *x = (double *)malloc(sizeof(double) * N);
        double *r = (double *)malloc(sizeof(double) * N);
        double *t = (double *)malloc(sizeof(double) * N);
        double *sc = (double *)malloc(sizeof(double) * N);
        build_system(n, K, Phi, xi + (size_t)s * K, NULL, fconst, NULL, a, aE, aN, Ab, b);
        for (int P = 0; P < N; ++P) sc[P] = 1.0 / sqrt(Ab[(size_t)P * (bw + 1)]);
        for (int P = 0; P < N; ++P)
            for (int d = 0; d <= bw && d <= P; ++d)
                Ab[(size_t)P * (bw + 1) + d] = rnd(f, sc[P] * Ab[(size_t)P * (bw + 1) + d] * sc[P - d]);
        int it = 0;
        double rr = INFINITY;
        int broke = band_cholesky_lowp(f, N, bw, Ab) != 0;
        if (!broke) {
            for (int P = 0; P < N; ++P) t[P] = rnd(f, sc[P] * b[P]);
            band_solve_lowp(f, N, bw, Ab, t);
            for (int P = 0; P < N; ++P) x[P] = sc[P] * t[P];
            double nb = norm2(N, b);
            for (;;) {
                stencil_apply(n, aE, aN, x, r);
                for (int P = 0; P < N; ++P) r[P] = b[P] - r[P];
                rr = norm2(N, r) / nb;
                if (rr < delta || it >= imax || !isfinite(rr)) break;
                for (int P = 0; P < N; ++P) t[P] = rnd(f, sc[P] * r[P]);
                band_solve_lowp(f, N, bw, Ab, t);
                for (int P = 0; P < N; ++P) x[P] += sc[P] * t[P];
                ++it;
            }
        }
        double q = 0.0;
        for (int P = 0; P < N; ++P) q += broke ? 0.0 : x[P];
        Q[s] = h * h * q;
        trips[s] = broke ? -1 : it;
        relres[s] = rr;
        if (!(rr < delta)) nfail += 1;
        free(a); free(aE); free(aN); free(Ab); free(b); free(x); free(r); free(t); free(sc);
    }
    return nfail;
}

/*
 * Adjoint gradient of Q = h^2 sum u with respect to xi (FP64).
 * Solves A lambda = w with w = h^2 * 1 (the gradient of Q in u), then
 * dQ/dZ_e = -sum over edges (e,o) of (lambda_e - lambda_o)(u_e - u_o)
 *           * 2 a_o^2 a_e / (a_e + a_o)^2   (boundary values of u, lambda: 0),
 * dQ/dxi_k = sum_e dQ/dZ_e Phi[e, k].
 * Outputs grad[S x K]; gZ (optional, [S x (n+1)^2]); lam (optional).
 */
int oracle_grad_batch(int n, int K, const double *Phi, int S, const double *xi, double fconst,
                      double *grad, double *gZ_out, double *lam_out)
{
    int m = n - 1, N = m * m, bw = m, np = (n + 1) * (n + 1);
    double h = 1.0 / n;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < S; ++s) {
        double *a = (double *)malloc(sizeof(double) * np);
        double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
        double *Ab = (double *)malloc(sizeof(double) * (size_t)N * (bw + 1));
        double *b = (double *)malloc(sizeof(double) * N);
        double *lam = (double *)malloc(sizeof(double) * N);
        double *U = (double *)calloc(np, sizeof(double));
        double *Lm = (double *)calloc(np, sizeof(double));
        double *gZ = (double *)calloc(np, sizeof(double));
        build_system(n, K, Phi, xi + (size_t)s * K, NULL, fconst, NULL, a, aE, aN, Ab, b);
        if (band_cholesky(N, bw, Ab)) {
#pragma omp critical
            fail = s + 1;
        } else {
            band_solve(N, bw, Ab, b, b); /* b now holds u */
            for (int P = 0; P < N; ++P) lam[P] = h * h;
            band_solve(N, bw, Ab, lam, lam);
            for (int iy = 1; iy <= m; ++iy)
                for (int ix = 1; ix <= m; ++ix) {
                    int P = (iy - 1) * m + (ix - 1), p = iy * (n + 1) + ix;
                    U[p] = b[P];
                    Lm[p] = lam[P];
                }
            /* horizontal edges */
            for (int iy = 0; iy <= n; ++iy)
                for (int ix = 0; ix < n; ++ix) {
                    int p = iy * (n + 1) + ix, q = p + 1;
                    double prod = (Lm[p] - Lm[q]) * (U[p] - U[q]);
                    if (g_disc) {
                        /* d/dZ of (2a_p + 2a_q + a_t1 + a_t2)/6, a = exp(Z) */
                        gZ[p] -= prod * 2.0 * a[p] / 6.0;
                        gZ[q] -= prod * 2.0 * a[q] / 6.0;
                        if (iy + 1 <= n) gZ[p + (n + 1) + 1] -= prod * a[p + (n + 1) + 1] / 6.0;
                        if (iy - 1 >= 0) gZ[p - (n + 1)] -= prod * a[p - (n + 1)] / 6.0;
                        continue;
                    }
                    double den = (a[p] + a[q]) * (a[p] + a[q]);
                    gZ[p] -= prod * 2.0 * a[q] * a[q] * a[p] / den;
                    gZ[q] -= prod * 2.0 * a[p] * a[p] * a[q] / den;
                }
            /* vertical edges */
            for (int iy = 0; iy < n; ++iy)
                for (int ix = 0; ix <= n; ++ix) {
                    int p = iy * (n + 1) + ix, q = p + (n + 1);
                    double prod = (Lm[p] - Lm[q]) * (U[p] - U[q]);
                    if (g_disc) {
                        gZ[p] -= prod * 2.0 * a[p] / 6.0;
                        gZ[q] -= prod * 2.0 * a[q] / 6.0;
                        if (ix + 1 <= n) gZ[q + 1] -= prod * a[q + 1] / 6.0;
                        if (ix - 1 >= 0) gZ[p - 1] -= prod * a[p - 1] / 6.0;
                        continue;
                    }
                    double den = (a[p] + a[q]) * (a[p] + a[q]);
                    gZ[p] -= prod * 2.0 * a[q] * a[q] * a[p] / den;
                    gZ[q] -= prod * 2.0 * a[p] * a[p] * a[q] / den;
                }
            for (int k = 0; k < K; ++k) {
                double g = 0.0;
                for (int p = 0; p < np; ++p) g += gZ[p] * Phi[(size_t)p * K + k];
                grad[(size_t)s * K + k] = g;
            }
            if (gZ_out) memcpy(gZ_out + (size_t)s * np, gZ, sizeof(double) * np);
            if (lam_out) memcpy(lam_out + (size_t)s * N, lam, sizeof(double) * N);
        }
        free(a); free(aE); free(aN); free(Ab); free(b); free(lam); free(U); free(Lm); free(gZ);
    }
    return fail;
}

/* Energy sum_edges a_e (u_p - u_q)^2 of a solution (boundary u = 0). */
double oracle_energy(int n, int K, const double *Phi, const double *xi, const double *u)
{
    int m = n - 1, np = (n + 1) * (n + 1);
    double *a = (double *)malloc(sizeof(double) * np);
    double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
    double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
    double *U = (double *)calloc(np, sizeof(double));
    field(n, K, Phi, xi, a);
    faces(n, a, aE, aN);
    for (int iy = 1; iy <= m; ++iy)
        for (int ix = 1; ix <= m; ++ix) U[iy * (n + 1) + ix] = u[(iy - 1) * m + (ix - 1)];
    double e = 0.0;
    for (int iy = 0; iy <= n; ++iy)
        for (int ix = 0; ix < n; ++ix) {
            double d = U[iy * (n + 1) + ix] - U[iy * (n + 1) + ix + 1];
            e += aE[iy * n + ix] * d * d;
        }
    for (int iy = 0; iy < n; ++iy)
        for (int ix = 0; ix <= n; ++ix) {
            double d = U[iy * (n + 1) + ix] - U[(iy + 1) * (n + 1) + ix];
            e += aN[iy * (n + 1) + ix] * d * d;
        }
    free(a); free(aE); free(aN); free(U);
    return e;
}

/* Dense matrix of one sample (for tiny-grid checks): A[N x N] row-major. */
int oracle_dense_matrix(int n, int K, const double *Phi, const double *xi, double *A)
{
    int m = n - 1, N = m * m, bw = m, np = (n + 1) * (n + 1);
    double *a = (double *)malloc(sizeof(double) * np);
    double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
    double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
    double *Ab = (double *)malloc(sizeof(double) * (size_t)N * (bw + 1));
    double *b = (double *)malloc(sizeof(double) * N);
    build_system(n, K, Phi, xi, NULL, 1.0, NULL, a, aE, aN, Ab, b);
    memset(A, 0, sizeof(double) * (size_t)N * N);
    for (int P = 0; P < N; ++P)
        for (int d = 0; d <= bw && d <= P; ++d) {
            A[(size_t)P * N + (P - d)] = Ab[(size_t)P * (bw + 1) + d];
            A[(size_t)(P - d) * N + P] = Ab[(size_t)P * (bw + 1) + d];
        }
    free(a); free(aE); free(aN); free(Ab); free(b);
    return 0;
}

/* Band of one sample's matrix in the lower storage of assemble_band
 * (Ab[P*(bw+1) + d] = A[P, P-d], bw = n-2), for the LAPACK banded CPU line. */
int oracle_band_matrix(int n, int K, const double *Phi, const double *xi, double *Ab)
{
    int m = n - 1, N = m * m, np = (n + 1) * (n + 1);
    double *a = (double *)malloc(sizeof(double) * np);
    double *aE = (double *)malloc(sizeof(double) * (n + 1) * n);
    double *aN = (double *)malloc(sizeof(double) * (n + 1) * n);
    double *b = (double *)malloc(sizeof(double) * N);
    build_system(n, K, Phi, xi, NULL, 1.0, NULL, a, aE, aN, Ab, b);
    free(a); free(aE); free(aN); free(b);
    return 0;
}

/* Set the number of OpenMP threads of later parallel regions. */
void oracle_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* Threads an OpenMP parallel region of this library uses. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
