/*
 * Plain FP64 CPU oracle for Fourier-accelerated steepest-descent Landau gauge
 * fixing of 4D SU(3) lattice gauge fields.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the GPU product path
 * never calls it.  It shares no code with the GPU library: links are kept as
 * full 3x3 complex matrices (array-of-structures), all nine matrix entries are
 * Fourier transformed with a recursive decimation-in-time FFT written here,
 * and every sum is Neumaier-compensated.
 *
 * Conventions (the paper's display equation for F_U[g] fixes the functional;
 * the rest is the reading of the cited steepest-descent method):
 *   sites s = x + Lx*(y + Ly*(z + Lz*t)), L = {Lx, Ly, Lz, Lt}, periodic;
 *   links U[((mu*V + s)*3 + i)*3 + j], mu = 0..3 for x, y, z, t;
 *   Nd = 4, Nc = 3, T^a = lambda_a / 2 (Gell-Mann matrices).
 *   F_U[g] = 1/(Nd Nc V) sum_x sum_mu Re Tr[g(x) U_mu(x) g(x+mu)^dagger]
 *   Delta(x) = A - Tr(A)/3, A = X - X^dagger, X = sum_mu [U_mu(x-mu) - U_mu(x)]
 *   theta = 1/(Nc V) sum_x Tr[Delta(x) Delta(x)^dagger]
 *   one iteration: g = reunit(1 + (alpha/2) * IFFT[K * FFT[Delta]]),
 *   K(p) = p2max / p2(p), K(0) = 0, p2(p) = sum_mu 4 sin^2(pi p_mu / L_mu),
 *   forward transform unnormalised, inverse with 1/V;
 *   then U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger for every link at once.
 *   reunit: Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1).
 * Variants of the step (orc_fix_ex flags): plain steepest descent (Delta in
 * place of the accelerated field) and the exact exponential
 * g = exp((alpha/2) * IFFT[K * FFT[Delta]]) (Taylor series with scaling and
 * squaring on the full 3x3 matrix).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define NC 3
#define ND 4

/* ------------------------------------------------------------------ */
/* lattice geometry                                                     */
/* ------------------------------------------------------------------ */

static int64_t volume(const int *L) { return (int64_t)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int *L, int64_t s, int c[4]) {
    for (int mu = 0; mu < 4; ++mu) { c[mu] = (int)(s % L[mu]); s /= L[mu]; }
}

static int64_t index_of(const int *L, const int c[4]) {
    return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}

/* neighbour of site s one step in direction mu (dir = +1 or -1), periodic */
static int64_t hop(const int *L, int64_t s, int mu, int dir) {
    int c[4];
    coords(L, s, c);
    c[mu] = (c[mu] + dir + L[mu]) % L[mu];
    return index_of(L, c);
}

/* ------------------------------------------------------------------ */
/* 3x3 complex matrices, row-major                                      */
/* ------------------------------------------------------------------ */

static void mat_mul(const cplx *a, const cplx *b, cplx *c) {
    cplx r[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 3; ++k) acc += a[3 * i + k] * b[3 * k + j];
            r[3 * i + j] = acc;
        }
    memcpy(c, r, sizeof r);
}

/* c = a * b^dagger */
static void mat_mul_dag(const cplx *a, const cplx *b, cplx *c) {
    cplx r[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 3; ++k) acc += a[3 * i + k] * conj(b[3 * j + k]);
            r[3 * i + j] = acc;
        }
    memcpy(c, r, sizeof r);
}

static void mat_dag(const cplx *a, cplx *c) {
    cplx r[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r[3 * i + j] = conj(a[3 * j + i]);
    memcpy(c, r, sizeof r);
}

static cplx mat_trace(const cplx *a) { return a[0] + a[4] + a[8]; }

/* reunitarise: Gram-Schmidt of rows 0,1; row 2 = conj(row0 x row1) */
static void reunit(const cplx *m, cplx *u) {
    cplx r0[3], r1[3];
    double n0 = 0;
    for (int j = 0; j < 3; ++j) n0 += creal(m[j] * conj(m[j]));
    n0 = sqrt(n0);
    for (int j = 0; j < 3; ++j) r0[j] = m[j] / n0;
    cplx ip = 0; /* <r0, m1> = sum conj(r0_j) m1_j */
    for (int j = 0; j < 3; ++j) ip += conj(r0[j]) * m[3 + j];
    for (int j = 0; j < 3; ++j) r1[j] = m[3 + j] - ip * r0[j];
    double n1 = 0;
    for (int j = 0; j < 3; ++j) n1 += creal(r1[j] * conj(r1[j]));
    n1 = sqrt(n1);
    for (int j = 0; j < 3; ++j) r1[j] /= n1;
    for (int j = 0; j < 3; ++j) { u[j] = r0[j]; u[3 + j] = r1[j]; }
    u[6] = conj(r0[1] * r1[2] - r0[2] * r1[1]);
    u[7] = conj(r0[2] * r1[0] - r0[0] * r1[2]);
    u[8] = conj(r0[0] * r1[1] - r0[1] * r1[0]);
}

/* Gell-Mann matrices lambda_a, a = 0..7 (lambda_1..lambda_8 in the usual count) */
static void gell_mann(int a, cplx *m) {
    for (int k = 0; k < 9; ++k) m[k] = 0;
    const double r3 = 1.0 / sqrt(3.0);
    switch (a) {
    case 0: m[1] = 1; m[3] = 1; break;
    case 1: m[1] = -I; m[3] = I; break;
    case 2: m[0] = 1; m[4] = -1; break;
    case 3: m[2] = 1; m[6] = 1; break;
    case 4: m[2] = -I; m[6] = I; break;
    case 5: m[5] = 1; m[7] = 1; break;
    case 6: m[5] = -I; m[7] = I; break;
    default: m[0] = r3; m[4] = r3; m[8] = -2 * r3; break;
    }
}

/* ------------------------------------------------------------------ */
/* compensated summation (Neumaier)                                     */
/* ------------------------------------------------------------------ */

static double neumaier_sum(const double *v, int64_t n) {
    double s = 0, c = 0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i])) c += (s - t) + v[i];
        else c += (v[i] - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------ */
/* threads                                                               */
/* ------------------------------------------------------------------ */

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* F, Delta, theta                                                       */
/* ------------------------------------------------------------------ */

/* F_U[g] of the paper's display equation; g == NULL means g = 1 everywhere. */
double orc_functional(const int *L, const cplx *U, const cplx *g) {
    const int64_t V = volume(L);
    double *site = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        double acc = 0;
        for (int mu = 0; mu < ND; ++mu) {
            const cplx *u = U + (mu * V + s) * 9;
            if (g) {
                cplx t[9];
                mat_mul(g + s * 9, u, t);
                mat_mul_dag(t, g + hop(L, s, mu, +1) * 9, t);
                acc += creal(mat_trace(t));
            } else {
                acc += creal(mat_trace(u));
            }
        }
        site[s] = acc;
    }
    double F = neumaier_sum(site, V) / ((double)ND * NC * (double)V);
    free(site);
    return F;
}

double orc_F(const int *L, const cplx *U) { return orc_functional(L, U, NULL); }

/* Delta(x) = A - Tr(A)/3 * 1, A = X - X^dagger, X = sum_mu U_mu(x-mu) - U_mu(x) */
void orc_delta(const int *L, const cplx *U, cplx *D) {
    const int64_t V = volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx X[9] = {0};
        for (int mu = 0; mu < ND; ++mu) {
            const cplx *um = U + (mu * V + hop(L, s, mu, -1)) * 9;
            const cplx *u = U + (mu * V + s) * 9;
            for (int k = 0; k < 9; ++k) X[k] += um[k] - u[k];
        }
        cplx A[9], Xd[9];
        mat_dag(X, Xd);
        for (int k = 0; k < 9; ++k) A[k] = X[k] - Xd[k];
        cplx tr = mat_trace(A) / 3.0;
        A[0] -= tr; A[4] -= tr; A[8] -= tr;
        memcpy(D + s * 9, A, sizeof A);
    }
}

/* theta = 1/(Nc V) sum_x Tr[Delta Delta^dagger] of the given Delta field */
double orc_theta_of_delta(const int *L, const cplx *D) {
    const int64_t V = volume(L);
    double *site = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        double acc = 0;
        for (int k = 0; k < 9; ++k) acc += creal(D[s * 9 + k] * conj(D[s * 9 + k]));
        site[s] = acc;
    }
    double th = neumaier_sum(site, V) / ((double)NC * (double)V);
    free(site);
    return th;
}

double orc_theta(const int *L, const cplx *U) {
    const int64_t V = volume(L);
    cplx *D = malloc(sizeof(cplx) * 9 * V);
    orc_delta(L, U, D);
    double th = orc_theta_of_delta(L, D);
    free(D);
    return th;
}

/* ------------------------------------------------------------------ */
/* FFT: recursive decimation in time along each axis                     */
/* ------------------------------------------------------------------ */

static int smallest_factor(int n) {
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* W[j] = exp(sign * 2 pi i j / n), computed in long double */
static cplx *twiddles(int n, int sign) {
    cplx *W = malloc(sizeof(cplx) * n);
    const long double twopi = 6.283185307179586476925286766559005768L;
    for (int j = 0; j < n; ++j) {
        long double a = twopi * (long double)j / (long double)n;
        W[j] = (double)cosl(a) + I * (double)(sign * sinl(a));
    }
    return W;
}

/*
 * out[k] = sum_j in[j*is] * exp(sign 2 pi i j k / n) for k < n.
 * W is the table for length n0 (a multiple of n), wstep = n0 / n.
 * Split n = p*m with p the smallest prime factor: transform the p
 * subsequences in[(j*p + r)*is] (length m), then combine
 * X[k + q*m] = sum_r W_n^{r*(k + q*m)} Y_r[k].
 */
static void dft_rec(const cplx *in, int64_t is, cplx *out, int n, const cplx *W, int n0, int wstep) {
    if (n == 1) { out[0] = in[0]; return; }
    const int p = smallest_factor(n), m = n / p;
    for (int r = 0; r < p; ++r) dft_rec(in + r * is, is * p, out + r * m, m, W, n0, wstep * p);
    cplx t[64]; /* p <= 64 is enforced by the caller's size check */
    for (int k = 0; k < m; ++k) {
        for (int r = 0; r < p; ++r) t[r] = out[r * m + k];
        for (int q = 0; q < p; ++q) {
            cplx acc = 0;
            const int e = k + q * m;
            for (int r = 0; r < p; ++r) acc += W[((int64_t)r * e % n) * wstep] * t[r];
            out[k + q * m] = acc;
        }
    }
}

/*
 * Unnormalised 4D DFT, in place, of every component of a[s*ncomp + c]:
 * a(n) <- sum_x a(x) exp(sign * 2 pi i sum_mu n_mu x_mu / L_mu).
 * Returns 0, or -1 if an extent has a prime factor above 64.
 */
int orc_fft4d(const int *L, cplx *a, int ncomp, int sign) {
    const int64_t V = volume(L);
    for (int mu = 0; mu < 4; ++mu) {
        int n = L[mu], q = n;
        while (q > 1) { int p = smallest_factor(q); if (p > 64) return -1; q /= p; }
    }
    int64_t stride = 1;
    for (int mu = 0; mu < 4; ++mu) {
        const int n = L[mu];
        cplx *W = twiddles(n, sign);
        const int64_t nlines = V / n * ncomp;
#pragma omp parallel
        {
            cplx *buf = malloc(sizeof(cplx) * n), *res = malloc(sizeof(cplx) * n);
#pragma omp for schedule(static)
            for (int64_t line = 0; line < nlines; ++line) {
                const int64_t c = line % ncomp, rest = line / ncomp;
                const int64_t lo = rest % stride, hi = rest / stride;
                const int64_t base = lo + hi * stride * n;
                for (int j = 0; j < n; ++j) buf[j] = a[(base + j * stride) * ncomp + c];
                dft_rec(buf, 1, res, n, W, n, 1);
                for (int j = 0; j < n; ++j) a[(base + j * stride) * ncomp + c] = res[j];
            }
            free(buf); free(res);
        }
        free(W);
        stride *= n;
    }
    return 0;
}

/* Brute-force 4D DFT of a single complex field (O(V^2)); for tiny lattices. */
void orc_dft4d_naive(const int *L, const cplx *in, cplx *out, int sign) {
    const int64_t V = volume(L);
    const long double twopi = 6.283185307179586476925286766559005768L;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < V; ++k) {
        int n[4];
        coords(L, k, n);
        cplx acc = 0;
        for (int64_t s = 0; s < V; ++s) {
            int x[4];
            coords(L, s, x);
            long double ph = 0;
            for (int mu = 0; mu < 4; ++mu)
                ph += (long double)(((int64_t)n[mu] * x[mu]) % L[mu]) / (long double)L[mu];
            ph *= twopi;
            acc += in[s] * ((double)cosl(ph) + I * (double)(sign * sinl(ph)));
        }
        out[k] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* Fourier acceleration                                                  */
/* ------------------------------------------------------------------ */

/* lattice momentum squared p2(n) = sum_mu 4 sin^2(pi n_mu / L_mu) */
static double p2_of(const int *L, const int n[4]) {
    const long double pi = 3.141592653589793238462643383279502884L;
    long double acc = 0;
    for (int mu = 0; mu < 4; ++mu) {
        long double sn = sinl(pi * (long double)n[mu] / (long double)L[mu]);
        acc += 4.0L * sn * sn;
    }
    return (double)acc;
}

double orc_p2max(const int *L) {
    const int64_t V = volume(L);
    double m = 0;
    for (int64_t k = 0; k < V; ++k) {
        int n[4];
        coords(L, k, n);
        double p2 = p2_of(L, n);
        if (p2 > m) m = p2;
    }
    return m;
}

/*
 * LD = IFFT[ K * FFT[D] ] with K(p) = p2max/p2(p), K(0) = 0, the forward
 * transform unnormalised and the inverse divided by V; all 9 entries.
 */
int orc_fourier_accelerate(const int *L, const cplx *D, cplx *LD) {
    const int64_t V = volume(L);
    memcpy(LD, D, sizeof(cplx) * 9 * V);
    if (orc_fft4d(L, LD, 9, -1)) return -1;
    const double p2max = orc_p2max(L);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < V; ++k) {
        int n[4];
        coords(L, k, n);
        double p2 = p2_of(L, n);
        double K = (k == 0) ? 0.0 : p2max / p2;
        for (int c = 0; c < 9; ++c) LD[k * 9 + c] *= K / (double)V;
    }
    return orc_fft4d(L, LD, 9, +1);
}

/* g(x) = reunit(1 + (alpha/2) LD(x)) for the current links */
int orc_gauge_field(const int *L, const cplx *U, double alpha, cplx *g) {
    const int64_t V = volume(L);
    cplx *D = malloc(sizeof(cplx) * 9 * V);
    cplx *LD = malloc(sizeof(cplx) * 9 * V);
    orc_delta(L, U, D);
    int rc = orc_fourier_accelerate(L, D, LD);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx M[9];
        for (int k = 0; k < 9; ++k) M[k] = 0.5 * alpha * LD[s * 9 + k];
        M[0] += 1; M[4] += 1; M[8] += 1;
        reunit(M, g + s * 9);
    }
    free(D); free(LD);
    return rc;
}

/* U_mu(x) <- g(x) U_mu(x) g(x+mu)^dagger for every link (old U, one g field) */
void orc_gauge_rotate(const int *L, cplx *U, const cplx *g) {
    const int64_t V = volume(L);
    cplx *Un = malloc(sizeof(cplx) * 9 * 4 * V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        for (int mu = 0; mu < ND; ++mu) {
            cplx t[9];
            mat_mul(g + s * 9, U + (mu * V + s) * 9, t);
            mat_mul_dag(t, g + hop(L, s, mu, +1) * 9, Un + (mu * V + s) * 9);
        }
    }
    memcpy(U, Un, sizeof(cplx) * 9 * 4 * V);
    free(Un);
}

/* exactly n gauge updates */
int orc_iterate(const int *L, cplx *U, double alpha, int n) {
    const int64_t V = volume(L);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    int rc = 0;
    for (int it = 0; it < n && !rc; ++it) {
        rc = orc_gauge_field(L, U, alpha, g);
        if (!rc) orc_gauge_rotate(L, U, g);
    }
    free(g);
    return rc;
}

/*
 * Iterate until theta < tol (tested before each update) or max_iter updates.
 * Outputs: *iters = updates applied; *F, *theta of the returned links;
 * F_hist/theta_hist (may be NULL) receive F_n, theta_n for n = 0..*iters.
 * Returns 0 if converged, 1 if max_iter was reached, 2 on non-finite theta.
 */
#define ORC_ACCELERATE 1 /* Fourier acceleration (else plain steepest descent) */
#define ORC_EXACT_EXP 2  /* g = exp((alpha/2) L Delta) instead of reunit(1 + ...) */

static void mat_exp(const cplx *X, cplx *E);

int orc_fix_ex(const int *L, cplx *U, double alpha, double tol, int max_iter, int flags,
               int *iters, double *F, double *theta, double *F_hist, double *theta_hist);

int orc_fix(const int *L, cplx *U, double alpha, double tol, int max_iter,
            int *iters, double *F, double *theta, double *F_hist, double *theta_hist) {
    return orc_fix_ex(L, U, alpha, tol, max_iter, ORC_ACCELERATE, iters, F, theta, F_hist,
                      theta_hist);
}

/*
 * As orc_fix, with the variants of the update step chosen by flags:
 *   without ORC_ACCELERATE: plain steepest descent (the method before Fourier
 *     acceleration), the step is built from Delta itself, no transform;
 *   with ORC_EXACT_EXP: the step matrix (alpha/2) L Delta is exponentiated
 *     exactly (mat_exp) instead of to first order plus reunitarisation.
 */
int orc_fix_ex(const int *L, cplx *U, double alpha, double tol, int max_iter, int flags,
               int *iters, double *F, double *theta, double *F_hist, double *theta_hist) {
    const int accelerate = flags & ORC_ACCELERATE, exact = flags & ORC_EXACT_EXP;
    const int64_t V = volume(L);
    cplx *D = malloc(sizeof(cplx) * 9 * V);
    cplx *LD = malloc(sizeof(cplx) * 9 * V);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    int n = 0, status = 1;
    for (;;) {
        orc_delta(L, U, D);
        const double th = orc_theta_of_delta(L, D);
        const double f = orc_F(L, U);
        if (F_hist) F_hist[n] = f;
        if (theta_hist) theta_hist[n] = th;
        *F = f; *theta = th;
        if (!isfinite(th)) { status = 2; break; }
        if (th < tol) { status = 0; break; }
        if (n >= max_iter) { status = 1; break; }
        if (accelerate) {
            if (orc_fourier_accelerate(L, D, LD)) { status = 2; break; }
        } else {
            memcpy(LD, D, sizeof(cplx) * 9 * V);
        }
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < V; ++s) {
            cplx M[9];
            for (int k = 0; k < 9; ++k) M[k] = 0.5 * alpha * LD[s * 9 + k];
            if (exact) {
                mat_exp(M, g + s * 9);
            } else {
                M[0] += 1; M[4] += 1; M[8] += 1;
                reunit(M, g + s * 9);
            }
        }
        orc_gauge_rotate(L, U, g);
        ++n;
    }
    *iters = n;
    free(D); free(LD); free(g);
    return status;
}

/* ------------------------------------------------------------------ */
/* gauge-invariant and group checks                                      */
/* ------------------------------------------------------------------ */

/* average plaquette 1/(6 Nc V) sum_x sum_{mu<nu} Re Tr U_mu(x)U_nu(x+mu)U_mu(x+nu)^+ U_nu(x)^+ */
double orc_plaquette(const int *L, const cplx *U) {
    const int64_t V = volume(L);
    double *site = malloc(sizeof(double) * V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        double acc = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                cplx a[9], b[9];
                mat_mul(U + (mu * V + s) * 9, U + (nu * V + hop(L, s, mu, +1)) * 9, a);
                mat_mul_dag(a, U + (mu * V + hop(L, s, nu, +1)) * 9, b);
                mat_mul_dag(b, U + (nu * V + s) * 9, a);
                acc += creal(mat_trace(a));
            }
        site[s] = acc;
    }
    double P = neumaier_sum(site, V) / (6.0 * NC * (double)V);
    free(site);
    return P;
}

/* max |(U U^+ - 1)_ij| and max |det U - 1| over nmat matrices */
void orc_unitarity(const cplx *U, int64_t nmat, double *max_unit, double *max_det) {
    double mu_ = 0, md = 0;
#pragma omp parallel for schedule(static) reduction(max : mu_, md)
    for (int64_t k = 0; k < nmat; ++k) {
        const cplx *u = U + k * 9;
        cplx p[9];
        mat_mul_dag(u, u, p);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double d = cabs(p[3 * i + j] - (i == j ? 1.0 : 0.0));
                if (d > mu_) mu_ = d;
            }
        cplx det = u[0] * (u[4] * u[8] - u[5] * u[7]) - u[1] * (u[3] * u[8] - u[5] * u[6]) +
                   u[2] * (u[3] * u[7] - u[4] * u[6]);
        double dd = cabs(det - 1.0);
        if (dd > md) md = dd;
    }
    *max_unit = mu_;
    *max_det = md;
}

/* ------------------------------------------------------------------ */
/* differentiation                                                       */
/* ------------------------------------------------------------------ */

/* X = i sum_a w_a T^a (anti-hermitian, traceless) */
static void su3_generator(const double *w, cplx *X) {
    for (int k = 0; k < 9; ++k) X[k] = 0;
    for (int a = 0; a < 8; ++a) {
        cplx lam[9];
        gell_mann(a, lam);
        for (int k = 0; k < 9; ++k) X[k] += 0.5 * I * w[a] * lam[k];
    }
}

/* exp(X) by scaling and squaring of the Taylor series */
static void mat_exp(const cplx *X, cplx *E) {
    double nrm = 0;
    for (int k = 0; k < 9; ++k) nrm += creal(X[k] * conj(X[k]));
    nrm = sqrt(nrm);
    int sq = 0;
    while (nrm > 0.25) { nrm *= 0.5; ++sq; }
    const double scale = ldexp(1.0, -sq);
    cplx Y[9], term[9], sum[9];
    for (int k = 0; k < 9; ++k) { Y[k] = X[k] * scale; term[k] = 0; sum[k] = 0; }
    term[0] = term[4] = term[8] = 1;
    sum[0] = sum[4] = sum[8] = 1;
    for (int n = 1; n <= 30; ++n) {
        mat_mul(term, Y, term);
        for (int k = 0; k < 9; ++k) { term[k] /= n; sum[k] += term[k]; }
    }
    for (int i = 0; i < sq; ++i) mat_mul(sum, sum, sum);
    memcpy(E, sum, sizeof sum);
}

/* g = exp(i sum_a w_a T^a) */
void orc_expm_su3(const double *w, cplx *g) {
    cplx X[9];
    su3_generator(w, X);
    mat_exp(X, g);
}

static void omega_to_g(const int *L, const double *omega, cplx *g) {
    const int64_t V = volume(L);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) orc_expm_su3(omega + s * 8, g + s * 9);
}

/* F_U[g] with g(x) = exp(i omega^a(x) T^a) */
double orc_functional_omega(const int *L, const cplx *U, const double *omega) {
    const int64_t V = volume(L);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    omega_to_g(L, omega, g);
    double F = orc_functional(L, U, g);
    free(g);
    return F;
}

/*
 * dF/domega^a(x) for F = F_U[exp(i omega T)].  With the gauge-transformed links
 * U^g, G^b(x) = -(i/(4 Nd Nc V)) Tr[lambda_b Delta[U^g](x)] is the derivative
 * along right-multiplied generators (delta g = i eps T^b g); the chain rule
 * through the exponential map uses
 *   d/deps exp(X + eps Y) = dexp_X(Y) exp(X),  dexp_X(Y) = sum_k ad_X^k(Y)/(k+1)!,
 * so dF/domega^a = sum_b J_ab G^b with J_ab = Tr[lambda_b (-i) dexp_X(i T^a)].
 */
double orc_functional_omega_grad(const int *L, const cplx *U, const double *omega, double *dF) {
    const int64_t V = volume(L);
    cplx *g = malloc(sizeof(cplx) * 9 * V);
    cplx *Ug = malloc(sizeof(cplx) * 9 * 4 * V);
    cplx *D = malloc(sizeof(cplx) * 9 * V);
    omega_to_g(L, omega, g);
    memcpy(Ug, U, sizeof(cplx) * 9 * 4 * V);
    orc_gauge_rotate(L, Ug, g);
    const double F = orc_F(L, Ug);
    orc_delta(L, Ug, D);
    const double norm = 1.0 / ((double)ND * NC * (double)V);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx lam[8][9];
        for (int b = 0; b < 8; ++b) gell_mann(b, lam[b]);
        double G[8];
        for (int b = 0; b < 8; ++b) {
            cplx t[9];
            mat_mul(lam[b], D + s * 9, t);
            G[b] = creal(-0.25 * I * norm * mat_trace(t));
        }
        cplx X[9];
        su3_generator(omega + s * 8, X);
        for (int a = 0; a < 8; ++a) {
            /* dexp_X(i T^a) = sum_k ad_X^k(Y)/(k+1)!, ad_X(Y) = XY - YX */
            cplx Y[9], term[9], sum[9];
            for (int k = 0; k < 9; ++k) { Y[k] = 0.5 * I * lam[a][k]; term[k] = Y[k]; sum[k] = Y[k]; }
            for (int k = 1; k <= 60; ++k) {
                cplx p[9], q[9];
                mat_mul(X, term, p);
                mat_mul(term, X, q);
                double tn = 0;
                for (int e = 0; e < 9; ++e) { term[e] = (p[e] - q[e]) / (k + 1); tn += cabs(term[e]); sum[e] += term[e]; }
                if (tn < 1e-20) break;
            }
            double acc = 0;
            for (int b = 0; b < 8; ++b) {
                cplx t[9];
                mat_mul(lam[b], sum, t);
                acc += creal(-I * mat_trace(t)) * G[b];
            }
            dF[s * 8 + a] = acc;
        }
    }
    free(g); free(Ug); free(D);
    return F;
}

/*
 * dtheta/deps^a_mu(x) for U_mu(x) -> exp(i eps^a T^a) U_mu(x):
 *   -(1/(Nc V)) Re Tr[i lambda_a (U D + D U^dagger)],  D = Delta(x+mu) - Delta(x).
 * Output layout dth[(mu*V + s)*8 + a].  Returns theta.
 */
double orc_theta_grad(const int *L, const cplx *U, double *dth) {
    const int64_t V = volume(L);
    cplx *D = malloc(sizeof(cplx) * 9 * V);
    orc_delta(L, U, D);
    const double th = orc_theta_of_delta(L, D);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx lam[8][9];
        for (int a = 0; a < 8; ++a) gell_mann(a, lam[a]);
        for (int mu = 0; mu < 4; ++mu) {
            const cplx *u = U + (mu * V + s) * 9;
            const cplx *dp = D + hop(L, s, mu, +1) * 9, *d0 = D + s * 9;
            cplx Dd[9], W1[9], W2[9], Ud[9], W[9];
            for (int k = 0; k < 9; ++k) Dd[k] = dp[k] - d0[k];
            mat_mul(u, Dd, W1);
            mat_dag(u, Ud);
            mat_mul(Dd, Ud, W2);
            for (int k = 0; k < 9; ++k) W[k] = W1[k] + W2[k];
            for (int a = 0; a < 8; ++a) {
                cplx t[9];
                mat_mul(lam[a], W, t);
                dth[(mu * V + s) * 8 + a] = -creal(I * mat_trace(t)) / ((double)NC * (double)V);
            }
        }
    }
    free(D);
    return th;
}
