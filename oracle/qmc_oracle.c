/*
 * qmc_oracle.c -- plain, slow, obviously correct CPU reference for randomized
 * rank-1 lattice quasi-Monte Carlo over sector-decomposed Feynman-parameter
 * integrands (arXiv:2305.19768, Sec. 2.1 "Disteval" and Sec. 2.2 "Median QMC rules").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file.  It shares no code, header,
 * table or constant with the HIP library; the two only consume the same seeded
 * inputs.
 *
 * Compile: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (x86-64 SSE2
 * doubles; no FMA contraction, so every rounding step below is the one written).
 *
 * Every routine follows one definition, in the order the mathematics states it:
 *   - lattice rule Q_{n,z}(f) = (1/n) sum_i f({i z / n + Delta}) with random shift
 *     Delta (Sec. 2.2, definition of Q_{n,z} next to the median rule, Eq. "median");
 *   - periodizing transforms korobov_r / baker (named in the Sec. 3.2 timing notes; the
 *     formulas are the standard ones: korobov_r is the regularized incomplete beta
 *     I_y(r+1, r+1) with density (2r+1)!/(r!)^2 y^r (1-y)^r, baker is the tent map);
 *   - integrand x^p U^a F^b sum_m c_{k,m} (log F)^m per epsilon order;
 *   - per-shift sums with Neumaier compensation;
 *   - the P_2 figure of merit of a lattice (Korobov space, alpha = 2, unit product
 *     weights; Sec. 2.2 first paragraph names this criterion for the CBC vectors).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NONFINITE 1
#define OR_INVAL 2

/* ---------------------------------------------------------------- lattice */

/* (a * b) mod n, exact for all 64-bit inputs. */
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t n)
{
    if (a < 0x100000000ull && b < 0x100000000ull)
        return (a * b) % n;
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) % (unsigned __int128)n);
}

/* y_j = frac(k_j / n + Delta_j), k_j = i z_j mod n (exact integer product). */
static void lattice_point(uint64_t n, int d, const uint64_t *z, const double *delta,
                          uint64_t i, double *y)
{
    for (int j = 0; j < d; ++j) {
        uint64_t k = mulmod(i, z[j], n);
        double q = (double)k / (double)n;        /* IEEE round-to-nearest quotient */
        double v = q + delta[j];
        if (v >= 1.0)
            v = v - 1.0;                         /* exact: v in [1, 2) */
        y[j] = v;
    }
}

void or_points(uint64_t n, int d, const uint64_t *z, const double *delta, uint64_t i0,
               uint64_t count, double *y_out)
{
    for (uint64_t t = 0; t < count; ++t)
        lattice_point(n, d, z, delta, i0 + t, y_out + t * (uint64_t)d);
}

/* -------------------------------------------------------------- transform */

static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i)
        r = r * (double)(n - k + i) / (double)i;
    return r;
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i)
        r *= x;
    return r;
}

/* kind: 0 = none, 1 = baker, r + 1 = korobov_r (r = 1..6). */
static void transform1(int kind, double y, double *x, double *w)
{
    if (kind == 0) {
        *x = y;
        *w = 1.0;
    } else if (kind == 1) {
        *x = 1.0 - fabs(2.0 * y - 1.0);
        *w = 1.0;
    } else {
        int r = kind - 1;
        int N = 2 * r + 1;
        /* phi(y) = sum_{j=r+1}^{2r+1} C(2r+1, j) y^j (1-y)^(2r+1-j) */
        double phi = 0.0;
        for (int j = r + 1; j <= N; ++j)
            phi += binom(N, j) * ipow(y, j) * ipow(1.0 - y, N - j);
        /* phi'(y) = (2r+1)!/(r!)^2 y^r (1-y)^r = (2r+1) C(2r, r) y^r (1-y)^r */
        double dens = (double)N * binom(2 * r, r) * ipow(y, r) * ipow(1.0 - y, r);
        *x = phi;
        *w = dens;
    }
}

void or_transform(int kind, uint64_t count, const double *y, double *x, double *w)
{
    for (uint64_t t = 0; t < count; ++t)
        transform1(kind, y[t], &x[t], &w[t]);
}

/* -------------------------------------------------------------- integrand */

typedef struct {
    int d, n_u, n_f, u_pow, f_pow2, K, M;
    const uint8_t *u_exp;
    const double *u_coef;
    const uint8_t *f_exp;
    const double *f_coef;
    const int32_t *x_pow2;
    const double *logc;
} integrand_t;

static double poly(int d, int nmono, const uint8_t *exps, const double *coef, const double *x)
{
    double s = 0.0;
    for (int t = 0; t < nmono; ++t) {
        double v = coef[t];
        for (int j = 0; j < d; ++j)
            v *= ipow(x[j], exps[t * d + j]);
        s += v;
    }
    return s;
}

/* out[k] = x^p U^a F^b sum_m logc[k][m] L^m, L = log F. */
static void integrand(const integrand_t *g, const double *x, double *out)
{
    double U = poly(g->d, g->n_u, g->u_exp, g->u_coef, x);
    double F = poly(g->d, g->n_f, g->f_exp, g->f_coef, x);
    double base = 1.0;
    for (int j = 0; j < g->d; ++j)
        if (g->x_pow2[j] != 0)
            base *= pow(x[j], 0.5 * (double)g->x_pow2[j]);
    if (g->u_pow != 0)
        base *= pow(U, (double)g->u_pow);
    if (g->f_pow2 != 0)
        base *= pow(F, 0.5 * (double)g->f_pow2);
    double L = (g->M > 0) ? log(F) : 0.0;
    for (int k = 0; k < g->K; ++k) {
        double s = 0.0;
        for (int m = 0; m <= g->M; ++m)
            s += g->logc[k * (g->M + 1) + m] * ipow(L, m);
        out[k] = base * s;
    }
}

int or_integrand(int d, int n_u, const uint8_t *u_exp, const double *u_coef, int n_f,
                 const uint8_t *f_exp, const double *f_coef, const int32_t *x_pow2,
                 int u_pow, int f_pow2, int K, int M, const double *logc,
                 uint64_t count, const double *x, double *out)
{
    integrand_t g = {d, n_u, n_f, u_pow, f_pow2, K, M, u_exp, u_coef, f_exp, f_coef,
                     x_pow2, logc};
    for (uint64_t t = 0; t < count; ++t)
        integrand(&g, x + t * (uint64_t)d, out + t * (uint64_t)K);
    return OR_OK;
}

/* ------------------------------------------------------------------- sums */

typedef struct {
    double s, c;
} neumaier_t;

static void neumaier_add(neumaier_t *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

/*
 * Shift estimates for one sector, shifts l0..l1-1.
 *   q_out[(l-l0)*K + k]   = (1/n) sum_i W(y_i) f_k(x(y_i))       (Neumaier)
 *   abs_out[(l-l0)*K + k] = (1/n) sum_i |W(y_i) f_k(x(y_i))|
 * A sample with W == 0 contributes 0 and the integrand is not evaluated there.
 * Returns OR_NONFINITE and writes the first offending (shift, index) to bad[0..1]
 * if a contribution is not finite.
 */
int or_sums(int d, int n_u, const uint8_t *u_exp, const double *u_coef, int n_f,
            const uint8_t *f_exp, const double *f_coef, const int32_t *x_pow2, int u_pow,
            int f_pow2, int K, int M, const double *logc, int transform, uint64_t n,
            const uint64_t *z, const double *shifts, int l0, int l1, double *q_out,
            double *abs_out, int64_t *bad)
{
    if (d < 1 || d > 16 || K < 1 || K > 16 || n < 1)
        return OR_INVAL;
    integrand_t g = {d, n_u, n_f, u_pow, f_pow2, K, M, u_exp, u_coef, f_exp, f_coef,
                     x_pow2, logc};
    double y[16], x[16], fk[16];
    for (int l = l0; l < l1; ++l) {
        neumaier_t acc[16], aab[16];
        memset(acc, 0, sizeof acc);
        memset(aab, 0, sizeof aab);
        for (uint64_t i = 0; i < n; ++i) {
            lattice_point(n, d, z, shifts + (size_t)l * d, i, y);
            double W = 1.0;
            for (int j = 0; j < d; ++j) {
                double w;
                transform1(transform, y[j], &x[j], &w);
                W *= w;
            }
            if (W == 0.0)
                continue;
            integrand(&g, x, fk);
            for (int k = 0; k < K; ++k) {
                double v = W * fk[k];
                if (!isfinite(v)) {
                    if (bad) {
                        bad[0] = l;
                        bad[1] = (int64_t)i;
                    }
                    return OR_NONFINITE;
                }
                neumaier_add(&acc[k], v);
                neumaier_add(&aab[k], fabs(v));
            }
        }
        for (int k = 0; k < K; ++k) {
            q_out[(l - l0) * K + k] = (acc[k].s + acc[k].c) / (double)n;
            if (abs_out)
                abs_out[(l - l0) * K + k] = (aab[k].s + aab[k].c) / (double)n;
        }
    }
    return OR_OK;
}

/* Neumaier sum of an array (exposed so the compensation itself can be pinned). */
double or_neumaier(const double *v, uint64_t count)
{
    neumaier_t a = {0.0, 0.0};
    for (uint64_t t = 0; t < count; ++t)
        neumaier_add(&a, v[t]);
    return a.s + a.c;
}

/* --------------------------------------------------------------------- P2 */

/*
 * P_2(z) = -1 + (1/n) sum_{k=0}^{n-1} prod_j [1 + 2 pi^2 B_2({k z_j / n})],
 * B_2(x) = x^2 - x + 1/6: the squared worst-case error of the lattice rule in the
 * Korobov space of smoothness alpha = 2 with unit product weights.
 */
double or_p2(uint64_t n, int d, const uint64_t *z)
{
    const double two_pi2 = 2.0 * M_PI * M_PI;
    neumaier_t acc = {0.0, 0.0};
    for (uint64_t k = 0; k < n; ++k) {
        double prod = 1.0;
        for (int j = 0; j < d; ++j) {
            uint64_t r = mulmod(k, z[j], n);
            double x = (double)r / (double)n;
            double b2 = x * x - x + 1.0 / 6.0;
            prod *= 1.0 + two_pi2 * b2;
        }
        neumaier_add(&acc, prod);
    }
    return -1.0 + (acc.s + acc.c) / (double)n;
}

/* splitmix64 (Steele, Lea, Flood, OOPSLA 2014): state += golden gamma, then the
 * variant-13 finalizer of MurmurHash3.  Counter-based use: value of counter c is
 * mix(seed + (c + 1) * gamma). */
uint64_t or_splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t x = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* ---------------------------------------------------- contour deformation */

/*
 * Contour deformation for integrands with F - i0 (physical kinematics), the standard
 * sector-decomposition choice (the paper's library call selects its parameter from
 * presamples, Sec. 3.1.3 library-call parameters):
 *
 *   z_j(x) = x_j - i lambda x_j (1 - x_j) dF/dx_j(x),      x real in the unit cube,
 *   J(x)   = det(dz/dx),  dz_j/dx_k = delta_jk - i lambda [delta_jk (1 - 2 x_j) dF/dx_j
 *                                                           + x_j (1 - x_j) d2F/dx_j dx_k],
 *   I      = int dx J(x) f(z(x)),
 *
 * with f the analytic continuation of the whole integrand (x^p, U, F and log F all at
 * z).  Logarithms and half-integer powers of F take the branch of F - i0: the argument
 * of F lies in [-pi, pi), a negative real F has argument -pi.  The contour is valid
 * (sign check) where Im F(z) <= 0; a sample violates it when Im F(z) > 2^-40 |F(z)|,
 * the margin keeping rounding noise of an exactly non-positive Im F (at points where
 * the deformation term cancels) from counting.
 */
#include <complex.h>

typedef double complex cplx;

/* Gradient g[j] and Hessian H[j*d+k] of a monomial sum at real x, term by term. */
static void poly_derivs(int d, int nmono, const uint8_t *exps, const double *coef,
                        const double *x, double *g, double *H)
{
    for (int j = 0; j < d; ++j) {
        g[j] = 0.0;
        for (int k = 0; k < d; ++k)
            H[j * d + k] = 0.0;
    }
    for (int t = 0; t < nmono; ++t) {
        const uint8_t *e = exps + t * d;
        for (int j = 0; j < d; ++j) {
            if (e[j] == 0)
                continue;
            double v = coef[t] * (double)e[j];
            for (int i = 0; i < d; ++i)
                v *= ipow(x[i], (int)e[i] - (i == j));
            g[j] += v;
            for (int k = 0; k < d; ++k) {
                int ek = (int)e[k] - (k == j);
                if (ek <= 0)
                    continue;
                double h = coef[t] * (double)e[j] * (double)ek;
                for (int i = 0; i < d; ++i)
                    h *= ipow(x[i], (int)e[i] - (i == j) - (i == k));
                H[j * d + k] += h;
            }
        }
    }
}

static cplx cipow(cplx z, int e)
{
    int a = e < 0 ? -e : e;
    cplx r = 1.0;
    for (int i = 0; i < a; ++i)
        r *= z;
    return e < 0 ? 1.0 / r : r;
}

static cplx cpoly(int d, int nmono, const uint8_t *exps, const double *coef, const cplx *z)
{
    cplx s = 0.0;
    for (int t = 0; t < nmono; ++t) {
        cplx v = coef[t];
        for (int j = 0; j < d; ++j)
            v *= cipow(z[j], exps[t * d + j]);
        s += v;
    }
    return s;
}

static int sign_violated(cplx F)
{
    return cimag(F) > 0x1p-40 * cabs(F);
}

/* log(F - i0): argument in [-pi, pi). */
static cplx log_minus_i0(cplx F)
{
    double arg = atan2(cimag(F), creal(F));
    if (cimag(F) == 0.0 && creal(F) < 0.0)
        arg = -M_PI;
    return log(cabs(F)) + I * arg;
}

/* Determinant by Gaussian elimination with partial pivoting (destroys A). */
static cplx det_lu(int d, cplx *A)
{
    cplx det = 1.0;
    for (int c = 0; c < d; ++c) {
        int p = c;
        for (int r = c + 1; r < d; ++r)
            if (cabs(A[r * d + c]) > cabs(A[p * d + c]))
                p = r;
        if (cabs(A[p * d + c]) == 0.0)
            return 0.0;
        if (p != c) {
            for (int k = 0; k < d; ++k) {
                cplx t = A[c * d + k];
                A[c * d + k] = A[p * d + k];
                A[p * d + k] = t;
            }
            det = -det;
        }
        det *= A[c * d + c];
        for (int r = c + 1; r < d; ++r) {
            cplx f = A[r * d + c] / A[c * d + c];
            for (int k = c + 1; k < d; ++k)
                A[r * d + k] -= f * A[c * d + k];
        }
    }
    return det;
}

/* z(x), J(x) and F(z) of one point. */
static void deform_point(const integrand_t *g, double lambda, const double *x, cplx *z,
                         cplx *J, cplx *Fz)
{
    const int d = g->d;
    double grad[16], H[256];
    cplx A[256];
    poly_derivs(d, g->n_f, g->f_exp, g->f_coef, x, grad, H);
    for (int j = 0; j < d; ++j) {
        double s = x[j] * (1.0 - x[j]);
        z[j] = x[j] - I * (lambda * s * grad[j]);
        for (int k = 0; k < d; ++k)
            A[j * d + k] = -I * (lambda * s * H[j * d + k]);
        A[j * d + j] += 1.0 - I * (lambda * (1.0 - 2.0 * x[j]) * grad[j]);
    }
    *J = det_lu(d, A);
    *Fz = cpoly(d, g->n_f, g->f_exp, g->f_coef, z);
}

/* out[k] = J(x) f_k(z(x)); *Fz_out = F(z). */
static void integrand_deformed(const integrand_t *g, double lambda, const double *x,
                               cplx *out, cplx *Fz_out)
{
    cplx z[16], J, F;
    deform_point(g, lambda, x, z, &J, &F);
    cplx U = cpoly(g->d, g->n_u, g->u_exp, g->u_coef, z);
    cplx base = J;
    for (int j = 0; j < g->d; ++j) {
        int p = g->x_pow2[j];
        if (p == 0)
            continue;
        if (p % 2 == 0)
            base *= cipow(z[j], p / 2);
        else
            base *= cipow(csqrt(z[j]), p);      /* Re z_j = x_j > 0: principal root */
    }
    if (g->u_pow != 0)
        base *= cipow(U, g->u_pow);
    cplx L = log_minus_i0(F);
    if (g->f_pow2 != 0) {
        if (g->f_pow2 % 2 == 0)
            base *= cipow(F, g->f_pow2 / 2);
        else
            base *= cipow(cexp(0.5 * L), g->f_pow2);
    }
    for (int k = 0; k < g->K; ++k) {
        cplx s = 0.0;
        for (int m = 0; m <= g->M; ++m)
            s += g->logc[k * (g->M + 1) + m] * cipow(L, m);
        out[k] = base * s;
    }
    *Fz_out = F;
}

/* J f_k(z(x)) at real points x [count][d]: out[(t*K + k)*2 + {0,1}]; viol[t] = 1 where
 * the sample violates the sign check (may be NULL). */
int or_integrand_deformed(int d, int n_u, const uint8_t *u_exp, const double *u_coef, int n_f,
                          const uint8_t *f_exp, const double *f_coef, const int32_t *x_pow2,
                          int u_pow, int f_pow2, int K, int M, const double *logc,
                          double lambda, uint64_t count, const double *x, double *out,
                          int32_t *viol)
{
    if (d < 1 || d > 16 || K < 1 || K > 16)
        return OR_INVAL;
    integrand_t g = {d, n_u, n_f, u_pow, f_pow2, K, M, u_exp, u_coef, f_exp, f_coef,
                     x_pow2, logc};
    cplx fk[16], F;
    for (uint64_t t = 0; t < count; ++t) {
        integrand_deformed(&g, lambda, x + t * (uint64_t)d, fk, &F);
        for (int k = 0; k < K; ++k) {
            out[(t * K + k) * 2] = creal(fk[k]);
            out[(t * K + k) * 2 + 1] = cimag(fk[k]);
        }
        if (viol)
            viol[t] = sign_violated(F);
    }
    return OR_OK;
}

/* z [d] (re, im), J (re, im), F(z) (re, im) at one real point x. */
void or_deform_point(int d, int n_f, const uint8_t *f_exp, const double *f_coef,
                     double lambda, const double *x, double *z_out, double *J_out,
                     double *F_out)
{
    integrand_t g = {d, 0, n_f, 0, 0, 1, 0, NULL, NULL, f_exp, f_coef, NULL, NULL};
    cplx z[16], J, F;
    deform_point(&g, lambda, x, z, &J, &F);
    for (int j = 0; j < d; ++j) {
        z_out[2 * j] = creal(z[j]);
        z_out[2 * j + 1] = cimag(z[j]);
    }
    J_out[0] = creal(J);
    J_out[1] = cimag(J);
    F_out[0] = creal(F);
    F_out[1] = cimag(F);
}

/*
 * Shift estimates of one sector on the deformed contour, shifts l0..l1-1:
 *   q_out[((l-l0)*K + k)*2 + {0,1}] = Re, Im of (1/n) sum_i W(y_i) J f_k(z(x(y_i)))
 *   abs_out[(l-l0)*K + k]           = (1/n) sum_i |W J f_k|
 * Real and imaginary parts are summed separately with Neumaier compensation.  Samples
 * with W == 0 are skipped.  sign[0] counts samples violating the sign check, sign[1..2]
 * hold the first one's (shift, index); the sums are formed regardless.
 */
int or_sums_deformed(int d, int n_u, const uint8_t *u_exp, const double *u_coef, int n_f,
                     const uint8_t *f_exp, const double *f_coef, const int32_t *x_pow2,
                     int u_pow, int f_pow2, int K, int M, const double *logc, double lambda,
                     int transform, uint64_t n, const uint64_t *z, const double *shifts,
                     int l0, int l1, double *q_out, double *abs_out, int64_t *bad,
                     int64_t *sign)
{
    if (d < 1 || d > 16 || K < 1 || K > 16 || n < 1)
        return OR_INVAL;
    integrand_t g = {d, n_u, n_f, u_pow, f_pow2, K, M, u_exp, u_coef, f_exp, f_coef,
                     x_pow2, logc};
    double y[16], x[16];
    cplx fk[16], F;
    if (sign) {
        sign[0] = 0;
        sign[1] = sign[2] = -1;
    }
    for (int l = l0; l < l1; ++l) {
        neumaier_t re[16], im[16], ab[16];
        memset(re, 0, sizeof re);
        memset(im, 0, sizeof im);
        memset(ab, 0, sizeof ab);
        for (uint64_t i = 0; i < n; ++i) {
            lattice_point(n, d, z, shifts + (size_t)l * d, i, y);
            double W = 1.0;
            for (int j = 0; j < d; ++j) {
                double w;
                transform1(transform, y[j], &x[j], &w);
                W *= w;
            }
            if (W == 0.0)
                continue;
            integrand_deformed(&g, lambda, x, fk, &F);
            if (sign && sign_violated(F)) {
                if (sign[0] == 0) {
                    sign[1] = l;
                    sign[2] = (int64_t)i;
                }
                sign[0] += 1;
            }
            for (int k = 0; k < K; ++k) {
                cplx v = W * fk[k];
                if (!isfinite(creal(v)) || !isfinite(cimag(v))) {
                    if (bad) {
                        bad[0] = l;
                        bad[1] = (int64_t)i;
                    }
                    return OR_NONFINITE;
                }
                neumaier_add(&re[k], creal(v));
                neumaier_add(&im[k], cimag(v));
                neumaier_add(&ab[k], cabs(v));
            }
        }
        for (int k = 0; k < K; ++k) {
            size_t o = (size_t)(l - l0) * K + k;
            q_out[2 * o] = (re[k].s + re[k].c) / (double)n;
            q_out[2 * o + 1] = (im[k].s + im[k].c) / (double)n;
            if (abs_out)
                abs_out[o] = (ab[k].s + ab[k].c) / (double)n;
        }
    }
    return OR_OK;
}

/* Number of samples (shifts l0..l1-1, all i) violating the sign check (no integrand). */
int64_t or_sign_violations(int d, int n_f, const uint8_t *f_exp, const double *f_coef,
                           double lambda, int transform, uint64_t n, const uint64_t *z,
                           const double *shifts, int l0, int l1)
{
    integrand_t g = {d, 0, n_f, 0, 0, 1, 0, NULL, NULL, f_exp, f_coef, NULL, NULL};
    double y[16], x[16];
    cplx zz[16], J, F;
    int64_t count = 0;
    for (int l = l0; l < l1; ++l)
        for (uint64_t i = 0; i < n; ++i) {
            lattice_point(n, d, z, shifts + (size_t)l * d, i, y);
            double W = 1.0;
            for (int j = 0; j < d; ++j) {
                double w;
                transform1(transform, y[j], &x[j], &w);
                W *= w;
            }
            if (W == 0.0)
                continue;
            deform_point(&g, lambda, x, zz, &J, &F);
            if (sign_violated(F))
                ++count;
        }
    return count;
}
