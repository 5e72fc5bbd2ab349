/*
 * qmcamp.h -- C ABI of the MI355X (gfx950) randomized rank-1 lattice QMC library
 * for sector-decomposed Feynman-parameter integrals and weighted sums of them
 * (amplitudes), after arXiv:2305.19768 (pySecDec 1.6), Sec. 2.1 and 2.2.
 *
 * The problem statement follows the paper's: a set of integrals, each a sum of
 * sectors; each sector an integrand over the unit cube expanded in epsilon up to a
 * fixed order; a rank-1 lattice of size n with generating vector z per sector, m
 * random shifts; weighted sums A = sum_i C_i I_i; value and error estimate out
 * (Sec. 2.1.1 usage, Sec. 2.1.3 adaptive weighted sums, Sec. 2.4 coefficients).
 *
 * Conventions
 *   - Plain C types only.  Pointers are host pointers unless the name starts with
 *     "dev_"; device pointers are HIP device addresses (e.g. a torch tensor's
 *     data_ptr()).  "stream" is a hipStream_t passed as void* (NULL = legacy stream).
 *   - The library copies every host input it needs during the call; the caller may
 *     free host buffers as soon as a call returns.
 *   - The library allocates no device memory: all device storage is the caller's
 *     workspace bound with qmc_bind_workspace() plus the caller's output buffers.
 *   - Errors are negative qmc_status codes; qmc_last_error() returns a thread-local
 *     message describing the most recent failure.  Argument checks happen before
 *     any launch, so a QMC_E_INVAL call has no device side effects.
 *   - Calls on one plan are not thread-safe; distinct plans are independent.
 */
#ifndef QMCAMP_H
#define QMCAMP_H

#ifndef __HIPCC_RTC__   /* run-time compiled kernels get the integer types built in */
#include <stddef.h>
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMC_OK = 0,
    QMC_E_INVAL = -1,      /* invalid argument; nothing was launched */
    QMC_E_NOMEM = -2,      /* host allocation failed or workspace too small */
    QMC_E_DEVICE = -3,     /* a HIP runtime call failed */
    QMC_E_NONFINITE = -4,  /* a per-shift sum is not finite; see qmc_query_status */
    QMC_E_TIMEOUT = -5,    /* amp_evaluate stopped at its time limit (results valid, flagged) */
    QMC_E_SIGNCHECK = -6,  /* deformed contour left the F - i0 half plane; see qmc_sign_violations */
    QMC_E_STATE = -7       /* call out of order (e.g. no workspace bound) */
} qmc_status;

/* Periodizing transforms (the paper's "korobov3" default and "baker", Sec. 3.2 timing notes). */
enum {
    QMC_TRANSFORM_NONE = 0,     /* x = y, w = 1 (tests only) */
    QMC_TRANSFORM_BAKER = 1,    /* tent map x = 1 - |2y - 1|, w = 1 */
    QMC_TRANSFORM_KOROBOV1 = 2, /* korobov_r = QMC_TRANSFORM_KOROBOV1 + r - 1, r = 1..6: */
    QMC_TRANSFORM_KOROBOV3 = 4, /*   x = I_y(r+1, r+1), w = (2r+1)!/(r!)^2 (y(1-y))^r    */
    QMC_TRANSFORM_KOROBOV6 = 7
};

enum { QMC_PREC_FP64 = 0, QMC_PREC_FP32 = 1 };

#define QMC_MAX_DIM 8      /* Feynman parameters per sector after the delta constraint */
#define QMC_MAX_ORDERS 4   /* epsilon orders per sector */
#define QMC_MAX_LOG 4      /* highest power of log F per order */
#define QMC_MAX_DEG 3      /* total degree of U and F (one- and two-loop graphs) */
#define QMC_MAX_SHIFTS 64
#define QMC_FLOW_LAYERS 4  /* affine coupling layers of a learned flow transform */
#define QMC_FLOW_HIDDEN 64 /* hidden width of each coupling layer's network */
#define QMC_FLOW_MAX_COND 4 /* conditioning features of a conditional flow (d + n_cond <= 16) */

/*
 * One sector integrand, expanded in epsilon (Sec. 2.3 and 3: sector-decomposed
 * parameter integrals, all orders up to the finite one are integrated):
 *
 *   f_k(x) = prod_j x_j^(x_pow2[j]/2) * U(x)^u_pow * F(x)^(f_pow2/2)
 *            * sum_{m=0}^{max_log} logc[k][m] * (log F(x))^m ,   k = 0 .. n_orders-1
 *
 * U and F are sums of monomials c * prod_j x_j^e_j with total degree <= QMC_MAX_DEG;
 * their monomials are rows u_off .. u_off+n_u-1 (f_off .. f_off+n_f-1) of the
 * problem's mono_exp / mono_coef arrays.  Repeated exponent rows are summed.
 *
 * Contour deformation (physical kinematics, F may change sign; the deformation
 * parameter is chosen from presamples in the paper's library call, Sec. 3.1.3): with
 * deform_lambda = lambda > 0 the sector is integrated over
 *   z_j(x) = x_j - i lambda x_j (1 - x_j) dF/dx_j(x),
 *   I_k = int dx det(dz/dx) f_k(z(x)),
 * f_k continued analytically (x^p, U, F, log F all at z); log F and half-integer powers
 * of F take the F - i0 branch (argument of F in [-pi, pi)).  The contour is valid where
 * Im F(z) <= 0; a sample with Im F(z) > 2^-40 |F(z)| is a sign-check violation.  A
 * problem with any deformed sector makes a complex plan: every sector's integrand is
 * complex (lambda = 0 sectors are integrated on the real contour with the F - i0
 * branch) and every per-order output carries (re, im) pairs.
 */
typedef struct {
    int32_t d;                        /* 1 .. QMC_MAX_DIM */
    int32_t integral;                 /* index of the integral this sector belongs to */
    int32_t n_u, n_f;                 /* number of monomials of U and F (n_f >= 1) */
    int64_t u_off, f_off;             /* first monomial row of U and F */
    int32_t x_pow2[QMC_MAX_DIM];      /* twice the exponent of x_j, |x_pow2| <= 16 */
    int32_t u_pow;                    /* exponent of U, |u_pow| <= 8 */
    int32_t f_pow2;                   /* twice the exponent of F, |f_pow2| <= 16 */
    int32_t transform;                /* QMC_TRANSFORM_* */
    int32_t reserved0;
    double logc[QMC_MAX_ORDERS][QMC_MAX_LOG + 1];
    uint64_t n;                       /* default lattice size (prime or any n >= 2) */
    uint64_t a;                       /* default Korobov parameter, z = (1, a, a^2, ...) mod n */
    double deform_lambda;             /* >= 0; > 0: contour deformation (see above) */
} qmc_sector_desc;

typedef struct {
    int32_t n_sectors;                /* >= 1 */
    int32_t n_orders;                 /* K, 1 .. QMC_MAX_ORDERS */
    int32_t order_lo;                 /* epsilon power of order 0 (informational) */
    int32_t max_log;                  /* 0 .. QMC_MAX_LOG */
    int32_t n_integrals;              /* >= 1; every sector's integral < n_integrals */
    int32_t reserved0;
    const qmc_sector_desc *sectors;   /* [n_sectors] */
    const uint8_t *mono_exp;          /* [rows][QMC_MAX_DIM] exponents, row-major */
    const double *mono_coef;          /* [rows] coefficients */
    int64_t n_mono_rows;
} qmc_problem;

typedef struct {
    int32_t m;                        /* random shifts per sector, 2 .. QMC_MAX_SHIFTS */
    int32_t precision;                /* QMC_PREC_FP64 (default) or QMC_PREC_FP32.
                                         FP32, real plans: korobov3 sectors whose U and F
                                         have no cancellation on the cube evaluate the
                                         transform and the integrand in FP32; the rest
                                         stay FP64.  FP32, complex plans: sectors with
                                         deform_lambda > 0 at plan time, or without
                                         cancellation, evaluate grad F, the Hessian of F,
                                         U(z) and F(z) in FP32 and the Jacobian, powers,
                                         logarithm and sign check from those in FP64
                                         (sign check margin 2^-20 |F| instead of 2^-40).
                                         Lattice points and sums are FP64 throughout.
                                         Error of the FP32 form: the first integration
                                         (and the first after qmc_set_shifts, a flow or a
                                         deformation change) integrates every sector on
                                         a calibration lattice (n = 1021, Korobov
                                         parameter of least P_2) with both forms and the
                                         plan's shifts, synchronizing the stream once;
                                         per (sector, order) -- per real and imaginary
                                         part in complex plans -- the shift differences
                                         D_l = Q32_l - Q64_l give the bound
                                         |mean D| + 3 x its standard error, which every
                                         err output of the plan then includes (0 for
                                         sectors evaluated in FP64). */
    uint64_t seed;                    /* seed of the built-in shift generator */
    uint64_t n_max;                   /* largest lattice size any call will use (sizes the
                                         workspace); 0 = max of the sectors' n */
    int32_t block;                    /* threads per workgroup (64..1024, multiple of 64);
                                         0 = tuned default */
    int32_t shift_tile;               /* shifts per workgroup, 1..16, divides m; 0 = tuned */
    int32_t shifts_per_pass;          /* shifts evaluated per lattice point in one pass:
                                         1, 2 or 4, divides shift_tile; 0 = tuned */
    int32_t reserved0;
} qmc_options;

typedef struct qmc_plan_s *qmc_plan_t;

/*
 * qmc_plan -- validate a problem and pack it for the device (the per-integrand
 * hoisting of Sec. 2.1: everything that does not depend on the lattice point is
 * prepared once).  Copies the host tables; computes each sector's dense nested-Horner
 * coefficient table for U and F; derives the shifts from opt->seed.  Host only: no
 * HIP call is made.  On success *out owns the plan (free with qmc_plan_free).
 * Errors: QMC_E_INVAL (bad dimension, degree > QMC_MAX_DEG, exponent out of range,
 * offsets outside the monomial arrays, non-finite coefficient, m out of range),
 * QMC_E_NOMEM.
 */
qmc_status qmc_plan(const qmc_problem *prob, const qmc_options *opt, qmc_plan_t *out);

/* Bytes of device workspace qmc_bind_workspace needs for this plan (0 on NULL). */
size_t qmc_workspace_bytes(qmc_plan_t plan);

/*
 * qmc_bind_workspace -- hand the plan a caller-owned device buffer of at least
 * qmc_workspace_bytes() bytes (256-byte aligned) and upload the packed tables on
 * `stream`.  The buffer must stay valid until the plan is freed or rebound.  The first
 * bind also creates the plan's side streams and events on the current device.
 * Errors: QMC_E_INVAL (NULL / misaligned), QMC_E_NOMEM (too small), QMC_E_DEVICE.
 */
qmc_status qmc_bind_workspace(qmc_plan_t plan, void *dev_workspace, size_t bytes, void *stream);

/*
 * qmc_set_shifts -- replace the shifts with caller values: host array
 * shifts[s][l][j], s < n_sectors, l < m, j < QMC_MAX_DIM (only j < d_s is read),
 * each in [0, 1).  Copied to the workspace on `stream` (without a bound workspace they
 * are kept on the host for qmc_integrate_static).
 * Built-in shifts (used until this is called): Delta_{s,l,j} =
 * (splitmix64(seed, (s << 32) | (l << 8) | j) >> 11) * 2^-53, where splitmix64(seed, c)
 * is the (c+1)-th output of Steele-Lea-Flood's SplitMix64 started from state `seed`.
 * Errors: QMC_E_INVAL (value outside [0,1) or not finite), QMC_E_DEVICE.
 */
qmc_status qmc_set_shifts(qmc_plan_t plan, const double *shifts, void *stream);

/*
 * qmc_integrate -- randomized rank-1 lattice rule for every sector (Sec. 2.1 and the
 * definition of Q_{n,z} in Sec. 2.2), on the device, asynchronous on `stream`:
 *
 *   Q[s][l][k] = (1/n_s) sum_{i=0}^{n_s-1} W(y) f_k(phi(y)),
 *   y_j = frac((i z_j mod n_s) / n_s + Delta_{s,l,j}),  z = (1, a_s, a_s^2, ...) mod n_s,
 *   x_j = phi(y_j), W = prod_j phi'(y_j)  (samples with W = 0 contribute 0);
 *   mean[s][k] = (1/m) sum_l Q[s][l][k];  err[s][k] = sqrt(sum_l (Q - mean)^2 / ((m-1) m)).
 *
 * n, a: host arrays [n_sectors] of lattice sizes and Korobov parameters, or NULL for
 * the sectors' defaults.  Requires 2 <= n_s <= n_max, n_s < 2^53, gcd(a_s^j, n_s) = 1
 * for j < d_s (checked on the host before launch: QMC_E_INVAL).
 * Outputs (device, caller-owned, float64): dev_q [n_sectors][m][K] (may be NULL),
 * dev_mean and dev_err [n_sectors][K]; in a complex plan (qmc_plan_complex) the
 * shapes are [n_sectors][m][K][2], [n_sectors][K][2] with (re, im) pairs and err holds
 * the standard errors of the real and imaginary parts.  Complex plans also count
 * sign-check violations per sector (qmc_sign_violations); the sums are formed
 * regardless.  Sums are compensated (TwoSum) within each
 * thread, across the wavefront and across workgroups, in a fixed order, so results
 * are bitwise reproducible.  Non-finite sums are reported by qmc_query_status, not
 * here (the call does not synchronize).  The launches of the different dimension
 * classes run concurrently on up to three side streams of the plan (created by
 * qmc_bind_workspace, non-blocking, default priority, destroyed by qmc_plan_free),
 * forked from `stream` and joined back to it with events inside the call: work queued
 * on `stream` afterwards sees every result, as with a single stream.
 */
qmc_status qmc_integrate(qmc_plan_t plan, const uint64_t *n, const uint64_t *a, void *stream,
                         double *dev_q, double *dev_mean, double *dev_err);

/*
 * qmc_integrate_vec -- qmc_integrate with general generating vectors instead of Korobov
 * parameters: z [n_sectors][QMC_MAX_DIM] host array, z[s][j] in [1, n_s) with
 * gcd(z[s][j], n_s) = 1 for j < d_s (entries beyond d_s ignored).  Otherwise identical.
 */
qmc_status qmc_integrate_vec(qmc_plan_t plan, const uint64_t *n, const uint64_t *z, void *stream,
                             double *dev_q, double *dev_mean, double *dev_err);

/*
 * qmc_integrate_static -- qmc_integrate for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and launches as qmc_integrate, except where the device state
 * of the call lives: the plan needs no bound workspace; its tables (sector records,
 * coefficients, shifts) and the call's lattice records, workgroup partials, Q (when
 * dev_q is NULL) and status word are placed in a device array that the library holds
 * per GPU, QMC_STATIC_SCRATCH_BYTES long, uploaded to on `stream` at every call.  The
 * caller passes the outputs (dev_q, dev_mean, dev_err) as before.  No device memory is
 * allocated: no hipMalloc, no workspace; the array is the current device's (call with
 * the device of `stream` current) and stays until the process ends.
 * Errors: as qmc_integrate; QMC_E_NOMEM (before any launch) if the call needs more than
 * QMC_STATIC_SCRATCH_BYTES (the partials take 16 B per workgroup, shift and column:
 * lower the launch target with qmc_set_launch_shape).
 * Sharing: every call on one GPU uses the same array, which keeps the last call's
 * contents (the status word and sign-check counters are reset by each call; everything
 * else is written before it is read).  Calls that overlap on one GPU (other streams,
 * other threads, other plans) race: serialize them.  qmc_query_status and
 * qmc_sign_violations after this call read the array, valid until the next static call
 * on that GPU.  The class launches run one after another on `stream`.
 */
#define QMC_STATIC_SCRATCH_BYTES (16u << 20)
qmc_status qmc_integrate_static(qmc_plan_t plan, const uint64_t *n, const uint64_t *a,
                                void *stream, double *dev_q, double *dev_mean, double *dev_err);

/*
 * Median QMC rule (Sec. 2.2, Eq. median): for every sector, the unshifted rank-1
 * estimates Q_{n,z_c} of r candidate generating vectors with components in
 * U_n = {1 <= z <= n-1 : gcd(z, n) = 1}, and the candidate whose estimate of epsilon
 * order `order` (negative: counted from the last) is the median (r odd: the middle; r
 * even: the lower middle; equal estimates keep candidate order).  The chosen vector is
 * then used with the m random shifts (qmc_integrate_vec).
 *   n: [n_sectors] lattice sizes or NULL (defaults); candidates: host
 *   [n_sectors][r][QMC_MAX_DIM] (the random draws are the caller's); dev_scratch: device
 *   buffer of qmc_median_workspace_bytes(plan, r) bytes, 256-byte aligned.
 * Outputs (host): z_out [n_sectors][QMC_MAX_DIM] chosen vectors; q_out [n_sectors][r]
 * (may be NULL) the candidates' estimates of the deciding order.  All candidates of all
 * sectors are integrated in one launch.  Synchronous.  Real plans only.
 */
size_t qmc_median_workspace_bytes(qmc_plan_t plan, int32_t r);
qmc_status qmc_median_lattice(qmc_plan_t plan, const uint64_t *n, int32_t r,
                              const uint64_t *candidates, int32_t order, void *dev_scratch,
                              size_t scratch_bytes, void *stream, uint64_t *z_out, double *q_out);

/*
 * qmc_query_status -- synchronize `stream` and report the device status word of the
 * last qmc_integrate: QMC_OK, or QMC_E_NONFINITE with *sector, *shift, *order set to
 * the first non-finite sum in (sector, shift, order) order; else, in a complex plan,
 * QMC_E_SIGNCHECK with *sector the first sector with a sign-check violation (*shift
 * and *order set to -1).
 */
qmc_status qmc_query_status(qmc_plan_t plan, void *stream, int32_t *sector, int32_t *shift,
                            int32_t *order);

/* 1 if the plan is complex (some sector deformed), 0 if real, -1 for NULL. */
int32_t qmc_plan_complex(qmc_plan_t plan);

/*
 * qmc_sign_violations -- synchronize `stream` and copy the per-sector counts of
 * sign-check violations (samples with Im F(z) > 2^-40 |F(z)|) of the last
 * qmc_integrate into the host array counts[n_sectors].  Real plans: all zero.
 */
qmc_status qmc_sign_violations(qmc_plan_t plan, void *stream, uint64_t *counts);

/*
 * qmc_set_deformation -- replace the deformation parameters of a complex plan with the
 * host array lambda[n_sectors] (each >= 0, finite); uploaded on `stream`.
 * Errors: QMC_E_INVAL (bad value), QMC_E_STATE (real plan or no workspace).
 */
qmc_status qmc_set_deformation(qmc_plan_t plan, const double *lambda, void *stream);

/*
 * qmc_choose_deformation -- the presample selection of the deformation parameter: for
 * every sector with lambda > 0, integrate at lattice size n_pre (Korobov parameters
 * a_pre[n_sectors], or NULL for the sectors' defaults) with the plan's shifts, and halve
 * lambda while any sample violates the sign check, at most max_halvings times.
 * Synchronous.  Writes the chosen parameters to lambda_out[n_sectors] and the number of
 * halvings to halvings_out[n_sectors] (either may be NULL) and leaves them set in the
 * plan.  Returns QMC_E_SIGNCHECK (parameters of the other sectors still chosen and set)
 * if some sector still violates after max_halvings.
 */
qmc_status qmc_choose_deformation(qmc_plan_t plan, uint64_t n_pre, const uint64_t *a_pre,
                                  int32_t max_halvings, void *stream, double *lambda_out,
                                  int32_t *halvings_out);

/*
 * qmc_integrate_deformed -- qmc_integrate of a complex plan with the sign-check fallback
 * built in (the deformation parameter chosen by presampling, Sec. 3.1.3, may still let
 * samples of the full lattice leave the F - i0 half plane): integrate every sector on
 * lattices (n, a) as qmc_integrate does, then re-integrate every sector with a
 * violating sample with its lambda halved, at most max_halvings times.  dev_q, dev_mean,
 * dev_err (layout of qmc_integrate; dev_q may be NULL) hold, for every sector, the
 * results at its final lambda: a sector keeps the sums of the last pass that integrated
 * it.  The same results as qmc_choose_deformation on these lattices followed by
 * qmc_integrate, without the second integration of the sectors that needed no halving.
 * Writes the final parameters to lambda_out[n_sectors] and the halvings of this call to
 * halvings_out[n_sectors] (either may be NULL) and leaves them set in the plan.
 * Synchronous.  Errors: QMC_E_INVAL, QMC_E_STATE (real plan, no workspace),
 * QMC_E_NONFINITE (a pass produced a non-finite sum, see qmc_query_status; the call
 * stops there: the plan keeps the parameters of that pass and lambda_out/halvings_out
 * are not written), QMC_E_SIGNCHECK (some sector still violates after max_halvings:
 * every output still written), and those of qmc_integrate.
 */
qmc_status qmc_integrate_deformed(qmc_plan_t plan, const uint64_t *n, const uint64_t *a,
                                  int32_t max_halvings, void *stream, double *dev_q,
                                  double *dev_mean, double *dev_err, double *lambda_out,
                                  int32_t *halvings_out);

/*
 * qmc_korobov_p2 -- figure of merit of Korobov lattices on the device:
 *   dev_p2[c] = -1 + (1/n) sum_{k<n} prod_{j<d} [1 + 2 pi^2 B2({k a_c^j / n})],
 *   B2(x) = x^2 - x + 1/6,
 * the worst-case error criterion (Korobov space alpha = 2, unit product weights) the
 * paper names for its lattices (Sec. 2.2).  candidates: host array [n_cand] of a,
 * 1 <= a < n.  Uses the plan's workspace as scratch (the plan must be bound; needs
 * n_cand <= 65536 and 2 <= n < 2^53).  Asynchronous on `stream`.
 */
qmc_status qmc_korobov_p2(qmc_plan_t plan, uint64_t n, int32_t d, const uint64_t *candidates,
                          int32_t n_cand, void *stream, double *dev_p2);

/*
 * qmc_korobov_search -- synchronous argmin of qmc_korobov_p2 over the candidates with
 * ties (relative 1e-12 of the minimum) broken towards the smallest a.  *a_out receives
 * the chosen parameter, *p2_out (may be NULL) its figure of merit.
 */
qmc_status qmc_korobov_search(qmc_plan_t plan, uint64_t n, int32_t d, const uint64_t *candidates,
                              int32_t n_cand, void *stream, uint64_t *a_out, double *p2_out);

/*
 * qmc_lattice_points -- the lattice-point step of qmc_integrate on its own, for
 * verification: dev_y[t][j] = y_j of point i = i0 + t, t < count, j < d, with
 *   k_j = i z_j mod n,  q_j = RN(k_j / n),  y_j = RN(q_j + shift[j]) (minus 1 if >= 1),
 * z = (1, a, a^2, ...) mod n (rank-1 lattice rule of Sec. 2.2).  The device walks the
 * points with the same per-thread stride arithmetic as the integration kernel.
 * dev_y: device float64 [count][d].  Requires i0 + count <= n, shift in [0,1)^d, gcd
 * conditions as qmc_integrate.  Asynchronous on `stream`.
 */
qmc_status qmc_lattice_points(uint64_t n, int32_t d, uint64_t a, const double *shift,
                              uint64_t i0, uint64_t count, void *stream, double *dev_y);

/*
 * Weighted sums of integrals A_t = sum_i C_ti I_i (Sec. 2.1.3; coefficient rows may be
 * sparse, Sec. 2.4): row t holds the entries row_ptr[t] .. row_ptr[t+1]-1 of col
 * (integral index) and coef_re / coef_im.  n_sums >= 1.
 * Coefficients may depend on the regulator (Sec. 2.4): with n_terms = P > 1 each entry
 * holds the P Laurent coefficients c_p of eps^(coef_order_lo + p), p < P, stored
 * [nnz][P] (qmc_coef_series produces them from expressions), and the sums are the
 * products of series
 *   A_t,j = sum_i sum_{p <= j} c_ti,p I_i,j-p,   j < n_orders,
 * i.e. output order j is eps^(order_lo + coef_order_lo + j); each term's variance is
 * |c|^2 var(I_i,j-p), the epsilon orders of an integral counted as independent.
 * Terms with p >= n_orders never contribute.  n_terms = 0 or 1 with coef_order_lo = 0:
 * constant coefficients.
 */
typedef struct {
    int32_t n_sums;
    int32_t n_terms;                  /* P: Laurent terms per coefficient (0 or 1: one) */
    const int64_t *row_ptr;           /* [n_sums + 1] */
    const int32_t *col;               /* [nnz] integral indices (< the problem's n_integrals) */
    const double *coef_re;            /* [nnz][P] */
    const double *coef_im;            /* [nnz][P], may be NULL (real coefficients) */
    int32_t coef_order_lo;            /* epsilon power of term p = 0 */
    int32_t reserved0;
} qmc_amplitude;

enum { QMC_AMP_HOST = 0, QMC_AMP_DEVICE = 1 };

/*
 * Options of the adaptive evaluation (Sec. 2.1.3): every epsilon order of every sum
 * must reach relative error epsrel (error definition of the Sec. 3.2 timing notes) or absolute error
 * epsabs.  Lattice sizes come from the ascending table lattice_n[n_lattice]; the
 * Korobov parameter of size lattice_n[l] for a sector of dimension d is
 * lattice_a[l * QMC_MAX_DIM + d - 1].
 * tau: per-sector cost of one evaluation (any unit), fixed for the whole evaluation; or
 * NULL: measured while the evaluation runs (Sec. 2.1.3, tau_i estimated on-line) --
 * every workgroup adds its duration on the device's constant 100 MHz clock to its
 * sector, and a sector's cost is its ticks per evaluation (n_s m per round) summed
 * over the rounds it was integrated in so far; a sector not yet integrated takes the
 * library's cost model (polynomial slots + transform + logarithm work, plus the network
 * of an attached flow).  Only cost ratios matter to the allocation.
 * tau_used: NULL, or a host array [max_rounds][n_sectors] whose row r receives the
 * costs the allocation after round r + 1 used (rows of allocations that did not take
 * place are left as they were; device mode writes at most QMC_AMP_TAU_ROWS rows).
 * mode QMC_AMP_DEVICE runs every round on the device: a round kernel, one persistent
 * kernel over the sectors without a flow (these must be korobov3 with integer powers of
 * U and F) and one over the flow-transformed sectors, then the reduction; the host only
 * polls the state between batches of rounds.  QMC_AMP_HOST integrates each round with
 * qmc_integrate.  With the same fixed costs both give the same rounds and lattice sizes
 * (measured costs differ between runs and forms).
 */
#define QMC_AMP_TAU_ROWS 64
typedef struct {
    double epsrel, epsabs;
    double timeout_s;                 /* wall-clock limit, <= 0: none */
    double alpha;                     /* variance decay exponent, var ~ w / n^alpha (2) */
    uint64_t n_presample;             /* initial lattice size (the paper's 1e4) */
    int32_t max_rounds;               /* allocation rounds after the presample (>= 1) */
    int32_t mode;                     /* QMC_AMP_HOST (host loop) or QMC_AMP_DEVICE */
    int32_t n_lattice;
    int32_t reserved0;
    const uint64_t *lattice_n;        /* [n_lattice], ascending, each <= the plan's n_max */
    const uint64_t *lattice_a;        /* [n_lattice][QMC_MAX_DIM] */
    const double *tau;                /* [n_sectors] or NULL (measured) */
    double *tau_used;                 /* output, [max_rounds][n_sectors] or NULL */
} qmc_amp_options;

typedef struct {
    int32_t rounds;                   /* integration rounds, presample included */
    int32_t converged;                /* 1 if every target met its error bound */
    int32_t timed_out;                /* 1 if stopped by timeout_s */
    int32_t lattice_limited;          /* 1 if some sector wanted more than the largest size */
    int64_t evaluations;              /* sum over rounds of n_s * m over integrated sectors */
    double seconds;                   /* wall time of the call */
    double max_eps_rel;               /* largest relative error over sums and orders */
} qmc_amp_stats;

/*
 * amp_evaluate -- adaptive evaluation of weighted sums of integrals (Sec. 2.1.3):
 * presample every sector at the smallest table size >= n_presample; then, per round,
 * form the integrals (sums of their sectors, variances added) and the sums
 * A_t = sum_i C_ti I_i with var(A_t) = sum_i |C_ti|^2 var(I_i) per order; stop when
 * every target meets its bound; otherwise, for every unmet target (sum t, order k) in
 * order, set V = max(epsrel^2 |A_tk|^2, epsabs^2), w_s = var_sk n_s^alpha and take the
 * closed-form sizes n_s = (alpha w_s lambda |C|^2 / tau_s)^(1/(alpha+1)) with
 * lambda = (1/alpha) [(1/V) sum_s (|C|^2 w_s tau_s^alpha)^(1/(alpha+1))]^((alpha+1)/alpha)
 * (the Lagrange solution of Eq. adaptive-solution with one consistent index), keep the
 * largest size any target asks for and never shrink, round up to the table and
 * re-integrate the sectors whose lattice changed.  Synchronous on `stream`.
 * With regulator-dependent coefficients the closed form's |C|^2 w_s becomes the sum over
 * the contributing terms, sum_p |c_p|^2 w_s,j-p.
 * Outputs (host, caller-owned): value and error [n_sums][n_orders][2] (re, im);
 * n_final [n_sectors] (may be NULL); stats (may be NULL).  Returns QMC_OK (converged
 * or not: see stats), QMC_E_TIMEOUT with valid results when the time limit stopped it,
 * QMC_E_INVAL / QMC_E_NONFINITE / QMC_E_DEVICE on failure.  Complex (deformed) plans
 * are not accepted (QMC_E_INVAL).
 * FP32 plans: the sectors' errors include the FP32 form's rounding bound (see the
 * precision option), which no lattice size lowers; a target whose bound, propagated
 * like the errors from the calibration estimates, exceeds half of max(epsrel |A|,
 * epsabs) is refused before any work with QMC_E_INVAL (evaluate those sums in FP64).
 */
qmc_status amp_evaluate(qmc_plan_t plan, const qmc_amplitude *amp, const qmc_amp_options *opt,
                        void *stream, double *value, double *error, uint64_t *n_final,
                        qmc_amp_stats *stats);

/*
 * Launch shape of the integrand kernels: threads per workgroup, shifts per workgroup,
 * shifts evaluated per lattice point in one pass, and the number of workgroups a launch
 * aims at (lattice points per thread follow from it).  All shapes give the same sums up
 * to rounding order.
 */
typedef struct {
    int32_t block;                    /* 64, 128 or 256 */
    int32_t shift_tile;               /* 1..16, divides m, shift_tile * columns <= 64 */
    int32_t shifts_per_pass;          /* 1, 2, 4 (divides shift_tile); 1 for complex plans */
    int32_t target_blocks;            /* 256 .. 32768 */
    double ms;                        /* qmc_autotune: measured time of the shape, ms */
} qmc_launch_shape;

qmc_status qmc_set_launch_shape(qmc_plan_t plan, const qmc_launch_shape *shape);
qmc_status qmc_get_launch_shape(qmc_plan_t plan, qmc_launch_shape *shape);

/*
 * qmc_autotune -- grid search over launch shapes (block 64/128/256, power-of-two shift
 * tiles dividing m, 1/2/4 shifts per pass where compiled, 8192/16384/32768 target
 * workgroups): each shape is timed with HIP events around `reps` qmc_integrate calls on
 * lattices n, a (NULL: the sectors' defaults), after one warm-up; the fastest (minimum
 * over the repetitions) is set on the plan and cached for the process under a key of
 * the plan's shape (sectors, dimensions, orders, precision, shifts, degrees, flows).
 * With use_cache != 0 a cached shape for the same key is applied without timing.
 * Synchronous; overwrites the plan's internal Q and statistics buffers.
 */
qmc_status qmc_autotune(qmc_plan_t plan, const uint64_t *n, const uint64_t *a, int32_t reps,
                        int32_t use_cache, void *stream, qmc_launch_shape *best);

/*
 * qmc_specialize -- plan-specialised integrand kernels (the per-integral generated
 * code of Sec. 2.1, where pySecDec compiles each integrand with its constants fixed):
 * for every launch class (dimension, precision) of the sectors of a real plan that have
 * no flow attached (FP64: every such sector; FP32: those with an FP32 form) write
 * straight-line code that evaluates only the monomials each sector has (multivariate
 * Horner by greedy factorisation), with the integer and half-integer powers of x_j, U
 * and F and the log-F polynomial of every order fixed (the sector's transform applied
 * as in the table-driven kernels), compile it for gfx950 with the
 * HIP run-time compiler and load it on the current device.  qmc_integrate then runs
 * these kernels for those classes; the results equal the table-driven kernels' up to
 * rounding order.  Each class kernel is compiled for two and for four shifts per pass
 * and for the shifts per pass of the launch shape at the time of the call (FP64 at
 * d >= 7: one), and for the sectors the class holds then; under a shape with other
 * shifts per pass, or after a sector enters the class (a flow detached), that class
 * runs the table-driven kernel until qmc_specialize is called again (kernels already
 * compiled are kept).  The amplitude evaluation's persistent kernels are unaffected.
 * flags: 0, QMC_SPEC_COMPILE_ONLY (generate and compile, load nothing: usable without
 * a GPU) or QMC_SPEC_OFF (unload every specialised kernel of the plan); with
 * QMC_SPEC_PERSISTENT, instead of the class kernels, the persistent kernel of
 * amp_evaluate's batched form (QMC_AMP_DEVICE) for the plan's sectors without a flow
 * and its number of orders: one program holding every sector, its integrand a switch on
 * the sector index inside the point loop (compiled in seconds for hundreds of sectors);
 * the batched form runs it while the plan's sectors without a flow and orders are those
 * it was compiled for.  Requires a real plan whose sectors have the batched form's
 * shape, and in FP32 an FP32 form for each (QMC_E_INVAL otherwise).
 * *seconds (may be NULL): wall time of the call.  Synchronous, host-side (no stream
 * work).  Errors: QMC_E_INVAL, QMC_E_DEVICE (compiler or module-load failure; the
 * message carries the compiler log).
 */
enum { QMC_SPEC_COMPILE_ONLY = 1, QMC_SPEC_OFF = 2, QMC_SPEC_PERSISTENT = 4 };
qmc_status qmc_specialize(qmc_plan_t plan, int32_t flags, double *seconds);

/*
 * qmc_gen_source -- the generated source of launch class (d, f32 != 0) of the plan as
 * qmc_specialize would compile it now (empty when the class has no sector, and for
 * complex plans): copied NUL-terminated into buf[cap] (truncated to cap - 1 bytes; buf may
 * be NULL), its full length in *len (may be NULL).  Host only.
 */
qmc_status qmc_gen_source(qmc_plan_t plan, int32_t d, int32_t f32, char *buf, size_t cap,
                          size_t *len);

/*
 * Learned coupling-flow transform (an alternative variable transform beside the
 * periodizing ones; not in the paper).  A flow for dimension d is a stack of
 * QMC_FLOW_LAYERS affine coupling layers in logit space of the unit cube: layer l keeps
 * the coordinates j with j % 2 == l % 2 and maps the others by z -> z exp(s) + t, where
 * (o_s, o_t) = W3 tanh(W2 tanh(W1 (m_l z) + b1) + b2) + b3 (widths d, 64, 64, 2d) and
 * s = 0.25 tanh(o_s), t = o_t, restricted to the moved coordinates.  The density
 * direction G: x -> u has log q(x) = log|det du/dx|; the sampling direction T = G^-1 is
 * what integration uses: x = T(u) after the sector's periodizing transform, weight
 * J_T(u) = 1/q(x).  The networks run on the matrix cores in bfloat16 with float32
 * accumulation; the coupling updates, logit and sigmoid are float64.
 *
 * Conditional flows (a flow shared by the points of a kinematic scan): n_cond
 * conditioning features c (0 <= n_cond <= QMC_FLOW_MAX_COND, d + n_cond <= 16) are
 * appended to every layer's network input, (m_l z, c), so W1 has d + n_cond columns; the
 * features are the caller's (e.g. scaled kinematic invariants), given per sample in
 * training and per sector when attached.
 *
 * Parameters (host float32, qmc_flow_param_count(d, n_cond) values) are laid out per
 * layer as W1 [64][d + n_cond], b1 [64], W2 [64][64], b2 [64], W3 [2d][64] (rows s then
 * t), b3 [2d].  A flow's device state (parameters, Adam moments, gradient, packed
 * operands) is a caller-owned, 256-byte aligned device buffer of qmc_flow_bytes(d,
 * n_cond) bytes.  Every call names the flow's (d, n_cond).
 */
enum { QMC_FLOW_SAMPLE = 0, QMC_FLOW_DENSITY = 1 };

typedef struct {
    float lr, beta1, beta2, eps;      /* Adam (Kingma and Ba 2015) */
    int32_t step;                     /* 1-based step number of this update (bias correction) */
    int32_t reserved0;
} qmc_flow_adam;

/* -1 / 0 if d is outside [1, QMC_MAX_DIM] or n_cond outside [0, QMC_FLOW_MAX_COND] */
int64_t qmc_flow_param_count(int32_t d, int32_t n_cond);
size_t qmc_flow_bytes(int32_t d, int32_t n_cond);

/* Upload parameters, zero the Adam moments and gradient, pack the matrix-core operands.
 * Synchronous.  Errors: QMC_E_INVAL (NULL, misaligned, non-finite parameter). */
qmc_status qmc_flow_load(void *dev_flow, int32_t d, int32_t n_cond, const float *params,
                         void *stream);

/* Copy parameters and/or the last gradient (either may be NULL) to the host.  Synchronous. */
qmc_status qmc_flow_read(const void *dev_flow, int32_t d, int32_t n_cond, float *params,
                         float *grad, void *stream);

/* dev_out[i][j], dev_logdet[i] for dev_in [count][d] (device float64, coordinates in
 * (0, 1)) and dev_cond [count][n_cond] (device float64; NULL when n_cond = 0):
 * QMC_FLOW_SAMPLE gives x = T(u) and log J_T(u); QMC_FLOW_DENSITY gives u = G(x) and
 * log q(x).  Asynchronous. */
qmc_status qmc_flow_transform(const void *dev_flow, int32_t d, int32_t n_cond, int32_t direction,
                              const double *dev_in, const double *dev_cond, int64_t count,
                              void *stream, double *dev_out, double *dev_logdet);

/* Device scratch bytes of qmc_flow_gradient over `count` points. */
size_t qmc_flow_scratch_bytes(int32_t d, int32_t n_cond, int64_t count);

/* Gradient of L = -(1/w_sum) sum_i w_i log q(x_i | c_i) (weighted maximum likelihood of
 * samples x [count][d] with weights w [count] and conditioning features cond
 * [count][n_cond] or NULL, device float64) into the flow's gradient buffer; *dev_loss
 * (device, may be NULL) receives L.  w_sum = 0: the library sums the weights on the
 * device (compensated, fixed order; no host synchronisation; L and the gradient are 0
 * if they sum to 0); w_sum > 0: the caller's normaliser.  Asynchronous; deterministic. */
qmc_status qmc_flow_gradient(void *dev_flow, int32_t d, int32_t n_cond, const double *dev_x,
                             const double *dev_w, const double *dev_cond, int64_t count,
                             double w_sum, void *dev_scratch, size_t scratch_bytes, void *stream,
                             double *dev_loss);

/* One Adam update of the parameters from the gradient buffer; repacks the operands. */
qmc_status qmc_flow_adam_step(void *dev_flow, int32_t d, int32_t n_cond, const qmc_flow_adam *opt,
                              void *stream);

/* Training: `epochs` passes over `batches` strided minibatches (batch b: samples
 * b, b + batches, ...), one gradient and one Adam step each (steps numbered from
 * opt->step).  w_sum: sum of all weights, or 0 to have the library sum them on the
 * device as qmc_flow_gradient does.  dev_loss_history (device, may be NULL) gets
 * each step's loss.  Scratch: qmc_flow_scratch_bytes(d, n_cond, count / batches).
 * Asynchronous. */
qmc_status qmc_flow_train(void *dev_flow, int32_t d, int32_t n_cond, const double *dev_x,
                          const double *dev_w, const double *dev_cond, int64_t count, double w_sum,
                          const qmc_flow_adam *opt, int32_t batches, int32_t epochs,
                          void *dev_scratch, size_t scratch_bytes, void *stream,
                          double *dev_loss_history);

/* Training samples of a sector: for the points i < n of the Korobov lattice (n, a) with
 * the plan's shift `shift`, dev_x[i][j] = phi(y_i)_j (the sector's periodizing transform)
 * and dev_w[i] = W(y_i) ||(f_k(x_i))_k||_2, the weight for which the optimal model
 * density is proportional to the root of the summed squares of the orders (0 where
 * W = 0 or f is not finite).  In a complex plan f is the deformed-contour integrand
 * J f(z(x)) and the norm runs over the real and imaginary parts of every order.
 * Asynchronous. */
qmc_status qmc_flow_samples(qmc_plan_t plan, int32_t sector, uint64_t n, uint64_t a, int32_t shift,
                            void *stream, double *dev_x, double *dev_w);

/* Integrate `sector` through the flow: per lattice sample y, u = phi(y) with weight W,
 * x = T(u | cond), contribution W J_T(u) f(x) (0 when a coordinate of u or x is not
 * inside (0, 1)); in a complex plan f is the deformed-contour integrand (FP64) and the
 * sign check counts as without a flow.  cond: host [n_cond] conditioning features of
 * this sector (NULL when n_cond = 0).  dev_flow NULL detaches.  The flow buffer must stay
 * valid while attached.  Synchronous. */
qmc_status qmc_flow_attach(qmc_plan_t plan, int32_t sector, const void *dev_flow, int32_t n_cond,
                           const double *cond, void *stream);

/*
 * qmc_coef_series -- a coefficient of a weighted sum given as an arithmetic expression
 * (Sec. 2.4): the symbols are replaced by the caller's values, the expression is
 * expanded into a Laurent series in the regulator in exact rational arithmetic, and
 * the series coefficients are rounded to the nearest double.  Host only (no HIP call).
 *   expr: numbers (integer, decimal, exponent notation; exact), symbols, the regulator
 *     named `regulator`, the imaginary unit I, + - * / and ^ (or **) with integer
 *     exponents, parentheses.  Functions and non-integer powers are rejected (they do
 *     not give rational series).
 *   names[k], values[k], k < n_symbols: symbol values, each an expression that may use
 *     the regulator, I and symbols given before it, e.g. "3/2", "-0.25", "1+2*I",
 *     "4-2*eps".
 *   Writes *leading_order (may be NULL): the lowest order with a non-zero coefficient
 *     (INT32_MAX for an identically zero expression), and for j < n_terms
 *     re[j] + i im[j] = the coefficient of regulator^(order_lo + j).
 * Errors: QMC_E_INVAL (syntax, unknown or repeated symbol, division by zero, an exponent
 * that is not an integer or depends on the regulator,
 * a non-zero term below order_lo when n_terms > 0 -- *leading_order is still set --,
 * a coefficient outside the double range, numbers beyond 2^21 bits), QMC_E_NOMEM.
 */
qmc_status qmc_coef_series(const char *expr, const char *regulator, int32_t n_symbols,
                           const char *const *names, const char *const *values, int32_t order_lo,
                           int32_t n_terms, int32_t *leading_order, double *re, double *im);

/*
 * qmc_enable_timing / qmc_read_timing -- kernel timing for measurement: while enabled,
 * every qmc_integrate records a HIP event pair on its stream around its main
 * (integrand) kernel.  Enabling (or disabling) clears the record; at most 4096
 * launches are recorded (QMC_E_STATE beyond).  qmc_read_timing synchronizes on the
 * recorded events and returns the summed kernel time in milliseconds and the number
 * of recorded launches (either pointer may be NULL).
 */
qmc_status qmc_enable_timing(qmc_plan_t plan, int32_t enable);
qmc_status qmc_read_timing(qmc_plan_t plan, double *ms_total, int32_t *launches);

/* Release a plan (host memory only; the workspace stays the caller's). NULL is a no-op. */
void qmc_plan_free(qmc_plan_t plan);

/* Thread-local description of the last failure ("" if none). */
const char *qmc_last_error(void);

/* Library version string. */
const char *qmc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QMCAMP_H */
