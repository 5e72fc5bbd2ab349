// qmc_kernels.hip -- gfx950 kernels of the randomized rank-1 lattice QMC library.
//
// One lattice sample = one (point i, shift l) pair of one sector, producing every
// epsilon order of that sector.  The hot kernel fuses, per sample (the fusion of
// lattice generation and integrand evaluation of Sec. 2.1 of arXiv:2305.19768):
//   lattice point  k_j = i z_j mod n (exact 64-bit), q_j = RN(k_j / n),
//                  y_j = q_j + Delta_j, minus 1 if >= 1           (Sec. 2.2, Q_{n,z})
//   transform      x_j = phi(y_j), W = prod_j phi'(y_j)            (korobov_r / baker)
//   integrand      U, F by dense nested Horner, B = x^p U^a F^b, L = log F,
//                  f_k = B sum_m c_{k,m} L^m
//   accumulation   W f_k into per-thread (sum, compensation) pairs per (shift, order)
// and ends with a wavefront TwoSum butterfly and an in-order cross-wave combine that
// writes one compensated partial per workgroup; a second kernel combines the
// partials of each sector in workgroup order (the on-device summation of Sec. 2.1),
// and a third forms the shift mean and its standard error.
//
// Mapping: every lane of a workgroup works on the same sector and the same shift at
// the same time, so all per-sector tables (coefficients, exponents, shifts, lattice
// vector) are wave-uniform and live in scalar registers; only the lattice point and
// the integrand values are per-lane.  The quotient RN(k/n) reuses RN(1/n) with one
// FMA correction (Markstein's theorem: with y = RN(1/n) and q0 = RN(k y), the value
// RN(q0 + RN(k - q0 n) y) is the correctly rounded k/n), and is shared by the
// SHIFT_TILE shifts a thread evaluates per point.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "qmc_internal.h"

namespace qmc {

// ----------------------------------------------------------- compensated sums

struct DD {
  double s, c;
};

// Knuth's TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void dd_add(DD &acc, double v) {
  double s, e;
  two_sum(acc.s, v, s, e);
  acc.s = s;
  acc.c += e;
}

__device__ __forceinline__ DD dd_combine(DD a, DD b) {
  DD r;
  double e;
  two_sum(a.s, b.s, r.s, e);
  r.c = (a.c + b.c) + e;
  return r;
}

__device__ __forceinline__ DD wave_reduce(DD v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    DD o;
    o.s = __shfl_xor(v.s, off, 64);
    o.c = __shfl_xor(v.c, off, 64);
    v = dd_combine(v, o);
  }
  return v;
}

// Opaque copy of a wave-uniform pointer: loads through the result cannot be hoisted
// out of the loop iteration that launders it, so the per-sector tables are re-read
// from the scalar cache each iteration instead of pinning hundreds of SGPRs.
// The tables are read through the constant address space, where wave-uniform loads
// are always scalar (s_load) loads.
template <typename T>
using cptr = const T __attribute__((address_space(4))) *;

template <typename T>
__device__ __forceinline__ cptr<T> launder_uniform(const T *p) {
  cptr<T> c = (cptr<T>)p;
  asm volatile("" : "+s"(c));
  return c;
}

// Launder that also waits for a per-lane value: the loads through the result cannot
// start before `after` is computed.  Chaining each group of table reads to the
// previous group's result bounds the number of table values held in SGPRs.
template <typename T>
__device__ __forceinline__ cptr<T> launder_after(cptr<T> c, double after) {
  asm volatile("" : "+s"(c) : "v"(after));
  return c;
}

// ------------------------------------------------------------- lattice points

// (a * b) mod n for a, b < n < 2^53 (double-and-add; used once per thread).
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, uint64_t n) {
  if ((a | b) < (1ull << 32)) return (a * b) % n;
  uint64_t r = 0;
  a %= n;
  while (b) {
    if (b & 1) {
      r += a;
      if (r >= n) r -= n;
    }
    a += a;
    if (a >= n) a -= n;
    b >>= 1;
  }
  return r;
}

// The lattice state k_j = i z_j mod n is carried as an exact double (k < n < 2^53).
__device__ __forceinline__ double quotient(double kd, double n_d, double inv_n) {
  const double q0 = kd * inv_n;
  const double r = __builtin_fma(-q0, n_d, kd);  // exact residual
  return __builtin_fma(r, inv_n, q0);
}

// k <- (k + dz) mod n as k - (n - dz), plus n if negative: every value is an integer of
// magnitude below 2^53, so both operations are exact.
__device__ __forceinline__ double lattice_step(double kd, double ndz, double n_d) {
  const double t = kd - ndz;
  return (t < 0.0) ? t + n_d : t;
}

// frac(q + Delta) for q, Delta in [0, 1): q + Delta < 2 and the fraction is exact.
__device__ __forceinline__ double shifted(double q, double delta) {
  return __builtin_amdgcn_fract(q + delta);
}

// ---------------------------------------------------------------- transforms

// korobov_r: x = I_y(r+1, r+1) = y^(r+1) * poly_r(y), w = C_r (y (1 - y))^r.
// Generic korobov_r for r = 1..6, coefficients of poly_r in ascending powers.
__device__ __forceinline__ void korobov_generic(int r, double y, double &x, double &w) {
  // poly_r(y) such that I_y(r+1, r+1) = y^(r+1) poly_r(y); C_r = (2r+1)!/(r!)^2.
  // r = 1: 3 - 2y;  r = 2: 10 - 15y + 6y^2;  r = 3: 35 - 84y + 70y^2 - 20y^3;
  // r = 4: 126 - 420y + 540y^2 - 315y^3 + 70y^4;
  // r = 5: 462 - 1980y + 3465y^2 - 3080y^3 + 1386y^4 - 252y^5;
  // r = 6: 1716 - 9009y + 20020y^2 - 24024y^3 + 16380y^4 - 6006y^5 + 924y^6.
  double t = y * (1.0 - y);
  double p, c, tr, yr;
  switch (r) {
    case 1:
      p = __builtin_fma(-2.0, y, 3.0);
      c = 6.0;
      tr = t;
      yr = y * y;
      break;
    case 2:
      p = __builtin_fma(__builtin_fma(6.0, y, -15.0), y, 10.0);
      c = 30.0;
      tr = t * t;
      yr = y * y * y;
      break;
    case 4:
      p = __builtin_fma(
          __builtin_fma(__builtin_fma(__builtin_fma(70.0, y, -315.0), y, 540.0), y, -420.0), y,
          126.0);
      c = 630.0;
      tr = (t * t) * (t * t);
      yr = (y * y) * (y * y) * y;
      break;
    case 5:
      p = __builtin_fma(
          __builtin_fma(
              __builtin_fma(__builtin_fma(__builtin_fma(-252.0, y, 1386.0), y, -3080.0), y,
                            3465.0),
              y, -1980.0),
          y, 462.0);
      c = 2772.0;
      tr = (t * t) * (t * t) * t;
      yr = (y * y) * (y * y) * (y * y);
      break;
    case 6:
      p = __builtin_fma(
          __builtin_fma(
              __builtin_fma(
                  __builtin_fma(__builtin_fma(__builtin_fma(924.0, y, -6006.0), y, 16380.0), y,
                                -24024.0),
                  y, 20020.0),
              y, -9009.0),
          y, 1716.0);
      c = 12012.0;
      tr = (t * t) * (t * t) * (t * t);
      yr = (y * y) * (y * y) * (y * y) * y;
      break;
    default:  // r = 3
      p = __builtin_fma(__builtin_fma(__builtin_fma(-20.0, y, 70.0), y, -84.0), y, 35.0);
      c = 140.0;
      tr = t * t * t;
      yr = (y * y) * (y * y);
      break;
  }
  w = c * tr;
  x = yr * p;
}

template <int D>
__device__ __forceinline__ double apply_transform(int kind, double w_scale, const double (&y)[D],
                                                  double (&x)[D]) {
  double W = 1.0;
  if (kind == QMC_TRANSFORM_KOROBOV3) {
    // x_j = y^4 (35 - 84 y + 70 y^2 - 20 y^3);  W = 140^d (prod_j y_j (1 - y_j))^3
    double T = 1.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double yj = y[j];
      const double p =
          __builtin_fma(__builtin_fma(__builtin_fma(-20.0, yj, 70.0), yj, -84.0), yj, 35.0);
      const double y2 = yj * yj;
      x[j] = (y2 * y2) * p;
      T *= yj * (1.0 - yj);
    }
    W = w_scale * (T * T * T);
  } else if (kind == QMC_TRANSFORM_BAKER) {
#pragma unroll
    for (int j = 0; j < D; ++j) x[j] = 1.0 - __builtin_fabs(2.0 * y[j] - 1.0);
  } else if (kind == QMC_TRANSFORM_NONE) {
#pragma unroll
    for (int j = 0; j < D; ++j) x[j] = y[j];
  } else {
    const int r = kind - QMC_TRANSFORM_KOROBOV1 + 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double w;
      korobov_generic(r, y[j], x[j], w);
      W *= w;
    }
  }
  return W;
}

// -------------------------------------------------------------- polynomials

// Dense nested Horner of total degree DEG (<= 3) over the degree-3 layout, for S
// points at once (each scalar coefficient feeds S FMAs).  The scalar loads of each
// (j, k) group go through a pointer laundered after the result of the group two steps
// back: a group's coefficients can arrive while the previous group computes, and at
// most two groups' coefficients (<= 2 (QMC_MAX_DIM + 1) doubles) occupy SGPRs.
#ifndef QMC_CHAIN_LAG
#define QMC_CHAIN_LAG 1
#endif
struct LoadChain {
  double dep1, dep2;   // results of the last two groups
  __device__ __forceinline__ cptr<double> next(cptr<double> c) const {
    return launder_after(c, QMC_CHAIN_LAG == 1 ? dep1 : dep2);
  }
  __device__ __forceinline__ void done(double v) {
    dep2 = dep1;
    dep1 = v;
  }
};

template <int D, int DEG, int S>
__device__ __forceinline__ void horner(cptr<double> c, const double (&x)[S][D], double (&out)[S],
                                       LoadChain &ch) {
  c = ch.next(c);
  double acc[S];
#pragma unroll
  for (int u = 0; u < S; ++u) acc[u] = c[0];
  int p = 1;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    c = ch.next(c);
    double g[S];
#pragma unroll
    for (int u = 0; u < S; ++u) g[u] = c[p];
    ++p;
    if (DEG >= 2) {
#pragma unroll
      for (int k = j; k < D; ++k) {
        if (DEG >= 3) c = ch.next(c);
        double h[S];
#pragma unroll
        for (int u = 0; u < S; ++u) h[u] = c[p];
        ++p;
        if (DEG >= 3) {
#pragma unroll
          for (int l = k; l < D; ++l)
#pragma unroll
            for (int u = 0; u < S; ++u) h[u] = __builtin_fma(c[p + l - k], x[u][l], h[u]);
          ch.done(h[0]);
        }
        p += D - k;
#pragma unroll
        for (int u = 0; u < S; ++u) g[u] = __builtin_fma(x[u][k], h[u], g[u]);
      }
    } else {
      p += (D - j) * (D - j + 3) / 2;   // skip the degree-2 and degree-3 slots of this j
    }
#pragma unroll
    for (int u = 0; u < S; ++u) acc[u] = __builtin_fma(x[u][j], g[u], acc[u]);
    ch.done(acc[0]);
  }
#pragma unroll
  for (int u = 0; u < S; ++u) out[u] = acc[u];
}

template <int D, int S>
__device__ __forceinline__ void poly(cptr<double> c, int deg, const double (&x)[S][D],
                                     double (&out)[S], LoadChain &ch) {
  if (deg >= 3) horner<D, 3, S>(c, x, out, ch);
  else if (deg == 2) horner<D, 2, S>(c, x, out, ch);
  else horner<D, 1, S>(c, x, out, ch);
}

// 1/v to within an ulp or two: hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double recip(double v) {
  double r = __builtin_amdgcn_rcp(v);
  r = __builtin_fma(__builtin_fma(-v, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-v, r, 1.0), r, r);
  return r;
}

// Natural logarithm of log F, accurate to a few ulp.  x = m 2^e with m in
// [sqrt(1/2), sqrt(2)); log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.1716, by the
// Taylor series atanh(s) = s sum_k s^(2k)/(2k+1) through s^19 (remainder below 2.4e-17
// relative); e ln 2 with ln 2 split into a 32-bit head (e * head exact) and a tail.
// log(0) = -inf, log(+inf) = +inf, negative or NaN input gives NaN.
__device__ __forceinline__ double log_f64(double x) {
  constexpr double kLn2Hi = 0x1.62e42ffp-1;
  constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
  double m = __builtin_amdgcn_frexp_mant(x);   // [0.5, 1) for finite non-zero x
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool low = m < 0.70710678118654752;
  m = low ? m + m : m;
  e = low ? e - 1 : e;
  const double s = (m - 1.0) * recip(m + 1.0);
  const double z = s * s;
  double p = 1.0 / 19.0;
  p = __builtin_fma(p, z, 1.0 / 17.0);
  p = __builtin_fma(p, z, 1.0 / 15.0);
  p = __builtin_fma(p, z, 1.0 / 13.0);
  p = __builtin_fma(p, z, 1.0 / 11.0);
  p = __builtin_fma(p, z, 1.0 / 9.0);
  p = __builtin_fma(p, z, 1.0 / 7.0);
  p = __builtin_fma(p, z, 1.0 / 5.0);
  p = __builtin_fma(p, z, 1.0 / 3.0);
  const double logm = 2.0 * __builtin_fma(s * z, p, s);
  const double ed = (double)e;
  double r = __builtin_fma(ed, kLn2Hi, __builtin_fma(ed, kLn2Lo, logm));
  const bool ok = x > 0.0 && x < __builtin_inf();
  return ok ? r : (x == 0.0 ? -__builtin_inf() : (x > 0.0 ? x : __builtin_nan("")));
}

__device__ __forceinline__ double ipow_u(double v, int e) {
  double r = 1.0;
  for (int t = 0; t < e; ++t) r *= v;
  return r;
}

// Per-sector scalars read once per workgroup (they stay in SGPRs).
struct SectorScalars {
  int flags, u_deg, f_deg, u_num, u_den, f_num, f_den, f_half, max_log;
  int u_off, f_off;
};

__device__ __forceinline__ SectorScalars load_scalars(const SectorDev *sd) {
  SectorScalars r;
  r.flags = sd->flags;
  r.u_deg = sd->u_deg;
  r.f_deg = sd->f_deg;
  r.u_num = sd->u_num;
  r.u_den = sd->u_den;
  r.f_num = sd->f_num;
  r.f_den = sd->f_den;
  r.f_half = sd->f_half;
  r.max_log = sd->max_log;
  r.u_off = sd->u_off;
  r.f_off = sd->f_off;
  return r;
}

// Integrand orders f_k(x) (without the transform weight) for S samples.
template <int D, int K, int S>
__device__ __forceinline__ void integrand(const SectorScalars &ss, cptr<SectorDev> sd,
                                          cptr<double> coef, const double (&x)[S][D],
                                          double (&f)[S][K]) {
  const int flags = ss.flags;
  double U[S], F[S];
  LoadChain ch{x[0][0], x[0][0]};
  poly<D, S>(coef + ss.u_off, ss.u_deg, x, U, ch);
  poly<D, S>(coef + ss.f_off, ss.f_deg, x, F, ch);
  double B[S];
  cptr<SectorDev> sx = launder_after(sd, F[0]);
#pragma unroll
  for (int u = 0; u < S; ++u) {
    double num = 1.0, den = 1.0, hn = 1.0, hd = 1.0;
    if (flags & SF_XPOW) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        num *= ipow_u(x[u][j], sx->x_num[j]);
        den *= ipow_u(x[u][j], sx->x_den[j]);
        const int h = sx->x_half[j];
        if (h > 0) hn *= x[u][j];
        if (h < 0) hd *= x[u][j];
      }
    }
    num *= ipow_u(U[u], ss.u_num);
    den *= ipow_u(U[u], ss.u_den);
    num *= ipow_u(F[u], ss.f_num);
    den *= ipow_u(F[u], ss.f_den);
    if (flags & SF_HALF) {
      if (ss.f_half > 0) hn *= F[u];
      if (ss.f_half < 0) hd *= F[u];
      // sqrt(hn / hd) = sqrt(hn hd) / hd
      B[u] = (num * sqrt(hn * hd)) * recip(den * hd);
    } else if (flags & SF_DEN) {
      B[u] = num * recip(den);
    } else {
      B[u] = num;
    }
  }
  const int M = ss.max_log;
  cptr<SectorDev> sl = launder_after(sd, B[0]);
  if (flags & SF_LOG) {
    double L[S];
#pragma unroll
    for (int u = 0; u < S; ++u) L[u] = log_f64(F[u]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double v[S];
#pragma unroll
      for (int u = 0; u < S; ++u) v[u] = sl->logc[k][M];
      for (int m = M - 1; m >= 0; --m) {
        const double cm = sl->logc[k][m];
#pragma unroll
        for (int u = 0; u < S; ++u) v[u] = __builtin_fma(v[u], L[u], cm);
      }
#pragma unroll
      for (int u = 0; u < S; ++u) f[u][k] = B[u] * v[u];
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int u = 0; u < S; ++u) f[u][k] = B[u] * sl->logc[k][0];
  }
}

// Integrand orders for the common sector shape (the plan sets SF_FAST): integer
// exponents of U and F only, no powers of x_j, and log F polynomials of degree at most
// K - 1 (the plan zero-pads them to that degree).  Straight-line code apart from the
// uniform exponent loops, which are shared by the S samples.
template <int D, int K, int S>
__device__ __forceinline__ void integrand_fast(const SectorScalars &ss, cptr<SectorDev> sd,
                                               cptr<double> coef, const double (&x)[S][D],
                                               double (&f)[S][K]) {
  double U[S], F[S];
  LoadChain ch{x[0][0], x[0][0]};
  poly<D, S>(coef + ss.u_off, ss.u_deg, x, U, ch);
  poly<D, S>(coef + ss.f_off, ss.f_deg, x, F, ch);
  double num[S], den[S];
#pragma unroll
  for (int u = 0; u < S; ++u) num[u] = den[u] = 1.0;
  for (int t = 0; t < ss.u_num; ++t)
#pragma unroll
    for (int u = 0; u < S; ++u) num[u] *= U[u];
  for (int t = 0; t < ss.u_den; ++t)
#pragma unroll
    for (int u = 0; u < S; ++u) den[u] *= U[u];
  for (int t = 0; t < ss.f_num; ++t)
#pragma unroll
    for (int u = 0; u < S; ++u) num[u] *= F[u];
  for (int t = 0; t < ss.f_den; ++t)
#pragma unroll
    for (int u = 0; u < S; ++u) den[u] *= F[u];
  double B[S];
#pragma unroll
  for (int u = 0; u < S; ++u) B[u] = num[u] * recip(den[u]);
  cptr<SectorDev> sl = launder_after(sd, B[0]);
  if (K > 1) {
    double L[S];
#pragma unroll
    for (int u = 0; u < S; ++u) L[u] = log_f64(F[u]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double v[S];
#pragma unroll
      for (int u = 0; u < S; ++u) v[u] = sl->logc[k][K - 1];
#pragma unroll
      for (int m = K - 2; m >= 0; --m) {
        const double cm = sl->logc[k][m];
#pragma unroll
        for (int u = 0; u < S; ++u) v[u] = __builtin_fma(v[u], L[u], cm);
      }
#pragma unroll
      for (int u = 0; u < S; ++u) f[u][k] = B[u] * v[u];
    }
  } else {
#pragma unroll
    for (int u = 0; u < S; ++u) f[u][0] = B[u] * sl->logc[0][0];
  }
}

// korobov3 on S samples: x = y^4 (35 - 84 y + 70 y^2 - 20 y^3), W = 140^d (prod y(1-y))^3.
template <int D, int S>
__device__ __forceinline__ void korobov3_fast(double w_scale, const double (&y)[S][D],
                                              double (&x)[S][D], double (&W)[S]) {
#pragma unroll
  for (int u = 0; u < S; ++u) {
    double T = 1.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double yj = y[u][j];
      const double p =
          __builtin_fma(__builtin_fma(__builtin_fma(-20.0, yj, 70.0), yj, -84.0), yj, 35.0);
      const double y2 = yj * yj;
      x[u][j] = (y2 * y2) * p;
      T *= yj * (1.0 - yj);
    }
    W[u] = w_scale * (T * T * T);
  }
}

// ------------------------------------------------------------- main kernel

// Workgroup -> sector by binary search over the launch's first-workgroup table.
__device__ __forceinline__ int find_sector(const int64_t *__restrict__ begin, int S, int64_t b) {
  int lo = 0, hi = S;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (begin[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Maximum shifts per workgroup and waves per workgroup (LDS staging of the partials).
constexpr int kMaxTile = 16;
constexpr int kMaxWaves = 4;

// Lattice points a thread sums in plain FP64 before folding the partial into its
// compensated (TwoSum) accumulator.
constexpr int kFold = 8;

// One workgroup: sector s, shifts [l_begin, l_begin + tile), lattice points of one
// chunk.  The shifts are processed S at a time: for each point the quotient k/n is
// formed once and reused by the S shifts of the pass, whose S*K accumulators stay in
// registers.  Each accumulator is a plain partial over at most kFold points folded
// into a (sum, compensation) pair.  After each pass the pairs are reduced over the
// wavefront and staged in LDS.
template <int D, int K, int S, bool FAST>
__device__ __forceinline__ void integrate_block(const LaunchArgs &a, int s, int l_begin, int tile,
                                                int64_t chunk_id, double (*red)[kMaxTile * 4][2]) {
  const SectorDev *__restrict__ sd = a.sectors + s;
  const LatticeDev *__restrict__ lt = a.lat + s;
  const uint64_t n = lt->n;
  const double n_d = lt->n_d, inv_n = lt->inv_n;
  const int64_t chunk = lt->chunk;
  const uint64_t i_begin = (uint64_t)(chunk_id * chunk);
  uint64_t i_end = i_begin + (uint64_t)chunk;
  if (i_end > n) i_end = n;
  const int kind = sd->transform;
  const double w_scale = sd->w_scale;
  const SectorScalars ss = load_scalars(sd);
  const uint64_t B = blockDim.x;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // every lane runs the same number of iterations; lanes past i_end contribute 0
  const int64_t n_iter = (int64_t)((i_end - i_begin + B - 1) / B);

  // lattice state of this thread at its first point i0: k_j = i0 z_j mod n
  double k0[D];
  const uint64_t i0 = i_begin + threadIdx.x;
#pragma unroll
  for (int j = 0; j < D; ++j) k0[j] = (double)mulmod(i0 % n, lt->z[j], n);

#pragma unroll 1
  for (int l0 = 0; l0 < tile; l0 += S) {
    DD acc[S][K];
#pragma unroll
    for (int u = 0; u < S; ++u)
#pragma unroll
      for (int kk = 0; kk < K; ++kk) acc[u][kk] = DD{0.0, 0.0};
    const double *__restrict__ sh = a.shifts + ((int64_t)s * a.m + l_begin + l0) * QMC_MAX_DIM;
    double k[D];
#pragma unroll
    for (int j = 0; j < D; ++j) k[j] = k0[j];

    uint64_t i = i0;
    int64_t it = 0;
#pragma unroll 1
    while (it < n_iter) {
      double part[S][K];
#pragma unroll
      for (int u = 0; u < S; ++u)
#pragma unroll
        for (int kk = 0; kk < K; ++kk) part[u][kk] = 0.0;
      const int64_t it_end = (n_iter - it < kFold) ? n_iter : it + kFold;
#pragma unroll 1
      for (; it < it_end; ++it, i += B) {
        const cptr<double> cl = launder_uniform(a.coef);
        const cptr<LatticeDev> ltl = launder_uniform(lt);
        const cptr<double> shl = launder_uniform(sh);
        double q[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          q[j] = quotient(k[j], n_d, inv_n);
          k[j] = lattice_step(k[j], ltl->ndz[j], n_d);
        }
        double y[S][D], x[S][D], W[S];
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
          for (int j = 0; j < D; ++j) y[u][j] = shifted(q[j], shl[u * QMC_MAX_DIM + j]);
        double f[S][K];
        if (FAST) {
          korobov3_fast<D, S>(w_scale, y, x, W);
          integrand_fast<D, K, S>(ss, (cptr<SectorDev>)sd, launder_after(cl, W[0]), x, f);
        } else {
#pragma unroll
          for (int u = 0; u < S; ++u) W[u] = apply_transform<D>(kind, w_scale, y[u], x[u]);
          integrand<D, K, S>(ss, (cptr<SectorDev>)sd, launder_after(cl, W[0]), x, f);
        }
        const bool valid = i < i_end;
#pragma unroll
        for (int u = 0; u < S; ++u) {
          const bool use = valid && (W[u] != 0.0);
#pragma unroll
          for (int kk = 0; kk < K; ++kk) part[u][kk] += use ? W[u] * f[u][kk] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < S; ++u)
#pragma unroll
        for (int kk = 0; kk < K; ++kk) dd_add(acc[u][kk], part[u][kk]);
    }
#pragma unroll
    for (int u = 0; u < S; ++u)
#pragma unroll
      for (int kk = 0; kk < K; ++kk) {
        const DD r = wave_reduce(acc[u][kk]);
        if (lane == 0) {
          red[wave][(l0 + u) * K + kk][0] = r.s;
          red[wave][(l0 + u) * K + kk][1] = r.c;
        }
      }
  }
}

// One launch per sector dimension D: workgroup blockIdx.x + block_base of the launch's
// global workgroup numbering (workgroups are numbered sector by sector, sectors ordered
// by dimension, so a dimension's workgroups are contiguous).
template <int D, int K, int S, bool FAST>
__global__ __launch_bounds__(256) void qmc_integrate_kernel(LaunchArgs a, int64_t block_base) {
  __shared__ double red[kMaxWaves][kMaxTile * 4][2];
  const int64_t b = block_base + blockIdx.x;
  const int s = a.order[find_sector(a.block_begin, a.n_sectors, b)];
  const LatticeDev *__restrict__ lt = a.lat + s;
  const int64_t local = b - lt->block_begin;
  const int nch = lt->n_chunks;
  const int tile_id = (int)(local / nch);
  const int64_t chunk_id = local - (int64_t)tile_id * nch;
  const int T = a.shift_tile;
  const int l_begin = tile_id * T;

  integrate_block<D, K, S, FAST>(a, s, l_begin, T, chunk_id, red);
  __syncthreads();
  // in-order combine of the waves, one thread per (shift in tile, order)
  const int nwaves = blockDim.x >> 6;
  if ((int)threadIdx.x < T * K) {
    DD r{red[0][threadIdx.x][0], red[0][threadIdx.x][1]};
    for (int w = 1; w < nwaves; ++w) r = dd_combine(r, DD{red[w][threadIdx.x][0], red[w][threadIdx.x][1]});
    double *out = a.partial + (b * (T * K) + threadIdx.x) * 2;
    out[0] = r.s;
    out[1] = r.c;
  }
}

// Combine the workgroup partials of one (sector, shift) in workgroup order: one wave
// per (sector, shift), lanes stride over the sector's chunks, then a TwoSum butterfly.
__global__ __launch_bounds__(64) void qmc_reduce_kernel(LaunchArgs a) {
  const int s = blockIdx.x / a.m;
  const int l = blockIdx.x - s * a.m;
  const int T = a.shift_tile;
  const int K = a.K;
  const int tile = l / T, lt_ = l - tile * T;
  const LatticeDev *__restrict__ lat = a.lat + s;
  if (!lat->active) return;   // sector not integrated by this launch: keep its Q
  const int nch = lat->n_chunks;
  const int64_t first = lat->block_begin + (int64_t)tile * nch;
  for (int kk = 0; kk < K; ++kk) {
    DD r{0.0, 0.0};
    for (int c = threadIdx.x; c < nch; c += 64) {
      const double *p = a.partial + ((first + c) * (T * K) + lt_ * K + kk) * 2;
      r = dd_combine(r, DD{p[0], p[1]});
    }
    r = wave_reduce(r);
    if (threadIdx.x == 0) {
      const double q = (r.s + r.c) / lat->n_d;
      a.q[((int64_t)s * a.m + l) * K + kk] = q;
      if (!isfinite(q)) {
        const int code = (s * a.m + l) * QMC_MAX_ORDERS + kk;
        atomicMin(a.status, code);
      }
    }
  }
}

// Shift mean and standard error per (sector, order).
__global__ void qmc_stats_kernel(LaunchArgs a) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.n_sectors * a.K) return;
  const int s = idx / a.K, kk = idx - s * a.K;
  const int m = a.m;
  const double *q = a.q + (int64_t)s * m * a.K + kk;
  DD sum{0.0, 0.0};
  for (int l = 0; l < m; ++l) dd_add(sum, q[(int64_t)l * a.K]);
  const double mean = (sum.s + sum.c) / (double)m;
  DD ss{0.0, 0.0};
  for (int l = 0; l < m; ++l) {
    const double dlt = q[(int64_t)l * a.K] - mean;
    dd_add(ss, dlt * dlt);
  }
  const double var = (ss.s + ss.c) / (double)(m - 1);
  a.mean[idx] = mean;
  a.err[idx] = sqrt(var / (double)m);
}

__global__ void qmc_status_reset_kernel(int32_t *status) {
  if (threadIdx.x == 0) status[0] = INT32_MAX;
}

// ------------------------------------------------------------ lattice points out

// The lattice step of the integration kernel on its own: thread t of workgroup b
// starts at i = i0 + b * steps * blockDim + t and walks `steps` points with stride
// blockDim, exactly like a workgroup of the integration kernel walks its chunk.
__global__ __launch_bounds__(256) void qmc_points_kernel(PointsArgs pa) {
  const uint64_t B = blockDim.x;
  const uint64_t first = pa.i0 + (uint64_t)blockIdx.x * pa.steps * B + threadIdx.x;
  const uint64_t end = pa.i0 + pa.count;
  double k[QMC_MAX_DIM];
  for (int j = 0; j < pa.d; ++j) k[j] = (double)mulmod(first % pa.n, pa.z[j], pa.n);
  uint64_t i = first;
  for (uint32_t r = 0; r < pa.steps && i < end; ++r, i += B) {
    for (int j = 0; j < pa.d; ++j) {
      const double q = quotient(k[j], pa.n_d, pa.inv_n);
      pa.out[(i - pa.i0) * pa.d + j] = shifted(q, pa.delta[j]);
      k[j] = lattice_step(k[j], pa.ndz[j], pa.n_d);
    }
  }
}

int launch_points(const PointsArgs &pa, unsigned grid, void *stream) {
  hipLaunchKernelGGL(qmc_points_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, pa);
  return (int)hipGetLastError();
}

// ----------------------------------------------------- Korobov figure of merit

// Partial sums of prod_j [1 + 2 pi^2 B2({k z_j / n})] over a chunk of k, for one
// candidate a per blockIdx.y.
__global__ __launch_bounds__(256) void qmc_p2_kernel(uint64_t n, int32_t d,
                                                     const uint64_t *__restrict__ cand,
                                                     int32_t chunks, double *partial) {
  const int c = blockIdx.y;
  const uint64_t a = cand[c];
  const double n_d = (double)n, inv_n = 1.0 / n_d;
  const double two_pi2 = 19.739208802178716;  // 2 pi^2
  const uint64_t per = (n + chunks - 1) / chunks;
  const uint64_t k_begin = (uint64_t)blockIdx.x * per;
  uint64_t k_end = k_begin + per;
  if (k_end > n) k_end = n;
  uint64_t z[QMC_MAX_DIM], kz[QMC_MAX_DIM], dz[QMC_MAX_DIM];
  uint64_t zj = 1;
  const uint64_t k0 = k_begin + threadIdx.x;
  for (int j = 0; j < QMC_MAX_DIM; ++j) {
    z[j] = zj;
    kz[j] = mulmod(k0 % n, zj, n);
    dz[j] = mulmod(blockDim.x % n, zj, n);
    zj = mulmod(zj, a, n);
  }
  DD acc{0.0, 0.0};
  for (uint64_t k = k0; k < k_end; k += blockDim.x) {
    double prod = 1.0;
    for (int j = 0; j < d; ++j) {
      const double x = quotient((double)kz[j], n_d, inv_n);
      const double b2 = __builtin_fma(x, x - 1.0, 1.0 / 6.0);
      prod *= __builtin_fma(two_pi2, b2, 1.0);
      const uint64_t kn = kz[j] + dz[j];
      kz[j] = (kn >= n) ? kn - n : kn;
    }
    dd_add(acc, prod);
  }
  (void)z;
  acc = wave_reduce(acc);
  __shared__ double red[4][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = acc.s;
    red[wave][1] = acc.c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    DD r{red[0][0], red[0][1]};
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = dd_combine(r, DD{red[w][0], red[w][1]});
    double *out = partial + ((int64_t)c * chunks + blockIdx.x) * 2;
    out[0] = r.s;
    out[1] = r.c;
  }
}

__global__ void qmc_p2_finish_kernel(uint64_t n, int32_t n_cand, int32_t chunks,
                                     const double *partial, double *p2) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cand) return;
  DD r{0.0, 0.0};
  for (int b = 0; b < chunks; ++b) {
    const double *p = partial + ((int64_t)c * chunks + b) * 2;
    r = dd_combine(r, DD{p[0], p[1]});
  }
  p2[c] = -1.0 + (r.s + r.c) / (double)n;
}

// ------------------------------------------------------------------ launchers

template <int D, int S, bool FAST>
static hipError_t launch_ds(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  dim3 grid((unsigned)dl.blocks), blk((unsigned)a.block);
  switch (a.K) {
    case 1: hipLaunchKernelGGL((qmc_integrate_kernel<D, 1, S, FAST>), grid, blk, 0, st, a, dl.base); break;
    case 2: hipLaunchKernelGGL((qmc_integrate_kernel<D, 2, S, FAST>), grid, blk, 0, st, a, dl.base); break;
    case 3: hipLaunchKernelGGL((qmc_integrate_kernel<D, 3, S, FAST>), grid, blk, 0, st, a, dl.base); break;
    default: hipLaunchKernelGGL((qmc_integrate_kernel<D, 4, S, FAST>), grid, blk, 0, st, a, dl.base); break;
  }
  return hipGetLastError();
}

// Sectors of the generic shape run one shift per pass (they are the uncommon case).
template <int D>
static hipError_t launch_d(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  if (!dl.fast) return launch_ds<D, 1, false>(a, dl, st);
  switch (a.shifts_per_pass) {
    case 1: return launch_ds<D, 1, true>(a, dl, st);
    case 4: return launch_ds<D, 4, true>(a, dl, st);
    default: return launch_ds<D, 2, true>(a, dl, st);
  }
}

static hipError_t launch_class(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  switch (dl.d) {
    case 1: return launch_d<1>(a, dl, st);
    case 2: return launch_d<2>(a, dl, st);
    case 3: return launch_d<3>(a, dl, st);
    case 4: return launch_d<4>(a, dl, st);
    case 5: return launch_d<5>(a, dl, st);
    case 6: return launch_d<6>(a, dl, st);
    case 7: return launch_d<7>(a, dl, st);
    default: return launch_d<8>(a, dl, st);
  }
}

bool tile_supported(int shift_tile, int shifts_per_pass, int block) {
  if (block < 64 || block > 64 * kMaxWaves || (block % 64) != 0) return false;
  if (shift_tile < 1 || shift_tile > kMaxTile) return false;
  if (shifts_per_pass != 1 && shifts_per_pass != 2 && shifts_per_pass != 4) return false;
  return shift_tile % shifts_per_pass == 0;
}

int launch_integrate(const LaunchArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (a.ev_start && (e = hipEventRecord((hipEvent_t)a.ev_start, st)) != hipSuccess) return (int)e;
  for (int t = 0; t < a.n_dim_launches; ++t) {
    const DimLaunch &dl = a.dims[t];
    if (dl.blocks == 0) continue;
    if ((e = launch_class(a, dl, st)) != hipSuccess) return (int)e;
  }
  if (a.ev_stop && (e = hipEventRecord((hipEvent_t)a.ev_stop, st)) != hipSuccess) return (int)e;
  hipLaunchKernelGGL(qmc_reduce_kernel, dim3((unsigned)(a.n_sectors * a.m)), dim3(64), 0, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  const int nk = a.n_sectors * a.K;
  hipLaunchKernelGGL(qmc_stats_kernel, dim3((unsigned)((nk + 127) / 128)), dim3(128), 0, st, a);
  return (int)hipGetLastError();
}

int launch_status_reset(int32_t *status, void *stream) {
  hipLaunchKernelGGL(qmc_status_reset_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, status);
  return (int)hipGetLastError();
}

int launch_korobov_p2(uint64_t n, int32_t d, const uint64_t *dev_cand, int32_t n_cand,
                      int32_t chunks, double *dev_partial, double *dev_p2, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(qmc_p2_kernel, dim3((unsigned)chunks, (unsigned)n_cand), dim3(256), 0, st,
                     n, d, dev_cand, chunks, dev_partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(qmc_p2_finish_kernel, dim3((unsigned)((n_cand + 127) / 128)), dim3(128), 0,
                     st, n, n_cand, chunks, dev_partial, dev_p2);
  return (int)hipGetLastError();
}

}  // namespace qmc
