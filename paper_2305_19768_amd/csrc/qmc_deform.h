// qmc_deform.h -- device helpers of the deformed-contour integrand (complex arithmetic,
// complex Horner, the Jacobian determinant, log(F - i0), the integrand in FP64 and with
// the FP32 polynomial bulk).  Shared by the deformed-contour kernels and the
// flow-transformed integration on the deformed contour.  Not part of the C ABI.
#pragma once

#include "qmc_device.h"

namespace qmc {


struct C2 {
  double r, i;
};

__device__ __forceinline__ C2 cmul(C2 a, C2 b) {
  return C2{__builtin_fma(a.r, b.r, -(a.i * b.i)), __builtin_fma(a.r, b.i, a.i * b.r)};
}

// a * b + c
__device__ __forceinline__ C2 cfma(C2 a, C2 b, C2 c) {
  return C2{__builtin_fma(a.r, b.r, __builtin_fma(-a.i, b.i, c.r)),
            __builtin_fma(a.r, b.i, __builtin_fma(a.i, b.r, c.i))};
}

__device__ __forceinline__ C2 crecip(C2 a) {
  const double inv = recip(__builtin_fma(a.r, a.r, a.i * a.i));
  return C2{a.r * inv, -a.i * inv};
}

__device__ __forceinline__ C2 cipow(C2 z, int e) {
  C2 r{1.0, 0.0};
  for (int t = 0; t < e; ++t) r = cmul(r, z);
  return r;
}

// Square root with the branch cut on the negative real axis taken from below
// (argument of a in [-pi, pi), so sqrt(-|a|) = -i sqrt|a|); for Re a >= 0 it is the
// principal root.
__device__ __forceinline__ C2 csqrt_minus_i0(C2 a) {
  const double r = sqrt(__builtin_fma(a.r, a.r, a.i * a.i));
  if (r == 0.0) return C2{0.0, 0.0};
  if (a.r >= 0.0) {
    const double t = sqrt(0.5 * (r + a.r));
    return C2{t, a.i * (0.5 * recip(t))};
  }
  const double t = sqrt(0.5 * (r - a.r));
  const double sgn = a.i > 0.0 ? 1.0 : -1.0;   // Im a = +-0: below the cut
  return C2{__builtin_fabs(a.i) * (0.5 * recip(t)), sgn * t};
}

// log(F - i0)
__device__ __forceinline__ C2 clog_minus_i0(C2 a) {
  const double lr = 0.5 * log_f64(__builtin_fma(a.r, a.r, a.i * a.i));
  const double arg = (a.i == 0.0 && a.r < 0.0) ? -3.141592653589793 : atan2(a.i, a.r);
  return C2{lr, arg};
}

// Dense nested Horner with complex variables over the degree-3 layout (coefficients
// real and wave-uniform), total degree DEG.
template <int D, int DEG>
__device__ __forceinline__ C2 horner_c(cptr<double> c, const C2 (&z)[D], LoadChain &ch) {
  c = ch.next(c);
  C2 acc{c[0], 0.0};
  int p = 1;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    c = ch.next(c);
    C2 g{c[p], 0.0};
    ++p;
    if (DEG >= 2) {
#pragma unroll
      for (int k = j; k < D; ++k) {
        if (DEG >= 3) c = ch.next(c);
        C2 h{c[p], 0.0};
        ++p;
        if (DEG >= 3) {
#pragma unroll
          for (int l = k; l < D; ++l) {
            h.r = __builtin_fma(c[p + l - k], z[l].r, h.r);
            h.i = __builtin_fma(c[p + l - k], z[l].i, h.i);
          }
          ch.done(h.r);
        }
        p += D - k;
        g = cfma(z[k], h, g);
      }
    } else {
      p += (D - j) * (D - j + 3) / 2;
    }
    acc = cfma(z[j], g, acc);
    ch.done(acc.r);
  }
  return acc;
}

template <int D>
__device__ __forceinline__ C2 poly_c(cptr<double> c, int deg, const C2 (&z)[D], LoadChain &ch) {
  if (deg >= 3) return horner_c<D, 3>(c, z, ch);
  if (deg == 2) return horner_c<D, 2>(c, z, ch);
  return horner_c<D, 1>(c, z, ch);
}

constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }   // lower triangle, j <= i

// Elimination determinant of the complex symmetric matrix A (lower triangle, packed by
// tri), without pivoting: the Hermitian part of A is the identity, so every pivot has
// real part >= 1.  A is overwritten.
template <int D>
__device__ __forceinline__ C2 det_sym(C2 (&A)[D * (D + 1) / 2]) {
  C2 det{1.0, 0.0};
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const C2 piv = A[tri(k, k)];
    det = cmul(det, piv);
    if (k + 1 < D) {
      const C2 r = crecip(piv);
#pragma unroll
      for (int i = k + 1; i < D; ++i) {
        const C2 t = cmul(A[tri(i, k)], r);
#pragma unroll
        for (int j = k + 1; j <= i; ++j) {   // A_ij -= t A_jk, four fused operations
          const C2 a = A[tri(j, k)], b = A[tri(i, j)];
          A[tri(i, j)] = C2{__builtin_fma(-t.r, a.r, __builtin_fma(t.i, a.i, b.r)),
                            __builtin_fma(-t.r, a.i, __builtin_fma(-t.i, a.r, b.i))};
        }
      }
    }
  }
  return det;
}

// The orders f_k = det x^p U^a F^b sum_m c_km (log F)^m on the contour point z, given
// U(z) and F(z): powers, roots, the division and the logarithm in FP64.
template <int D, int NK>
__device__ __forceinline__ void deform_finish(const SectorScalars &ss, cptr<SectorDev> sd, C2 det,
                                              const C2 (&z)[D], C2 U, C2 F, C2 (&f)[NK]) {
  const int flags = ss.flags;
  cptr<SectorDev> sx = launder_after(sd, F.r);
  C2 num = det, den{1.0, 0.0};
  if (flags & SF_XPOW) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      num = cmul(num, cipow(z[j], sx->x_num[j]));
      den = cmul(den, cipow(z[j], sx->x_den[j]));
      const int h = sx->x_half[j];
      if (h != 0) {
        const C2 r = csqrt_minus_i0(z[j]);   // Re z_j = x_j >= 0: principal root
        if (h > 0) num = cmul(num, r);
        else den = cmul(den, r);
      }
    }
  }
  num = cmul(num, cipow(U, ss.u_num));
  den = cmul(den, cipow(U, ss.u_den));
  num = cmul(num, cipow(F, ss.f_num));
  den = cmul(den, cipow(F, ss.f_den));
  if (ss.f_half != 0) {
    const C2 r = csqrt_minus_i0(F);
    if (ss.f_half > 0) num = cmul(num, r);
    else den = cmul(den, r);
  }
  const C2 B = (flags & SF_DEN) ? cmul(num, crecip(den)) : num;
  const int M = ss.max_log;
  cptr<SectorDev> sl = launder_after(sd, B.r);
  if (flags & SF_LOG) {
    const C2 L = clog_minus_i0(F);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      C2 v{sl->logc[k][M], 0.0};
      for (int m = M - 1; m >= 0; --m) v = cfma(v, L, C2{sl->logc[k][m], 0.0});
      f[k] = cmul(B, v);
    }
  } else {
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const double c0 = sl->logc[k][0];
      f[k] = C2{B.r * c0, B.i * c0};
    }
  }
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The Hessian H_jk(x) = h0_jk + L_jk(x) of F (degree <= 3: L_jk is linear and homogeneous)
// and the gradient from it by Euler's theorem on the homogeneous parts of F,
// dF/dx_j = c_j + sum_k x_k (h0_jk + L_jk(x) / 2) with c_j = dF/dx_j at x = 0 (packed
// by the plan): about a third of the operations of D dense gradient polynomials of
// degree 2.  Fills A with I - i lambda (D1 + S H S) (lower
// triangle) and g with the gradient.  T: the polynomial arithmetic (double or float).
template <int D, class T, class P, class Chain>
__device__ __forceinline__ void hessian_and_gradient(P coef, int grad_off, int hess_off,
                                                     double lam, const double (&x)[D],
                                                     const T (&xt)[D], Chain &ch, double (&g)[D],
                                                     C2 (&A)[D * (D + 1) / 2]) {
  double sq[D];
  T gt[D];
  {
    const P cg = ch.next(coef + grad_off);
#pragma unroll
    for (int j = 0; j < D; ++j) gt[j] = cg[j];
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const double s = x[j] * (1.0 - x[j]);
    // korobov3 evaluated with fused multiply-adds can round x a few ulp above 1 near
    // y = 1, making s a tiny negative number; the symmetric scaling takes its root
    sq[j] = sqrt(__builtin_fmax(s, 0.0));
  }
  int t = 0;
#pragma unroll
  for (int j = 0; j < D; ++j)
#pragma unroll
    for (int k = j; k < D; ++k, ++t) {
      const P c = ch.next(coef + hess_off + t * dense_len1(D));
      T L = c[1] * xt[0];
#pragma unroll
      for (int l = 1; l < D; ++l) L = fma_t(c[1 + l], xt[l], L);
      ch.done(L);
      const T h0 = c[0];
      const T w = fma_t((T)0.5, L, h0);
      gt[j] = fma_t(xt[k], w, gt[j]);
      if (k != j) gt[k] = fma_t(xt[j], w, gt[k]);
      const double v = -lam * sq[j] * sq[k] * (double)(L + h0);
      if (k == j) A[tri(j, j)] = C2{1.0, v};
      else A[tri(k, j)] = C2{0.0, v};
    }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    g[j] = (double)gt[j];
    A[tri(j, j)].i += -lam * (1.0 - 2.0 * x[j]) * g[j];
  }
}

// J f_k(z(x)) for every order; returns whether the sample violates the sign check.
template <int D, int NK>
__device__ __forceinline__ bool integrand_deform(const SectorScalars &ss, cptr<SectorDev> sd,
                                                 cptr<double> coef, int grad_off, int hess_off,
                                                 double lam, const double (&x)[D], C2 (&f)[NK]) {
  LoadChain ch{x[0], x[0]};
  double g[D];
  C2 A[D * (D + 1) / 2];
  hessian_and_gradient<D, double>(coef, grad_off, hess_off, lam, x, x, ch, g, A);
  const C2 det = det_sym<D>(A);
  // the contour point, formed after the elimination so that it is not live across it
  C2 z[D];
#pragma unroll
  for (int j = 0; j < D; ++j) z[j] = C2{x[j], -lam * (x[j] * (1.0 - x[j])) * g[j]};
  const C2 U = poly_c<D>(coef + ss.u_off, ss.u_deg, z, ch);
  const C2 F = poly_c<D>(coef + ss.f_off, ss.f_deg, z, ch);
  const bool viol = F.i > 0.0 && F.i * F.i > 0x1p-80 * __builtin_fma(F.r, F.r, F.i * F.i);
  deform_finish<D, NK>(ss, sd, det, z, U, F, f);
  return viol;
}

// ------------------------------------------------------------- FP32 bulk form
// The polynomial work of a sample -- the gradient and Hessian of F at x, U(z) and F(z)
// -- in FP32 from the FP32 copy of the tables; the lattice point, the transform, the
// Jacobian matrix and its determinant, the powers, the division, the logarithm and
// every accumulation stay FP64.

struct C2f {
  float r, i;
};

// a * b + c with real-coefficient Horner operands of the FP32 polynomials
__device__ __forceinline__ C2f cfmaf(C2f a, C2f b, C2f c) {
  return C2f{__builtin_fmaf(a.r, b.r, __builtin_fmaf(-a.i, b.i, c.r)),
             __builtin_fmaf(a.r, b.i, __builtin_fmaf(a.i, b.r, c.i))};
}

template <int D, int DEG>
__device__ __forceinline__ C2f horner_cf(cptr<float> c, const C2f (&z)[D], LoadChainF &ch) {
  c = ch.next(c);
  C2f acc{c[0], 0.0f};
  int p = 1;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    c = ch.next(c);
    C2f g{c[p], 0.0f};
    ++p;
    if (DEG >= 2) {
#pragma unroll
      for (int k = j; k < D; ++k) {
        if (DEG >= 3) c = ch.next(c);
        C2f h{c[p], 0.0f};
        ++p;
        if (DEG >= 3) {
#pragma unroll
          for (int l = k; l < D; ++l) {
            h.r = __builtin_fmaf(c[p + l - k], z[l].r, h.r);
            h.i = __builtin_fmaf(c[p + l - k], z[l].i, h.i);
          }
          ch.done(h.r);
        }
        p += D - k;
        g = cfmaf(z[k], h, g);
      }
    } else {
      p += (D - j) * (D - j + 3) / 2;
    }
    acc = cfmaf(z[j], g, acc);
    ch.done(acc.r);
  }
  return acc;
}

template <int D>
__device__ __forceinline__ C2f poly_cf(cptr<float> c, int deg, const C2f (&z)[D], LoadChainF &ch) {
  if (deg >= 3) return horner_cf<D, 3>(c, z, ch);
  if (deg == 2) return horner_cf<D, 2>(c, z, ch);
  return horner_cf<D, 1>(c, z, ch);
}

// integrand_deform with the polynomial bulk in FP32.  The sign check uses the FP32
// value of F(z) with a margin above FP32 rounding: Im F(z) > 2^-20 |F(z)|.
template <int D, int NK>
__device__ __forceinline__ bool integrand_deform_f32(const SectorScalars &ss, cptr<SectorDev> sd,
                                                     cptr<float> coef, int grad_off, int hess_off,
                                                     double lam, const double (&x)[D],
                                                     C2 (&f)[NK]) {
  float xf[D];
#pragma unroll
  for (int j = 0; j < D; ++j) xf[j] = (float)x[j];
  LoadChainF ch{xf[0]};
  double g[D];
  C2 A[D * (D + 1) / 2];
  hessian_and_gradient<D, float>(coef, grad_off, hess_off, lam, x, xf, ch, g, A);
  const C2 det = det_sym<D>(A);
  C2 z[D];
  C2f zf[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    z[j] = C2{x[j], -lam * (x[j] * (1.0 - x[j])) * g[j]};
    zf[j] = C2f{xf[j], (float)z[j].i};
  }
  const C2f Uf = poly_cf<D>(coef + ss.u_off32, ss.u_deg, zf, ch);
  const C2f Ff = poly_cf<D>(coef + ss.f_off32, ss.f_deg, zf, ch);
  const C2 U{(double)Uf.r, (double)Uf.i}, F{(double)Ff.r, (double)Ff.i};
  const bool viol = F.i > 0.0 && F.i * F.i > 0x1p-40 * __builtin_fma(F.r, F.r, F.i * F.i);
  deform_finish<D, NK>(ss, sd, det, z, U, F, f);
  return viol;
}

}  // namespace qmc
