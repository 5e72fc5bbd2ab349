// qmc_device.h -- device functions of the lattice QMC kernels (gfx950): compensated
// sums, exact lattice points, periodizing transforms, dense nested-Horner polynomials,
// the integrand orders in FP64 and FP32, and the body of one integration workgroup.
#pragma once

// The header is also compiled at run time (hiprtc) for plan-specialised integrands,
// where the runtime and integer types are built in.
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <stdint.h>
#endif

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

// A wave-uniform 64-bit value moved into scalar registers (a copy when it already is).
__device__ __forceinline__ uint64_t to_sgpr64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ cptr<T> launder_uniform(const T *p) {
  cptr<T> c = (cptr<T>)to_sgpr64((uint64_t)(uintptr_t)p);
  asm volatile("" : "+s"(c));
  return c;
}

// Launder that also waits for a per-lane value: the loads through the result cannot
// start before `after` is computed.  Chaining each group of table reads to the
// previous group's result bounds the number of table values held in SGPRs.
template <typename T>
__device__ __forceinline__ cptr<T> launder_after(cptr<T> c, double after) {
  c = (cptr<T>)to_sgpr64((uint64_t)c);
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
// One Newton step on the hardware reciprocal (about 2^-25 relative on gfx950): within
// about 11 ulp of 1/v (measured over 4M random arguments; two steps: within half an ulp).
// Used where a relative error of a few 1e-15 in a factor of the integrand is immaterial.
__device__ __forceinline__ double recip1(double v) {
  const double r = __builtin_amdgcn_rcp(v);
  return __builtin_fma(__builtin_fma(-v, r, 1.0), r, r);
}

// Natural logarithm of log F, accurate to a few ulp.  x = m 2^e with m in
// [sqrt(1/2), sqrt(2)); log m = 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.1716, by the
// Taylor series atanh(s) = s sum_k s^(2k)/(2k+1) through s^19 (remainder below 2.4e-17
// relative); e ln 2 with ln 2 split into a 32-bit head (e * head exact) and a tail.
// log(0) = -inf, log(+inf) = +inf, negative or NaN input gives NaN.
// log_pos: the same for x known to be positive and finite (F with non-negative
// coefficients and a positive constant term, on the unit cube), without the special
// cases (no compare-and-select, no divergent branch).
__device__ __forceinline__ double log_pos(double x) {
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
  return __builtin_fma(ed, kLn2Hi, __builtin_fma(ed, kLn2Lo, logm));
}

// Logarithm by table reduction, for the plan-specialised kernels (x positive and
// finite).  x = m 2^e with m in [1/2, 1); the top six bits of m's mantissa pick
// c_i = (1 + (i + 1/2)/64)/2, the centre of m's bucket, so r = m / c_i - 1 lies within
// +-1/129; log x = e ln 2 + ln c_i + log1p(r), with log1p(r) = r (1 - r/2 + ... + r^6/7)
// (the next term, r^8/8, is below 2e-18).  kLogTab[i] = {RN(1/c_i), RN(ln c_i)}; r is
// formed as fma(m, RN(1/c_i), -1).  Absolute error a few 1e-16 (relative accuracy near
// x = 1 is not kept; the integrands use log x only multiplied into smooth terms).  The
// table lives in LDS (LogTable, filled once per workgroup by fill_log_table).
constexpr double kLogTab[64][2] = {
    {0x1.fc07f01fc07f0p+0, -0x1.5ee82aa241920p-1},
    {0x1.f44659e4a4271p+0, -0x1.5707a26bb8c66p-1},
    {0x1.ecc07b301ecc0p+0, -0x1.4f45a835a4e19p-1},
    {0x1.e573ac901e574p+0, -0x1.47a1527e8a2d3p-1},
    {0x1.de5d6e3f8868ap+0, -0x1.4019c2125ca93p-1},
    {0x1.d77b654b82c34p+0, -0x1.38ae2171976e7p-1},
    {0x1.d0cb58f6ec074p+0, -0x1.315da4434068bp-1},
    {0x1.ca4b3055ee191p+0, -0x1.2a2786d0ec107p-1},
    {0x1.c3f8f01c3f8f0p+0, -0x1.230b0d8bebc98p-1},
    {0x1.bdd2b899406f7p+0, -0x1.1c07849ae6007p-1},
    {0x1.b7d6c3dda338bp+0, -0x1.151c3f6f29612p-1},
    {0x1.b2036406c80d9p+0, -0x1.0e4898611cce1p-1},
    {0x1.ac5701ac5701bp+0, -0x1.078bf0533c568p-1},
    {0x1.a6d01a6d01a6dp+0, -0x1.00e5ae5b207abp-1},
    {0x1.a16d3f97a4b02p+0, -0x1.f4aa7ee03192dp-2},
    {0x1.9c2d14ee4a102p+0, -0x1.e7b42c3ddad73p-2},
    {0x1.970e4f80cb872p+0, -0x1.dae75484c9616p-2},
    {0x1.920fb49d0e229p+0, -0x1.ce42f18064743p-2},
    {0x1.8d3018d3018d3p+0, -0x1.c1c60693fa39ep-2},
    {0x1.886e5f0abb04ap+0, -0x1.b56fa04462909p-2},
    {0x1.83c977ab2beddp+0, -0x1.a93ed3c8ad9e3p-2},
    {0x1.7f405fd017f40p+0, -0x1.9d32bea15ed3bp-2},
    {0x1.7ad2208e0ecc3p+0, -0x1.914a8635bf68ap-2},
    {0x1.767dce434a9b1p+0, -0x1.85855776dcbfbp-2},
    {0x1.724287f46debcp+0, -0x1.79e26687cfb3ep-2},
    {0x1.6e1f76b4337c7p+0, -0x1.6e60ee6af1972p-2},
    {0x1.6a13cd1537290p+0, -0x1.630030b3aac49p-2},
    {0x1.661ec6a5122f9p+0, -0x1.57bf753c8d1fbp-2},
    {0x1.623fa77016240p+0, -0x1.4c9e09e172c3cp-2},
    {0x1.5e75bb8d015e7p+0, -0x1.419b423d5e8c7p-2},
    {0x1.5ac056b015ac0p+0, -0x1.36b6776be1117p-2},
    {0x1.571ed3c506b3ap+0, -0x1.2bef07cdc9354p-2},
    {0x1.5390948f40febp+0, -0x1.214456d0eb8d4p-2},
    {0x1.5015015015015p+0, -0x1.16b5ccbacfb73p-2},
    {0x1.4cab88725af6ep+0, -0x1.0c42d676162e3p-2},
    {0x1.49539e3b2d067p+0, -0x1.01eae5626c691p-2},
    {0x1.460cbc7f5cf9ap+0, -0x1.ef5ade4dcffe6p-3},
    {0x1.42d6625d51f87p+0, -0x1.db13db0d48940p-3},
    {0x1.3fb013fb013fbp+0, -0x1.c6ffbc6f00f71p-3},
    {0x1.3c995a47babe7p+0, -0x1.b31d8575bce3dp-3},
    {0x1.3991c2c187f63p+0, -0x1.9f6c407089664p-3},
    {0x1.3698df3de0748p+0, -0x1.8beafeb38fe8cp-3},
    {0x1.33ae45b57bcb2p+0, -0x1.7898d85444c73p-3},
    {0x1.30d190130d190p+0, -0x1.6574ebe8c133ap-3},
    {0x1.2e025c04b8097p+0, -0x1.527e5e4a1b58dp-3},
    {0x1.2b404ad012b40p+0, -0x1.3fb45a59928ccp-3},
    {0x1.288b01288b013p+0, -0x1.2d1610c86813ap-3},
    {0x1.25e22708092f1p+0, -0x1.1aa2b7e23f72ap-3},
    {0x1.23456789abcdfp+0, -0x1.08598b59e3a07p-3},
    {0x1.20b470c67c0d9p+0, -0x1.ec739830a1120p-4},
    {0x1.1e2ef3b3fb874p+0, -0x1.c885801bc4b23p-4},
    {0x1.1bb4a4046ed29p+0, -0x1.a4e7640b1bc38p-4},
    {0x1.19453808ca29cp+0, -0x1.8197e2f40e3f0p-4},
    {0x1.16e0689427379p+0, -0x1.5e95a4d9791cbp-4},
    {0x1.1485f0e0acd3bp+0, -0x1.3bdf5a7d1ee64p-4},
    {0x1.12358e75d3033p+0, -0x1.1973bd1465567p-4},
    {0x1.0fef010fef011p+0, -0x1.eea31c006b87cp-5},
    {0x1.0db20a88f4696p+0, -0x1.aaef2d0fb10fcp-5},
    {0x1.0b7e6ec259dc8p+0, -0x1.67c94f2d4bb58p-5},
    {0x1.0953f39010954p+0, -0x1.252f32f8d183fp-5},
    {0x1.073260a47f7c6p+0, -0x1.c63d2ec14aaf2p-6},
    {0x1.05197f7d73404p+0, -0x1.432a925980cc1p-6},
    {0x1.03091b51f5e1ap+0, -0x1.82448a388a2aap-7},
    {0x1.0101010101010p+0, -0x1.0080559588b35p-8},
};
struct LogTable {
  double v[64][2];
};
__device__ __forceinline__ void fill_log_table(LogTable &t) {
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    t.v[i][0] = kLogTab[i][0];
    t.v[i][1] = kLogTab[i][1];
  }
}
__device__ __forceinline__ double log_tab(double x, const LogTable &t) {
  constexpr double kLn2Hi = 0x1.62e42ffp-1;
  constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
  const double m = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
  const int e = __builtin_amdgcn_frexp_exp(x);
  const unsigned hi = (unsigned)(__builtin_bit_cast(unsigned long long, m) >> 32);
  const int i = (int)((hi >> 14) & 63u);             // top six mantissa bits
  const double inv_c = t.v[i][0], log_c = t.v[i][1];
  const double r = __builtin_fma(m, inv_c, -1.0);
  double p = 1.0 / 7.0;
  p = __builtin_fma(p, r, -1.0 / 6.0);
  p = __builtin_fma(p, r, 1.0 / 5.0);
  p = __builtin_fma(p, r, -1.0 / 4.0);
  p = __builtin_fma(p, r, 1.0 / 3.0);
  p = __builtin_fma(p, r, -0.5);
  p = __builtin_fma(p, r, 1.0);
  const double ed = (double)e;
  return __builtin_fma(ed, kLn2Hi, __builtin_fma(ed, kLn2Lo, __builtin_fma(r, p, log_c)));
}

__device__ __forceinline__ double log_f64(double x) {
  const double r = log_pos(x);
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
  int u_off, f_off, u_off32, f_off32;
};

template <typename P>
__device__ __forceinline__ SectorScalars load_scalars(P sd) {
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
  r.u_off32 = sd->u_off32;
  r.f_off32 = sd->f_off32;
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
// Coefficients of the korobov_3 polynomial held in registers for a whole loop.  A
// float64 operation takes at most one literal, so with literal operands every point
// would rebuild one of them with two moves; the opaque copies below are made once.
struct KorobovConsts {
  double c0, c1, c2, c3;
};
__device__ __forceinline__ double opaque_vgpr(double v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ KorobovConsts korobov3_consts() {
  return KorobovConsts{opaque_vgpr(35.0), opaque_vgpr(-84.0), opaque_vgpr(70.0),
                       opaque_vgpr(-20.0)};
}

template <int D, int S>
__device__ __forceinline__ void korobov3_fast(double w_scale, const KorobovConsts &c,
                                              const double (&y)[S][D], double (&x)[S][D],
                                              double (&W)[S]) {
#pragma unroll
  for (int u = 0; u < S; ++u) {
    double T = 1.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double yj = y[u][j];
      const double p =
          __builtin_fma(__builtin_fma(__builtin_fma(c.c3, yj, c.c2), yj, c.c1), yj, c.c0);
      const double y2 = yj * yj;
      x[u][j] = (y2 * y2) * p;
      // y (1 - y) = y - y^2 in one rounding (the exact value, correctly rounded)
      T *= __builtin_fma(-yj, yj, yj);
    }
    W[u] = w_scale * (T * T * T);
  }
}

// --------------------------------------------------------- FP32 integrand form
// The same fast-path integrand with the transform, polynomials, powers, logarithm and
// orders in FP32 (coefficients from the FP32 copy of the tables); the lattice point
// stays FP64 and every contribution is accumulated in FP64.  Used for sectors whose F
// has no cancellation and a positive constant term (SF_F32OK), where FP32 keeps a
// relative accuracy of a few ulp in every factor.
__device__ __forceinline__ cptr<float> launder_after_f(cptr<float> c, float after) {
  c = (cptr<float>)to_sgpr64((uint64_t)c);
  asm volatile("" : "+s"(c) : "v"(after));
  return c;
}

struct LoadChainF {
  float dep1;
  __device__ __forceinline__ cptr<float> next(cptr<float> c) const { return launder_after_f(c, dep1); }
  __device__ __forceinline__ void done(float v) { dep1 = v; }
};

template <int D, int DEG, int S>
__device__ __forceinline__ void horner_f32(cptr<float> c, const float (&x)[S][D], float (&out)[S],
                                           LoadChainF &ch) {
  c = ch.next(c);
  float acc[S];
#pragma unroll
  for (int u = 0; u < S; ++u) acc[u] = c[0];
  int p = 1;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    c = ch.next(c);
    float g[S];
#pragma unroll
    for (int u = 0; u < S; ++u) g[u] = c[p];
    ++p;
    if (DEG >= 2) {
#pragma unroll
      for (int k = j; k < D; ++k) {
        if (DEG >= 3) c = ch.next(c);
        float h[S];
#pragma unroll
        for (int u = 0; u < S; ++u) h[u] = c[p];
        ++p;
        if (DEG >= 3) {
#pragma unroll
          for (int l = k; l < D; ++l)
#pragma unroll
            for (int u = 0; u < S; ++u) h[u] = __builtin_fmaf(c[p + l - k], x[u][l], h[u]);
          ch.done(h[0]);
        }
        p += D - k;
#pragma unroll
        for (int u = 0; u < S; ++u) g[u] = __builtin_fmaf(x[u][k], h[u], g[u]);
      }
    } else {
      p += (D - j) * (D - j + 3) / 2;
    }
#pragma unroll
    for (int u = 0; u < S; ++u) acc[u] = __builtin_fmaf(x[u][j], g[u], acc[u]);
    ch.done(acc[0]);
  }
#pragma unroll
  for (int u = 0; u < S; ++u) out[u] = acc[u];
}

template <int D, int S>
__device__ __forceinline__ void poly_f32(cptr<float> c, int deg, const float (&x)[S][D],
                                         float (&out)[S], LoadChainF &ch) {
  if (deg >= 3) horner_f32<D, 3, S>(c, x, out, ch);
  else if (deg == 2) horner_f32<D, 2, S>(c, x, out, ch);
  else horner_f32<D, 1, S>(c, x, out, ch);
}

template <int D, int K, int S>
__device__ __forceinline__ void integrand_fast_f32(const SectorScalars &ss, cptr<SectorDev> sd,
                                                   cptr<float> coef, const float (&x)[S][D],
                                                   float (&f)[S][K]) {
  float U[S], F[S];
  LoadChainF ch{x[0][0]};
  poly_f32<D, S>(coef + ss.u_off32, ss.u_deg, x, U, ch);
  poly_f32<D, S>(coef + ss.f_off32, ss.f_deg, x, F, ch);
  float num[S], den[S];
#pragma unroll
  for (int u = 0; u < S; ++u) num[u] = den[u] = 1.0f;
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
  float B[S];
#pragma unroll
  for (int u = 0; u < S; ++u) {
    float r = __builtin_amdgcn_rcpf(den[u]);
    r = __builtin_fmaf(__builtin_fmaf(-den[u], r, 1.0f), r, r);   // one Newton step
    B[u] = num[u] * r;
  }
  cptr<SectorDev> sl = launder_after(sd, (double)B[0]);
  if (K > 1) {
    float L[S];
#pragma unroll
    for (int u = 0; u < S; ++u) L[u] = __builtin_amdgcn_logf(F[u]) * 0.693147180559945309f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float v[S];
#pragma unroll
      for (int u = 0; u < S; ++u) v[u] = sl->logc32[k][K - 1];
#pragma unroll
      for (int m = K - 2; m >= 0; --m) {
        const float cm = sl->logc32[k][m];
#pragma unroll
        for (int u = 0; u < S; ++u) v[u] = __builtin_fmaf(v[u], L[u], cm);
      }
#pragma unroll
      for (int u = 0; u < S; ++u) f[u][k] = B[u] * v[u];
    }
  } else {
#pragma unroll
    for (int u = 0; u < S; ++u) f[u][0] = B[u] * sl->logc32[0][0];
  }
}

template <int D, int S>
__device__ __forceinline__ void korobov3_f32(float w_scale, const float (&y)[S][D],
                                             float (&x)[S][D], float (&W)[S]) {
#pragma unroll
  for (int u = 0; u < S; ++u) {
    float T = 1.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const float yj = y[u][j];
      const float p =
          __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(-20.0f, yj, 70.0f), yj, -84.0f), yj, 35.0f);
      const float y2 = yj * yj;
      x[u][j] = (y2 * y2) * p;
      T *= __builtin_fmaf(-yj, yj, yj);
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

// The work of one workgroup of an integration launch: workgroup b of the launch's
// global numbering holds sector s, shifts [l_begin, l_begin + tile) and one chunk of its
// lattice points (workgroups are numbered sector by sector in workgroup order, each
// sector's shift tiles one after another).
struct BlockWork {
  int64_t b, chunk_id;
  int s, l_begin, tile;
  uint64_t t0;   // start on the constant clock (cost accounting)
};

// Cost accounting for the adaptive loop (the cost per evaluation of each sector is
// measured while the evaluation runs, Sec. 2.1.3): with a.sector_ticks set, thread 0 of
// a workgroup adds the workgroup's duration on the constant 100 MHz clock to its
// sector's counter once the workgroup's partial is stored.
__device__ __forceinline__ uint64_t ticks_now() { return __builtin_amdgcn_s_memrealtime(); }
__device__ __forceinline__ void ticks_add(const LaunchArgs &a, int s, uint64_t t0) {
  if (a.sector_ticks && threadIdx.x == 0)
    atomicAdd(a.sector_ticks + s, (unsigned long long)(ticks_now() - t0));
}

__device__ __forceinline__ BlockWork block_work(const LaunchArgs &a, int64_t block_base) {
  BlockWork w;
  w.t0 = ticks_now();
  w.b = block_base + blockIdx.x;
  w.s = a.order[find_sector(a.block_begin, a.n_sectors, w.b)];
  const LatticeDev *__restrict__ lt = a.lat + w.s;
  const int64_t local = w.b - lt->block_begin;
  const int nch = lt->n_chunks;
  const int tile_id = (int)(local / nch);
  w.chunk_id = local - (int64_t)tile_id * nch;
  w.tile = a.shift_tile;
  w.l_begin = tile_id * w.tile;
  return w;
}

// In-order combine of the waves' partials (one thread per (shift in tile, order)) into
// the workgroup's partial; call after the workgroup barrier that follows the block.
__device__ __forceinline__ void block_store(const LaunchArgs &a, const BlockWork &w,
                                            double (*red)[kMaxTile * 4][2]) {
  const int nwaves = blockDim.x >> 6;
  const int cols = w.tile * a.K;
  if ((int)threadIdx.x < cols) {
    DD r{red[0][threadIdx.x][0], red[0][threadIdx.x][1]};
    for (int v = 1; v < nwaves; ++v) r = dd_combine(r, DD{red[v][threadIdx.x][0], red[v][threadIdx.x][1]});
    double *out = a.partial + (w.b * cols + threadIdx.x) * 2;
    out[0] = r.s;
    out[1] = r.c;
  }
  ticks_add(a, w.s, w.t0);
}

// Maximum shifts per workgroup and waves per workgroup (LDS staging of the partials).

// Lattice points a thread sums in plain FP64 before folding the partial into its
// compensated (TwoSum) accumulator.
constexpr int kFold = 8;

// One workgroup: sector s, shifts [l_begin, l_begin + tile), lattice points of one
// chunk.  The shifts are processed S at a time: for each point the quotient k/n is
// formed once and reused by the S shifts of the pass, whose S*K accumulators stay in
// registers.  Each accumulator is a plain partial over at most kFold points folded
// into a (sum, compensation) pair.  After each pass the pairs are reduced over the
// wavefront and staged in LDS.
// REGCONST: hold the korobov_3 coefficients in registers for the whole block (fewer
// instructions per point; the persistent kernel, tighter on registers, uses literals).
//
// GEN: a plan-specialised integrand (generated straight-line code, compiled at run time,
// its coefficients as literals: one sector's, or a switch among several on the sector
// index s) with static members f64<S>(x, f, C, log_table, s) and f32<S>(x, f, C, s) that
// give the orders f_k of S transformed samples of sector s (C, the coefficient table +
// gen_off, is passed for generators that read it) and `korobov3` (else the transform
// runs through apply_transform; FP32 sectors are korobov_3); NoGen selects the
// table-driven forms.
struct NoGen {};
template <class T>
struct IsGen {
  static constexpr bool value = true;
};
template <>
struct IsGen<NoGen> {
  static constexpr bool value = false;
};
// A generated integrand with finite = true is finite on the whole closed cube (F, and U
// where it divides, positive there), so a sample of weight 0 contributes 0 without a
// test and lanes past the chunk only need weight 0.
template <class T>
struct GenFinite {
  static constexpr bool value = T::finite;
};
template <>
struct GenFinite<NoGen> {
  static constexpr bool value = false;
};

template <int D, int K, int S, bool FAST, bool F32, bool REGCONST = true, class GEN = NoGen>
__device__ __forceinline__ void integrate_block(const LaunchArgs &a, int s, int l_begin, int tile,
                                                int64_t chunk_id, double (*red)[kMaxTile * 4][2],
                                                int64_t gen_off = 0) {
  const SectorDev *__restrict__ sd = a.sectors + s;
  const LatticeDev *__restrict__ lt = a.lat + s;
  const uint64_t n = lt->n;
  const int64_t chunk = lt->chunk;
  const uint64_t i_begin = (uint64_t)(chunk_id * chunk);
  uint64_t i_end = i_begin + (uint64_t)chunk;
  if (i_end > n) i_end = n;
  const int kind = sd->transform;
  const uint64_t B = blockDim.x;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // every lane runs the same number of iterations; lanes past i_end contribute 0
  const int64_t n_iter = (int64_t)((i_end - i_begin + B - 1) / B);

  // the logarithm table of the generated FP64 integrands, in LDS for the workgroup
  __shared__ LogTable log_table;
  if constexpr (IsGen<GEN>::value && !F32) {
    fill_log_table(log_table);
    __syncthreads();
  }
  KorobovConsts kc{35.0, -84.0, 70.0, -20.0};
  if constexpr (REGCONST) kc = korobov3_consts();
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
    // shifts of this pass inside the tile: S, or fewer on the last pass of a tile that is
    // not a multiple of S; the surplus slots re-read the pass's first shift (in bounds)
    // and their sums are dropped
    const int live = (tile - l0 < S) ? tile - l0 : S;
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
        const cptr<float> cl32 = launder_uniform(a.coef32);
        const cptr<LatticeDev> ltl = launder_uniform(lt);
        const cptr<double> shl = launder_uniform(sh);
        // per-sector scalars re-read each iteration (scalar loads) rather than kept live
        // across it, where they would be spilled and restored with vector instructions
        const cptr<SectorDev> sdl = launder_uniform(sd);
        const SectorScalars ss = load_scalars(sdl);
        const double n_d = ltl->n_d, inv_n = ltl->inv_n, w_scale = sdl->w_scale;
        double q[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          q[j] = quotient(k[j], n_d, inv_n);
          k[j] = lattice_step(k[j], ltl->ndz[j], n_d);
          // step now, while the table value is in a register: sunk to the end of the
          // iteration, the loaded values would be spilled across the integrand
          asm volatile("" : "+v"(k[j]));
        }
        double y[S][D], x[S][D], W[S];
#pragma unroll
        for (int u = 0; u < S; ++u)
#pragma unroll
          for (int j = 0; j < D; ++j)
            y[u][j] = shifted(q[j], shl[(u < live ? u : 0) * QMC_MAX_DIM + j]);
        double f[S][K];
        const bool valid = i < i_end;
        if constexpr (IsGen<GEN>::value) {
          if constexpr (F32) {
            float yf[S][D], xf[S][D], Wf[S], ff[S][K];
#pragma unroll
            for (int u = 0; u < S; ++u)
#pragma unroll
              for (int j = 0; j < D; ++j) yf[u][j] = (float)y[u][j];
            korobov3_f32<D, S>((float)w_scale, yf, xf, Wf);
            GEN::template f32<S>(xf, ff, launder_after_f(cl32 + gen_off, Wf[0]), s);
#pragma unroll
            for (int u = 0; u < S; ++u) {
              if constexpr (GenFinite<GEN>::value) Wf[u] = valid ? Wf[u] : 0.0f;
              W[u] = (double)Wf[u];
#pragma unroll
              for (int kk = 0; kk < K; ++kk) f[u][kk] = (double)(Wf[u] * ff[u][kk]);
            }
          } else {
            if constexpr (GEN::korobov3) {
              korobov3_fast<D, S>(w_scale, kc, y, x, W);
            } else {
#pragma unroll
              for (int u = 0; u < S; ++u) W[u] = apply_transform<D>(kind, w_scale, y[u], x[u]);
            }
            GEN::template f64<S>(x, f, launder_after(cl + gen_off, W[0]), log_table, s);
          }
        } else if (F32) {
          float yf[S][D], xf[S][D], Wf[S], ff[S][K];
#pragma unroll
          for (int u = 0; u < S; ++u)
#pragma unroll
            for (int j = 0; j < D; ++j) yf[u][j] = (float)y[u][j];
          korobov3_f32<D, S>((float)w_scale, yf, xf, Wf);
          integrand_fast_f32<D, K, S>(ss, (cptr<SectorDev>)sd, launder_after_f(cl32, Wf[0]), xf, ff);
#pragma unroll
          for (int u = 0; u < S; ++u) {
            W[u] = (double)Wf[u];
#pragma unroll
            for (int kk = 0; kk < K; ++kk) f[u][kk] = (double)(Wf[u] * ff[u][kk]);
          }
        } else if (FAST) {
          korobov3_fast<D, S>(w_scale, kc, y, x, W);
          integrand_fast<D, K, S>(ss, (cptr<SectorDev>)sd, launder_after(cl, W[0]), x, f);
        } else {
#pragma unroll
          for (int u = 0; u < S; ++u) W[u] = apply_transform<D>(kind, w_scale, y[u], x[u]);
          integrand<D, K, S>(ss, (cptr<SectorDev>)sd, launder_after(cl, W[0]), x, f);
        }
        if constexpr (GenFinite<GEN>::value) {
#pragma unroll
          for (int u = 0; u < S; ++u) {
            if constexpr (F32) {   // the weight (0 past the chunk) is in f already
#pragma unroll
              for (int kk = 0; kk < K; ++kk) part[u][kk] += f[u][kk];
            } else {
              const double w = valid ? W[u] : 0.0;
#pragma unroll
              for (int kk = 0; kk < K; ++kk) part[u][kk] = __builtin_fma(w, f[u][kk], part[u][kk]);
            }
          }
        } else {
#pragma unroll
          for (int u = 0; u < S; ++u) {
            const bool use = valid && (W[u] != 0.0);
#pragma unroll
            for (int kk = 0; kk < K; ++kk)
              part[u][kk] += use ? (F32 ? f[u][kk] : W[u] * f[u][kk]) : 0.0;
          }
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
        if (lane == 0 && u < live) {
          red[wave][(l0 + u) * K + kk][0] = r.s;
          red[wave][(l0 + u) * K + kk][1] = r.c;
        }
      }
  }
}

}  // namespace qmc
