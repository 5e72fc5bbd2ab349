// qmc_api.cpp -- host planner and C ABI of the lattice QMC library (see include/qmcamp.h).
//
// The planner does, once per problem, the per-integrand work that does not depend
// on the lattice point (the hoisting of Sec. 2.1 of arXiv:2305.19768): it validates
// the sectors, converts the monomial lists of U and F into dense nested-Horner
// tables (degree <= 3), splits every exponent into integer / half-integer parts and
// numerator / denominator factors, and derives the random shifts.  Per call it
// builds the lattice table (n, z = (1, a, a^2, ...) mod n, RN(1/n), workgroup
// ranges) and launches the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qmc_plan.h"

using namespace qmc;

namespace qmc {

thread_local std::string g_last_error;

qmc_status fail(qmc_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

qmc_status hip_fail(int e, const char *what) {
  return fail(QMC_E_DEVICE, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t n) {
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) % (unsigned __int128)n);
}

uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// SplitMix64 (Steele, Lea, Flood 2014), counter-based: output number `counter` (0-based)
// of the generator started from state `seed`.
uint64_t splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t x = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace qmc

static void layout(qmc_plan_s *p) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  // the partial buffer holds any tunable launch shape: at most target + S (m / tile) + 64
  // workgroups (one rounding workgroup per sector and tile), tile * KC pairs each
  const int tiles = (p->m + p->tile - 1) / p->tile;
  p->max_blocks = kTargetBlocks + (int64_t)p->S * tiles + 64;
  p->partial_doubles = 2 * (size_t)p->KC *
                       ((size_t)kTargetBlocksMax * kMaxTile + (size_t)p->S * p->m + 64 * kMaxTile);
  p->off_sec = take(sizeof(SectorDev) * p->S);
  p->off_coef = take(sizeof(double) * p->coef.size());
  p->off_coef32 = take(sizeof(float) * p->coef.size());
  {  // batched amplitude evaluation: state and tables, bounded by kAmpMaxSums sums and
     // kAmpMaxLattice table entries
    const size_t S = p->S, NI = p->n_integrals, K = p->K;
    p->amp_bytes = align256(sizeof(AmpState)) + 6 * align256(4 * S) + align256(4 * (NI + 1)) +
                   4 * align256(8 * S) + align256(8 * S * QMC_AMP_TAU_ROWS) +
                   3 * align256(8 * kAmpMaxSums * NI * K) + 2 * align256(8 * NI * K) +
                   4 * align256(8 * kAmpMaxSums * K) + align256(4 * kAmpMaxSums * K) +
                   align256(8 * kAmpMaxLattice) + align256(8 * kAmpMaxLattice * QMC_MAX_DIM);
    p->off_amp = take(p->amp_bytes);
  }
  p->off_shift = take(sizeof(double) * p->shifts.size());
  p->off_lat = take(sizeof(LatticeDev) * p->S);
  p->off_begin = take(sizeof(int64_t) * (p->S + 1));
  p->off_order = take(sizeof(int32_t) * p->S);
  p->off_q = take(sizeof(double) * (size_t)p->S * p->m * p->KC);
  p->off_mean = take(sizeof(double) * (size_t)p->S * p->KC);
  p->off_err = take(sizeof(double) * (size_t)p->S * p->KC);
  p->off_status = take(256);
  p->off_sign = take(sizeof(unsigned long long) * (size_t)p->S);
  p->off_ticks = take(sizeof(unsigned long long) * (size_t)p->S);
  // FP32 calibration: Q of both forms [2][S][m][KC], their means and errors [2][S][KC],
  // and the resulting bound [S][KC]
  p->off_cal = take(sizeof(double) * (2 * (size_t)p->S * p->m * p->KC + 2 * (size_t)p->S * p->KC));
  p->off_bound = take(sizeof(double) * (size_t)p->S * p->KC);
  p->off_partial = take(sizeof(double) * p->partial_doubles);
  p->off_p2cand = take(sizeof(uint64_t) * kP2MaxCand);
  p->off_p2part = take(sizeof(double) * kP2PartialDoubles);
  p->off_p2vals = take(sizeof(double) * kP2MaxCand);
  p->total = o;
}

// Position of each monomial in the dense nested-Horner layout (degree <= 3).
static int dense_pos(int D, const uint8_t *e, int *deg_out) {
  int var[3], g = 0;
  for (int j = 0; j < D; ++j)
    for (int t = 0; t < e[j]; ++t) {
      if (g >= 3) return -1;
      var[g++] = j;
    }
  *deg_out = g;
  if (g == 0) return 0;
  int p = 1;
  for (int j = 0; j < D; ++j) {
    if (g == 1 && var[0] == j) return p;
    ++p;
    for (int k = j; k < D; ++k) {
      if (g == 2 && var[0] == j && var[1] == k) return p;
      ++p;
      for (int l = k; l < D; ++l) {
        if (g == 3 && var[0] == j && var[1] == k && var[2] == l) return p;
        ++p;
      }
    }
  }
  return -1;
}

// Complex plans: the gradient of F at x = 0 (dF/dx_a(0), D values; the device forms the
// gradient at x from the Hessian by Euler's theorem) and dense tables of d2F/dx_a dx_b
// for b >= a (degree 1, D(D+1)/2 tables), differentiated monomial by monomial.
static void pack_derivatives(int D, const qmc_problem *prob, int64_t off, int32_t count,
                             std::vector<double> &coef, int32_t *grad_off, int32_t *hess_off) {
  const size_t gbase = coef.size();
  const size_t hbase = gbase + (size_t)D;
  coef.resize(hbase + (size_t)(D * (D + 1) / 2) * dense_len1(D), 0.0);
  *grad_off = (int32_t)gbase;
  *hess_off = (int32_t)hbase;
  for (int32_t r = 0; r < count; ++r) {
    const uint8_t *er = prob->mono_exp + (size_t)(off + r) * QMC_MAX_DIM;
    const double c = prob->mono_coef[off + r];
    int e[QMC_MAX_DIM];
    int deg = 0;
    for (int j = 0; j < D; ++j) {
      e[j] = er[j];
      deg += e[j];
    }
    // first derivatives at x = 0: only the monomials c x_a contribute (c)
    if (deg == 1)
      for (int a = 0; a < D; ++a)
        if (e[a] == 1) coef[gbase + (size_t)a] += c;
    // second derivatives d2/dx_i dx_k, k >= i: c e_i (e_k - [i == k]) x^(e - 1_i - 1_k)
    int t = 0;
    for (int i = 0; i < D; ++i)
      for (int k = i; k < D; ++k, ++t) {
        int eik[QMC_MAX_DIM];
        for (int j = 0; j < D; ++j) eik[j] = e[j];
        const double fi = (double)eik[i];
        eik[i] -= 1;
        const double fk = (double)eik[k];
        eik[k] -= 1;
        if (fi <= 0.0 || fk <= 0.0) continue;
        int var = -1;
        for (int j = 0; j < D; ++j)
          if (eik[j] > 0) var = j;   // remaining degree <= 1
        coef[hbase + (size_t)t * dense_len1(D) + (var < 0 ? 0 : 1 + var)] += c * fi * fk;
      }
  }
}

static qmc_status pack_poly(int D, const qmc_problem *prob, int64_t off, int32_t count,
                            std::vector<double> &coef, int32_t *table_off, int32_t *deg_out,
                            double *abs_sum, int s, const char *name) {
  if (count < 0 || off < 0 || off + count > prob->n_mono_rows)
    return fail(QMC_E_INVAL, "sector %d: %s monomial rows [%lld, %lld) outside [0, %lld)", s, name,
                (long long)off, (long long)(off + count), (long long)prob->n_mono_rows);
  const int len = dense_len(D);
  const size_t base = coef.size();
  coef.resize(base + len, 0.0);
  *table_off = (int32_t)base;
  int deg = 0;
  double a = 0.0;
  for (int32_t t = 0; t < count; ++t) {
    const uint8_t *e = prob->mono_exp + (off + t) * QMC_MAX_DIM;
    const double c = prob->mono_coef[off + t];
    if (!std::isfinite(c)) return fail(QMC_E_INVAL, "sector %d: non-finite %s coefficient", s, name);
    for (int j = D; j < QMC_MAX_DIM; ++j)
      if (e[j] != 0)
        return fail(QMC_E_INVAL, "sector %d: %s monomial uses x_%d beyond d = %d", s, name, j + 1, D);
    int g;
    const int pos = dense_pos(D, e, &g);
    if (pos < 0)
      return fail(QMC_E_INVAL, "sector %d: %s monomial of total degree > %d", s, name, QMC_MAX_DEG);
    coef[base + pos] += c;
    if (c != 0.0) deg = std::max(deg, g);
    a += std::fabs(c);
  }
  *deg_out = std::max(deg, 1);
  if (abs_sum) *abs_sum = a;
  return QMC_OK;
}

// FP32 eligibility of a fast-path sector (integer powers of U and F).  The FP32 form
// evaluates U, F, num = U^u_num F^f_num, den = U^u_den F^f_den, B = num / den and
// log F in FP32, so it needs (1) no cancellation: every coefficient of U and F is
// non-negative, which makes both monotone on the cube, between their constant term
// (at x = 0) and the sum of their coefficients (at x = 1), each evaluated with a
// relative error of a few ulp per monomial; and (2) every one of those quantities,
// and the weighted orders W B (log F)^m, inside FP32's normal range with a wide margin
// (2^-100 .. 2^100; FP32 normals span 2^-126 .. 2^128), so that no intermediate is
// denormal, zero or infinite.  The weight W is at most (140/64)^d and |log F| at most
// max(|log min F|, |log max F|).  Other sectors keep the FP64 integrand.
static bool fp32_range_ok(const SectorDev &sd, const std::vector<double> &coef, int D) {
  double u_lo = coef[sd.u_off], u_hi = 0.0, f_lo = coef[sd.f_off], f_hi = 0.0;
  for (int i = 0; i < dense_len(D); ++i) {
    if (coef[sd.u_off + i] < 0.0 || coef[sd.f_off + i] < 0.0) return false;
    u_hi += coef[sd.u_off + i];
    f_hi += coef[sd.f_off + i];
  }
  if (!(f_lo > 0.0)) return false;                              // F vanishes at x = 0
  if (!(u_lo > 0.0) && (sd.u_num > 0 || sd.u_den > 0)) return false;
  const double lo = -100.0, hi = 100.0;
  auto in = [&](double l2) { return l2 >= lo && l2 <= hi; };
  const double lu_lo = (sd.u_num + sd.u_den) ? std::log2(u_lo) : 0.0, lu_hi = std::log2(u_hi);
  const double lf_lo = std::log2(f_lo), lf_hi = std::log2(f_hi);
  // every partial power of U and F (the FP32 products are built one factor at a time)
  for (int t = 1; t <= std::max(sd.u_num, sd.u_den); ++t)
    if (!in(t * lu_lo) || !in(t * lu_hi)) return false;
  for (int t = 1; t <= std::max(sd.f_num, sd.f_den); ++t)
    if (!in(t * lf_lo) || !in(t * lf_hi)) return false;
  const double num_lo = sd.u_num * lu_lo + sd.f_num * lf_lo, num_hi = sd.u_num * lu_hi + sd.f_num * lf_hi;
  const double den_lo = sd.u_den * lu_lo + sd.f_den * lf_lo, den_hi = sd.u_den * lu_hi + sd.f_den * lf_hi;
  if (!in(num_lo) || !in(num_hi) || !in(den_lo) || !in(den_hi)) return false;
  const double b_lo = num_lo - den_hi, b_hi = num_hi - den_lo;   // log2 of the range of B
  const double w_hi = D * std::log2(140.0 / 64.0);
  const double lmax = std::max(std::fabs(std::log(f_lo)), std::fabs(std::log(f_hi)));
  double v_hi = 0.0;   // largest |sum_m c_km L^m| over the orders
  for (int k = 0; k < sd.n_orders; ++k) {
    double v = 0.0;
    for (int m = 0; m <= QMC_MAX_LOG; ++m) v += std::fabs(sd.logc[k][m]) * std::pow(lmax, m);
    v_hi = std::max(v_hi, v);
  }
  return in(b_lo) && in(b_hi + w_hi + std::log2(std::max(v_hi, 1.0)));
}

// 0: generic path, 1: fast path in FP64, 2: fast path in FP32, 3: deformed (complex plan),
// 4: attached flow transform, 5: deformed with the FP32 polynomial bulk, 6: deformed with
// an attached flow transform.
static int path_class(const qmc_plan_s *p, int s) {
  if (p->cplx)
    return p->sec[s].flow ? 6 : (p->precision == QMC_PREC_FP32 && (p->sec[s].flags & SF_CF32)) ? 5 : 3;
  if (p->sec[s].flow) return 4;
  const int f = p->sec[s].flags;
  if (!(f & SF_FAST)) return 0;
  return (p->precision == QMC_PREC_FP32 && (f & SF_F32OK)) ? 2 : 1;
}

namespace qmc {
// Workgroup order: by dimension, then path class, then sector index.
void plan_reorder(qmc_plan_s *p) {
  p->order.resize(p->S);
  for (int s = 0; s < p->S; ++s) p->order[s] = s;
  std::stable_sort(p->order.begin(), p->order.end(), [&](int32_t x, int32_t y) {
    const int fx = path_class(p, x), fy = path_class(p, y);
    return p->dims[x] != p->dims[y] ? p->dims[x] < p->dims[y] : fx < fy;
  });
}
}  // namespace qmc

static void split_pow2(int32_t e2, int32_t *num, int32_t *den, int32_t *half) {
  const int32_t mag = e2 < 0 ? -e2 : e2;
  *num = e2 > 0 ? mag / 2 : 0;
  *den = e2 < 0 ? mag / 2 : 0;
  *half = (mag & 1) ? (e2 > 0 ? 1 : -1) : 0;
}

extern "C" {

const char *qmc_last_error(void) { return g_last_error.c_str(); }

const char *qmc_version(void) { return "qmcamp 0.1 (gfx950)"; }

qmc_status qmc_plan(const qmc_problem *prob, const qmc_options *opt, qmc_plan_t *out) {
  g_last_error.clear();
  if (!prob || !opt || !out) return fail(QMC_E_INVAL, "NULL argument");
  *out = nullptr;
  if (prob->n_sectors < 1 || !prob->sectors)
    return fail(QMC_E_INVAL, "n_sectors must be >= 1 with a sector array");
  if (prob->n_orders < 1 || prob->n_orders > QMC_MAX_ORDERS)
    return fail(QMC_E_INVAL, "n_orders must be in [1, %d]", QMC_MAX_ORDERS);
  if (prob->max_log < 0 || prob->max_log > QMC_MAX_LOG)
    return fail(QMC_E_INVAL, "max_log must be in [0, %d]", QMC_MAX_LOG);
  if (prob->n_integrals < 1) return fail(QMC_E_INVAL, "n_integrals must be >= 1");
  if (prob->n_mono_rows < 0 || (prob->n_mono_rows > 0 && (!prob->mono_exp || !prob->mono_coef)))
    return fail(QMC_E_INVAL, "monomial arrays missing");
  if (opt->m < 2 || opt->m > QMC_MAX_SHIFTS)
    return fail(QMC_E_INVAL, "m must be in [2, %d]", QMC_MAX_SHIFTS);
  if (opt->precision != QMC_PREC_FP64 && opt->precision != QMC_PREC_FP32)
    return fail(QMC_E_INVAL, "unknown precision %d", opt->precision);
  // complex plan: some sector integrated on a deformed contour
  int cplx = 0;
  for (int s = 0; s < prob->n_sectors; ++s) {
    const double lam = prob->sectors[s].deform_lambda;
    if (!(lam >= 0.0) || !std::isfinite(lam))
      return fail(QMC_E_INVAL, "sector %d: deform_lambda must be finite and >= 0", s);
    if (lam > 0.0) cplx = 1;
  }
  const int KC = cplx ? 2 * prob->n_orders : prob->n_orders;
  const int block = opt->block ? opt->block : 256;
  int tile = opt->shift_tile;
  if (!tile)  // largest power of two <= 16 dividing m (and fitting 64 columns per workgroup)
    for (tile = 16; tile > 1 && (opt->m % tile != 0 || tile * KC > 64); tile >>= 1) {
    }
  const int spp = cplx ? 1
                       : (opt->shifts_per_pass ? opt->shifts_per_pass : (tile % 2 == 0 ? 2 : 1));
  if (cplx && opt->shifts_per_pass > 1)
    return fail(QMC_E_INVAL, "unsupported launch shape: deformed sectors run one shift per pass");
  if (!tile_supported(tile, spp, block) || tile * KC > 64)
    return fail(QMC_E_INVAL, "unsupported launch shape: shift_tile %d, shifts_per_pass %d, block %d",
                tile, spp, block);
  if (opt->m % tile != 0)
    return fail(QMC_E_INVAL, "m = %d is not a multiple of shift_tile = %d", opt->m, tile);

  qmc_plan_s *p = new (std::nothrow) qmc_plan_s();
  if (!p) return fail(QMC_E_NOMEM, "out of host memory");
  p->S = prob->n_sectors;
  p->K = prob->n_orders;
  p->cplx = cplx;
  p->KC = KC;
  p->M = prob->max_log;
  p->n_integrals = prob->n_integrals;
  p->m = opt->m;
  p->precision = opt->precision;
  p->block = block;
  p->tile = tile;
  p->spp = spp;
  p->sec.resize(p->S);
  p->n_default.resize(p->S);
  p->a_default.resize(p->S);
  p->dims.resize(p->S);
  uint64_t nmax = 0;
  for (int s = 0; s < p->S; ++s) {
    const qmc_sector_desc &in = prob->sectors[s];
    SectorDev &sd = p->sec[s];
    std::memset(&sd, 0, sizeof sd);
    const int D = in.d;
    if (D < 1 || D > QMC_MAX_DIM) {
      delete p;
      return fail(QMC_E_INVAL, "sector %d: d = %d outside [1, %d]", s, D, QMC_MAX_DIM);
    }
    if (in.integral < 0 || in.integral >= prob->n_integrals) {
      delete p;
      return fail(QMC_E_INVAL, "sector %d: integral %d outside [0, %d)", s, in.integral,
                  prob->n_integrals);
    }
    if (in.transform < QMC_TRANSFORM_NONE || in.transform > QMC_TRANSFORM_KOROBOV6) {
      delete p;
      return fail(QMC_E_INVAL, "sector %d: unknown transform %d", s, in.transform);
    }
    if (in.n_f < 1) {
      delete p;
      return fail(QMC_E_INVAL, "sector %d: F needs at least one monomial", s);
    }
    if (in.u_pow < -8 || in.u_pow > 8 || in.f_pow2 < -16 || in.f_pow2 > 16) {
      delete p;
      return fail(QMC_E_INVAL, "sector %d: exponent of U or F out of range", s);
    }
    sd.d = D;
    sd.transform = in.transform;
    sd.w_scale = std::pow(140.0, D);   // exact: 140^8 < 2^53 * 2^16
    sd.integral = in.integral;
    sd.n_orders = p->K;
    sd.max_log = p->M;
    p->dims[s] = D;
    p->d_max = std::max(p->d_max, D);
    qmc_status st;
    if (in.n_u == 0) {
      // U absent: constant 1
      const size_t base = p->coef.size();
      p->coef.resize(base + dense_len(D), 0.0);
      p->coef[base] = 1.0;
      sd.u_off = (int32_t)base;
      sd.u_deg = 1;
    } else if ((st = pack_poly(D, prob, in.u_off, in.n_u, p->coef, &sd.u_off, &sd.u_deg, nullptr,
                               s, "U")) != QMC_OK) {
      delete p;
      return st;
    }
    if ((st = pack_poly(D, prob, in.f_off, in.n_f, p->coef, &sd.f_off, &sd.f_deg, &sd.f_abs, s,
                        "F")) != QMC_OK) {
      delete p;
      return st;
    }
    if (cplx) {
      pack_derivatives(D, prob, in.f_off, in.n_f, p->coef, &sd.grad_off, &sd.hess_off);
      sd.lambda = in.deform_lambda;
    }
    int flags = 0;
    for (int j = 0; j < QMC_MAX_DIM; ++j) {
      const int32_t e2 = j < D ? in.x_pow2[j] : 0;
      if (j >= D && in.x_pow2[j] != 0) {
        delete p;
        return fail(QMC_E_INVAL, "sector %d: x_pow2[%d] set beyond d", s, j);
      }
      if (e2 < -16 || e2 > 16) {
        delete p;
        return fail(QMC_E_INVAL, "sector %d: x_pow2[%d] = %d out of range", s, j, e2);
      }
      split_pow2(e2, &sd.x_num[j], &sd.x_den[j], &sd.x_half[j]);
      if (e2 != 0) flags |= SF_XPOW;
      if (sd.x_half[j] != 0) flags |= SF_HALF;
      if (sd.x_den[j] != 0 || sd.x_half[j] < 0) flags |= SF_DEN;
    }
    sd.u_num = in.u_pow > 0 ? in.u_pow : 0;
    sd.u_den = in.u_pow < 0 ? -in.u_pow : 0;
    int32_t fh;
    split_pow2(in.f_pow2, &sd.f_num, &sd.f_den, &fh);
    sd.f_half = fh;
    if (fh != 0) flags |= SF_HALF;
    if (sd.u_den || sd.f_den || fh < 0) flags |= SF_DEN;
    if (p->M > 0) flags |= SF_LOG;
    if (in.transform == QMC_TRANSFORM_KOROBOV3 && !(flags & (SF_XPOW | SF_HALF)) &&
        p->M <= p->K - 1)
      flags |= SF_FAST;

    // FP32 bulk on the deformed contour: where the contour moves off the real cube F(z)
    // keeps a non-zero imaginary part inside it; on the real contour only without
    // cancellation (as for SF_F32OK)
    // the log coefficients first: the FP32 range test below reads them
    for (int k = 0; k < QMC_MAX_ORDERS; ++k)
      for (int mm = 0; mm <= QMC_MAX_LOG; ++mm) {
        const double c = (k < p->K && mm <= p->M) ? in.logc[k][mm] : 0.0;
        if (!std::isfinite(c)) {
          delete p;
          return fail(QMC_E_INVAL, "sector %d: non-finite logc[%d][%d]", s, k, mm);
        }
        sd.logc[k][mm] = c;
        sd.logc32[k][mm] = (float)c;
      }
    // FP32 eligibility: no cancellation in U or F on the cube, every FP32 intermediate
    // inside the normal range
    if ((flags & SF_FAST) && fp32_range_ok(sd, p->coef, D)) flags |= SF_F32OK;
    if (p->cplx && p->precision == QMC_PREC_FP32) {
      // real-contour sectors under the same rule as SF_F32OK (the deformed ones keep a
      // non-zero imaginary part of F(z) inside the cube)
      bool ok = in.deform_lambda > 0.0;
      if (!ok) ok = fp32_range_ok(sd, p->coef, D);
      if (ok) flags |= SF_CF32;
    }
    sd.flags = flags;
    sd.u_off32 = sd.u_off;
    sd.f_off32 = sd.f_off;
    p->n_default[s] = in.n;
    p->a_default[s] = in.a;
    nmax = std::max<uint64_t>(nmax, in.n);
  }
  p->n_max = opt->n_max ? opt->n_max : nmax;
  if (p->n_max < 2 || p->n_max >= (1ull << 53)) {
    const unsigned long long bad = (unsigned long long)p->n_max;
    delete p;
    return fail(QMC_E_INVAL, "n_max = %llu outside [2, 2^53)", bad);
  }
  // built-in shifts
  p->shifts.assign((size_t)p->S * p->m * QMC_MAX_DIM, 0.0);
  for (int s = 0; s < p->S; ++s)
    for (int l = 0; l < p->m; ++l)
      for (int j = 0; j < QMC_MAX_DIM; ++j) {
        const uint64_t c = ((uint64_t)s << 32) | ((uint64_t)l << 8) | (uint64_t)j;
        p->shifts[((size_t)s * p->m + l) * QMC_MAX_DIM + j] =
            (double)(splitmix64(opt->seed, c) >> 11) * 0x1.0p-53;
      }
  p->coef32.assign(p->coef.begin(), p->coef.end());
  plan_reorder(p);
  layout(p);
  p->lat.resize(p->S);
  p->begin.resize(p->S + 1);
  *out = p;
  return QMC_OK;
}

size_t qmc_workspace_bytes(qmc_plan_t p) { return p ? p->total : 0; }

qmc_status qmc_bind_workspace(qmc_plan_t p, void *dev, size_t bytes, void *stream) {
  g_last_error.clear();
  if (!p || !dev) return fail(QMC_E_INVAL, "NULL plan or workspace");
  if (((uintptr_t)dev & 255) != 0) return fail(QMC_E_INVAL, "workspace not 256-byte aligned");
  if (bytes < p->total)
    return fail(QMC_E_NOMEM, "workspace of %zu bytes, %zu needed", bytes, p->total);
  p->ws = (char *)dev;
  p->ws_bytes = bytes;
  p->lat_valid = false;
  hipStream_t st = (hipStream_t)stream;
  int e;
  if (!p->side.fork) {
    hipEvent_t f;
    if ((e = hipEventCreateWithFlags(&f, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "create fork event");
    p->side.fork = f;
    for (int i = 0; i < kSideStreams; ++i) {
      hipStream_t s;
      hipEvent_t j;
      if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "create side stream");
      if ((e = hipEventCreateWithFlags(&j, hipEventDisableTiming)) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(e, "create join event");
      }
      p->side.stream[i] = s;
      p->side.join[i] = j;
      p->side.n = i + 1;
    }
  }
  if ((e = hipMemcpyAsync(p->ws + p->off_sec, p->sec.data(), sizeof(SectorDev) * p->S,
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload sectors");
  if (!p->coef.empty() &&
      (e = hipMemcpyAsync(p->ws + p->off_coef, p->coef.data(), sizeof(double) * p->coef.size(),
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload coefficients");
  if (!p->coef32.empty() &&
      (e = hipMemcpyAsync(p->ws + p->off_coef32, p->coef32.data(), sizeof(float) * p->coef32.size(),
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload FP32 coefficients");
  if ((e = hipMemcpyAsync(p->ws + p->off_shift, p->shifts.data(),
                          sizeof(double) * p->shifts.size(), hipMemcpyHostToDevice, st)) !=
      hipSuccess)
    return hip_fail(e, "upload shifts");
  if ((e = hipMemcpyAsync(p->ws + p->off_order, p->order.data(), sizeof(int32_t) * p->S,
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload sector order");
  if ((e = launch_status_reset((int32_t *)(p->ws + p->off_status), stream)) != hipSuccess)
    return hip_fail(e, "status reset");
  return QMC_OK;
}

qmc_status qmc_set_shifts(qmc_plan_t p, const double *shifts, void *stream) {
  g_last_error.clear();
  if (!p || !shifts) return fail(QMC_E_INVAL, "NULL argument");
  for (int s = 0; s < p->S; ++s)
    for (int l = 0; l < p->m; ++l)
      for (int j = 0; j < p->dims[s]; ++j) {
        const double v = shifts[((size_t)s * p->m + l) * QMC_MAX_DIM + j];
        if (!(v >= 0.0 && v < 1.0))
          return fail(QMC_E_INVAL, "shift[%d][%d][%d] = %g outside [0, 1)", s, l, j, v);
      }
  for (int s = 0; s < p->S; ++s)
    for (int l = 0; l < p->m; ++l)
      for (int j = 0; j < QMC_MAX_DIM; ++j) {
        const size_t at = ((size_t)s * p->m + l) * QMC_MAX_DIM + j;
        p->shifts[at] = j < p->dims[s] ? shifts[at] : 0.0;
      }
  p->cal_valid = false;
  if (!p->ws) return QMC_OK;   // kept on the host (uploaded at bind, or by qmc_integrate_static)
  int e = hipMemcpyAsync(p->ws + p->off_shift, p->shifts.data(), sizeof(double) * p->shifts.size(),
                         hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "upload shifts");
  return QMC_OK;
}

}  // extern "C"

namespace qmc {

// Calibration lattice of the FP32 rounding bound: n = 1021 (prime) with the Korobov
// parameter of least P_2 per dimension (exhaustive over a in [1, n/2], smallest a on
// ties), computed once per process on the host.
constexpr uint64_t kCalN = 1021;

static uint64_t cal_korobov(int d) {
  static std::mutex mu;
  static uint64_t cache[QMC_MAX_DIM + 1] = {};
  std::lock_guard<std::mutex> lk(mu);
  if (cache[d]) return cache[d];
  const double two_pi2 = 2.0 * M_PI * M_PI;
  double best = INFINITY;
  uint64_t best_a = 1;
  for (uint64_t a = 1; a <= kCalN / 2; ++a) {
    uint64_t z[QMC_MAX_DIM];
    z[0] = 1;
    for (int j = 1; j < d; ++j) z[j] = z[j - 1] * a % kCalN;
    double sum = 0.0;
    for (uint64_t k = 0; k < kCalN; ++k) {
      double prod = 1.0;
      for (int j = 0; j < d; ++j) {
        const double x = (double)(k * z[j] % kCalN) / (double)kCalN;
        prod *= 1.0 + two_pi2 * (x * x - x + 1.0 / 6.0);
      }
      sum += prod;
    }
    const double p2 = sum / (double)kCalN - 1.0;
    if (p2 < best * (1.0 - 1e-12)) {
      best = p2;
      best_a = a;
    }
  }
  cache[d] = best_a;
  return best_a;
}

qmc_status fp32_calibrate(qmc_plan_s *p, void *stream, char *static_base, size_t static_cap) {
  if (p->precision != QMC_PREC_FP32) return QMC_OK;
  const size_t S = p->S, KC = p->KC, m = p->m;
  p->f32_bound.assign(S * KC, 0.0);
  p->cal_mean.assign(S * KC, 0.0);
  bool any = false;   // a sector with an FP32 form (real: the fast path; complex: FP32 bulk)
  for (size_t s = 0; s < S; ++s)
    any = any || (!p->sec[s].flow && (p->cplx ? (p->sec[s].flags & SF_CF32) != 0
                                              : (p->sec[s].flags & SF_FAST) && (p->sec[s].flags & SF_F32OK)));
  if (!any) {
    p->cal_valid = true;
    return QMC_OK;
  }
  // the two forms' Q, means and errors
  const size_t qn = S * m * KC, need = sizeof(double) * (2 * qn + 2 * S * KC);
  char *cal;
  size_t cap = static_cap;
  if (static_base) {
    if (align256(need) > static_cap) return fail(QMC_E_NOMEM, "static scratch too small for the FP32 calibration");
    cap = static_cap - align256(need);
    cal = static_base + cap;
  } else {
    cal = p->ws + p->off_cal;
  }
  double *q64 = (double *)cal, *q32 = q64 + qn, *mean = q32 + qn, *err = mean + S * KC;
  const uint64_t n_c = std::min<uint64_t>(kCalN, p->n_max);
  std::vector<uint64_t> n(S, n_c), a(S);
  for (size_t s = 0; s < S; ++s) a[s] = n_c == kCalN ? cal_korobov(p->dims[s]) : 1;
  const int prec = p->precision;
  const bool timing = p->timing;
  p->bound_off = true;
  p->timing = false;
  p->precision = QMC_PREC_FP64;
  qmc_status r = integrate_sectors(p, n.data(), a.data(), nullptr, stream, q64, mean, err, nullptr,
                                   static_base, cap);
  p->precision = prec;
  if (r == QMC_OK)
    r = integrate_sectors(p, n.data(), a.data(), nullptr, stream, q32, mean, err, nullptr,
                          static_base, cap);
  p->bound_off = false;
  p->timing = timing;
  if (r != QMC_OK) return r;
  std::vector<double> h64(qn), h32(qn);
  hipStream_t st = (hipStream_t)stream;
  int e;
  if ((e = hipMemcpyAsync(h64.data(), q64, sizeof(double) * qn, hipMemcpyDeviceToHost, st)) ||
      (e = hipMemcpyAsync(h32.data(), q32, sizeof(double) * qn, hipMemcpyDeviceToHost, st)) ||
      (e = hipStreamSynchronize(st)))
    return hip_fail(e, "read the FP32 calibration");
  // per (sector, column): the shift differences D_l = Q32_l - Q64_l on the same points
  // estimate the FP32 form's error; bound = |mean D| + 3 x its standard error
  for (size_t s = 0; s < S; ++s)
    for (size_t k = 0; k < KC; ++k) {
      double md = 0.0, m64 = 0.0;
      for (size_t l = 0; l < m; ++l) {
        const size_t at = (s * m + l) * KC + k;
        md += h32[at] - h64[at];
        m64 += h64[at];
      }
      md /= (double)m;
      double ss = 0.0;
      for (size_t l = 0; l < m; ++l) {
        const size_t at = (s * m + l) * KC + k;
        const double dl = h32[at] - h64[at] - md;
        ss += dl * dl;
      }
      const double se = m > 1 ? std::sqrt(ss / ((double)(m - 1) * (double)m)) : std::fabs(md);
      p->f32_bound[s * KC + k] = std::fabs(md) + 3.0 * se;
      p->cal_mean[s * KC + k] = m64 / (double)m;
    }
  p->cal_valid = true;
  p->bound_in_ws = false;   // uploaded by the next integration on the workspace
  return QMC_OK;
}

qmc_status integrate_sectors(qmc_plan_s *p, const uint64_t *n_in, const uint64_t *a_in,
                             const uint8_t *active, void *stream, double *dev_q, double *dev_mean,
                             double *dev_err, const uint64_t *zvec, char *static_base,
                             size_t static_cap) {
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (!dev_mean || !dev_err) return fail(QMC_E_INVAL, "dev_mean and dev_err are required");
  const bool in_static = static_base != nullptr;
  if (!in_static && !p->ws) return fail(QMC_E_STATE, "no workspace bound");
  const bool with_bound = p->precision == QMC_PREC_FP32 && !p->bound_off;
  if (with_bound && !p->cal_valid) {
    qmc_status r = fp32_calibrate(p, stream, static_base, static_cap);
    if (r != QMC_OK) return r;
  }
  const int tiles = p->m / p->tile;
  // lattice table
  __int128 total = 0;
  for (int s = 0; s < p->S; ++s) {
    LatticeDev &L = p->lat[s];
    if (active && !active[s]) {   // keeps its previous Q; no workgroups
      std::memset(&L, 0, sizeof L);
      continue;
    }
    const uint64_t n = n_in ? n_in[s] : p->n_default[s];
    if (n < 2 || n > p->n_max || n >= (1ull << 53))
      return fail(QMC_E_INVAL, "sector %d: n = %llu outside [2, n_max = %llu]", s,
                  (unsigned long long)n, (unsigned long long)p->n_max);
    const uint64_t a = (a_in ? a_in[s] : p->a_default[s]) % n;
    std::memset(&L, 0, sizeof L);
    L.active = 1;
    L.n = n;
    L.n_d = (double)n;
    L.inv_n = 1.0 / (double)n;
    uint64_t z = 1 % n;
    for (int j = 0; j < QMC_MAX_DIM; ++j) {
      if (j < p->dims[s]) {
        if (zvec) {   // general generating vector
          z = zvec[(size_t)s * QMC_MAX_DIM + j];
          if (z < 1 || z >= n)
            return fail(QMC_E_INVAL, "sector %d: z_%d = %llu outside [1, n)", s, j + 1,
                        (unsigned long long)z);
        }
        if (gcd_u64(z, n) != 1)
          return fail(QMC_E_INVAL, "sector %d: z_%d = %llu shares a factor with n = %llu", s,
                      j + 1, (unsigned long long)z, (unsigned long long)n);
        L.z[j] = z;
        L.dz[j] = mulmod_host((uint64_t)p->block % n, z, n);
        L.ndz[j] = (double)(n - L.dz[j]);
      }
      if (!zvec) z = mulmod_host(z, a, n);
    }
    total += (__int128)n * tiles;
  }
  // points per thread: enough that the launch has about target_blocks workgroups
  const __int128 per_block = (__int128)p->target_blocks * p->block;
  int64_t ppt = (int64_t)((total + per_block - 1) / per_block);
  if (ppt < 1) ppt = 1;
  const int64_t chunk = ppt * p->block;
  int64_t b = 0;
  DimLaunch dl[4 * QMC_MAX_DIM];
  int n_dl = 0;
  for (int t = 0; t < p->S; ++t) {
    const int s = p->order[t];
    LatticeDev &L = p->lat[s];
    L.chunk = chunk;
    L.n_chunks = L.active ? (int32_t)((L.n + chunk - 1) / chunk) : 0;
    L.block_begin = b;
    p->begin[t] = b;
    const int cls = path_class(p, s);
    const int fast = (cls == 1 || cls == 2) ? 1 : 0, f32 = (cls == 2 || cls == 5) ? 1 : 0;
    const int deform = (cls == 3 || cls == 5 || cls == 6) ? 1 : 0;
    const int flow = (cls == 4 || cls == 6) ? 1 : 0;
    if (n_dl == 0 || dl[n_dl - 1].d != p->dims[s] || dl[n_dl - 1].fast != fast ||
        dl[n_dl - 1].f32 != f32 || dl[n_dl - 1].deform != deform || dl[n_dl - 1].flow != flow) {
      if (n_dl == 4 * QMC_MAX_DIM) return fail(QMC_E_STATE, "too many launch classes");
      dl[n_dl].d = p->dims[s];
      dl[n_dl].base = b;
      dl[n_dl].blocks = 0;
      dl[n_dl].fast = fast;
      dl[n_dl].f32 = f32;
      dl[n_dl].deform = deform;
      dl[n_dl].flow = flow;
      dl[n_dl].pad = 0;
      dl[n_dl].gen = (!deform && !flow) ? gen_lookup(p, p->dims[s], f32 != 0) : 0;
      ++n_dl;
    }
    const int64_t nb = (int64_t)L.n_chunks * tiles;
    dl[n_dl - 1].blocks += nb;
    b += nb;
  }
  p->begin[p->S] = b;
  hipStream_t st = (hipStream_t)stream;
  int e;
  // device regions of this call: the plan's workspace, or a layout in the static scratch
  char *r_sec, *r_coef, *r_coef32, *r_shift, *r_lat, *r_begin, *r_order, *r_q, *r_status, *r_sign,
      *r_partial, *r_bound;
  if (in_static) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
      char *at = static_base + o;
      o = align256(o + bytes);
      return at;
    };
    r_sec = take(sizeof(SectorDev) * p->S);
    r_coef = take(sizeof(double) * p->coef.size());
    r_coef32 = take(sizeof(float) * p->coef32.size());
    r_shift = take(sizeof(double) * p->shifts.size());
    r_lat = take(sizeof(LatticeDev) * p->S);
    r_begin = take(sizeof(int64_t) * (p->S + 1));
    r_order = take(sizeof(int32_t) * p->S);
    r_q = dev_q ? nullptr : take(sizeof(double) * (size_t)p->S * p->m * p->KC);
    r_status = take(256);
    r_sign = p->cplx ? take(sizeof(unsigned long long) * (size_t)p->S) : nullptr;
    r_bound = with_bound ? take(sizeof(double) * p->f32_bound.size()) : nullptr;
    r_partial = take(sizeof(double) * 2 * (size_t)b * p->tile * p->KC);
    if (o > static_cap)
      return fail(QMC_E_NOMEM,
                  "the call needs %zu bytes of static scratch (%lld workgroups), the library "
                  "holds %zu; lower the launch target (qmc_set_launch_shape) or the shifts",
                  o, (long long)b, static_cap);
    auto up = [&](char *dst, const void *src, size_t bytes) {
      return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    if ((e = up(r_sec, p->sec.data(), sizeof(SectorDev) * p->S)) ||
        (e = up(r_coef, p->coef.data(), sizeof(double) * p->coef.size())) ||
        (e = up(r_coef32, p->coef32.data(), sizeof(float) * p->coef32.size())) ||
        (e = up(r_shift, p->shifts.data(), sizeof(double) * p->shifts.size())) ||
        (e = up(r_lat, p->lat.data(), sizeof(LatticeDev) * p->S)) ||
        (e = up(r_begin, p->begin.data(), sizeof(int64_t) * (p->S + 1))) ||
        (e = up(r_order, p->order.data(), sizeof(int32_t) * p->S)) ||
        (with_bound && (e = up(r_bound, p->f32_bound.data(), sizeof(double) * p->f32_bound.size()))))
      return hip_fail(e, "upload tables to the static scratch");
    p->static_status = (int32_t *)r_status;
    p->static_sign = (unsigned long long *)r_sign;
  } else {
    if ((size_t)b * p->tile * p->KC * 2 > p->partial_doubles)
      return fail(QMC_E_NOMEM, "launch needs %lld workgroups, workspace holds %lld", (long long)b,
                  (long long)(p->partial_doubles / (2 * (size_t)p->tile * p->KC)));
    r_sec = p->ws + p->off_sec;
    r_coef = p->ws + p->off_coef;
    r_coef32 = p->ws + p->off_coef32;
    r_shift = p->ws + p->off_shift;
    r_lat = p->ws + p->off_lat;
    r_begin = p->ws + p->off_begin;
    r_order = p->ws + p->off_order;
    r_q = p->ws + p->off_q;
    r_status = p->ws + p->off_status;
    r_sign = p->ws + p->off_sign;
    r_partial = p->ws + p->off_partial;
    r_bound = with_bound ? p->ws + p->off_bound : nullptr;
    if (with_bound && !p->bound_in_ws) {
      if ((e = hipMemcpyAsync(r_bound, p->f32_bound.data(), sizeof(double) * p->f32_bound.size(),
                              hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail(e, "upload the FP32 bound");
      p->bound_in_ws = true;
    }
    p->static_status = nullptr;
    p->static_sign = nullptr;
  }
  const bool same = in_static ||
                    (p->lat_valid && p->lat_uploaded.size() == p->lat.size() &&
                     std::memcmp(p->lat_uploaded.data(), p->lat.data(),
                                 sizeof(LatticeDev) * p->lat.size()) == 0);
  if (!same) {
    if ((e = hipMemcpyAsync(p->ws + p->off_lat, p->lat.data(), sizeof(LatticeDev) * p->S,
                            hipMemcpyHostToDevice, st)) != hipSuccess)
      return hip_fail(e, "upload lattice table");
    if ((e = hipMemcpyAsync(p->ws + p->off_begin, p->begin.data(), sizeof(int64_t) * (p->S + 1),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
      return hip_fail(e, "upload workgroup table");
    p->lat_uploaded = p->lat;
    p->lat_valid = true;
  }
  LaunchArgs la;
  std::memset(&la, 0, sizeof la);
  la.sectors = (const SectorDev *)r_sec;
  la.coef = (const double *)r_coef;
  la.coef32 = (const float *)r_coef32;
  la.shifts = (const double *)r_shift;
  la.lat = (const LatticeDev *)r_lat;
  la.block_begin = (const int64_t *)r_begin;
  la.order = (const int32_t *)r_order;
  la.n_dim_launches = n_dl;
  for (int t = 0; t < n_dl; ++t) la.dims[t] = dl[t];
  la.partial = (double *)r_partial;
  la.q = dev_q ? dev_q : (double *)r_q;
  la.mean = dev_mean;
  la.err = dev_err;
  la.status = (int32_t *)r_status;
  la.n_sectors = p->S;
  la.m = p->m;
  la.K = p->KC;
  la.cplx = p->cplx;
  la.sign_count = (unsigned long long *)r_sign;
  la.sector_ticks = (p->ticks_on && !in_static) ? (unsigned long long *)(p->ws + p->off_ticks)
                                                : nullptr;
  la.f32_bound = (const double *)r_bound;
  la.shift_tile = p->tile;
  la.shifts_per_pass = p->spp;
  la.block = p->block;
  la.total_blocks = b;
  la.d_max = p->d_max;
  la.precision = p->precision;
  if (p->timing && !in_static) {
    if (p->ev_used + 2 > p->ev.size()) {
      if (p->ev.size() >= 2 * 4096) return fail(QMC_E_STATE, "timing record full; re-enable timing");
      for (int t = 0; t < 2; ++t) {
        hipEvent_t h;
        if ((e = hipEventCreate(&h)) != hipSuccess) return hip_fail(e, "create timing event");
        p->ev.push_back(h);
      }
    }
    la.ev_start = p->ev[p->ev_used];
    la.ev_stop = p->ev[p->ev_used + 1];
    p->ev_used += 2;
  }
  if ((e = launch_status_reset(la.status, stream)) != hipSuccess) return hip_fail(e, "status reset");
  if (p->cplx && (e = launch_clear_u64(la.sign_count, p->S, stream)) != hipSuccess)
    return hip_fail(e, "sign-check counter reset");
  // the static form runs every class launch on the caller's stream (no side streams)
  if ((e = launch_integrate(la, stream, in_static ? nullptr : &p->side)) != hipSuccess)
    return hip_fail(e, "integrate launch");
  return QMC_OK;
}

}  // namespace qmc

namespace qmc {
qmc_status p2_check_args(uint64_t n, int32_t d, const uint64_t *cand, int32_t n_cand) {
  if (n < 2 || n >= (1ull << 53)) return fail(QMC_E_INVAL, "n = %llu outside [2, 2^53)",
                                              (unsigned long long)n);
  if (d < 1 || d > QMC_MAX_DIM) return fail(QMC_E_INVAL, "d = %d outside [1, %d]", d, QMC_MAX_DIM);
  if (n_cand < 1 || n_cand > kP2MaxCand)
    return fail(QMC_E_INVAL, "n_cand = %d outside [1, %d]", n_cand, kP2MaxCand);
  for (int32_t c = 0; c < n_cand; ++c)
    if (cand[c] < 1 || cand[c] >= n)
      return fail(QMC_E_INVAL, "candidate %d: a = %llu outside [1, n)", c,
                  (unsigned long long)cand[c]);
  return QMC_OK;
}

int64_t p2_chunks(uint64_t n, int32_t n_cand) {
  // workgroups per candidate: about 128 points per thread, within the partial buffer
  int64_t chunks = (int64_t)((n + 256 * 128 - 1) / (256 * 128));
  const int64_t cap = (int64_t)(kP2PartialDoubles / 2) / n_cand;
  return std::max<int64_t>(1, std::min<int64_t>(chunks, std::min<int64_t>(cap, 65535)));
}
}  // namespace qmc

extern "C" {

qmc_status qmc_integrate(qmc_plan_t p, const uint64_t *n_in, const uint64_t *a_in, void *stream,
                         double *dev_q, double *dev_mean, double *dev_err) {
  g_last_error.clear();
  return integrate_sectors(p, n_in, a_in, nullptr, stream, dev_q, dev_mean, dev_err);
}

qmc_status qmc_integrate_vec(qmc_plan_t p, const uint64_t *n_in, const uint64_t *z, void *stream,
                             double *dev_q, double *dev_mean, double *dev_err) {
  g_last_error.clear();
  if (!z) return fail(QMC_E_INVAL, "NULL generating vectors");
  return integrate_sectors(p, n_in, nullptr, nullptr, stream, dev_q, dev_mean, dev_err, z);
}

// ------------------------------------------------------------ median QMC rules

static constexpr int64_t kMedianTarget = 16384;

struct MedianLayout {
  size_t sec, lat, shift, begin, order, q, mean, err, status, partial, total;
};

static MedianLayout median_layout(const qmc_plan_s *p, int32_t r) {
  const size_t V = (size_t)p->S * r;
  MedianLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = o;
    o = align256(o + b);
    return at;
  };
  L.sec = take(sizeof(SectorDev) * V);
  L.lat = take(sizeof(LatticeDev) * V);
  L.shift = take(sizeof(double) * V * QMC_MAX_DIM);
  L.begin = take(sizeof(int64_t) * (V + 1));
  L.order = take(sizeof(int32_t) * V);
  L.q = take(sizeof(double) * V * p->KC);
  L.mean = take(sizeof(double) * V * p->KC);
  L.err = take(sizeof(double) * V * p->KC);
  L.status = take(256);
  L.partial = take(sizeof(double) * 2 * (size_t)p->KC * (kMedianTarget + V + 64));
  L.total = o;
  return L;
}

size_t qmc_median_workspace_bytes(qmc_plan_t p, int32_t r) {
  if (!p || r < 1) return 0;
  return median_layout(p, r).total;
}

qmc_status qmc_median_lattice(qmc_plan_t p, const uint64_t *n_in, int32_t r,
                              const uint64_t *cand, int32_t order, void *dev_scratch,
                              size_t scratch_bytes, void *stream, uint64_t *z_out, double *q_out) {
  g_last_error.clear();
  if (!p || !cand || !z_out || !dev_scratch) return fail(QMC_E_INVAL, "NULL argument");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  if (p->cplx) return fail(QMC_E_INVAL, "median rules take real plans");
  if (r < 1 || r > 1024) return fail(QMC_E_INVAL, "r = %d outside [1, 1024]", r);
  if (order < -p->K || order >= p->K)
    return fail(QMC_E_INVAL, "order %d outside [-%d, %d)", order, p->K, p->K);
  const int k_sel = order < 0 ? p->K + order : order;
  const MedianLayout ML = median_layout(p, r);
  if (scratch_bytes < ML.total)
    return fail(QMC_E_NOMEM, "scratch of %zu bytes, %zu needed", scratch_bytes, ML.total);
  if (((uintptr_t)dev_scratch & 255) != 0) return fail(QMC_E_INVAL, "scratch not 256-byte aligned");
  const int S = p->S, V = S * r, K = p->KC;
  std::vector<SectorDev> sec(V);
  std::vector<LatticeDev> lat(V);
  std::vector<int32_t> ord(V);
  std::vector<int64_t> begin(V + 1);
  __int128 total = 0;
  for (int s = 0; s < S; ++s) {
    const uint64_t n = n_in ? n_in[s] : p->n_default[s];
    if (n < 2 || n > p->n_max || n >= (1ull << 53))
      return fail(QMC_E_INVAL, "sector %d: n = %llu outside [2, n_max]", s, (unsigned long long)n);
    for (int c = 0; c < r; ++c) {
      const int v = s * r + c;
      sec[v] = p->sec[s];
      LatticeDev &L = lat[v];
      std::memset(&L, 0, sizeof L);
      L.active = 1;
      L.n = n;
      L.n_d = (double)n;
      L.inv_n = 1.0 / (double)n;
      for (int j = 0; j < p->dims[s]; ++j) {
        const uint64_t z = cand[((size_t)s * r + c) * QMC_MAX_DIM + j];
        if (z < 1 || z >= n || gcd_u64(z, n) != 1)
          return fail(QMC_E_INVAL, "sector %d, candidate %d: z_%d = %llu not in U_n", s, c, j + 1,
                      (unsigned long long)z);
        L.z[j] = z;
        L.dz[j] = mulmod_host((uint64_t)p->block % n, z, n);
        L.ndz[j] = (double)(n - L.dz[j]);
      }
      total += (__int128)n;
    }
  }
  for (int v = 0; v < V; ++v) ord[v] = v;
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
    const int sx = x / r, sy = y / r;
    const int fx = path_class(p, sx), fy = path_class(p, sy);
    return p->dims[sx] != p->dims[sy] ? p->dims[sx] < p->dims[sy] : fx < fy;
  });
  const __int128 per_block = (__int128)kMedianTarget * p->block;
  int64_t ppt = (int64_t)((total + per_block - 1) / per_block);
  if (ppt < 1) ppt = 1;
  const int64_t chunk = ppt * p->block;
  int64_t b = 0;
  DimLaunch dl[4 * QMC_MAX_DIM];
  int n_dl = 0;
  for (int t = 0; t < V; ++t) {
    const int v = ord[t], s = v / r;
    LatticeDev &L = lat[v];
    L.chunk = chunk;
    L.n_chunks = (int32_t)((L.n + chunk - 1) / chunk);
    L.block_begin = b;
    begin[t] = b;
    const int cls = path_class(p, s);
    const int fast = (cls == 1 || cls == 2) ? 1 : 0, f32 = cls == 2 ? 1 : 0, flow = cls == 4 ? 1 : 0;
    if (n_dl == 0 || dl[n_dl - 1].d != p->dims[s] || dl[n_dl - 1].fast != fast ||
        dl[n_dl - 1].f32 != f32 || dl[n_dl - 1].flow != flow) {
      if (n_dl == 4 * QMC_MAX_DIM) return fail(QMC_E_STATE, "too many launch classes");
      dl[n_dl] = DimLaunch{b, 0, p->dims[s], fast, f32, 0, flow, 0, 0};
      ++n_dl;
    }
    dl[n_dl - 1].blocks += L.n_chunks;
    b += L.n_chunks;
  }
  begin[V] = b;
  if ((size_t)(b + 0) > (size_t)(kMedianTarget + V + 64))
    return fail(QMC_E_STATE, "median launch needs %lld workgroups", (long long)b);
  char *w = (char *)dev_scratch;
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> zero((size_t)V * QMC_MAX_DIM, 0.0);
  int e;
  if ((e = hipMemcpyAsync(w + ML.sec, sec.data(), sizeof(SectorDev) * V, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(w + ML.lat, lat.data(), sizeof(LatticeDev) * V, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(w + ML.shift, zero.data(), sizeof(double) * zero.size(), hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(w + ML.begin, begin.data(), sizeof(int64_t) * (V + 1), hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(w + ML.order, ord.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, st)))
    return hip_fail(e, "upload median tables");
  LaunchArgs la;
  std::memset(&la, 0, sizeof la);
  la.sectors = (const SectorDev *)(w + ML.sec);
  la.coef = (const double *)(p->ws + p->off_coef);
  la.coef32 = (const float *)(p->ws + p->off_coef32);
  la.shifts = (const double *)(w + ML.shift);
  la.lat = (const LatticeDev *)(w + ML.lat);
  la.block_begin = (const int64_t *)(w + ML.begin);
  la.order = (const int32_t *)(w + ML.order);
  la.n_dim_launches = n_dl;
  for (int t = 0; t < n_dl; ++t) la.dims[t] = dl[t];
  la.partial = (double *)(w + ML.partial);
  la.q = (double *)(w + ML.q);
  la.mean = (double *)(w + ML.mean);
  la.err = (double *)(w + ML.err);
  la.status = (int32_t *)(w + ML.status);
  la.n_sectors = V;
  la.m = 1;
  la.K = K;
  la.shift_tile = 1;
  la.shifts_per_pass = 1;
  la.block = p->block;
  la.total_blocks = b;
  la.d_max = p->d_max;
  la.precision = p->precision;
  if ((e = launch_status_reset(la.status, stream)) != hipSuccess) return hip_fail(e, "status reset");
  if ((e = launch_integrate(la, stream, &p->side)) != hipSuccess) return hip_fail(e, "median launch");
  std::vector<double> q((size_t)V * K);
  int32_t code = 0;
  if ((e = hipMemcpyAsync(q.data(), w + ML.q, sizeof(double) * q.size(), hipMemcpyDeviceToHost, st)) ||
      (e = hipMemcpyAsync(&code, w + ML.status, sizeof code, hipMemcpyDeviceToHost, st)) ||
      (e = hipStreamSynchronize(st)))
    return hip_fail(e, "read median estimates");
  if (code != INT32_MAX) {
    const int v = code / QMC_MAX_ORDERS;
    return fail(QMC_E_NONFINITE, "non-finite estimate: sector %d, candidate %d", v / r, v % r);
  }
  std::vector<int> idx(r);
  for (int s = 0; s < S; ++s) {
    for (int c = 0; c < r; ++c) idx[c] = c;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
      return q[((size_t)s * r + x) * K + k_sel] < q[((size_t)s * r + y) * K + k_sel];
    });
    const int c = idx[(r - 1) / 2];
    for (int j = 0; j < QMC_MAX_DIM; ++j)
      z_out[(size_t)s * QMC_MAX_DIM + j] = j < p->dims[s] ? cand[((size_t)s * r + c) * QMC_MAX_DIM + j] : 0;
    if (q_out)
      for (int cc = 0; cc < r; ++cc) q_out[(size_t)s * r + cc] = q[((size_t)s * r + cc) * K + k_sel];
  }
  return QMC_OK;
}

qmc_status qmc_query_status(qmc_plan_t p, void *stream, int32_t *sector, int32_t *shift,
                            int32_t *order) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (!p->ws && !p->static_status) return fail(QMC_E_STATE, "no workspace bound");
  int32_t code = 0;
  hipStream_t st = (hipStream_t)stream;
  const void *at = p->static_status ? (const void *)p->static_status : p->ws + p->off_status;
  int e = hipMemcpyAsync(&code, at, sizeof code, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "read status");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronize");
  if (code == INT32_MAX) {
    if (!p->cplx) return QMC_OK;
    std::vector<uint64_t> cnt(p->S);
    qmc_status sc = qmc_sign_violations(p, stream, cnt.data());
    if (sc != QMC_OK) return sc;
    for (int s = 0; s < p->S; ++s)
      if (cnt[s]) {
        if (sector) *sector = s;
        if (shift) *shift = -1;
        if (order) *order = -1;
        return fail(QMC_E_SIGNCHECK, "sign check failed: sector %d, %llu samples with Im F(z) > 0",
                    s, (unsigned long long)cnt[s]);
      }
    return QMC_OK;
  }
  const int ko = code % QMC_MAX_ORDERS;
  const int sl = code / QMC_MAX_ORDERS;
  if (sector) *sector = sl / p->m;
  if (shift) *shift = sl % p->m;
  if (order) *order = ko;
  return fail(QMC_E_NONFINITE, "non-finite sum: sector %d, shift %d, order %d", sl / p->m,
              sl % p->m, ko);
}

int32_t qmc_plan_complex(qmc_plan_t p) { return p ? p->cplx : -1; }

qmc_status qmc_sign_violations(qmc_plan_t p, void *stream, uint64_t *counts) {
  if (!p || !counts) return fail(QMC_E_INVAL, "NULL argument");
  if (!p->ws && !p->static_status) return fail(QMC_E_STATE, "no workspace bound");
  if (!p->cplx) {
    for (int s = 0; s < p->S; ++s) counts[s] = 0;
    return QMC_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  const void *at = p->static_sign ? (const void *)p->static_sign : p->ws + p->off_sign;
  int e = hipMemcpyAsync(counts, at, sizeof(uint64_t) * p->S, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return hip_fail(e, "read sign-check counters");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronize");
  return QMC_OK;
}

qmc_status qmc_set_deformation(qmc_plan_t p, const double *lambda, void *stream) {
  g_last_error.clear();
  if (!p || !lambda) return fail(QMC_E_INVAL, "NULL argument");
  if (!p->cplx) return fail(QMC_E_STATE, "the plan is real (no deformed sector)");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  for (int s = 0; s < p->S; ++s)
    if (!(lambda[s] >= 0.0) || !std::isfinite(lambda[s]))
      return fail(QMC_E_INVAL, "lambda[%d] must be finite and >= 0", s);
  for (int s = 0; s < p->S; ++s) p->sec[s].lambda = lambda[s];
  p->cal_valid = false;   // the contour changed
  int e = hipMemcpyAsync(p->ws + p->off_sec, p->sec.data(), sizeof(SectorDev) * p->S,
                         hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "upload sectors");
  return QMC_OK;
}

qmc_status qmc_choose_deformation(qmc_plan_t p, uint64_t n_pre, const uint64_t *a_pre,
                                  int32_t max_halvings, void *stream, double *lambda_out,
                                  int32_t *halvings_out) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (!p->cplx) return fail(QMC_E_STATE, "the plan is real (no deformed sector)");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  if (max_halvings < 0 || max_halvings > 60)
    return fail(QMC_E_INVAL, "max_halvings = %d outside [0, 60]", max_halvings);
  const int S = p->S;
  std::vector<uint64_t> n(S, n_pre), a(S), cnt(S);
  std::vector<uint8_t> active(S);
  std::vector<int32_t> halv(S, 0);
  std::vector<double> lam(S);
  for (int s = 0; s < S; ++s) {
    a[s] = a_pre ? a_pre[s] : p->a_default[s];
    lam[s] = p->sec[s].lambda;
    active[s] = lam[s] > 0.0;
  }
  double *mean = (double *)(p->ws + p->off_mean), *err = (double *)(p->ws + p->off_err);
  bool failed = false;
  int first_failed = -1;
  for (;;) {
    bool any = false;
    for (int s = 0; s < S; ++s) any = any || active[s];
    if (!any) break;
    qmc_status st = qmc_set_deformation(p, lam.data(), stream);
    if (st != QMC_OK) return st;
    p->bound_off = true;   // only the sign-check counts are wanted here
    st = integrate_sectors(p, n.data(), a.data(), active.data(), stream, nullptr, mean, err);
    p->bound_off = false;
    if (st != QMC_OK) return st;
    if ((st = qmc_sign_violations(p, stream, cnt.data())) != QMC_OK) return st;
    for (int s = 0; s < S; ++s) {
      if (!active[s] || cnt[s] == 0) {
        active[s] = 0;
        continue;
      }
      if (halv[s] < max_halvings) {
        lam[s] *= 0.5;
        ++halv[s];
      } else {
        active[s] = 0;
        if (!failed) first_failed = s;
        failed = true;
      }
    }
  }
  qmc_status st = qmc_set_deformation(p, lam.data(), stream);
  if (st != QMC_OK) return st;
  for (int s = 0; s < S; ++s) {
    if (lambda_out) lambda_out[s] = lam[s];
    if (halvings_out) halvings_out[s] = halv[s];
  }
  if (failed)
    return fail(QMC_E_SIGNCHECK, "sector %d: sign check still fails after %d halvings",
                first_failed, max_halvings);
  return QMC_OK;
}

qmc_status qmc_integrate_deformed(qmc_plan_t p, const uint64_t *n_in, const uint64_t *a_in,
                                  int32_t max_halvings, void *stream, double *dev_q,
                                  double *dev_mean, double *dev_err, double *lambda_out,
                                  int32_t *halvings_out) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (!p->cplx) return fail(QMC_E_STATE, "the plan is real (no deformed sector)");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  if (!dev_mean || !dev_err) return fail(QMC_E_INVAL, "dev_mean and dev_err are required");
  if (max_halvings < 0 || max_halvings > 60)
    return fail(QMC_E_INVAL, "max_halvings = %d outside [0, 60]", max_halvings);
  const int S = p->S;
  std::vector<uint64_t> cnt(S);
  std::vector<uint8_t> active(S, 1);   // the first pass integrates every sector
  std::vector<int32_t> halv(S, 0);
  std::vector<double> lam(S);
  for (int s = 0; s < S; ++s) lam[s] = p->sec[s].lambda;
  bool failed = false, changed = false;
  int first_failed = -1;
  for (;;) {
    bool any = false;
    for (int s = 0; s < S; ++s) any = any || active[s];
    if (!any) break;
    qmc_status st;
    if (changed && (st = qmc_set_deformation(p, lam.data(), stream)) != QMC_OK) return st;
    changed = false;
    // a later pass re-integrates only the sectors whose lambda was halved: the others
    // keep the sums (and, through the statistics over every sector, the errors) of the
    // pass at their final lambda
    st = integrate_sectors(p, n_in, a_in, active.data(), stream, dev_q, dev_mean, dev_err);
    if (st != QMC_OK) return st;
    int32_t sec = -1, shift = -1, order = -1;
    st = qmc_query_status(p, stream, &sec, &shift, &order);
    if (st == QMC_E_NONFINITE) return st;
    g_last_error.clear();
    if ((st = qmc_sign_violations(p, stream, cnt.data())) != QMC_OK) return st;
    for (int s = 0; s < S; ++s) {
      if (!active[s] || cnt[s] == 0) {
        active[s] = 0;
        continue;
      }
      if (halv[s] < max_halvings) {
        lam[s] *= 0.5;
        ++halv[s];
        changed = true;
      } else {
        active[s] = 0;
        if (!failed) first_failed = s;
        failed = true;
      }
    }
  }
  for (int s = 0; s < S; ++s) {
    if (lambda_out) lambda_out[s] = lam[s];
    if (halvings_out) halvings_out[s] = halv[s];
  }
  if (failed)
    return fail(QMC_E_SIGNCHECK, "sector %d: sign check still fails after %d halvings",
                first_failed, max_halvings);
  return QMC_OK;
}

// ------------------------------------------------------------------ autotuner

static std::mutex g_tune_mu;
static std::map<std::string, qmc_launch_shape> g_tune_cache;

// Cache key: what decides the best launch shape of the integrand kernels.
static std::string tune_key(const qmc_plan_s *p) {
  long long mono = 0, flows = 0;
  for (const SectorDev &sd : p->sec) {
    mono += sd.u_deg * 1000 + sd.f_deg;
    flows += sd.flow != 0;
  }
  char buf[256];
  // the plan-specialised kernels (qmc_specialize) change which kernels a shape runs
  std::snprintf(buf, sizeof buf, "S%d d%d K%d M%d p%d m%d c%d f%lld u%lld g%zu", p->S, p->d_max,
                p->K, p->M, p->precision, p->m, p->cplx, flows, mono, p->gen.size());
  return buf;
}

qmc_status qmc_set_launch_shape(qmc_plan_t p, const qmc_launch_shape *sh) {
  g_last_error.clear();
  if (!p || !sh) return fail(QMC_E_INVAL, "NULL argument");
  const int spp = p->cplx ? 1 : sh->shifts_per_pass;
  if (!tile_supported(sh->shift_tile, spp, sh->block) || sh->shift_tile * p->KC > 64 ||
      p->m % sh->shift_tile != 0 || (p->cplx && sh->shifts_per_pass != 1))
    return fail(QMC_E_INVAL, "unsupported launch shape: block %d, shift_tile %d, shifts_per_pass %d",
                sh->block, sh->shift_tile, sh->shifts_per_pass);
  if (sh->target_blocks < 256 || sh->target_blocks > kTargetBlocksMax)
    return fail(QMC_E_INVAL, "target_blocks = %d outside [256, %lld]", sh->target_blocks,
                (long long)kTargetBlocksMax);
  p->block = sh->block;
  p->tile = sh->shift_tile;
  p->spp = spp;
  p->target_blocks = sh->target_blocks;
  for (int &g : p->persistent_grid) g = 0;   // occupancy depends on the block size
  for (GenKernel &g : p->gen) g.grid = 0;
  p->lat_valid = false;
  return QMC_OK;
}

qmc_status qmc_get_launch_shape(qmc_plan_t p, qmc_launch_shape *sh) {
  if (!p || !sh) return fail(QMC_E_INVAL, "NULL argument");
  sh->block = p->block;
  sh->shift_tile = p->tile;
  sh->shifts_per_pass = p->spp;
  sh->target_blocks = (int32_t)p->target_blocks;
  sh->ms = 0.0;
  return QMC_OK;
}

qmc_status qmc_autotune(qmc_plan_t p, const uint64_t *n, const uint64_t *a, int32_t reps,
                        int32_t use_cache, void *stream, qmc_launch_shape *best) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  if (reps < 1 || reps > 100) return fail(QMC_E_INVAL, "reps = %d outside [1, 100]", reps);
  const std::string key = tune_key(p);
  if (use_cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      qmc_status st = qmc_set_launch_shape(p, &it->second);
      if (st == QMC_OK && best) *best = it->second;
      return st;
    }
  }
  qmc_launch_shape keep;
  qmc_get_launch_shape(p, &keep);
  hipStream_t hs = (hipStream_t)stream;
  double *mean = (double *)(p->ws + p->off_mean), *err = (double *)(p->ws + p->off_err);
  hipEvent_t e0, e1;
  int e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "create event");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "create event");
  }
  qmc_launch_shape top = keep;
  top.ms = 1e300;
  qmc_status res = QMC_OK;
  const int blocks[] = {64, 128, 256};
  const int spps[] = {1, 2, 4};
  const int targets[] = {8192, 16384, 32768};
  for (int bl : blocks)
    for (int tile = 1; tile <= kMaxTile && res == QMC_OK; tile *= 2)
      for (int spp : spps)
        for (int tg : targets) {
          qmc_launch_shape c{bl, tile, spp, tg, 0.0};
          if (p->cplx && spp != 1) continue;
          // FP32 at four shifts per pass: the specialised kernels take four, the
          // table-driven ones run two (no FP32 table kernel is compiled for four)
          if (p->precision == QMC_PREC_FP32 && spp == 4 && p->gen.empty()) continue;
          if (qmc_set_launch_shape(p, &c) != QMC_OK) continue;
          // warm-up (uploads the lattice table), then the timed repetitions
          if ((res = integrate_sectors(p, n, a, nullptr, stream, nullptr, mean, err)) != QMC_OK)
            break;
          float best_ms = 1e30f;
          for (int r = 0; r < reps && res == QMC_OK; ++r) {
            if ((e = hipEventRecord(e0, hs)) != hipSuccess) res = hip_fail(e, "record event");
            else if ((res = integrate_sectors(p, n, a, nullptr, stream, nullptr, mean, err)) != QMC_OK) {
            } else if ((e = hipEventRecord(e1, hs)) != hipSuccess) res = hip_fail(e, "record event");
            else if ((e = hipEventSynchronize(e1)) != hipSuccess) res = hip_fail(e, "synchronize");
            else {
              float ms = 0.0f;
              if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) res = hip_fail(e, "elapsed time");
              best_ms = std::min(best_ms, ms);
            }
          }
          if (res == QMC_OK && best_ms < top.ms) {
            top = c;
            top.ms = best_ms;
          }
        }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res != QMC_OK) {
    qmc_set_launch_shape(p, &keep);
    return res;
  }
  res = qmc_set_launch_shape(p, &top);
  if (res != QMC_OK) return res;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = top;
  }
  if (best) *best = top;
  return QMC_OK;
}


qmc_status qmc_korobov_p2(qmc_plan_t p, uint64_t n, int32_t d, const uint64_t *cand,
                          int32_t n_cand, void *stream, double *dev_p2) {
  g_last_error.clear();
  if (!p || !cand || !dev_p2) return fail(QMC_E_INVAL, "NULL argument");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  qmc_status chk = p2_check_args(n, d, cand, n_cand);
  if (chk != QMC_OK) return chk;
  const int64_t chunks = p2_chunks(n, n_cand);
  hipStream_t st = (hipStream_t)stream;
  int e = hipMemcpyAsync(p->ws + p->off_p2cand, cand, sizeof(uint64_t) * n_cand,
                         hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "upload candidates");
  e = launch_korobov_p2(n, d, (const uint64_t *)(p->ws + p->off_p2cand), n_cand, (int32_t)chunks,
                        (double *)(p->ws + p->off_p2part), dev_p2, stream);
  if (e != hipSuccess) return hip_fail(e, "P2 launch");
  return QMC_OK;
}

qmc_status qmc_korobov_search(qmc_plan_t p, uint64_t n, int32_t d, const uint64_t *cand,
                              int32_t n_cand, void *stream, uint64_t *a_out, double *p2_out) {
  if (!a_out) return fail(QMC_E_INVAL, "NULL a_out");
  if (!p || !p->ws) return fail(p ? QMC_E_STATE : QMC_E_INVAL, "plan not bound");
  double *dev_vals = (double *)(p->ws + p->off_p2vals);
  qmc_status st = qmc_korobov_p2(p, n, d, cand, n_cand, stream, dev_vals);
  if (st != QMC_OK) return st;
  std::vector<double> v(n_cand);
  hipStream_t hs = (hipStream_t)stream;
  int e = hipMemcpyAsync(v.data(), dev_vals, sizeof(double) * n_cand, hipMemcpyDeviceToHost, hs);
  if (e != hipSuccess) return hip_fail(e, "read P2 values");
  if ((e = hipStreamSynchronize(hs)) != hipSuccess) return hip_fail(e, "synchronize");
  double vmin = v[0];
  for (double x : v) vmin = std::min(vmin, x);
  uint64_t best = 0;
  double bestv = 0.0;
  bool have = false;
  for (int32_t c = 0; c < n_cand; ++c)
    if (v[c] <= vmin * (1.0 + 1e-12) && (!have || cand[c] < best)) {
      best = cand[c];
      bestv = v[c];
      have = true;
    }
  *a_out = best;
  if (p2_out) *p2_out = bestv;
  return QMC_OK;
}

qmc_status qmc_enable_timing(qmc_plan_t p, int32_t enable) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  p->timing = enable != 0;
  p->ev_used = 0;
  return QMC_OK;
}

qmc_status qmc_read_timing(qmc_plan_t p, double *ms_total, int32_t *launches) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  double tot = 0.0;
  for (size_t t = 0; t + 1 < p->ev_used; t += 2) {
    int e = hipEventSynchronize(p->ev[t + 1]);
    if (e != hipSuccess) return hip_fail(e, "synchronize timing event");
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, p->ev[t], p->ev[t + 1])) != hipSuccess)
      return hip_fail(e, "elapsed time");
    tot += ms;
  }
  if (ms_total) *ms_total = tot;
  if (launches) *launches = (int32_t)(p->ev_used / 2);
  return QMC_OK;
}

qmc_status qmc_lattice_points(uint64_t n, int32_t d, uint64_t a, const double *shift,
                              uint64_t i0, uint64_t count, void *stream, double *dev_y) {
  g_last_error.clear();
  if (!shift || !dev_y) return fail(QMC_E_INVAL, "NULL argument");
  if (n < 2 || n >= (1ull << 53)) return fail(QMC_E_INVAL, "n = %llu outside [2, 2^53)",
                                              (unsigned long long)n);
  if (d < 1 || d > QMC_MAX_DIM) return fail(QMC_E_INVAL, "d = %d outside [1, %d]", d, QMC_MAX_DIM);
  if (count == 0) return QMC_OK;
  if (i0 >= n || count > n - i0) return fail(QMC_E_INVAL, "points [%llu, %llu) outside [0, n)",
                                             (unsigned long long)i0,
                                             (unsigned long long)(i0 + count));
  PointsArgs pa;
  std::memset(&pa, 0, sizeof pa);
  pa.n = n;
  pa.n_d = (double)n;
  pa.inv_n = 1.0 / (double)n;
  pa.d = d;
  pa.i0 = i0;
  pa.count = count;
  pa.out = dev_y;
  pa.steps = 16;
  const uint64_t am = a % n;
  uint64_t z = 1 % n;
  for (int j = 0; j < d; ++j) {
    if (gcd_u64(z, n) != 1)
      return fail(QMC_E_INVAL, "z_%d = %llu shares a factor with n", j + 1, (unsigned long long)z);
    if (!(shift[j] >= 0.0 && shift[j] < 1.0))
      return fail(QMC_E_INVAL, "shift[%d] = %g outside [0, 1)", j, shift[j]);
    pa.z[j] = z;
    pa.dz[j] = mulmod_host(256 % n, z, n);
    pa.ndz[j] = (double)(n - pa.dz[j]);
    pa.delta[j] = shift[j];
    z = mulmod_host(z, am, n);
  }
  const uint64_t per = 256ull * pa.steps;
  const uint64_t grid = (count + per - 1) / per;
  if (grid > 0x7fffffffull) return fail(QMC_E_INVAL, "too many points for one call");
  int e = launch_points(pa, (unsigned)grid, stream);
  if (e != hipSuccess) return hip_fail(e, "points launch");
  return QMC_OK;
}

void qmc_plan_free(qmc_plan_t p) { delete p; }

}  // extern "C"
