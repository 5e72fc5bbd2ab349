// qmc_gen.cpp -- plan-specialised integrand kernels, generated and compiled at run time.
//
// pySecDec writes and compiles integrand code per integral (Sec. 2.1 of arXiv:2305.19768:
// the integrand kernels are generated code, with the per-integrand constants hoisted
// out of the point loop).  The table-driven kernels of this library instead evaluate
// U and F by a dense nested Horner over every monomial slot of total degree <= 3,
// which at d = 6 visits 84 slots for the 10-30 monomials F actually has.  This file
// writes, for every real-contour sector without a flow, straight-line code that
// evaluates only its own monomials, with the epsilon-order polynomials in log F and the
// powers of x_j, U and F (integer or half-integer) fixed, and compiles it with hiprtc for the device the plan runs on: one kernel
// per (dimension, precision) launch class, a uniform switch over the class's sectors
// choosing the sector's code (every workgroup holds one sector).  Everything else --
// lattice points, transform, accumulation, reductions -- is the library's own block
// body (qmc_device.h), compiled into the same kernel from the embedded header text.
//
// Polynomial evaluation: multivariate Horner by greedy factorisation.  P = x_v Q + R
// where x_v occurs in the most monomials of P (ties: smallest v), Q = (the monomials
// containing x_v) / x_v and R the rest, recursively; each split costs one FMA (one
// multiplication when R is empty), so a polynomial of M monomials takes at most one
// operation per monomial per variable occurrence and usually about M.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "qmc_plan.h"

using namespace qmc;

namespace qmc {
// Text of the device headers, embedded at build time (qmc_rtc_headers.cpp, generated).
extern const char *const kRtcHeaderText[];
extern const char *const kRtcHeaderName[];
extern const int kRtcHeaderCount;
}  // namespace qmc

namespace {

struct Mono {
  int e[QMC_MAX_DIM];
  double c;
};

// Monomials (exponent vector, coefficient) of a dense degree-3 nested-Horner table, in
// its slot order: c0; per j: x_j, then per k >= j: x_j x_k, then x_j x_k x_l, l >= k.
std::vector<Mono> sparse_monomials(const double *tab, int D) {
  std::vector<Mono> out;
  auto add = [&](int p, int a, int b, int c) {
    if (tab[p] == 0.0) return;
    Mono m;
    std::memset(m.e, 0, sizeof m.e);
    if (a >= 0) ++m.e[a];
    if (b >= 0) ++m.e[b];
    if (c >= 0) ++m.e[c];
    m.c = tab[p];
    out.push_back(m);
  };
  int p = 0;
  add(p++, -1, -1, -1);
  for (int j = 0; j < D; ++j) {
    add(p++, j, -1, -1);
    for (int k = j; k < D; ++k) {
      add(p++, j, k, -1);
      for (int l = k; l < D; ++l) add(p++, j, k, l);
    }
  }
  return out;
}

std::string lit(double v, bool f32) {
  char buf[64];
  if (f32) {
    const float f = (float)v;
    if (f == 0.0f) return "0.0f";
    std::snprintf(buf, sizeof buf, "%af", (double)f);
  } else {
    if (v == 0.0) return "0.0";
    std::snprintf(buf, sizeof buf, "%a", v);
  }
  return buf;
}

struct Emitter {
  bool f32;
  std::string body;
  int n = 0;
  const char *T() const { return f32 ? "float" : "double"; }
  const char *fma() const { return f32 ? "__builtin_fmaf" : "__builtin_fma"; }
  std::string tmp() { return "t" + std::to_string(++n); }
  void line(const std::string &s) { body += "      " + s + "\n"; }

  // Returns an expression for P (a temporary or a literal); "" for the zero polynomial.
  std::string poly(const std::vector<Mono> &P, int D) {
    double c0 = 0.0;
    bool has_c0 = false;
    std::vector<const Mono *> nc;
    for (const Mono &m : P) {
      int g = 0;
      for (int j = 0; j < D; ++j) g += m.e[j];
      if (g == 0) {
        c0 += m.c;
        has_c0 = true;
      } else {
        nc.push_back(&m);
      }
    }
    if (nc.empty()) return (has_c0 && c0 != 0.0) ? lit(c0, f32) : std::string();
    int v = 0, best = -1;
    for (int j = 0; j < D; ++j) {
      int cnt = 0;
      for (const Mono *m : nc) cnt += m->e[j] > 0;
      if (cnt > best) {
        best = cnt;
        v = j;
      }
    }
    std::vector<Mono> Q, R;
    for (const Mono &m : P) {
      if (m.e[v] > 0) {
        Mono q = m;
        --q.e[v];
        Q.push_back(q);
      } else {
        R.push_back(m);
      }
    }
    const std::string q = poly(Q, D);
    const std::string r = poly(R, D);
    const std::string t = tmp();
    const std::string xv = "x[u][" + std::to_string(v) + "]";
    if (r.empty())
      line(std::string("const ") + T() + " " + t + " = " + xv + " * " + q + ";");
    else
      line(std::string("const ") + T() + " " + t + " = " + fma() + "(" + xv + ", " + q + ", " + r + ");");
    return t;
  }
};

// Non-negative coefficients and a positive constant term: the polynomial is at least
// that constant on [0, 1]^d.
bool positive_on_cube(const std::vector<Mono> &P, int D) {
  bool c0 = false;
  for (const Mono &mo : P) {
    if (mo.c < 0.0) return false;
    int g = 0;
    for (int j = 0; j < D; ++j) g += mo.e[j];
    c0 = c0 || (g == 0 && mo.c > 0.0);
  }
  return c0;
}

std::string product(const std::string &base, int times, const std::string &one) {
  if (times == 0) return one;
  std::string s = base;
  for (int t = 1; t < times; ++t) s += " * " + base;
  return s;
}

// The generated integrand of one sector: struct G<s> with f64<S> or f32<S> giving the
// orders f_k (without the transform weight) of S transformed samples; `korobov3` tells
// the block body which transform to apply (korobov_3 inline, the others through
// apply_transform).
std::string sector_struct(const qmc_plan_s *p, int s, bool f32, bool *finite_out = nullptr,
                          bool *korobov3_out = nullptr) {
  const SectorDev &sd = p->sec[s];
  const int D = sd.d, K = p->K;
  Emitter em{f32, std::string(), 0};
  const std::vector<Mono> U = sparse_monomials(p->coef.data() + sd.u_off, D);
  const std::vector<Mono> F = sparse_monomials(p->coef.data() + sd.f_off, D);
  const char *T = em.T();
  const std::string one = f32 ? "1.0f" : "1.0";
  std::string u = em.poly(U, D), f = em.poly(F, D);
  if (u.empty()) u = f32 ? "0.0f" : "0.0";
  if (f.empty()) f = f32 ? "0.0f" : "0.0";
  em.line(std::string("const ") + T + " U = " + u + ";");
  em.line(std::string("const ") + T + " F = " + f + ";");
  // B = U^u_num F^f_num prod_j x_j^x_num / (U^u_den F^f_den prod_j x_j^x_den), times
  // sqrt(hn / hd) = sqrt(hn hd) / hd for the half-integer exponents (hn: the factors with
  // exponent +1/2, hd: those with -1/2); FP32 sectors have integer exponents of U and F only
  std::string num, den, hn, hd;
  auto mul = [](std::string &acc, const std::string &t) { acc += (acc.empty() ? "" : " * ") + t; };
  if (sd.u_num) mul(num, product("U", sd.u_num, one));
  if (sd.f_num) mul(num, product("F", sd.f_num, one));
  if (sd.u_den) mul(den, product("U", sd.u_den, one));
  if (sd.f_den) mul(den, product("F", sd.f_den, one));
  bool neg_x = false;
  for (int j = 0; j < D; ++j) {
    const std::string xj = "x[u][" + std::to_string(j) + "]";
    if (sd.x_num[j]) mul(num, product(xj, sd.x_num[j], one));
    if (sd.x_den[j]) mul(den, product(xj, sd.x_den[j], one));
    if (sd.x_half[j] > 0) mul(hn, xj);
    if (sd.x_half[j] < 0) mul(hd, xj);
    neg_x = neg_x || sd.x_den[j] != 0 || sd.x_half[j] < 0;
  }
  if (sd.f_half > 0) mul(hn, "F");
  if (sd.f_half < 0) mul(hd, "F");
  if (!hn.empty() || !hd.empty()) {
    std::string h = hn;
    if (!hd.empty()) mul(h, hd);
    em.line("const double hs = __builtin_sqrt(" + h + ");");
    mul(num, "hs");
    if (!hd.empty()) mul(den, hd);
  }
  if (num.empty()) num = one;
  if (den.empty()) {
    em.line(std::string("const ") + T + " B = " + num + ";");
  } else {
    em.line(std::string("const ") + T + " den = " + den + ";");
    if (f32) {
      em.line("float r = __builtin_amdgcn_rcpf(den);");
      em.line("r = __builtin_fmaf(__builtin_fmaf(-den, r, 1.0f), r, r);");
      em.line("const float B = (" + num + ") * r;");
    } else {
      em.line("const double B = (" + num + ") * qmc::recip1(den);");
    }
  }
  // orders: f_k = sum_m logc[k][m] B L^m, from the terms BL_m = B L^m
  int mmax = 0;
  for (int k = 0; k < K; ++k)
    for (int m = 0; m <= p->M; ++m)
      if (sd.logc[k][m] != 0.0) mmax = std::max(mmax, m);
  // F > 0 on the whole cube when its coefficients are non-negative and its constant
  // term positive: then the logarithm needs no special cases, and with U positive too
  // (where it divides) the integrand is finite on the closed cube
  const bool f_pos = positive_on_cube(F, D);
  const bool finite = f_pos && (sd.u_den == 0 || positive_on_cube(U, D)) && !neg_x;
  if (mmax > 0) {
    em.line(f32 ? "const float L = __builtin_amdgcn_logf(F) * 0.693147180559945309f;"
                : f_pos ? "const double L = qmc::log_tab(F, lt);" : "const double L = qmc::log_f64(F);");
    em.line(std::string("const ") + T + " BL0 = B;");
    for (int m = 1; m <= mmax; ++m)
      em.line(std::string("const ") + T + " BL" + std::to_string(m) + " = BL" +
              std::to_string(m - 1) + " * L;");
  } else {
    em.line(std::string("const ") + T + " BL0 = B;");
  }
  for (int k = 0; k < K; ++k) {
    std::string acc;
    for (int m = 0; m <= mmax; ++m) {
      const double c = f32 ? (double)sd.logc32[k][m] : sd.logc[k][m];
      if (c == 0.0) continue;
      const std::string term = "BL" + std::to_string(m);
      if (acc.empty())
        acc = (c == 1.0) ? term : lit(c, f32) + " * " + term;
      else
        acc = std::string(em.fma()) + "(" + lit(c, f32) + ", " + term + ", " + acc + ")";
    }
    em.line("f[u][" + std::to_string(k) + "] = " + (acc.empty() ? (f32 ? "0.0f" : "0.0") : acc) + ";");
  }
  if (finite_out) *finite_out = finite;
  if (korobov3_out) *korobov3_out = sd.transform == QMC_TRANSFORM_KOROBOV3;
  char head[600];
  std::snprintf(head, sizeof head,
                "struct G%d {\n"
                "  static constexpr bool finite = %s;\n"
                "  static constexpr bool korobov3 = %s;\n"
                "  template <int S>\n"
                "  __device__ static __forceinline__ void %s(const %s (&x)[S][%d], %s (&f)[S][%d],\n"
                "                                          qmc::cptr<%s>%s, int) {\n"
                "#pragma unroll\n"
                "    for (int u = 0; u < S; ++u) {\n",
                s, finite ? "true" : "false",
                sd.transform == QMC_TRANSFORM_KOROBOV3 ? "true" : "false", f32 ? "f32" : "f64", T,
                D, T, K, T,
                f32 ? "" : ", const qmc::LogTable &lt");
  return std::string(head) + em.body + "    }\n  }\n};\n";
}

const char *kPrelude =
    "// integer types of the run-time compiler (no C library headers there)\n"
    "typedef __hip_internal::int8_t int8_t;\n"
    "typedef __hip_internal::uint8_t uint8_t;\n"
    "typedef __hip_internal::int16_t int16_t;\n"
    "typedef __hip_internal::uint16_t uint16_t;\n"
    "typedef __hip_internal::int32_t int32_t;\n"
    "typedef __hip_internal::uint32_t uint32_t;\n"
    "typedef __hip_internal::int64_t int64_t;\n"
    "typedef __hip_internal::uint64_t uint64_t;\n"
    "typedef unsigned long uintptr_t;\n"
    "#include \"qmc_device.h\"\n";

}  // namespace

namespace qmc {

std::string gen_persistent_name(bool f32) {
  return f32 ? "qmc_gen_persistent_f32" : "qmc_gen_persistent_f64";
}

std::string gen_kernel_name(int D, bool f32, int S) {
  char buf[64];
  std::snprintf(buf, sizeof buf, "qmc_gen_d%d_%s_s%d", D, f32 ? "f32" : "f64", S);
  return buf;
}

// Source of the kernel of launch class (D, f32) with S shifts per pass: the generated
// integrands of the class's sectors and the kernel that switches between them.
std::string gen_class_source(const qmc_plan_s *p, int D, bool f32, int S,
                             const std::vector<int> &sectors) {
  std::string src = kPrelude;
  src += "namespace qmc_gen {\n";
  for (int s : sectors) src += sector_struct(p, s, f32);
  src += "}  // namespace qmc_gen\n\n";
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "extern \"C\" __global__ __launch_bounds__(256) void %s(qmc::LaunchArgs a, "
                "int64_t block_base) {\n"
                "  __shared__ double red[qmc::kMaxWaves][qmc::kMaxTile * 4][2];\n"
                "  const qmc::BlockWork w = qmc::block_work(a, block_base);\n"
                "  switch (w.s) {\n",
                gen_kernel_name(D, f32, S).c_str());
  src += buf;
  for (int s : sectors) {
    std::snprintf(buf, sizeof buf,
                  "    case %d:\n"
                  "      qmc::integrate_block<%d, %d, %d, true, %s, true, qmc_gen::G%d>(a, w.s, "
                  "w.l_begin, w.tile, w.chunk_id, red);\n"
                  "      break;\n",
                  s, D, p->K, S, f32 ? "true" : "false", s);
    src += buf;
  }
  src +=
      "    default:\n"
      "      break;\n"
      "  }\n"
      "  __syncthreads();\n"
      "  qmc::block_store(a, w, red);\n"
      "}\n";
  return src;
}

// A struct whose integrand switches on the (wave-uniform) sector index among the
// given sectors' generated integrands: the form a persistent kernel takes, where one
// program holds every sector (the switch sits inside the point loop around the integrand
// alone, so the lattice, transform and accumulation code is compiled once per
// dimension, not once per sector).  Finite, or korobov_3, where every sector is.
std::string gen_switch_struct(const qmc_plan_s *p, const std::string &name, int D, bool f32,
                              const std::vector<int> &sectors, const std::vector<bool> &finite,
                              const std::vector<bool> &korobov3) {
  bool fin = true, k3 = true;
  for (size_t i = 0; i < sectors.size(); ++i) {
    fin = fin && finite[i];
    k3 = k3 && korobov3[i];
  }
  const char *T = f32 ? "float" : "double";
  char buf[768];
  std::snprintf(buf, sizeof buf,
                "struct %s {\n"
                "  static constexpr bool finite = %s;\n"
                "  static constexpr bool korobov3 = %s;\n"
                "  template <int S>\n"
                "  __device__ static __forceinline__ void %s(const %s (&x)[S][%d], %s (&f)[S][%d],\n"
                "                                          qmc::cptr<%s> c%s, int s) {\n"
                "    switch (s) {\n",
                name.c_str(), fin ? "true" : "false", k3 ? "true" : "false", f32 ? "f32" : "f64",
                T, D, T, p->K, T, f32 ? "" : ", const qmc::LogTable &lt");
  std::string src = buf;
  for (int s : sectors) {
    std::snprintf(buf, sizeof buf, "      case %d: G%d::template %s<S>(x, f, c%s, s); break;\n", s,
                  s, f32 ? "f32" : "f64", f32 ? "" : ", lt");
    src += buf;
  }
  std::snprintf(buf, sizeof buf,
                "      default:   // every work item of the launch is one of the sectors above\n"
                "#pragma unroll\n"
                "        for (int u = 0; u < S; ++u)\n"
                "#pragma unroll\n"
                "          for (int k = 0; k < %d; ++k) f[u][k] = 0;\n"
                "    }\n"
                "  }\n"
                "};\n",
                p->K);
  return src + buf;
}

// Source of the batched form's persistent kernel specialised to the plan: the generated
// integrands of the given sectors (every one without a flow), one switch struct per
// dimension, and the persistent loop of the library (qmc_persist.h) with a work-item
// runner that dispatches on the sector's dimension.  S shifts per pass (FP64 one, FP32
// two, as the library's persistent kernels).
std::string gen_persistent_source(const qmc_plan_s *p, bool f32, int S,
                                  const std::vector<int> &sectors) {
  std::string src = kPrelude;
  src += "#include \"qmc_persist.h\"\n";
  src += "namespace qmc_gen {\n";
  int dmax = 1;
  std::vector<std::vector<int>> by_d(QMC_MAX_DIM + 1);
  std::vector<std::vector<bool>> fin_d(QMC_MAX_DIM + 1), k3_d(QMC_MAX_DIM + 1);
  for (int s : sectors) {
    bool fin = false, k3 = false;
    src += sector_struct(p, s, f32, &fin, &k3);
    const int d = p->sec[s].d;
    by_d[d].push_back(s);
    fin_d[d].push_back(fin);
    k3_d[d].push_back(k3);
    dmax = std::max(dmax, d);
  }
  for (int d = 1; d <= QMC_MAX_DIM; ++d)
    if (!by_d[d].empty())
      src += gen_switch_struct(p, "C" + std::to_string(d), d, f32, by_d[d], fin_d[d], k3_d[d]);
  src += "}  // namespace qmc_gen\n\n";
  char buf[512];
  src +=
      "struct RunGen {\n"
      "  __device__ static __forceinline__ void run(const qmc::LaunchArgs &a, int s, int l_begin, "
      "int T,\n"
      "                                             int64_t chunk_id, double (*red)[qmc::kMaxTile * 4][2]) {\n"
      "    switch (a.sectors[s].d) {\n";
  for (int d = 1; d <= QMC_MAX_DIM; ++d) {
    if (by_d[d].empty()) continue;
    std::snprintf(buf, sizeof buf,
                  "      case %d: qmc::integrate_block<%d, %d, %d, true, %s, false, qmc_gen::C%d>(a, s, "
                  "l_begin, T, chunk_id, red); break;\n",
                  d, d, p->K, S, f32 ? "true" : "false", d);
    src += buf;
  }
  src += "      default: break;\n    }\n  }\n};\n\n";
  char waves[96];   // the occupancy the library's persistent kernel of the same form asks
  std::snprintf(waves, sizeof waves, "qmc::persistent_waves<%d, %s, false>()", dmax,
                f32 ? "true" : "false");
  std::snprintf(buf, sizeof buf,
                "extern \"C\" __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu("
                "%s))) void %s(qmc::LaunchArgs a, qmc::AmpState *st) {\n"
                "  __shared__ double red[qmc::kMaxWaves][qmc::kMaxTile * 4][2];\n"
                "  __shared__ int64_t item;\n"
                "  qmc::persistent_loop<%d, RunGen>(a, st, red, item);\n"
                "}\n",
                waves, gen_persistent_name(f32).c_str(), p->K);
  return src + buf;
}

// Code objects of sources compiled in this process (plans of the same problem share
// them); at most kGenCacheMax entries, the oldest dropped first.
std::mutex g_gen_mu;
std::vector<std::pair<std::string, std::vector<char>>> g_gen_cache;
constexpr size_t kGenCacheMax = 64;

// Compiles one class kernel for gfx950; returns the code object or an error message.
bool gen_compile(const std::string &src, const std::string &name, std::vector<char> &code,
                 std::string &err) {
  {
    std::lock_guard<std::mutex> lk(g_gen_mu);
    for (const auto &e : g_gen_cache)
      if (e.first == src) {
        code = e.second;
        return true;
      }
  }
  hiprtcProgram prog;
  hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), (name + ".hip").c_str(), kRtcHeaderCount,
                                       kRtcHeaderText, kRtcHeaderName);
  if (r != HIPRTC_SUCCESS) {
    err = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
    return false;
  }
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                        // no packed FP32 math, as for the library's own kernels
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    err = std::string("hiprtcCompileProgram: ") + hiprtcGetErrorString(r) + "\n" +
          log.substr(0, 2000);
    hiprtcDestroyProgram(&prog);
    return false;
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  code.resize(n);
  if (n) hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  if (n == 0) {
    err = "empty code object";
    return false;
  }
  std::lock_guard<std::mutex> lk(g_gen_mu);
  if (g_gen_cache.size() >= kGenCacheMax) g_gen_cache.erase(g_gen_cache.begin());
  g_gen_cache.emplace_back(src, code);
  return true;
}

// Shifts per pass a class kernel runs with under a launch shape of `spp` shifts per
// pass (FP64 at d >= 7 one shift per pass: two overflow the registers).
int gen_spp_for(int spp, int D, bool f32) { return (!f32 && D >= 7) ? 1 : spp; }
int gen_spp(const qmc_plan_s *p, int D, bool f32) { return gen_spp_for(p->spp, D, f32); }

// The sectors of launch class (D, f32) of the plan: real-contour sectors without a flow;
// FP32 takes the fast-path sectors with an FP32 form, FP64 every other one (fast path
// and generic shape alike).
std::vector<int> gen_class_sectors(const qmc_plan_s *p, int D, bool f32) {
  std::vector<int> out;
  if (p->cplx) return out;
  for (int s = 0; s < p->S; ++s) {
    const SectorDev &sd = p->sec[s];
    if (sd.d != D || sd.flow) continue;
    const bool s32 = p->precision == QMC_PREC_FP32 && (sd.flags & SF_FAST) && (sd.flags & SF_F32OK);
    if (s32 == f32) out.push_back(s);
  }
  return out;
}

GenKernel *gen_persistent_lookup(qmc_plan_s *p, bool f32, int K, const std::vector<int> &sectors) {
  for (GenKernel &g : p->gen)
    if (g.persistent && g.f32 == (int)f32 && g.K == K && g.sectors == sectors) return &g;
  return nullptr;
}

uint64_t gen_lookup(const qmc_plan_s *p, int D, bool f32) {
  if (p->gen.empty()) return 0;
  const int S = gen_spp(p, D, f32);
  for (const GenKernel &g : p->gen)
    if (!g.persistent && g.d == D && g.f32 == (int)f32 && g.spp == S)
      // a sector that joined the class later (a flow detached) has no case in the switch
      return g.sectors == gen_class_sectors(p, D, f32) ? (uint64_t)(uintptr_t)g.fn : 0;
  return 0;
}

}  // namespace qmc

extern "C" {

qmc_status qmc_gen_source(qmc_plan_t p, int32_t d, int32_t f32, char *buf, size_t cap,
                          size_t *len) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (d < 1 || d > QMC_MAX_DIM) return fail(QMC_E_INVAL, "d = %d outside [1, %d]", d, QMC_MAX_DIM);
  const std::vector<int> secs = gen_class_sectors(p, d, f32 != 0);
  const std::string src =
      secs.empty() ? std::string()
                   : gen_class_source(p, d, f32 != 0, gen_spp(p, d, f32 != 0), secs);
  if (len) *len = src.size();
  if (buf && cap) {
    const size_t n = std::min(cap - 1, src.size());
    std::memcpy(buf, src.data(), n);
    buf[n] = '\0';
  }
  return QMC_OK;
}

qmc_status qmc_specialize(qmc_plan_t p, int32_t flags, double *seconds) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (flags & ~(QMC_SPEC_COMPILE_ONLY | QMC_SPEC_OFF | QMC_SPEC_PERSISTENT))
    return fail(QMC_E_INVAL, "unknown flags 0x%x", flags);
  const auto t0 = std::chrono::steady_clock::now();
  if (flags & QMC_SPEC_OFF) {
    for (GenKernel &g : p->gen) (void)hipModuleUnload((hipModule_t)g.mod);
    p->gen.clear();
    if (seconds) *seconds = 0.0;
    return QMC_OK;
  }
  struct Job {
    int d, f32, spp;
    std::vector<int> sectors;
    std::string name, src, err;
    std::vector<char> code;
    bool ok = false;
  };
  std::vector<Job> jobs;
  if (flags & QMC_SPEC_PERSISTENT) {
    // the batched form's persistent kernel over every sector without a flow: real plans
    // whose sectors have the common shape (as the batched form requires), FP64 or FP32
    // with an FP32 form for every such sector
    if (p->cplx) return fail(QMC_E_INVAL, "the batched form takes real plans");
    const bool f32 = p->precision == QMC_PREC_FP32;
    std::vector<int> secs;
    for (int s = 0; s < p->S; ++s) {
      const SectorDev &sd = p->sec[s];
      if (sd.flow) continue;
      if (!(sd.flags & SF_FAST))
        return fail(QMC_E_INVAL, "sector %d does not have the common shape of the batched form", s);
      if (f32 && !(sd.flags & SF_F32OK))
        return fail(QMC_E_INVAL, "sector %d has no FP32 form: the FP32 plan is mixed", s);
      secs.push_back(s);
    }
    if (secs.empty() || gen_persistent_lookup(p, f32, p->K, secs)) {
      if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return QMC_OK;
    }
    Job j;
    j.d = 0;
    j.f32 = f32;
    j.spp = f32 ? 2 : 1;
    j.sectors = secs;
    j.name = gen_persistent_name(f32);
    j.src = gen_persistent_source(p, f32, j.spp, secs);
    jobs.push_back(std::move(j));
  }
  // every class for the shifts per pass of the current launch shape and of the shapes
  // the autotuner prefers (two and four), so that a change of shape keeps the
  // specialised kernels
  for (int D = 1; D <= QMC_MAX_DIM && !(flags & QMC_SPEC_PERSISTENT); ++D)
    for (int f32 = 0; f32 <= 1; ++f32) {
      const std::vector<int> secs = gen_class_sectors(p, D, f32 != 0);
      if (secs.empty()) continue;
      std::vector<int> spps;
      for (int spp : {p->spp, 2, 4}) {
        const int S = gen_spp_for(spp, D, f32 != 0);
        if (std::find(spps.begin(), spps.end(), S) == spps.end()) spps.push_back(S);
      }
      for (int S : spps) {
        bool have = false;
        for (const GenKernel &g : p->gen)
          have |= g.d == D && g.f32 == f32 && g.spp == S && g.sectors == secs;
        if (have) continue;
        Job j;
        j.d = D;
        j.f32 = f32;
        j.spp = S;
        j.sectors = secs;
        j.name = gen_kernel_name(D, f32 != 0, S);
        j.src = gen_class_source(p, D, f32 != 0, S, secs);
        jobs.push_back(std::move(j));
      }
    }
  // the classes compile concurrently (independent programs)
  std::vector<std::thread> th;
  for (Job &j : jobs) th.emplace_back([&j] { j.ok = gen_compile(j.src, j.name, j.code, j.err); });
  for (std::thread &t : th) t.join();
  for (Job &j : jobs)
    if (!j.ok) return fail(QMC_E_DEVICE, "compiling %s: %s", j.name.c_str(), j.err.c_str());
  if (!(flags & QMC_SPEC_COMPILE_ONLY)) {
    for (Job &j : jobs) {
      GenKernel g{};
      g.d = j.d;
      g.f32 = j.f32;
      g.spp = j.spp;
      g.persistent = j.d == 0;
      g.K = p->K;
      hipModule_t mod;
      hipFunction_t fn;
      int e = hipModuleLoadData(&mod, j.code.data());
      if (e != hipSuccess) return hip_fail(e, "load generated kernels");
      if ((e = hipModuleGetFunction(&fn, mod, j.name.c_str())) != hipSuccess) {
        (void)hipModuleUnload(mod);
        return hip_fail(e, "find generated kernel");
      }
      g.mod = mod;
      g.fn = fn;
      g.sectors = j.sectors;
      p->gen.push_back(g);
    }
  }
  if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return QMC_OK;
}

}  // extern "C"
