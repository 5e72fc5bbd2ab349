// qmc_amp.cpp -- adaptive evaluation of weighted sums of integrals (amplitudes).
//
// Implements the allocation of Sec. 2.1.3 of arXiv:2305.19768: each sector (the unit
// with its own lattice size n_s, cost tau_s and convergence constant w_s) is first
// sampled on a presample lattice; then every round forms the integrals, the weighted
// sums and their variances, and for every sum/order that misses its error bound
// chooses the sizes that minimise sum_s tau_s n_s subject to the target variance
// (Lagrange closed form), keeping the largest request per sector, never shrinking,
// rounding up to the table of available lattices.  Only sectors whose lattice changed
// are integrated again.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "qmc_plan.h"

using namespace qmc;

namespace {

struct Target {
  int t, k;
};

// Cost of one evaluation in the units of the dense polynomial work: the slots the
// nested Horner visits for U and F, the transform and the logarithm; an attached flow
// transform adds its four coupling networks, measured at 60-75 times a plain d = 6
// evaluation (about 230 units).
constexpr double kFlowCost = 16000.0;

double cost_model(const SectorDev &sd) {
  const int d = sd.d;
  auto slots = [d](int deg) {
    const double c1 = d, c2 = d * (d + 1) / 2.0, c3 = d * (d + 1) * (d + 2) / 6.0;
    return 1.0 + c1 + (deg >= 2 ? c2 : 0.0) + (deg >= 3 ? c3 : 0.0);
  };
  return slots(sd.u_deg) + slots(sd.f_deg) + 10.0 * d + ((sd.flags & SF_LOG) ? 40.0 : 0.0) +
         20.0 + (sd.flow ? kFlowCost : 0.0);
}

size_t ladder_ceil(const std::vector<uint64_t> &lad, double want, bool *limited) {
  for (size_t l = 0; l < lad.size(); ++l)
    if ((double)lad[l] >= want) return l;
  if (limited) *limited = true;
  return lad.size() - 1;
}

// Batched form: the rounds run on the device (round kernel, persistent integrand kernel
// over the plain sectors, a second one over the flow-transformed sectors, reduction,
// statistics); the host queues a few rounds at a time and only reads the state word
// between them.
qmc_status amp_device(qmc_plan_s *p, int T, int NI, int P, const std::vector<double> &cre,
                      const std::vector<double> &cim, const std::vector<double> &c2,
                      const std::vector<uint64_t> &lad, const qmc_amp_options *opt,
                      const std::vector<double> &tau, void *stream, double *value, double *error,
                      uint64_t *n_final, qmc_amp_stats *stats,
                      std::chrono::steady_clock::time_point t_start) {
  const int S = p->S, K = p->K;
  for (int s = 0; s < S; ++s)
    if (!p->sec[s].flow && !(p->sec[s].flags & SF_FAST))
      return fail(QMC_E_INVAL, "device mode evaluates sectors of the common shape only "
                               "(korobov3, integer powers of U and F, or a flow attached); "
                               "sector %d is not", s);
  if (T > kAmpMaxSums) return fail(QMC_E_INVAL, "device mode: at most %d sums", kAmpMaxSums);
  if ((int)lad.size() > kAmpMaxLattice)
    return fail(QMC_E_INVAL, "device mode: at most %d lattice sizes", kAmpMaxLattice);
  const bool f32 = p->precision == QMC_PREC_FP32;
  // workgroup order of the batched form: the sectors without a flow (for the persistent
  // kernel), then those with one (for the flow persistent kernel), each in plan order
  std::vector<int32_t> order_dev;
  order_dev.reserve(S);
  for (int q = 0; q < S; ++q)
    if (!p->sec[p->order[q]].flow) order_dev.push_back(p->order[q]);
  const int n_plain = (int)order_dev.size();
  for (int q = 0; q < S; ++q)
    if (p->sec[p->order[q]].flow) order_dev.push_back(p->order[q]);
  bool all_f32 = true;
  for (int s = 0; s < S; ++s)
    all_f32 = all_f32 && (p->sec[s].flow || (p->sec[s].flags & SF_F32OK));
  const int variant = !f32 ? kPersistentF64 : all_f32 ? kPersistentF32 : kPersistentF32Mixed;
  // the plan-specialised persistent kernel (qmc_specialize with QMC_SPEC_PERSISTENT), if
  // it was compiled for these sectors and orders
  std::vector<int> plain_secs;
  for (int s = 0; s < S; ++s)
    if (!p->sec[s].flow) plain_secs.push_back(s);
  GenKernel *gk = variant == kPersistentF32Mixed ? nullptr : gen_persistent_lookup(p, f32, K, plain_secs);
  int &grid = gk ? gk->grid : p->persistent_grid[variant];
  int e;
  if (!grid) {
    if (gk) {
      int dev = 0, cus = 0, per = 0;
      if ((e = hipGetDevice(&dev)) != hipSuccess ||
          (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
          (e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per, (hipFunction_t)gk->fn,
                                                                 p->block, 0)) != hipSuccess)
        return hip_fail(e, "occupancy query");
      grid = cus * (per > 0 ? per : 1);
    } else if ((e = persistent_grid(p->d_max, variant, K, p->block, &grid)) != hipSuccess) {
      return hip_fail(e, "occupancy query");
    }
  }
  int flow_grid = 0;
  if (n_plain < S && (e = persistent_flow_grid(p->block, &flow_grid)) != hipSuccess)
    return hip_fail(e, "occupancy query");
  // ---- device tables in the workspace
  char *base = p->ws + p->off_amp;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *at = base + o;
    o += align256(bytes);
    return at;
  };
  AmpState *dst = (AmpState *)take(sizeof(AmpState));
  int32_t *d_integral = (int32_t *)take(4 * S), *d_dims = (int32_t *)take(4 * S);
  int32_t *d_lidx = (int32_t *)take(4 * S), *d_active = (int32_t *)take(4 * S);
  int32_t *d_iptr = (int32_t *)take(4 * (NI + 1)), *d_isec = (int32_t *)take(4 * S);
  int32_t *d_order = (int32_t *)take(4 * S);
  double *d_want = (double *)take(8 * S), *d_tau = (double *)take(8 * S);
  double *d_tick_sum = (double *)take(8 * S), *d_eval_sum = (double *)take(8 * S);
  double *d_trace = (double *)take(8 * (size_t)S * QMC_AMP_TAU_ROWS);
  double *d_c2 = (double *)take(8 * kAmpMaxSums * NI * K);
  double *d_cre = (double *)take(8 * kAmpMaxSums * NI * K);
  double *d_cim = (double *)take(8 * kAmpMaxSums * NI * K);
  double *d_I = (double *)take(8 * NI * K), *d_VI = (double *)take(8 * NI * K);
  double *d_Are = (double *)take(8 * kAmpMaxSums * K), *d_Aim = (double *)take(8 * kAmpMaxSums * K);
  double *d_Vre = (double *)take(8 * kAmpMaxSums * K), *d_Vim = (double *)take(8 * kAmpMaxSums * K);
  int32_t *d_unmet = (int32_t *)take(4 * kAmpMaxSums * K);
  uint64_t *d_ln = (uint64_t *)take(8 * kAmpMaxLattice);
  uint64_t *d_la = (uint64_t *)take(8 * kAmpMaxLattice * QMC_MAX_DIM);
  if (o > p->amp_bytes) return fail(QMC_E_NOMEM, "amplitude region too small");
  std::vector<int32_t> integral(S), lidx(S);
  size_t l0 = lad.size() - 1;
  for (size_t l = 0; l < lad.size(); ++l)
    if ((double)lad[l] >= (double)std::max<uint64_t>(opt->n_presample, 2)) {
      l0 = l;
      break;
    }
  for (int s = 0; s < S; ++s) {
    integral[s] = p->sec[s].integral;
    lidx[s] = (int32_t)l0;
  }
  // sectors grouped by integral, ascending within each (the order of the sums)
  std::vector<int32_t> iptr(NI + 1, 0), isec(S);
  for (int s = 0; s < S; ++s) ++iptr[integral[s] + 1];
  for (int c = 0; c < NI; ++c) iptr[c + 1] += iptr[c];
  {
    std::vector<int32_t> fill(iptr.begin(), iptr.end() - 1);
    for (int s = 0; s < S; ++s) isec[fill[integral[s]]++] = s;
  }
  AmpState init;
  std::memset(&init, 0, sizeof init);
  hipStream_t st = (hipStream_t)stream;
  // every table goes up in one copy: a host image of the region (the tables at their
  // device offsets, zeros between and in the arrays the kernels write before they read),
  // in pinned memory kept by the plan, so that the copy is not staged or pinned per call
  // (the previous call's copy has finished: every call synchronises before it returns)
  if (p->amp_host_bytes < o) {
    if (p->amp_host) (void)hipHostFree(p->amp_host);
    p->amp_host = nullptr;
    p->amp_host_bytes = 0;
    if ((e = hipHostMalloc(&p->amp_host, o, hipHostMallocDefault)) != hipSuccess)
      return hip_fail(e, "pinned host image of the amplitude tables");
    p->amp_host_bytes = o;
  }
  char *image = (char *)p->amp_host;
  std::memset(image, 0, o);
  auto put = [&](void *dst_, const void *src, size_t bytes) {
    if (bytes) std::memcpy(image + ((char *)dst_ - base), src, bytes);
  };
  put(dst, &init, sizeof init);
  put(d_integral, integral.data(), 4 * S);
  put(d_dims, p->dims.data(), 4 * S);
  put(d_lidx, lidx.data(), 4 * S);
  put(d_iptr, iptr.data(), 4 * (NI + 1));
  put(d_isec, isec.data(), 4 * S);
  put(d_order, order_dev.data(), 4 * S);
  put(d_tau, tau.data(), 8 * S);
  put(d_c2, c2.data(), 8 * c2.size());
  put(d_cre, cre.data(), 8 * cre.size());
  put(d_cim, cim.data(), 8 * cim.size());
  put(d_ln, lad.data(), 8 * lad.size());
  put(d_trace, opt->tau_used,
      opt->tau_used ? 8 * (size_t)S * std::min(opt->max_rounds, QMC_AMP_TAU_ROWS) : 0);
  put(d_la, opt->lattice_a, 8 * lad.size() * QMC_MAX_DIM);
  if ((e = hipMemcpyAsync(base, image, o, hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload amplitude tables");
  AmpArgs g;
  std::memset(&g, 0, sizeof g);
  g.state = dst;
  g.S = S;
  g.K = K;
  g.T = T;
  g.NI = NI;
  g.m = p->m;
  g.tile = p->tile;
  g.block = p->block;
  g.n_lattice = (int32_t)lad.size();
  g.max_rounds = opt->max_rounds;
  g.P = P;
  g.epsrel = opt->epsrel;
  g.epsabs = opt->epsabs;
  g.alpha = opt->alpha;
  g.integral = d_integral;
  g.int_ptr = d_iptr;
  g.int_sec = d_isec;
  g.dims = d_dims;
  g.order = d_order;
  g.n_plain = n_plain;
  g.lidx = d_lidx;
  g.active = d_active;
  g.unmet = d_unmet;
  g.want = d_want;
  g.tau = d_tau;
  g.ticks = (unsigned long long *)(p->ws + p->off_ticks);
  g.tick_sum = d_tick_sum;
  g.eval_sum = d_eval_sum;
  g.measure_tau = opt->tau ? 0 : 1;
  g.tau_trace = opt->tau_used ? d_trace : nullptr;
  g.trace_rows = std::min(opt->max_rounds, QMC_AMP_TAU_ROWS);
  g.c2 = d_c2;
  g.cre = d_cre;
  g.cim = d_cim;
  g.I = d_I;
  g.VI = d_VI;
  g.Are = d_Are;
  g.Aim = d_Aim;
  g.Vre = d_Vre;
  g.Vim = d_Vim;
  g.mean = (const double *)(p->ws + p->off_mean);
  g.err = (const double *)(p->ws + p->off_err);
  g.lattice_n = d_ln;
  g.lattice_a = d_la;
  g.lat = (LatticeDev *)(p->ws + p->off_lat);
  g.block_begin = (int64_t *)(p->ws + p->off_begin);
  LaunchArgs la;
  std::memset(&la, 0, sizeof la);
  la.sectors = (const SectorDev *)(p->ws + p->off_sec);
  la.coef = (const double *)(p->ws + p->off_coef);
  la.coef32 = (const float *)(p->ws + p->off_coef32);
  la.shifts = (const double *)(p->ws + p->off_shift);
  la.lat = (const LatticeDev *)(p->ws + p->off_lat);
  la.block_begin = (const int64_t *)(p->ws + p->off_begin);
  la.order = d_order;
  la.partial = (double *)(p->ws + p->off_partial);
  la.q = (double *)(p->ws + p->off_q);
  la.mean = (double *)(p->ws + p->off_mean);
  la.err = (double *)(p->ws + p->off_err);
  la.status = (int32_t *)(p->ws + p->off_status);
  p->static_status = nullptr;   // qmc_query_status reads the workspace's status word
  p->static_sign = nullptr;
  la.n_sectors = S;
  la.m = p->m;
  la.K = K;
  la.shift_tile = p->tile;
  la.shifts_per_pass = 2;
  la.block = p->block;
  la.d_max = p->d_max;
  la.precision = p->precision;
  la.done = &dst->done;
  la.sector_ticks = g.ticks;
  if (f32) {   // the sectors' errors include the FP32 form's rounding bound
    if (!p->bound_in_ws) {
      if ((e = hipMemcpyAsync(p->ws + p->off_bound, p->f32_bound.data(),
                              sizeof(double) * p->f32_bound.size(), hipMemcpyHostToDevice, st)) !=
          hipSuccess)
        return hip_fail(e, "upload the FP32 bound");
      p->bound_in_ws = true;
    }
    la.f32_bound = (const double *)(p->ws + p->off_bound);
  }
  p->lat_valid = false;   // the device rewrites the lattice records
  if ((e = launch_status_reset(la.status, stream)) != hipSuccess) return hip_fail(e, "status reset");
  if ((e = launch_clear_u64(g.ticks, S, stream)) != hipSuccess) return hip_fail(e, "tick reset");
  AmpState hs;
  bool timed_out = false;
  for (;;) {
    for (int r = 0; r < 4; ++r) {   // queue a few rounds; finished rounds return at once
      if ((e = launch_amp_round(g, stream)) != hipSuccess) return hip_fail(e, "round kernel");
      if (gk) {
        LaunchArgs la_k = la;
        AmpState *st_k = dst;
        void *params[] = {&la_k, &st_k};
        e = hipModuleLaunchKernel((hipFunction_t)gk->fn, (unsigned)grid, 1, 1, (unsigned)p->block,
                                  1, 1, 0, st, params, nullptr);
      } else {
        e = launch_persistent(la, dst, p->d_max, variant, (unsigned)grid, stream);
      }
      if (e != hipSuccess) return hip_fail(e, "persistent kernel");
      if (n_plain < S &&
          (e = launch_persistent_flow(la, dst, (unsigned)flow_grid, stream)) != hipSuccess)
        return hip_fail(e, "flow persistent kernel");
      if ((e = launch_reduce_stats(la, stream)) != hipSuccess) return hip_fail(e, "reduction");
    }
    if ((e = launch_amp_round(g, stream)) != hipSuccess) return hip_fail(e, "round kernel");
    // the state and the status word in one synchronisation; a non-finite sum is then
    // reported by qmc_query_status
    int32_t code = 0;
    if ((e = hipMemcpyAsync(&hs, dst, sizeof hs, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(&code, la.status, sizeof code, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "read state");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronize");
    if (code != INT32_MAX) {
      qmc_status r = qmc_query_status(p, stream, nullptr, nullptr, nullptr);
      if (r != QMC_OK) return r;
    }
    if (hs.done) break;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (opt->timeout_s > 0.0 && secs >= opt->timeout_s) {
      timed_out = true;
      break;
    }
  }
  // the four result arrays are consecutive in the region: one copy
  std::vector<char> res((char *)d_Vim - (char *)d_Are + 8 * T * K);
  if ((e = hipMemcpyAsync(res.data(), d_Are, res.size(), hipMemcpyDeviceToHost, st)) ||
      (e = hipMemcpyAsync(lidx.data(), d_lidx, 4 * S, hipMemcpyDeviceToHost, st)))
    return hip_fail(e, "read results");
  // the trace rows the rounds could have written (the others still hold the caller's
  // values, uploaded at the start)
  const int rows = std::min<int>(hs.rounds, g.trace_rows);
  if (opt->tau_used && rows > 0 &&
      (e = hipMemcpyAsync(opt->tau_used, d_trace, 8 * (size_t)S * rows, hipMemcpyDeviceToHost,
                          st)) != hipSuccess)
    return hip_fail(e, "read costs");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "read results");
  auto result = [&](const double *at, int i) {
    double v;
    std::memcpy(&v, res.data() + ((const char *)at - (const char *)d_Are) + 8 * (size_t)i, 8);
    return v;
  };
  for (int i = 0; i < T * K; ++i) {
    value[2 * i] = result(d_Are, i);
    value[2 * i + 1] = result(d_Aim, i);
    error[2 * i] = std::sqrt(result(d_Vre, i));
    error[2 * i + 1] = std::sqrt(result(d_Vim, i));
  }
  if (n_final)
    for (int s = 0; s < S; ++s) n_final[s] = lad[lidx[s]];
  if (stats) {
    stats->rounds = hs.rounds;
    stats->converged = hs.done == 1;
    stats->timed_out = timed_out;
    stats->lattice_limited = hs.limited;
    stats->evaluations = hs.evaluations;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    stats->max_eps_rel = hs.max_eps;
  }
  if (timed_out)
    return fail(QMC_E_TIMEOUT, "stopped after the time limit with max relative error %.3g",
                hs.max_eps);
  return QMC_OK;
}

}  // namespace

extern "C" qmc_status amp_evaluate(qmc_plan_t p, const qmc_amplitude *amp,
                                   const qmc_amp_options *opt, void *stream, double *value,
                                   double *error, uint64_t *n_final, qmc_amp_stats *stats) {
  g_last_error.clear();
  const auto t_start = std::chrono::steady_clock::now();
  if (!p || !amp || !opt || !value || !error) return fail(QMC_E_INVAL, "NULL argument");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  if (p->cplx) return fail(QMC_E_INVAL, "amp_evaluate does not take complex (deformed) plans");
  const int S = p->S, K = p->K, m = p->m, NI = p->n_integrals;
  const int T = amp->n_sums;
  // ---- validate the sums
  if (T < 1 || !amp->row_ptr) return fail(QMC_E_INVAL, "n_sums must be >= 1 with row_ptr");
  if (amp->row_ptr[0] != 0) return fail(QMC_E_INVAL, "row_ptr[0] must be 0");
  for (int t = 0; t < T; ++t)
    if (amp->row_ptr[t + 1] < amp->row_ptr[t]) return fail(QMC_E_INVAL, "row_ptr not ascending");
  const int64_t nnz = amp->row_ptr[T];
  if (nnz > 0 && (!amp->col || !amp->coef_re)) return fail(QMC_E_INVAL, "missing coefficients");
  if (amp->n_terms < 0 || amp->n_terms > 64)
    return fail(QMC_E_INVAL, "n_terms = %d outside [0, 64]", amp->n_terms);
  if (amp->coef_order_lo < -1000 || amp->coef_order_lo > 1000)
    return fail(QMC_E_INVAL, "coef_order_lo = %d outside [-1000, 1000]", amp->coef_order_lo);
  const int Pin = amp->n_terms > 0 ? amp->n_terms : 1;
  const int P = std::min(Pin, K);   // term p reaches output order j >= p only
  for (int64_t e = 0; e < nnz; ++e) {
    if (amp->col[e] < 0 || amp->col[e] >= NI)
      return fail(QMC_E_INVAL, "coefficient %lld: integral %d outside [0, %d)", (long long)e,
                  amp->col[e], NI);
    for (int q = 0; q < Pin; ++q) {
      const double im = amp->coef_im ? amp->coef_im[e * Pin + q] : 0.0;
      if (!std::isfinite(amp->coef_re[e * Pin + q]) || !std::isfinite(im))
        return fail(QMC_E_INVAL, "coefficient %lld (term %d) is not finite", (long long)e, q);
    }
  }
  // ---- validate the options
  if (!(opt->epsrel >= 0.0) || !(opt->epsabs >= 0.0) || (opt->epsrel == 0.0 && opt->epsabs == 0.0))
    return fail(QMC_E_INVAL, "need epsrel >= 0, epsabs >= 0, not both 0");
  if (!(opt->alpha > 0.0) || !std::isfinite(opt->alpha)) return fail(QMC_E_INVAL, "alpha must be > 0");
  if (opt->max_rounds < 1) return fail(QMC_E_INVAL, "max_rounds must be >= 1");
  if (opt->mode != QMC_AMP_HOST && opt->mode != QMC_AMP_DEVICE)
    return fail(QMC_E_INVAL, "unknown mode %d", opt->mode);
  if (opt->n_lattice < 1 || !opt->lattice_n || !opt->lattice_a)
    return fail(QMC_E_INVAL, "a lattice table is required");
  std::vector<uint64_t> lad(opt->lattice_n, opt->lattice_n + opt->n_lattice);
  for (size_t l = 0; l < lad.size(); ++l) {
    if (lad[l] < 2 || lad[l] > p->n_max)
      return fail(QMC_E_INVAL, "lattice size %llu outside [2, n_max = %llu]",
                  (unsigned long long)lad[l], (unsigned long long)p->n_max);
    if (l && lad[l] <= lad[l - 1]) return fail(QMC_E_INVAL, "lattice sizes must ascend");
    for (int d = 1; d <= QMC_MAX_DIM; ++d) {
      bool used = false;
      for (int s = 0; s < S && !used; ++s) used = p->dims[s] == d;
      if (!used) continue;
      const uint64_t n = lad[l], a = opt->lattice_a[l * QMC_MAX_DIM + d - 1] % n;
      uint64_t z = 1 % n;
      for (int j = 0; j < d; ++j, z = mulmod_host(z, a, n))
        if (gcd_u64(z, n) != 1)
          return fail(QMC_E_INVAL, "lattice %llu, d = %d: a = %llu gives z_%d sharing a factor with n",
                      (unsigned long long)n, d, (unsigned long long)a, j + 1);
    }
  }
  std::vector<double> tau(S);
  for (int s = 0; s < S; ++s) {
    tau[s] = opt->tau ? opt->tau[s] : cost_model(p->sec[s]);
    if (!(tau[s] > 0.0) || !std::isfinite(tau[s])) return fail(QMC_E_INVAL, "tau[%d] must be > 0", s);
  }
  // coefficient terms c_p and |c_p|^2 of each integral in each sum, [T][NI][P]
  const size_t TNP = (size_t)T * NI * P;
  std::vector<double> c2(TNP, 0.0), cre(TNP, 0.0), cim(TNP, 0.0);
  for (int t = 0; t < T; ++t)
    for (int64_t e = amp->row_ptr[t]; e < amp->row_ptr[t + 1]; ++e)
      for (int q = 0; q < P; ++q) {
        const size_t at = ((size_t)t * NI + amp->col[e]) * P + q;
        cre[at] += amp->coef_re[e * Pin + q];
        cim[at] += amp->coef_im ? amp->coef_im[e * Pin + q] : 0.0;
      }
  for (size_t i = 0; i < c2.size(); ++i) c2[i] = cre[i] * cre[i] + cim[i] * cim[i];
  // FP32 plans: the rounding bound of the FP32 form, measured on the calibration lattice,
  // is a floor that no lattice size lowers.  A target below twice the floor the bound
  // sets for a sum (propagated like the errors, from the calibration estimates) is
  // refused before any work: such sums need the FP64 form.
  if (p->precision == QMC_PREC_FP32) {
    if (!p->cal_valid) {
      qmc_status r = fp32_calibrate(p, stream);
      if (r != QMC_OK) return r;
    }
    std::vector<double> Ic((size_t)NI * K, 0.0), B2((size_t)NI * K, 0.0);
    for (int s = 0; s < S; ++s)
      for (int k = 0; k < K; ++k) {
        const double b = p->f32_bound[(size_t)s * K + k];
        Ic[(size_t)p->sec[s].integral * K + k] += p->cal_mean[(size_t)s * K + k];
        B2[(size_t)p->sec[s].integral * K + k] += b * b;
      }
    for (int t = 0; t < T; ++t)
      for (int k = 0; k < K; ++k) {
        double re = 0.0, im = 0.0, fl2 = 0.0;
        for (int i = 0; i < NI; ++i)
          for (int q = 0; q < P && q <= k; ++q) {
            const size_t at = ((size_t)t * NI + i) * P + q;
            re += cre[at] * Ic[(size_t)i * K + k - q];
            im += cim[at] * Ic[(size_t)i * K + k - q];
            fl2 += c2[at] * B2[(size_t)i * K + k - q];
          }
        const double floor = std::sqrt(fl2);
        const double allowed = std::max(opt->epsrel * std::sqrt(re * re + im * im), opt->epsabs);
        if (floor > 0.0 && 2.0 * floor > allowed)
          return fail(QMC_E_INVAL,
                      "sum %d, order %d: the FP32 form's rounding bound (%.3g, relative %.3g) "
                      "exceeds half the requested error; evaluate in FP64", t, k, floor,
                      floor / std::sqrt(re * re + im * im));
      }
  }

  if (opt->mode == QMC_AMP_DEVICE)
    return amp_device(p, T, NI, P, cre, cim, c2, lad, opt, tau, stream, value, error, n_final,
                      stats, t_start);
  // measured costs: the integrand kernels add every workgroup's ticks to its sector
  const bool measure = opt->tau == nullptr;
  unsigned long long *dev_ticks = (unsigned long long *)(p->ws + p->off_ticks);
  std::vector<unsigned long long> ticks(S, 0);
  std::vector<double> tick_sum(S, 0.0), eval_sum(S, 0.0);
  struct TicksOff {   // the plan records ticks only inside this loop
    qmc_plan_s *p;
    ~TicksOff() { p->ticks_on = false; }
  } ticks_off{p};
  if (measure) {
    int e = launch_clear_u64(dev_ticks, S, stream);
    if (e != hipSuccess) return hip_fail(e, "tick reset");
    p->ticks_on = true;
  }
  // ---- presample
  bool limited = false;
  std::vector<size_t> lidx(S, ladder_ceil(lad, (double)std::max<uint64_t>(opt->n_presample, 2), &limited));
  std::vector<uint64_t> n(S), a(S);
  std::vector<uint8_t> active(S, 1);
  std::vector<double> mean((size_t)S * K), err((size_t)S * K);
  double *dev_mean = (double *)(p->ws + p->off_mean), *dev_err = (double *)(p->ws + p->off_err);
  hipStream_t st = (hipStream_t)stream;
  int64_t evals = 0;
  int rounds = 0;
  bool converged = false, timed_out = false;
  double max_eps = 0.0;
  std::vector<double> Are((size_t)T * K), Aim((size_t)T * K), Vre((size_t)T * K), Vim((size_t)T * K);
  qmc_status status = QMC_OK;
  for (;;) {
    for (int s = 0; s < S; ++s) {
      n[s] = lad[lidx[s]];
      a[s] = opt->lattice_a[lidx[s] * QMC_MAX_DIM + p->dims[s] - 1];
      if (active[s]) evals += (int64_t)n[s] * m;
    }
    qmc_status r = integrate_sectors(p, n.data(), a.data(), active.data(), stream, nullptr,
                                     dev_mean, dev_err);
    if (r != QMC_OK) return r;
    ++rounds;
    int e;
    if ((e = hipMemcpyAsync(mean.data(), dev_mean, sizeof(double) * mean.size(),
                            hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "read sector means");
    if ((e = hipMemcpyAsync(err.data(), dev_err, sizeof(double) * err.size(),
                            hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "read sector errors");
    if (measure) {
      if ((e = hipMemcpyAsync(ticks.data(), dev_ticks, sizeof(unsigned long long) * S,
                              hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "read sector ticks");
      if ((e = launch_clear_u64(dev_ticks, S, stream)) != hipSuccess) return hip_fail(e, "tick reset");
    }
    if ((r = qmc_query_status(p, stream, nullptr, nullptr, nullptr)) != QMC_OK) return r;
    if (measure)
      for (int s = 0; s < S; ++s) {
        if (active[s]) {
          tick_sum[s] += (double)ticks[s];
          eval_sum[s] += (double)n[s] * (double)m;
        }
        if (tick_sum[s] > 0.0) tau[s] = tick_sum[s] / eval_sum[s];
      }
    // ---- integrals and sums
    std::vector<double> I((size_t)NI * K, 0.0), VI((size_t)NI * K, 0.0);
    for (int s = 0; s < S; ++s)
      for (int k = 0; k < K; ++k) {
        I[(size_t)p->sec[s].integral * K + k] += mean[(size_t)s * K + k];
        VI[(size_t)p->sec[s].integral * K + k] += err[(size_t)s * K + k] * err[(size_t)s * K + k];
      }
    std::vector<Target> unmet;
    max_eps = 0.0;
    for (int t = 0; t < T; ++t)
      for (int k = 0; k < K; ++k) {
        double re = 0.0, im = 0.0, vre = 0.0, vim = 0.0;
        for (int i = 0; i < NI; ++i)
          for (int q = 0; q < P && q <= k; ++q) {
            const size_t at = ((size_t)t * NI + i) * P + q;
            const double cr = cre[at], ci = cim[at];
            const double v = I[(size_t)i * K + k - q], vv = VI[(size_t)i * K + k - q];
            re += cr * v;
            im += ci * v;
            vre += cr * cr * vv;
            vim += ci * ci * vv;
          }
        const size_t at = (size_t)t * K + k;
        Are[at] = re;
        Aim[at] = im;
        Vre[at] = vre;
        Vim[at] = vim;
        const double mag2 = re * re + im * im, var = vre + vim;
        const double eps = mag2 > 0.0 ? std::sqrt(var / mag2) : (var > 0.0 ? INFINITY : 0.0);
        max_eps = std::max(max_eps, eps);
        const bool ok = eps <= opt->epsrel || std::sqrt(var) <= opt->epsabs;
        if (!ok) unmet.push_back({t, k});
      }
    if (unmet.empty()) {
      converged = true;
      break;
    }
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (opt->timeout_s > 0.0 && secs >= opt->timeout_s) {
      timed_out = true;
      status = fail(QMC_E_TIMEOUT, "stopped after %.3f s with max relative error %.3g", secs,
                    max_eps);
      break;
    }
    if (rounds > opt->max_rounds) break;
    // ---- allocation (sequential over the unmet targets, largest request kept)
    if (opt->tau_used) std::memcpy(opt->tau_used + (size_t)(rounds - 1) * S, tau.data(), 8 * (size_t)S);
    const double al = opt->alpha;
    std::vector<double> want(S);
    for (int s = 0; s < S; ++s) want[s] = (double)n[s];
    for (const Target &tg : unmet) {
      const size_t at = (size_t)tg.t * K + tg.k;
      const double mag2 = Are[at] * Are[at] + Aim[at] * Aim[at];
      const double V = std::max(opt->epsrel * opt->epsrel * mag2, opt->epsabs * opt->epsabs);
      if (!(V > 0.0)) continue;
      // cw[s] = |C|^2 w_s of the closed form: sum over the coefficient terms reaching
      // this order of |c_p|^2 var_s,k-p n_s^alpha
      double sum = 0.0;
      std::vector<double> cw(S, 0.0);
      for (int s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int q = 0; q < P && q <= tg.k; ++q) {
          const double e = err[(size_t)s * K + tg.k - q];
          acc += c2[((size_t)tg.t * NI + p->sec[s].integral) * P + q] * e * e;
        }
        cw[s] = acc * std::pow((double)n[s], al);
        if (cw[s] > 0.0) sum += std::pow(cw[s] * std::pow(tau[s], al), 1.0 / (al + 1.0));
      }
      if (!(sum > 0.0)) continue;
      const double lam = (1.0 / al) * std::pow(sum / V, (al + 1.0) / al);
      for (int s = 0; s < S; ++s)
        if (cw[s] > 0.0)
          want[s] = std::max(want[s], std::pow(al * cw[s] * lam / tau[s], 1.0 / (al + 1.0)));
    }
    bool any = false;
    for (int s = 0; s < S; ++s) {
      const size_t l = std::max(lidx[s], ladder_ceil(lad, want[s], &limited));
      active[s] = l != lidx[s];
      any = any || active[s];
      lidx[s] = l;
    }
    if (!any) break;   // every sector that matters already sits on the largest lattice
  }
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < K; ++k) {
      const size_t at = (size_t)t * K + k;
      value[at * 2] = Are[at];
      value[at * 2 + 1] = Aim[at];
      error[at * 2] = std::sqrt(Vre[at]);
      error[at * 2 + 1] = std::sqrt(Vim[at]);
    }
  if (n_final)
    for (int s = 0; s < S; ++s) n_final[s] = lad[lidx[s]];
  if (stats) {
    stats->rounds = rounds;
    stats->converged = converged ? 1 : 0;
    stats->timed_out = timed_out ? 1 : 0;
    stats->lattice_limited = limited ? 1 : 0;
    stats->evaluations = evals;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    stats->max_eps_rel = max_eps;
  }
  return status;
}
