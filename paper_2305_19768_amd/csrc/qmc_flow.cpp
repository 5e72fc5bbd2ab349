// qmc_flow.cpp -- C ABI of the learned coupling-flow transform: state management,
// transform, training (gradient, Adam, epochs over QMC samples), training samples
// from a plan's sector, and attaching a flow to a sector of a plan.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "qmc_flow.h"
#include "qmc_plan.h"

using namespace qmc;

namespace qmc {
void plan_reorder(qmc_plan_s *p);
}  // namespace qmc

static bool dim_ok(int32_t d) { return d >= 1 && d <= QMC_MAX_DIM; }
static bool shape_ok(int32_t d, int32_t c) {
  return dim_ok(d) && c >= 0 && c <= kFlowMaxCond && d + c <= kFlowIn;
}
#define CHECK_SHAPE(d, c)                                                                     \
  if (!shape_ok(d, c))                                                                        \
    return fail(QMC_E_INVAL, "flow shape d = %d, n_cond = %d outside d in [1, %d], n_cond in " \
                             "[0, %d]", d, c, QMC_MAX_DIM, kFlowMaxCond);

extern "C" {

int64_t qmc_flow_param_count(int32_t d, int32_t n_cond) {
  return shape_ok(d, n_cond) ? flow_params(d, n_cond) : -1;
}

size_t qmc_flow_bytes(int32_t d, int32_t n_cond) {
  return shape_ok(d, n_cond) ? (size_t)flow_total_bytes(d, n_cond) : 0;
}

qmc_status qmc_flow_load(void *dev_flow, int32_t d, int32_t c, const float *params, void *stream) {
  g_last_error.clear();
  if (!dev_flow || !params) return fail(QMC_E_INVAL, "NULL argument");
  CHECK_SHAPE(d, c);
  if (((uintptr_t)dev_flow & 255) != 0) return fail(QMC_E_INVAL, "flow buffer not 256-byte aligned");
  const int64_t P = flow_params(d, c);
  for (int64_t k = 0; k < P; ++k)
    if (!std::isfinite(params[k])) return fail(QMC_E_INVAL, "parameter %lld not finite", (long long)k);
  hipStream_t st = (hipStream_t)stream;
  FlowHeader h;
  std::memset(&h, 0, sizeof h);
  h.d = d;
  h.n_cond = c;
  char *f = (char *)dev_flow;
  int e;
  if ((e = hipMemcpyAsync(f, &h, sizeof h, hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload flow header");
  if ((e = hipMemcpyAsync(f + flow_off_params(d, c), params, sizeof(float) * P,
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload flow parameters");
  // Adam moments and gradient: zero with a fill kernel (capturable, no memset nodes)
  if ((e = launch_flow_clear((float *)(f + flow_off_m(d, c)),
                             (flow_off_pack(d, c) - flow_off_m(d, c)) / 4, stream)) != hipSuccess)
    return hip_fail(e, "clear flow state");
  if ((e = launch_flow_pack(dev_flow, d, c, stream)) != hipSuccess) return hip_fail(e, "pack flow");
  // the header copy reads a stack object: finish before returning
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronize");
  return QMC_OK;
}

qmc_status qmc_flow_read(const void *dev_flow, int32_t d, int32_t c, float *params, float *grad,
                         void *stream) {
  g_last_error.clear();
  if (!dev_flow) return fail(QMC_E_INVAL, "NULL flow");
  CHECK_SHAPE(d, c);
  hipStream_t st = (hipStream_t)stream;
  const int64_t P = flow_params(d, c);
  const char *f = (const char *)dev_flow;
  int e;
  if (params && (e = hipMemcpyAsync(params, f + flow_off_params(d, c), sizeof(float) * P,
                                    hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(e, "read flow parameters");
  if (grad && (e = hipMemcpyAsync(grad, f + flow_off_grad(d, c), sizeof(float) * P,
                                  hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(e, "read flow gradient");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronize");
  return QMC_OK;
}

qmc_status qmc_flow_transform(const void *dev_flow, int32_t d, int32_t c, int32_t direction,
                              const double *dev_in, const double *dev_cond, int64_t count,
                              void *stream, double *dev_out, double *dev_logdet) {
  g_last_error.clear();
  if (!dev_flow || (count > 0 && (!dev_in || !dev_out || !dev_logdet || (c > 0 && !dev_cond))))
    return fail(QMC_E_INVAL, "NULL argument");
  CHECK_SHAPE(d, c);
  if (direction != QMC_FLOW_SAMPLE && direction != QMC_FLOW_DENSITY)
    return fail(QMC_E_INVAL, "unknown direction %d", direction);
  if (count < 0) return fail(QMC_E_INVAL, "count < 0");
  int e = launch_flow_transform(dev_flow, d, c, dev_in, dev_cond, count, dev_out, dev_logdet,
                                direction == QMC_FLOW_SAMPLE ? 0 : 1, stream);
  if (e != hipSuccess) return hip_fail(e, "flow transform launch");
  return QMC_OK;
}

size_t qmc_flow_scratch_bytes(int32_t d, int32_t c, int64_t count) {
  if (!shape_ok(d, c) || count < 1) return 0;
  const int64_t waves = flow_grad_waves(count);
  return align256(sizeof(double) * 8 * kFlowLayers * (size_t)count) +
         align256(sizeof(float) * (size_t)waves * flow_params(d, c)) +
         align256(sizeof(double) * (size_t)waves) + 256;
}

// Scratch layout of a gradient over `count` points: layer inputs, per-wavefront
// gradients, per-wavefront losses, then the on-device weight sum (one double).
static size_t wsum_offset(int32_t d, int32_t c, int64_t count) {
  const int64_t waves = flow_grad_waves(count);
  return align256(sizeof(double) * 8 * kFlowLayers * (size_t)count) +
         align256(sizeof(float) * (size_t)waves * flow_params(d, c)) +
         align256(sizeof(double) * (size_t)waves);
}

// gradient of L = -scale sum_i w_i log q(x_i) over samples offset + i * stride, where
// scale = inv_wsum, or inv_wsum / *dev_wsum when the weight sum is on the device
static qmc_status flow_gradient(void *dev_flow, int32_t d, int32_t c, const double *x,
                                const double *w, const double *cond, int64_t count,
                                int64_t offset, int64_t stride, double inv_wsum,
                                const double *dev_wsum, void *scratch, size_t bytes, void *stream,
                                double *dev_loss) {
  if (bytes < qmc_flow_scratch_bytes(d, c, count))
    return fail(QMC_E_NOMEM, "scratch of %zu bytes, %zu needed", bytes,
                qmc_flow_scratch_bytes(d, c, count));
  char *s = (char *)scratch;
  const int64_t waves = flow_grad_waves(count);
  double *zs = (double *)s;
  float *gpart = (float *)(s + align256(sizeof(double) * 8 * kFlowLayers * (size_t)count));
  double *lpart =
      (double *)((char *)gpart + align256(sizeof(float) * (size_t)waves * flow_params(d, c)));
  int e = launch_flow_grad(dev_flow, d, c, x, w, cond, count, offset, stride, inv_wsum, dev_wsum,
                           zs, gpart, lpart, dev_loss, stream);
  if (e != hipSuccess) return hip_fail(e, "flow gradient launch");
  return QMC_OK;
}

// w_sum > 0: the caller's normaliser; 0: the weights are summed on the device into the
// scratch's last slot (*dev_wsum set), with no host synchronisation.
static qmc_status weight_sum(int32_t d, int32_t c, int64_t per, const double *dev_w, int64_t count,
                             double w_sum, void *scratch, void *stream, const double **dev_wsum) {
  *dev_wsum = nullptr;
  if (w_sum > 0.0 && std::isfinite(w_sum)) return QMC_OK;
  if (w_sum != 0.0) return fail(QMC_E_INVAL, "w_sum must be > 0 (or 0: summed on the device)");
  double *slot = (double *)((char *)scratch + wsum_offset(d, c, per));
  int e = launch_flow_wsum(dev_w, count, slot, stream);
  if (e != hipSuccess) return hip_fail(e, "weight sum launch");
  *dev_wsum = slot;
  return QMC_OK;
}

qmc_status qmc_flow_gradient(void *dev_flow, int32_t d, int32_t c, const double *dev_x,
                             const double *dev_w, const double *dev_cond, int64_t count,
                             double w_sum, void *dev_scratch, size_t scratch_bytes, void *stream,
                             double *dev_loss) {
  g_last_error.clear();
  if (!dev_flow || !dev_x || !dev_w || !dev_scratch || (c > 0 && !dev_cond))
    return fail(QMC_E_INVAL, "NULL argument");
  CHECK_SHAPE(d, c);
  if (count < 1) return fail(QMC_E_INVAL, "count must be >= 1");
  if (!(w_sum >= 0.0) || !std::isfinite(w_sum))
    return fail(QMC_E_INVAL, "w_sum must be > 0 (or 0: summed on the device)");
  if (scratch_bytes < qmc_flow_scratch_bytes(d, c, count))
    return fail(QMC_E_NOMEM, "scratch of %zu bytes, %zu needed", scratch_bytes,
                qmc_flow_scratch_bytes(d, c, count));
  const double *dev_wsum;
  qmc_status st = weight_sum(d, c, count, dev_w, count, w_sum, dev_scratch, stream, &dev_wsum);
  if (st != QMC_OK) return st;
  return flow_gradient(dev_flow, d, c, dev_x, dev_w, dev_cond, count, 0, 1,
                       dev_wsum ? 1.0 : 1.0 / w_sum, dev_wsum, dev_scratch, scratch_bytes, stream,
                       dev_loss);
}

qmc_status qmc_flow_adam_step(void *dev_flow, int32_t d, int32_t c, const qmc_flow_adam *opt,
                              void *stream) {
  g_last_error.clear();
  if (!dev_flow || !opt) return fail(QMC_E_INVAL, "NULL argument");
  CHECK_SHAPE(d, c);
  if (!(opt->lr > 0.0f) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) ||
      !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) || !(opt->eps > 0.0f))
    return fail(QMC_E_INVAL, "Adam parameters out of range");
  if (opt->step < 1) return fail(QMC_E_INVAL, "step must be >= 1");
  const float c1 = 1.0f - std::pow(opt->beta1, (float)opt->step);
  const float c2 = 1.0f - std::pow(opt->beta2, (float)opt->step);
  int e = launch_flow_adam(dev_flow, d, c, opt->lr, opt->beta1, opt->beta2, opt->eps, c1, c2,
                           stream);
  if (e != hipSuccess) return hip_fail(e, "Adam launch");
  return QMC_OK;
}

qmc_status qmc_flow_train(void *dev_flow, int32_t d, int32_t c, const double *dev_x,
                          const double *dev_w, const double *dev_cond, int64_t count, double w_sum,
                          const qmc_flow_adam *opt, int32_t batches, int32_t epochs,
                          void *dev_scratch, size_t scratch_bytes, void *stream,
                          double *dev_loss_history) {
  g_last_error.clear();
  if (!dev_flow || !dev_x || !dev_w || !dev_scratch || !opt || (c > 0 && !dev_cond))
    return fail(QMC_E_INVAL, "NULL argument");
  CHECK_SHAPE(d, c);
  if (batches < 1 || epochs < 1 || count < batches)
    return fail(QMC_E_INVAL, "need 1 <= batches <= count and epochs >= 1");
  if (!(w_sum >= 0.0) || !std::isfinite(w_sum))
    return fail(QMC_E_INVAL, "w_sum must be > 0 (or 0: summed on the device)");
  // batch b holds samples b, b + batches, b + 2 batches, ...: lattice points in index
  // order fill the cube in slabs, so strided batches are spread over the whole cube
  const int64_t per = count / batches;
  if (scratch_bytes < qmc_flow_scratch_bytes(d, c, per))
    return fail(QMC_E_NOMEM, "scratch of %zu bytes, %zu needed", scratch_bytes,
                qmc_flow_scratch_bytes(d, c, per));
  const double *dev_wsum;
  qmc_status st0 = weight_sum(d, c, per, dev_w, count, w_sum, dev_scratch, stream, &dev_wsum);
  if (st0 != QMC_OK) return st0;
  // the batch's weights are normalised by the share of the total it should carry,
  // w_sum * per / count
  const double share = (double)count / (double)per;
  const double inv_b = dev_wsum ? share : share / w_sum;
  qmc_flow_adam a = *opt;
  int64_t t = 0;
  for (int32_t ep = 0; ep < epochs; ++ep)
    for (int32_t b = 0; b < batches; ++b, ++t) {
      qmc_status st = flow_gradient(dev_flow, d, c, dev_x, dev_w, dev_cond, per, b, batches,
                                    inv_b, dev_wsum, dev_scratch, scratch_bytes, stream,
                                    dev_loss_history ? dev_loss_history + t : nullptr);
      if (st != QMC_OK) return st;
      a.step = opt->step + (int32_t)t;
      if ((st = qmc_flow_adam_step(dev_flow, d, c, &a, stream)) != QMC_OK) return st;
    }
  return QMC_OK;
}

qmc_status qmc_flow_samples(qmc_plan_t p, int32_t sector, uint64_t n, uint64_t a, int32_t shift,
                            void *stream, double *dev_x, double *dev_w) {
  g_last_error.clear();
  if (!p || !dev_x || !dev_w) return fail(QMC_E_INVAL, "NULL argument");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  if (sector < 0 || sector >= p->S) return fail(QMC_E_INVAL, "sector %d out of range", sector);
  if (shift < 0 || shift >= p->m) return fail(QMC_E_INVAL, "shift %d out of range", shift);
  if (n < 2 || n >= (1ull << 53)) return fail(QMC_E_INVAL, "n outside [2, 2^53)");
  const int d = p->dims[sector];
  FlowSampleArgs fa;
  std::memset(&fa, 0, sizeof fa);
  fa.sd = (const SectorDev *)(p->ws + p->off_sec) + sector;
  fa.coef = (const double *)(p->ws + p->off_coef);
  fa.n = n;
  fa.n_d = (double)n;
  fa.inv_n = 1.0 / (double)n;
  uint64_t z = 1 % n;
  for (int j = 0; j < d; ++j) {
    if (gcd_u64(z, n) != 1) return fail(QMC_E_INVAL, "z_%d shares a factor with n", j + 1);
    fa.z[j] = z;
    z = mulmod_host(z, a % n, n);
  }
  for (int j = 0; j < d; ++j)
    fa.shift[j] = p->shifts[((size_t)sector * p->m + shift) * QMC_MAX_DIM + j];
  fa.K = p->K;
  fa.cplx = p->cplx;
  fa.x = dev_x;
  fa.w = dev_w;
  int e = launch_flow_samples(fa, d, stream);
  if (e != hipSuccess) return hip_fail(e, "flow samples launch");
  return QMC_OK;
}

qmc_status qmc_flow_attach(qmc_plan_t p, int32_t sector, const void *dev_flow, int32_t n_cond,
                           const double *cond, void *stream) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  if (!p->ws) return fail(QMC_E_STATE, "no workspace bound");
  if (sector < 0 || sector >= p->S) return fail(QMC_E_INVAL, "sector %d out of range", sector);
  if (dev_flow && ((uintptr_t)dev_flow & 255) != 0)
    return fail(QMC_E_INVAL, "flow buffer not 256-byte aligned");
  if (dev_flow) {
    CHECK_SHAPE(p->dims[sector], n_cond);
    if (n_cond > 0 && !cond) return fail(QMC_E_INVAL, "NULL conditioning features");
    for (int32_t k = 0; k < n_cond; ++k)
      if (!std::isfinite(cond[k])) return fail(QMC_E_INVAL, "conditioning feature %d not finite", k);
    // the kernels locate the operands from (d, n_cond): they must be the flow's own
    FlowHeader h;
    int e0 = hipMemcpyAsync(&h, dev_flow, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e0 == hipSuccess) e0 = hipStreamSynchronize((hipStream_t)stream);
    if (e0 != hipSuccess) return hip_fail(e0, "read flow header");
    if (h.d != p->dims[sector] || h.n_cond != n_cond)
      return fail(QMC_E_INVAL, "flow of shape (d = %d, n_cond = %d) attached as (%d, %d)", h.d,
                  h.n_cond, p->dims[sector], n_cond);
  }
  SectorDev &sd = p->sec[sector];
  sd.flow = (uint64_t)(uintptr_t)dev_flow;
  sd.flow_cond = dev_flow ? n_cond : 0;
  for (int k = 0; k < kFlowMaxCond; ++k) sd.cond[k] = (dev_flow && k < n_cond) ? cond[k] : 0.0;
  plan_reorder(p);
  p->cal_valid = false;   // the sector's integrand form changed
  hipStream_t st = (hipStream_t)stream;
  int e;
  if ((e = hipMemcpyAsync(p->ws + p->off_sec, p->sec.data(), sizeof(SectorDev) * p->S,
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload sectors");
  if ((e = hipMemcpyAsync(p->ws + p->off_order, p->order.data(), sizeof(int32_t) * p->S,
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "upload sector order");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "synchronize");
  p->lat_valid = false;
  return QMC_OK;
}

}  // extern "C"
