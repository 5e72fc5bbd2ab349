// qmc_flow.h -- device layout of a learned coupling-flow transform (one per sector).
// Not part of the C ABI.
#pragma once

#include <stdint.h>

#include "../../include/qmcamp.h"
#include "qmc_internal.h"

namespace qmc {

constexpr int kFlowLayers = QMC_FLOW_LAYERS;   // affine coupling layers
constexpr int kFlowHidden = QMC_FLOW_HIDDEN;   // hidden width of each layer's network
constexpr int kFlowIn = 16;                    // network input, padded (d + n_cond <= 16)
constexpr int kFlowOut = 16;                   // network output rows: s (d), t (d), zero rest
constexpr int kFlowMaxCond = QMC_FLOW_MAX_COND;

// Parameters of one coupling layer in the natural layout (float32), for d coordinates
// and c conditioning features (network input width d + c):
//   W1 [64][d + c], b1 [64], W2 [64][64], b2 [64], W3 [2d][64], b3 [2d]
__host__ __device__ constexpr int64_t flow_layer_params(int d, int c) {
  return (int64_t)kFlowHidden * (d + c) + kFlowHidden + kFlowHidden * kFlowHidden + kFlowHidden +
         2 * d * kFlowHidden + 2 * d;
}
__host__ __device__ constexpr int64_t flow_params(int d, int c) {
  return kFlowLayers * flow_layer_params(d, c);
}

// Offsets (in floats) of the blocks of layer l's parameters.
struct FlowParamOffsets {
  int64_t W1, b1, W2, b2, W3, b3;
};
__host__ __device__ inline FlowParamOffsets flow_offsets(int d, int c, int l) {
  FlowParamOffsets o;
  o.W1 = (int64_t)l * flow_layer_params(d, c);
  o.b1 = o.W1 + (int64_t)kFlowHidden * (d + c);
  o.W2 = o.b1 + kFlowHidden;
  o.b2 = o.W2 + kFlowHidden * kFlowHidden;
  o.W3 = o.b2 + kFlowHidden;
  o.b3 = o.W3 + 2 * d * kFlowHidden;
  return o;
}

// Packed bfloat16 A operands of the matrix-core products of one layer, in lane order
// (each lane's operand contiguous):
//   F1  W1      [rb 4][lane 64][4]        16x16x16: rows hidden, k = network inputs
//   F2  W2      [rb 4][ks 2][lane 64][8]  16x16x32: rows hidden, k = hidden (permuted)
//   F3  W3      [ks 2][lane 64][8]        16x16x32: rows outputs, k = hidden (permuted)
//   B3  W3^T    [rb 4][lane 64][4]        16x16x16: rows hidden, k = outputs
//   B2  W2^T    [rb 4][ks 2][lane 64][8]  16x16x32: rows hidden in, k = hidden out (permuted)
//   B1  W1^T    [ks 2][lane 64][8]        16x16x32: rows network inputs, k = hidden (permuted)
// The hidden index of k slot 8g + j (lane group g, element j) of k step ks is
//   32 ks + (j < 4 ? 4g + j : 16 + 4g + j - 4),
// exactly the hidden rows a lane of group g holds in the 16x16 result tiles of the
// previous product, so results feed the next product without leaving registers.
constexpr int kPackF1 = 0, kPackF2 = 1024, kPackF3 = 5120, kPackB3 = 6144, kPackB2 = 7168,
              kPackB1 = 11264, kPackLayer = 12288;   // bfloat16 elements

__host__ __device__ constexpr int flow_perm(int ks, int slot) {
  return 32 * ks + ((slot & 7) < 4 ? 4 * (slot >> 3) + (slot & 7) : 16 + 4 * (slot >> 3) + (slot & 7) - 4);
}

// Device state of one flow (caller-owned buffer of qmc_flow_bytes(d, c) bytes).
struct FlowHeader {
  int32_t d, step, n_cond;   // dimension, Adam steps taken, conditioning features
  int32_t pad[61];
};
__host__ __device__ inline int64_t flow_padded(int d, int c) {
  return 4 * ((flow_params(d, c) + 63) / 64 * 64);
}
__host__ __device__ inline int64_t flow_off_params(int, int) { return 256; }
__host__ __device__ inline int64_t flow_off_m(int d, int c) { return 256 + flow_padded(d, c); }
__host__ __device__ inline int64_t flow_off_v(int d, int c) { return flow_off_m(d, c) + flow_padded(d, c); }
__host__ __device__ inline int64_t flow_off_grad(int d, int c) { return flow_off_v(d, c) + flow_padded(d, c); }
__host__ __device__ inline int64_t flow_off_pack(int d, int c) { return flow_off_grad(d, c) + flow_padded(d, c); }
__host__ __device__ inline int64_t flow_total_bytes(int d, int c) {
  return flow_off_pack(d, c) + 2 * (int64_t)kFlowLayers * kPackLayer;
}

int launch_flow_pack(void *flow, int d, int c, void *stream);
int launch_flow_transform(const void *flow, int d, int c, const double *u, const double *cond,
                          int64_t count, double *x, double *logJ, int dir, void *stream);
int flow_grad_waves(int64_t count);
// inv_wsum: 1 / (sum of weights) when dev_wsum is NULL; else the weights are divided
// on the device by *dev_wsum and the result multiplied by inv_wsum (a batch's share).
int launch_flow_grad(void *flow, int d, int c, const double *x, const double *w,
                     const double *cond, int64_t count, int64_t offset, int64_t stride,
                     double inv_wsum, const double *dev_wsum, double *zs, float *gpart,
                     double *lpart, double *loss, void *stream);
// *out = sum of w[0 .. count) (one workgroup, fixed order)
int launch_flow_wsum(const double *w, int64_t count, double *out, void *stream);
int launch_flow_adam(void *flow, int d, int c, float lr, float b1, float b2, float eps, float c1,
                     float c2, void *stream);
int launch_flow_clear(float *p, int64_t count, void *stream);

// Training samples of one sector (see qmc_flow_samples); on the deformed contour (cplx)
// the weight is W |J f| over the orders of the complex integrand.
struct FlowSampleArgs {
  const SectorDev *sd;
  const double *coef;
  uint64_t n;
  double n_d, inv_n;
  uint64_t z[QMC_MAX_DIM];
  double shift[QMC_MAX_DIM];
  int K;
  int cplx;
  double *x, *w;
};
int launch_flow_samples(const FlowSampleArgs &fa, int d, void *stream);

}  // namespace qmc
