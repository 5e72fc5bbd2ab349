// qmc_flow_kernels.hip -- learned coupling-flow variable transform on the matrix cores.
//
// A flow is a stack of kFlowLayers affine coupling layers in logit space of the unit
// cube; layer l conditions on the coordinates j with j % 2 == l % 2 and moves the
// others by z <- z exp(s) + t (density direction x -> u) or z <- (z - t) exp(-s)
// (sampling direction u -> x), with (s, t) from a d-64-64-2d network with tanh
// activations and s = 0.25 tanh(o_s).  The sampling direction replaces x = u after the
// periodizing transform, x = T(u), with weight J_T(u) = 1 / q(x).  Training maximises
// the weighted log-likelihood of QMC samples of the integrand (weights |W f|), which
// needs no derivative of the integrand.  A conditional flow appends c conditioning
// features (kinematic invariants of the sector) to every network input: (m_l z, cond).
//
// Matrix-core mapping: the points of a wavefront are the N dimension of every product,
// in four groups of 16 (bfloat16 16x16x16 and 16x16x32 products, float32 accumulation).
// A 16x16 result tile leaves lane (p, g) = (lane % 16, lane / 16) holding rows 4g..4g+3
// of column p; with the weight columns permuted at packing time (flow_perm), those
// registers are exactly the B operand of the next product, so the network runs from
// registers.  Only the network input and output pass through LDS, where each lane
// hands its point's coordinates to the lanes that feed them to the matrix core.
#include "qmc_deform.h"
#include "qmc_flow.h"

namespace qmc {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf_bits(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}

// tanh in float32, one formula for every argument: x P(x^2) / Q(x^2) with P, Q of degree
// 4 and P(0) = Q(0) = 1, the argument clamped to [-9, 9] (tanh(9) rounds to the largest
// float32 below 1).  The coefficients are a minimax fit on the relative error (csrc/fit_tanh.py:
// 2.1e-8 in exact arithmetic, below 3.5e-7 evaluated in float32 with one reciprocal).  One
// transcendental instruction per element and no divergent branch.  The results are rounded
// to bfloat16 (8 significant bits) before use.
__device__ __forceinline__ float tanh_f(float x) {
  const float c = __builtin_amdgcn_fmed3f(x, -9.0f, 9.0f);
  const float t = c * c;
  float p = 0x1.cd1634p-27f;
  p = __builtin_fmaf(p, t, 0x1.5aa224p-16f);
  p = __builtin_fmaf(p, t, 0x1.ca9e3ap-9f);
  p = __builtin_fmaf(p, t, 0x1.121a86p-3f);
  p = __builtin_fmaf(p, t, 1.0f);
  float q = 0x1.a300fcp-21f;
  q = __builtin_fmaf(q, t, 0x1.591658p-12f);
  q = __builtin_fmaf(q, t, 0x1.a82f1cp-6f);
  q = __builtin_fmaf(q, t, 0x1.de629p-2f);
  q = __builtin_fmaf(q, t, 1.0f);
  return (c * p) * __builtin_amdgcn_rcpf(q);
}

__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma32(v8b a, v8b b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Biases of one layer staged as float: b1 [64], b2 [64], b3 [16] (zero beyond 2d); read
// four at a time (16-byte aligned).
struct alignas(16) FlowBias {
  float b1[kFlowHidden], b2[kFlowHidden], b3[kFlowOut];
};

__device__ __forceinline__ void stage_bias(const char *flow, int d, int c, FlowBias *sb, int tid,
                                           int nt) {
  const float *P = (const float *)(flow + flow_off_params(d, c));
  for (int e = tid; e < kFlowLayers * (2 * kFlowHidden + kFlowOut); e += nt) {
    const int l = e / (2 * kFlowHidden + kFlowOut), r = e % (2 * kFlowHidden + kFlowOut);
    const FlowParamOffsets o = flow_offsets(d, c, l);
    float v;
    if (r < kFlowHidden) v = P[o.b1 + r];
    else if (r < 2 * kFlowHidden) v = P[o.b2 + r - kFlowHidden];
    else v = (r - 2 * kFlowHidden) < 2 * d ? P[o.b3 + r - 2 * kFlowHidden] : 0.0f;
    float *dst = &sb[l].b1[0];
    dst[r] = v;
  }
}

// The network of one layer for the 64 points of a wavefront.  zin: [64][16] bfloat16
// inputs (point-major, masked); pk: the layer's packed operands.  Returns the outputs
// o[q] (rows 4g..4g+3 of the 16 output rows, column p of point group q), and with KEEP
// the hidden activations h1, h2 [q][rb] (rows 16 rb + 4g + i).
template <bool KEEP>
__device__ __forceinline__ void flow_mlp(const unsigned short *pk, const FlowBias &bs,
                                         const unsigned short *zin, int lane, v4f (&o)[4],
                                         v4f (*h1)[4], v4f (*h2)[4]) {
  const int p = lane & 15, g = lane >> 4;
  // the biases enter as the accumulator operand of each layer's first product (the
  // rows 16 rb + 4 g + i of the lane's result tiles)
  v4s B1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) B1[q] = *(const v4s *)(zin + (16 * q + p) * kFlowIn + 4 * g);
  v4f C[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const v4s A = *(const v4s *)(pk + kPackF1 + (rb * 64 + lane) * 4);
    const v4f b = *(const v4f *)(bs.b1 + 16 * rb + 4 * g);
#pragma unroll
    for (int q = 0; q < 4; ++q) C[q][rb] = mfma16(A, B1[q], b);
  }
  v8b H[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = tanh_f(C[q][rb][i]);
        if (KEEP) h1[q][rb][i] = v;
        H[q][rb >> 1][(rb & 1) * 4 + i] = (__bf16)v;
      }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const v4f b = *(const v4f *)(bs.b2 + 16 * rb + 4 * g);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const v8b A = *(const v8b *)(pk + kPackF2 + ((rb * 2 + ks) * 64 + lane) * 8);
#pragma unroll
      for (int q = 0; q < 4; ++q) C[q][rb] = mfma32(A, H[q][ks], ks == 0 ? b : C[q][rb]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = tanh_f(C[q][rb][i]);
        if (KEEP) h2[q][rb][i] = v;
        H[q][rb >> 1][(rb & 1) * 4 + i] = (__bf16)v;
      }
  const v4f b3 = *(const v4f *)(bs.b3 + 4 * g);
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const v8b A = *(const v8b *)(pk + kPackF3 + (ks * 64 + lane) * 8);
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = mfma32(A, H[q][ks], ks == 0 ? b3 : o[q]);
  }
}

// Per-wave LDS exchange areas: network input (bfloat16) and output (float).
struct FlowXchg {
  unsigned short zin[64 * kFlowIn];
  float out[64 * kFlowOut];
};

// Per-wave LDS of the backward pass: output gradients (bfloat16, point-major) and two
// transposed tiles [feature][16 points] for the parameter products.
struct FlowBack {
  unsigned short gout[64 * kFlowOut];
  unsigned short ta[kFlowHidden * 16], tb[kFlowHidden * 16];
};

__device__ __forceinline__ bool conditioning(int j, int l) { return (j & 1) == (l & 1); }

// Orders the LDS exchanges of one wavefront, which stay within the wave's own FlowXchg /
// FlowBack area: a wave's LDS operations complete in issue order, so the lanes only need
// the compiler not to move accesses across this point (no workgroup barrier: the other
// waves of the workgroup run on independently).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One coupling layer applied to the lane's point (z in logit space, d coordinates),
// all lanes of the workgroup together.  dir 0: sampling (inverse affine), 1: density.
// Network input of layer l for the lane's point: the kept coordinates, then the c
// conditioning features, zero elsewhere.
template <int DMAX>
__device__ __forceinline__ void put_input(unsigned short *zin, const double (&z)[DMAX], int d, int c,
                                          const float (&cond)[kFlowMaxCond], int l) {
#pragma unroll
  for (int j = 0; j < kFlowIn; ++j) {
    unsigned short v = 0;
    if (j < d && j < DMAX && conditioning(j, l)) v = bf_bits((float)z[j < DMAX ? j : 0]);
    else if (j >= d && j < d + c) v = bf_bits(cond[(j - d) & (kFlowMaxCond - 1)]);
    zin[j] = v;
  }
}

// tanh of a float32 network output in FP64 from one exponential: with e = exp(-2|o|),
// tanh(o) = sign(o) (1 - e) / (1 + e).  The absolute error is a few units of 2^-53 (for
// small |o| the cancellation in 1 - e costs relative accuracy only); the flow uses
// s = tanh(o) / 4 as an exponent, where the absolute error is what matters.
__device__ __forceinline__ double tanh_out(float o) {
  const double e = exp(-2.0 * __builtin_fabs((double)o));
  const double th = (1.0 - e) / (1.0 + e);
  return o < 0.0f ? -th : th;
}

// The coupling moves each transformed coordinate by z <- (z - t) exp(-s) (dir 0) or
// z exp(s) + t (dir 1); ssum accumulates s and jac multiplies the factors exp(-+s)
// themselves (the Jacobian of the layer, exactly the factor the map applied).
template <int DMAX>
__device__ __forceinline__ void coupling(const unsigned short *pk, const FlowBias &bs,
                                         FlowXchg &xc, int d, int c, const float (&cond)[kFlowMaxCond],
                                         int l, int dir, int lane, double (&z)[DMAX],
                                         double &ssum, double &jac) {
  put_input<DMAX>(xc.zin + lane * kFlowIn, z, d, c, cond, l);
  wave_sync();
  v4f o[4];
  flow_mlp<false>(pk, bs, xc.zin, lane, o, nullptr, nullptr);
  const int p = lane & 15, g = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) xc.out[(16 * q + p) * kFlowOut + 4 * g + i] = o[q][i];
  wave_sync();
#pragma unroll
  for (int j = 0; j < DMAX; ++j) {
    if (j >= d || conditioning(j, l)) continue;
    const double s = 0.25 * tanh_out(xc.out[lane * kFlowOut + j]);
    const double t = (double)xc.out[lane * kFlowOut + d + j];
    const double e = exp(dir == 0 ? -s : s);
    z[j] = dir == 0 ? (z[j] - t) * e : __builtin_fma(z[j], e, t);
    ssum += s;
    jac *= e;
  }
  wave_sync();
}

// ------------------------------------------------------------------- packing

__global__ void flow_pack_kernel(char *flow, int d, int c) {
  const int l = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kPackLayer) return;
  const float *P = (const float *)(flow + flow_off_params(d, c));
  const FlowParamOffsets o = flow_offsets(d, c, l);
  const int din = d + c;   // network inputs
  float v = 0.0f;
  if (e < kPackF2) {                      // W1: rows hidden, k = inputs
    const int rb = e / 256, lane = (e / 4) % 64, el = e % 4;
    const int row = 16 * rb + lane % 16, k = 4 * (lane / 16) + el;
    v = k < din ? P[o.W1 + row * din + k] : 0.0f;
  } else if (e < kPackF3) {               // W2: rows hidden, k = hidden (permuted)
    const int t = e - kPackF2, rb = t / 1024, ks = (t / 512) % 2, lane = (t / 8) % 64, j = t % 8;
    const int row = 16 * rb + lane % 16, slot = 8 * (lane / 16) + j;
    v = P[o.W2 + row * kFlowHidden + flow_perm(ks, slot)];
  } else if (e < kPackB3) {               // W3: rows outputs, k = hidden (permuted)
    const int t = e - kPackF3, ks = t / 512, lane = (t / 8) % 64, j = t % 8;
    const int row = lane % 16, slot = 8 * (lane / 16) + j;
    v = row < 2 * d ? P[o.W3 + row * kFlowHidden + flow_perm(ks, slot)] : 0.0f;
  } else if (e < kPackB2) {               // W3^T: rows hidden, k = outputs
    const int t = e - kPackB3, rb = t / 256, lane = (t / 4) % 64, el = t % 4;
    const int row = 16 * rb + lane % 16, k = 4 * (lane / 16) + el;
    v = k < 2 * d ? P[o.W3 + k * kFlowHidden + row] : 0.0f;
  } else if (e < kPackB1) {               // W2^T: rows hidden in, k = hidden out (permuted)
    const int t = e - kPackB2, rb = t / 1024, ks = (t / 512) % 2, lane = (t / 8) % 64, j = t % 8;
    const int row = 16 * rb + lane % 16, slot = 8 * (lane / 16) + j;
    v = P[o.W2 + flow_perm(ks, slot) * kFlowHidden + row];
  } else {                                // W1^T: rows inputs, k = hidden (permuted)
    const int t = e - kPackB1, ks = t / 512, lane = (t / 8) % 64, j = t % 8;
    const int row = lane % 16, slot = 8 * (lane / 16) + j;
    v = row < din ? P[o.W1 + flow_perm(ks, slot) * din + row] : 0.0f;
  }
  ((unsigned short *)(flow + flow_off_pack(d, c)))[(int64_t)l * kPackLayer + e] = bf_bits(v);
}

// ----------------------------------------------------------- transform alone

// dir 0: u -> x = T(u) and log J_T(u); dir 1: x -> u = G(x) and log q(x).  Points with a
// coordinate outside (0, 1) get a NaN log-determinant.
__global__ __launch_bounds__(256) void flow_transform_kernel(const char *flow, int d, int c,
                                                             const double *in, const double *cond,
                                                             int64_t count, double *out,
                                                             double *logdet, int dir) {
  __shared__ FlowBias sb[kFlowLayers];
  __shared__ FlowXchg xc[4];
  stage_bias(flow, d, c, sb, threadIdx.x, blockDim.x);
  __syncthreads();
  const unsigned short *pk = (const unsigned short *)(flow + flow_off_pack(d, c));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < count;
  float cf[kFlowMaxCond];
#pragma unroll
  for (int k = 0; k < kFlowMaxCond; ++k) cf[k] = (valid && k < c) ? (float)cond[i * c + k] : 0.0f;
  double z[8], a[8];
  double lsum = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (valid && j < d) ? in[i * d + j] : 0.5;
    z[j] = 0.0;
    if (j < d) {   // logit and log(a (1 - a)) from the same two logarithms
      const double la = log(a[j]), lb = log(1.0 - a[j]);
      z[j] = la - lb;
      lsum += la + lb;
    }
  }
  double ssum = 0.0, jac = 1.0;
  for (int step = 0; step < kFlowLayers; ++step) {
    const int l = dir == 0 ? kFlowLayers - 1 - step : step;
    coupling<8>(pk + (int64_t)l * kPackLayer, sb[l], xc[wave], d, c, cf, l, dir, lane, z, ssum,
                jac);
  }
  double rsum = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j >= d) continue;
    const double r = 1.0 / (1.0 + exp(-z[j]));
    if (valid) out[i * d + j] = r;
    rsum += log(r * (1.0 - r));
  }
  if (valid) logdet[i] = dir == 0 ? rsum - lsum - ssum : rsum - lsum + ssum;
}

// ------------------------------------------------------------------- training

// Loss L = -sum_i w_i log q(x_i) * inv_wsum and its gradient for the points of this
// launch.  Every wavefront handles 64 points: the density direction forward (layer
// inputs kept in scratch), then the layers backwards with the network recomputed.
// Input gradients run through the packed transposed weights; parameter gradients are
// products over the points (K = 16 points of a group, bfloat16 tiles transposed through
// LDS).  Each wavefront writes its complete parameter gradient to its own slice of
// scratch, summed over wavefronts in a fixed order by flow_reduce_kernel.
struct FlowTrainArgs {
  char *flow;
  int d, c;                // coordinates, conditioning features
  const double *x, *w;
  const double *cond;      // [samples][c] or NULL
  int64_t count;     // points of this batch: sample index offset + i * stride
  int64_t offset, stride;
  double inv_wsum;
  double *zs;        // [L][count][8] layer inputs
  float *gpart;      // [waves][P] per-wavefront parameter gradients
  double *lpart;     // [waves] per-wavefront loss
};

// Sum over the 16 lanes of a lane group (same g, all p).
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Transposed tile of a result held in the 16x16 layout (rows 16 rb + 4g + i, point p).
__device__ __forceinline__ void put_tile(unsigned short *t, const v4f (&v)[4], int p, int g) {
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) t[(16 * rb + 4 * g + i) * 16 + p] = bf_bits(v[rb][i]);
}

__global__ __launch_bounds__(256) void flow_grad_kernel(FlowTrainArgs a) {
  __shared__ FlowBias sb[kFlowLayers];
  __shared__ FlowXchg xc[4];
  __shared__ FlowBack bk[4];
  const int d = a.d, c = a.c, din = d + c;
  stage_bias(a.flow, d, c, sb, threadIdx.x, blockDim.x);
  __syncthreads();
  const unsigned short *pk = (const unsigned short *)(a.flow + flow_off_pack(d, c));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15, g = lane >> 4;
  const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in_range = i < a.count;
  const int64_t gi = a.offset + i * a.stride;   // sample index
  const int64_t P = flow_params(d, c);
  FlowXchg &X = xc[wave];
  FlowBack &Bk = bk[wave];
  // a sample on (or rounded beyond) a face of the cube carries no weight
  double xs[8];
  bool inside = in_range;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xs[j] = (in_range && j < d) ? a.x[gi * d + j] : 0.5;
    if (j < d) inside = inside && xs[j] > 0.0 && xs[j] < 1.0;
  }
  const bool valid = inside;
  double wi = valid ? a.w[gi] * a.inv_wsum : 0.0;
  float cf[kFlowMaxCond];
#pragma unroll
  for (int k = 0; k < kFlowMaxCond; ++k) cf[k] = (in_range && k < c) ? (float)a.cond[gi * c + k] : 0.0f;

  // forward, density direction
  double z[8];
  double lx = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    z[j] = 0.0;
    if (j < d) {
      const double xj = valid ? xs[j] : 0.5;
      const double la = log(xj), lb = log(1.0 - xj);
      z[j] = la - lb;
      lx += la + lb;
    }
  }
  double ssum = 0.0, jac = 1.0;
  for (int l = 0; l < kFlowLayers; ++l) {
    if (valid)
#pragma unroll
      for (int j = 0; j < 8; ++j) a.zs[((int64_t)l * a.count + i) * 8 + j] = z[j];
    coupling<8>(pk + (int64_t)l * kPackLayer, sb[l], X, d, c, cf, l, 1, lane, z, ssum, jac);
  }
  double uu[8];
  bool u_in = true;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    uu[j] = 0.5;
    if (j >= d) continue;
    uu[j] = 1.0 / (1.0 + exp(-z[j]));
    u_in = u_in && uu[j] > 0.0 && uu[j] < 1.0;
  }
  // a sample whose image rounds onto a face of the cube carries no weight either
  if (!u_in) wi = 0.0;
  double dz[8], lu = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j < d && u_in) lu += log(uu[j] * (1.0 - uu[j]));
    dz[j] = j < d ? -wi * (1.0 - 2.0 * uu[j]) : 0.0;   // d/dz of -w log(u (1 - u))
  }
  double lq = (valid && u_in) ? -wi * (lu - lx + ssum) : 0.0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) lq += __shfl_xor(lq, o, 64);
  if (lane == 0) a.lpart[gw] = lq;

  float *G = a.gpart + gw * P;
  const v4f zero = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int l = kFlowLayers - 1; l >= 0; --l) {
    const unsigned short *pl = pk + (int64_t)l * kPackLayer;
    const FlowParamOffsets po = flow_offsets(d, c, l);
    double zl[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) zl[j] = valid ? a.zs[((int64_t)l * a.count + i) * 8 + j] : 0.0;
    put_input<8>(X.zin + lane * kFlowIn, zl, d, c, cf, l);
    wave_sync();
    v4f o[4], h1[4][4], h2[4][4];
    flow_mlp<true>(pl, sb[l], X.zin, lane, o, h1, h2);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) X.out[(16 * q + p) * kFlowOut + 4 * g + ii] = o[q][ii];
    wave_sync();
    // coupling backward on the lane's own point: gradient of the 2d network outputs
    float dof[kFlowOut];
#pragma unroll
    for (int r = 0; r < kFlowOut; ++r) dof[r] = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j >= d || conditioning(j, l)) continue;
      const double th = tanh_out(X.out[lane * kFlowOut + j]);
      const double es = exp(0.25 * th);
      const double ds = dz[j] * zl[j] * es - wi;       // log q carries + s
      dof[j] = (float)(ds * 0.25 * (1.0 - th * th));
      dof[d + j] = (float)dz[j];
      dz[j] *= es;
    }
#pragma unroll
    for (int r = 0; r < kFlowOut; ++r) Bk.gout[lane * kFlowOut + r] = bf_bits(dof[r]);
    // bias of the last product: sum over the wavefront's points
#pragma unroll
    for (int r = 0; r < kFlowOut; ++r) {
      float v = dof[r];
#pragma unroll
      for (int sft = 32; sft >= 1; sft >>= 1) v += __shfl_xor(v, sft, 64);
      if (lane == 0 && r < 2 * d) G[po.b3 + r] = v;
    }
    wave_sync();

    // dh2 = (W3^T do) (1 - h2^2)
    v4f dh[4][4];
    {
      v4s Bo[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) Bo[q] = *(const v4s *)(Bk.gout + (16 * q + p) * kFlowOut + 4 * g);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const v4s A = *(const v4s *)(pl + kPackB3 + (rb * 64 + lane) * 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) dh[q][rb] = mfma16(A, Bo[q], zero);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) dh[q][rb][ii] *= 1.0f - h2[q][rb][ii] * h2[q][rb][ii];
    // gW3 = sum_points do h2^T (rows: outputs, columns: hidden), then gb2
    {
      v4f acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = zero;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        put_tile(Bk.ta, h2[q], p, g);
        if (g == q)
#pragma unroll
          for (int r = 0; r < kFlowOut; ++r) Bk.tb[r * 16 + p] = Bk.gout[lane * kFlowOut + r];
        wave_sync();
        const v4s Ao = *(const v4s *)(Bk.tb + p * 16 + 4 * g);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[c] = mfma16(Ao, *(const v4s *)(Bk.ta + (16 * c + p) * 16 + 4 * g), acc[c]);
        wave_sync();
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
          if (4 * g + ii < 2 * d) G[po.W3 + (4 * g + ii) * kFlowHidden + 16 * c + p] = acc[c][ii];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          float v = 0.0f;
#pragma unroll
          for (int q = 0; q < 4; ++q) v += dh[q][rb][ii];
          v = group_sum(v);
          if (p == 0) G[po.b2 + 16 * rb + 4 * g + ii] = v;
        }
    }
    // dh1 = (W2^T dh2) (1 - h1^2)
    v4f dg[4][4];
    {
      v8b Hb[4][2];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) Hb[q][rb >> 1][(rb & 1) * 4 + ii] = (__bf16)dh[q][rb][ii];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) dg[q][rb] = zero;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const v8b A = *(const v8b *)(pl + kPackB2 + ((rb * 2 + ks) * 64 + lane) * 8);
#pragma unroll
          for (int q = 0; q < 4; ++q) dg[q][rb] = mfma32(A, Hb[q][ks], dg[q][rb]);
        }
    }
    // gW2 = sum_points dh2 h1^T (rows: hidden out, columns: hidden in)
    {
      v4f acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = zero;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        put_tile(Bk.ta, h1[q], p, g);
        put_tile(Bk.tb, dh[q], p, g);
        wave_sync();
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const v4s Bh = *(const v4s *)(Bk.ta + (16 * c + p) * 16 + 4 * g);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[r][c] = mfma16(*(const v4s *)(Bk.tb + (16 * r + p) * 16 + 4 * g), Bh, acc[r][c]);
        }
        wave_sync();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii)
            G[po.W2 + (16 * r + 4 * g + ii) * kFlowHidden + 16 * c + p] = acc[r][c][ii];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) dg[q][rb][ii] *= 1.0f - h1[q][rb][ii] * h1[q][rb][ii];
    // gb1, gW1 = sum_points dh1 v^T (columns: network inputs), dv = W1^T dh1
    {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          float v = 0.0f;
#pragma unroll
          for (int q = 0; q < 4; ++q) v += dg[q][rb][ii];
          v = group_sum(v);
          if (p == 0) G[po.b1 + 16 * rb + 4 * g + ii] = v;
        }
      v4f acc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = zero;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        put_tile(Bk.ta, dg[q], p, g);
        if (g == q)
#pragma unroll
          for (int r = 0; r < kFlowIn; ++r) Bk.tb[r * 16 + p] = X.zin[lane * kFlowIn + r];
        wave_sync();
        const v4s Bv = *(const v4s *)(Bk.tb + p * 16 + 4 * g);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[r] = mfma16(*(const v4s *)(Bk.ta + (16 * r + p) * 16 + 4 * g), Bv, acc[r]);
        wave_sync();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii)
          if (p < din) G[po.W1 + (16 * r + 4 * g + ii) * din + p] = acc[r][ii];
      v8b Hb[4][2];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) Hb[q][rb >> 1][(rb & 1) * 4 + ii] = (__bf16)dg[q][rb][ii];
      v4f dv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) dv[q] = zero;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const v8b A = *(const v8b *)(pl + kPackB1 + (ks * 64 + lane) * 8);
#pragma unroll
        for (int q = 0; q < 4; ++q) dv[q] = mfma32(A, Hb[q][ks], dv[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) X.out[(16 * q + p) * kFlowOut + 4 * g + ii] = dv[q][ii];
      wave_sync();
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < d && conditioning(j, l)) dz[j] += (double)X.out[lane * kFlowOut + j];
      wave_sync();
    }
  }
}

// grad[k] = sum over wavefronts of gpart[w][k] (fixed order); loss likewise.
// A workgroup of 256 takes 64 parameters; its four wavefronts sum the slices w = g,
// g + 4, ... (g = wavefront) for them, and the four partial sums are added in order g =
// 0..3.  The first workgroup also sums the loss over its 256 threads and a fixed tree.
// Every assignment is fixed, so the sums are deterministic.
// With wsum (device) set, the per-sample weights entered unnormalised and both sums are
// multiplied by scale / *wsum (0 when the weights sum to zero); else by scale.
constexpr int kReduceParams = 64;
__global__ __launch_bounds__(256) void flow_reduce_kernel(char *flow, int d, int c,
                                                          const float *gpart,
                                                          const double *lpart, int64_t waves,
                                                          double *loss, const double *wsum,
                                                          double scale) {
  __shared__ double part[4][kReduceParams];
  __shared__ double lp[256];
  if (wsum) scale = (*wsum > 0.0) ? scale / *wsum : 0.0;
  const int64_t P = flow_params(d, c);
  const int kk = threadIdx.x & (kReduceParams - 1), g = threadIdx.x / kReduceParams;
  const int64_t k = (int64_t)blockIdx.x * kReduceParams + kk;
  float *grad = (float *)(flow + flow_off_grad(d, c));
  double s = 0.0;
  if (k < P)
    for (int64_t w = g; w < waves; w += 4) s += (double)gpart[w * P + k];
  part[g][kk] = s;
  __syncthreads();
  if (g == 0 && k < P)
    grad[k] = (float)((((part[0][kk] + part[1][kk]) + part[2][kk]) + part[3][kk]) * scale);
  if (blockIdx.x == 0 && loss) {
    double t = 0.0;
    for (int64_t w = threadIdx.x; w < waves; w += 256) t += lpart[w];
    lp[threadIdx.x] = t;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) lp[threadIdx.x] += lp[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss = lp[0] * scale;
  }
}

// Sum of the training weights w[0 .. count) into *out: one workgroup; thread t sums
// the samples t, t + 256, ... with TwoSum compensation, then a fixed tree over the
// threads' (sum, compensation) pairs (deterministic).
__global__ __launch_bounds__(256) void flow_wsum_kernel(const double *w, int64_t count,
                                                        double *out) {
  __shared__ double ps[256], pc[256];
  DD acc{0.0, 0.0};
  for (int64_t i = threadIdx.x; i < count; i += 256) dd_add(acc, w[i]);
  ps[threadIdx.x] = acc.s;
  pc[threadIdx.x] = acc.c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const DD r = dd_combine(DD{ps[threadIdx.x], pc[threadIdx.x]},
                              DD{ps[threadIdx.x + o], pc[threadIdx.x + o]});
      ps[threadIdx.x] = r.s;
      pc[threadIdx.x] = r.c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = ps[0] + pc[0];
}

// Adam (Kingma and Ba 2015) on the float32 master parameters; c1, c2 are the bias
// corrections 1 - beta^t of this step.
__global__ void flow_adam_kernel(char *flow, int d, int c, float lr, float b1, float b2, float eps,
                                 float c1, float c2) {
  const int64_t P = flow_params(d, c);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  float *prm = (float *)(flow + flow_off_params(d, c));
  float *m = (float *)(flow + flow_off_m(d, c));
  float *v = (float *)(flow + flow_off_v(d, c));
  const float gk = ((const float *)(flow + flow_off_grad(d, c)))[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  prm[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void flow_clear_kernel(float *p, int64_t count) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) p[k] = 0.0f;
}

// ------------------------------------------------------- integration with a flow

// LDS of one workgroup of the flow-transformed integration: the forward operands of all
// layers (F1, F2, F3: the first kPackF3 + 1024 elements of each layer's pack), biases
// and the per-wave exchange areas.
constexpr int kPackFwd = kPackB3;   // forward part of a layer's pack
struct FlowIntegrateLds {
  unsigned short pack[kFlowLayers][kPackFwd];
  FlowBias bias[kFlowLayers];
  FlowXchg xc[4];
};

// A workgroup's share of a sector with an attached flow: per sample y, u = phi(y) with
// weight W (the sector's periodizing transform), x = T(u | cond) and J_T(u) by the flow,
// then the integrand at x; W J_T f accumulated as on the real contour.  A sample with a
// coordinate of u or x outside (0, 1) contributes 0.  CPLX: the integrand is the
// deformed-contour one, J f(z(x)) in FP64, accumulated as (re, im) columns, with the
// sign check counted as on the contour without a flow.  All QMC_MAX_ORDERS orders are
// formed (the tables are zero beyond the plan's); the first a.K columns are kept.
template <int D, bool CPLX>
__device__ __forceinline__ void flow_block(const LaunchArgs &a, int s, int l_begin, int tile,
                                           int64_t chunk_id, double (*red)[kMaxTile * 4][2],
                                           FlowIntegrateLds &L) {
  constexpr int NK = QMC_MAX_ORDERS;
  constexpr int KC = CPLX ? 2 * NK : NK;
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
  const int K = a.K;   // columns kept
  const int fc = sd->flow_cond;
  float cf[kFlowMaxCond];
#pragma unroll
  for (int k = 0; k < kFlowMaxCond; ++k) cf[k] = k < fc ? (float)sd->cond[k] : 0.0f;
  const double lam = sd->lambda;
  const int grad_off = sd->grad_off, hess_off = sd->hess_off;
  const uint64_t B = blockDim.x;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n_iter = (int64_t)((i_end - i_begin + B - 1) / B);
  double k0[D];
  const uint64_t i0 = i_begin + threadIdx.x;
#pragma unroll
  for (int j = 0; j < D; ++j) k0[j] = (double)mulmod(i0 % n, lt->z[j], n);
  uint32_t viol = 0;

#pragma unroll 1
  for (int l0 = 0; l0 < tile; ++l0) {
    DD acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = DD{0.0, 0.0};
    const double *__restrict__ sh = a.shifts + ((int64_t)s * a.m + l_begin + l0) * QMC_MAX_DIM;
    double k[D];
#pragma unroll
    for (int j = 0; j < D; ++j) k[j] = k0[j];
    uint64_t i = i0;
#pragma unroll 1
    for (int64_t it = 0; it < n_iter; ++it, i += B) {
      const cptr<double> cl = launder_uniform(a.coef);
      const cptr<LatticeDev> ltl = launder_uniform(lt);
      const cptr<double> shl = launder_uniform(sh);
      double y[D], u[D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double q = quotient(k[j], n_d, inv_n);
        k[j] = lattice_step(k[j], ltl->ndz[j], n_d);
        y[j] = shifted(q, shl[j]);
      }
      const double Wk = apply_transform<D>(kind, w_scale, y, u);
      // J_T(u) = prod_j x_j (1 - x_j) / (u_j (1 - u_j)) times the coupling factors; the two
      // products are kept as mantissa in [1/2, 1) and binary exponent (no underflow)
      bool inside = true;
      double z[D], mu = 1.0;
      int eu = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        inside = inside && u[j] > 0.0 && u[j] < 1.0;
        const double uj = (u[j] > 0.0 && u[j] < 1.0) ? u[j] : 0.5;
        z[j] = log(uj) - log(1.0 - uj);
        const double v = mu * (uj * (1.0 - uj));
        mu = __builtin_amdgcn_frexp_mant(v);
        eu += __builtin_amdgcn_frexp_exp(v);
      }
      double ssum = 0.0, jac = 1.0;
      for (int step = 0; step < kFlowLayers; ++step) {
        const int l = kFlowLayers - 1 - step;
        coupling<D>(L.pack[l], L.bias[l], L.xc[wave], D, fc, cf, l, 0, lane, z, ssum, jac);
      }
      double x[1][D], mx = 1.0;
      int ex = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double r = 1.0 / (1.0 + exp(-z[j]));
        inside = inside && r > 0.0 && r < 1.0;
        x[0][j] = (r > 0.0 && r < 1.0) ? r : 0.5;
        const double v = mx * (x[0][j] * (1.0 - x[0][j]));
        mx = __builtin_amdgcn_frexp_mant(v);
        ex += __builtin_amdgcn_frexp_exp(v);
      }
      const double W = Wk * __builtin_amdgcn_ldexp((mx / mu) * jac, ex - eu);
      const bool use = (i < i_end) && inside && (W != 0.0);
      if constexpr (CPLX) {
        C2 f[NK];
        const bool bad = integrand_deform<D, NK>(ss, (cptr<SectorDev>)sd, launder_after(cl, W),
                                                 grad_off, hess_off, lam, x[0], f);
        viol += (use && bad) ? 1u : 0u;
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
          dd_add(acc[2 * kk], use ? W * f[kk].r : 0.0);
          dd_add(acc[2 * kk + 1], use ? W * f[kk].i : 0.0);
        }
      } else {
        double f[1][NK];
        integrand<D, NK, 1>(ss, (cptr<SectorDev>)sd, launder_after(cl, W), x, f);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) dd_add(acc[kk], use ? W * f[0][kk] : 0.0);
      }
    }
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      if (c >= K) break;
      const DD r = wave_reduce(acc[c]);
      if (lane == 0) {
        red[wave][l0 * K + c][0] = r.s;
        red[wave][l0 * K + c][1] = r.c;
      }
    }
  }
  if constexpr (CPLX) {   // sign-check violations: one vector atomic per wave
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) viol += (uint32_t)__shfl_xor((int)viol, o, 64);
    if (lane == 0 && viol != 0) atomicAdd(a.sign_count + s, (unsigned long long)viol);
  }
}

// The forward operands and biases of sector s's flow, into the workgroup's LDS.
__device__ __forceinline__ void stage_flow(const LaunchArgs &a, int s, FlowIntegrateLds &L) {
  const char *flow = (const char *)a.sectors[s].flow;
  const int d = a.sectors[s].d, c = a.sectors[s].flow_cond;
  const uint4 *src = (const uint4 *)(flow + flow_off_pack(d, c));
  for (int l = 0; l < kFlowLayers; ++l) {
    const uint4 *sl = src + (int64_t)l * kPackLayer / 8;
    uint4 *dl = (uint4 *)L.pack[l];
    for (int e = threadIdx.x; e < kPackFwd / 8; e += blockDim.x) dl[e] = sl[e];
  }
  stage_bias(flow, d, c, L.bias, threadIdx.x, blockDim.x);
}

// Two waves per SIMD (256 registers, a few spilled at d >= 4): with one, every latency of
// the network's LDS exchanges, matrix products and transcendentals was exposed.
template <int D, bool CPLX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void qmc_flow_integrate_kernel(LaunchArgs a, int64_t block_base) {
  __shared__ double red[kMaxWaves][kMaxTile * 4][2];
  __shared__ FlowIntegrateLds L;
  const uint64_t t0 = ticks_now();
  const int64_t b = block_base + blockIdx.x;
  const int s = a.order[find_sector(a.block_begin, a.n_sectors, b)];
  const LatticeDev *__restrict__ lt = a.lat + s;
  stage_flow(a, s, L);
  __syncthreads();
  const int64_t local = b - lt->block_begin;
  const int nch = lt->n_chunks;
  const int tile_id = (int)(local / nch);
  const int64_t chunk_id = local - (int64_t)tile_id * nch;
  const int T = a.shift_tile;
  flow_block<D, CPLX>(a, s, tile_id * T, T, chunk_id, red, L);
  __syncthreads();
  const int nwaves = blockDim.x >> 6;
  const int cols = T * a.K;
  if ((int)threadIdx.x < cols) {
    DD r{red[0][threadIdx.x][0], red[0][threadIdx.x][1]};
    for (int w = 1; w < nwaves; ++w) r = dd_combine(r, DD{red[w][threadIdx.x][0], red[w][threadIdx.x][1]});
    double *out = a.partial + (b * cols + threadIdx.x) * 2;
    out[0] = r.s;
    out[1] = r.c;
  }
  ticks_add(a, s, t0);
}

// The batched form's flow-transformed sectors (real contour): the round's work items
// [plain_blocks, total_blocks) drained from their own atomic counter, one item per
// workgroup at a time; a workgroup restages the flow's operands only when its sector
// changes.  Every workgroup exits once the counter passes the round's total.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void qmc_persistent_flow_kernel(LaunchArgs a, AmpState *st) {
  __shared__ double red[kMaxWaves][kMaxTile * 4][2];
  __shared__ FlowIntegrateLds L;
  __shared__ int64_t item;
  __shared__ int staged;
  if (st->done) return;
  const int64_t begin = st->plain_blocks, total = st->total_blocks;
  if (threadIdx.x == 0) staged = -1;
  const int T = a.shift_tile;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item = begin + (int64_t)atomicAdd(&st->flow_counter, 1u);
    __syncthreads();
    const int64_t b = item;
    if (b >= total) break;
    const uint64_t t0 = ticks_now();
    const int s = a.order[find_sector(a.block_begin, a.n_sectors, b)];
    if (s != staged) {
      stage_flow(a, s, L);
      __syncthreads();
      if (threadIdx.x == 0) staged = s;
    }
    const LatticeDev *__restrict__ lt = a.lat + s;
    const int64_t local = b - lt->block_begin;
    const int nch = lt->n_chunks;
    const int tile_id = (int)(local / nch);
    const int64_t chunk_id = local - (int64_t)tile_id * nch;
    switch (a.sectors[s].d) {
      case 1: flow_block<1, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
      case 2: flow_block<2, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
      case 3: flow_block<3, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
      case 4: flow_block<4, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
      case 5: flow_block<5, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
      case 6: flow_block<6, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
      case 7: flow_block<7, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
      default: flow_block<8, false>(a, s, tile_id * T, T, chunk_id, red, L); break;
    }
    __syncthreads();
    const int nwaves = blockDim.x >> 6;
    const int cols = T * a.K;
    if ((int)threadIdx.x < cols) {
      DD r{red[0][threadIdx.x][0], red[0][threadIdx.x][1]};
      for (int w = 1; w < nwaves; ++w) r = dd_combine(r, DD{red[w][threadIdx.x][0], red[w][threadIdx.x][1]});
      double *out = a.partial + (b * cols + threadIdx.x) * 2;
      out[0] = r.s;
      out[1] = r.c;
    }
    ticks_add(a, s, t0);
  }
}

// Training samples of one sector: x_i = phi(y_i) for the points of lattice (n, z) with
// one shift, and weights w_i = W(y_i) ||f(x_i)||_2 over the orders (0 where W = 0); on
// the deformed contour f is J f(z(x)) and the norm runs over real and imaginary parts.
template <int D>
__global__ __launch_bounds__(256) void qmc_flow_samples_kernel(FlowSampleArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const SectorScalars ss = load_scalars(a.sd);
  double y[D], x[1][D];
#pragma unroll
  for (int j = 0; j < D; ++j)
    y[j] = shifted(quotient((double)mulmod(i, a.z[j], a.n), a.n_d, a.inv_n), a.shift[j]);
  const double W = apply_transform<D>(a.sd->transform, a.sd->w_scale, y, x[0]);
  double nrm = 0.0;
  const cptr<double> cl = launder_after(launder_uniform(a.coef), W);
  if (a.cplx) {
    C2 f[QMC_MAX_ORDERS];
    integrand_deform<D, QMC_MAX_ORDERS>(ss, (cptr<SectorDev>)a.sd, cl, a.sd->grad_off,
                                        a.sd->hess_off, a.sd->lambda, x[0], f);
#pragma unroll
    for (int k = 0; k < QMC_MAX_ORDERS; ++k)
      if (k < a.K) nrm = __builtin_fma(f[k].r, f[k].r, __builtin_fma(f[k].i, f[k].i, nrm));
  } else {
    double f[1][QMC_MAX_ORDERS];
    integrand<D, QMC_MAX_ORDERS, 1>(ss, (cptr<SectorDev>)a.sd, cl, x, f);
#pragma unroll
    for (int k = 0; k < QMC_MAX_ORDERS; ++k)
      if (k < a.K) nrm = __builtin_fma(f[0][k], f[0][k], nrm);
  }
  const double wi = W != 0.0 ? W * sqrt(nrm) : 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) a.x[i * D + j] = x[0][j];
  a.w[i] = isfinite(wi) ? wi : 0.0;
}

template <bool CPLX>
static void launch_flow_integrate_p(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  dim3 grid((unsigned)dl.blocks), blk((unsigned)a.block);
  switch (dl.d) {
    case 1: hipLaunchKernelGGL((qmc_flow_integrate_kernel<1, CPLX>), grid, blk, 0, st, a, dl.base); break;
    case 2: hipLaunchKernelGGL((qmc_flow_integrate_kernel<2, CPLX>), grid, blk, 0, st, a, dl.base); break;
    case 3: hipLaunchKernelGGL((qmc_flow_integrate_kernel<3, CPLX>), grid, blk, 0, st, a, dl.base); break;
    case 4: hipLaunchKernelGGL((qmc_flow_integrate_kernel<4, CPLX>), grid, blk, 0, st, a, dl.base); break;
    case 5: hipLaunchKernelGGL((qmc_flow_integrate_kernel<5, CPLX>), grid, blk, 0, st, a, dl.base); break;
    case 6: hipLaunchKernelGGL((qmc_flow_integrate_kernel<6, CPLX>), grid, blk, 0, st, a, dl.base); break;
    case 7: hipLaunchKernelGGL((qmc_flow_integrate_kernel<7, CPLX>), grid, blk, 0, st, a, dl.base); break;
    default: hipLaunchKernelGGL((qmc_flow_integrate_kernel<8, CPLX>), grid, blk, 0, st, a, dl.base); break;
  }
}

int launch_persistent_flow(const LaunchArgs &a, AmpState *st, unsigned grid, void *stream) {
  hipLaunchKernelGGL(qmc_persistent_flow_kernel, dim3(grid), dim3(a.block), 0,
                     (hipStream_t)stream, a, st);
  return (int)hipGetLastError();
}

int persistent_flow_grid(int block, int *grid) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)qmc_persistent_flow_kernel,
                                                   block, 0);
  if (e != hipSuccess) return (int)e;
  *grid = cus * (per > 0 ? per : 1);
  return 0;
}

int launch_flow_integrate(const LaunchArgs &a, const DimLaunch &dl, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dl.deform) launch_flow_integrate_p<true>(a, dl, st);
  else launch_flow_integrate_p<false>(a, dl, st);
  return (int)hipGetLastError();
}

int launch_flow_samples(const FlowSampleArgs &fa, int d, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  dim3 grid((unsigned)((fa.n + 255) / 256)), blk(256);
  switch (d) {
    case 1: hipLaunchKernelGGL(qmc_flow_samples_kernel<1>, grid, blk, 0, st, fa); break;
    case 2: hipLaunchKernelGGL(qmc_flow_samples_kernel<2>, grid, blk, 0, st, fa); break;
    case 3: hipLaunchKernelGGL(qmc_flow_samples_kernel<3>, grid, blk, 0, st, fa); break;
    case 4: hipLaunchKernelGGL(qmc_flow_samples_kernel<4>, grid, blk, 0, st, fa); break;
    case 5: hipLaunchKernelGGL(qmc_flow_samples_kernel<5>, grid, blk, 0, st, fa); break;
    case 6: hipLaunchKernelGGL(qmc_flow_samples_kernel<6>, grid, blk, 0, st, fa); break;
    case 7: hipLaunchKernelGGL(qmc_flow_samples_kernel<7>, grid, blk, 0, st, fa); break;
    default: hipLaunchKernelGGL(qmc_flow_samples_kernel<8>, grid, blk, 0, st, fa); break;
  }
  return (int)hipGetLastError();
}

// ------------------------------------------------------------------ launchers

int launch_flow_pack(void *flow, int d, int c, void *stream) {
  hipLaunchKernelGGL(flow_pack_kernel, dim3((kPackLayer + 255) / 256, kFlowLayers), dim3(256), 0,
                     (hipStream_t)stream, (char *)flow, d, c);
  return (int)hipGetLastError();
}

int launch_flow_transform(const void *flow, int d, int c, const double *u, const double *cond,
                          int64_t count, double *x, double *logJ, int dir, void *stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(flow_transform_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, (const char *)flow, d, c, u, cond, count, x, logJ, dir);
  return (int)hipGetLastError();
}

int flow_grad_waves(int64_t count) { return (int)((count + 255) / 256) * 4; }

int launch_flow_wsum(const double *w, int64_t count, double *out, void *stream) {
  hipLaunchKernelGGL(flow_wsum_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, w, count, out);
  return (int)hipGetLastError();
}

int launch_flow_grad(void *flow, int d, int c, const double *x, const double *w,
                     const double *cond, int64_t count, int64_t offset, int64_t stride,
                     double inv_wsum, const double *dev_wsum, double *zs, float *gpart,
                     double *lpart, double *loss, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  // with a device weight sum the kernel takes the raw weights and the reduction scales
  FlowTrainArgs a{(char *)flow, d, c, x, w, cond, count, offset, stride,
                  dev_wsum ? 1.0 : inv_wsum, zs, gpart, lpart};
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(flow_grad_kernel, dim3(blocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  const int64_t P = flow_params(d, c);
  hipLaunchKernelGGL(flow_reduce_kernel, dim3((unsigned)((P + kReduceParams - 1) / kReduceParams)),
                     dim3(256), 0, st,
                     (char *)flow, d, c, (const float *)gpart, (const double *)lpart,
                     (int64_t)blocks * 4, loss, dev_wsum, dev_wsum ? inv_wsum : 1.0);
  return (int)hipGetLastError();
}

int launch_flow_adam(void *flow, int d, int c, float lr, float b1, float b2, float eps, float c1,
                     float c2, void *stream) {
  const int64_t P = flow_params(d, c);
  hipLaunchKernelGGL(flow_adam_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, (char *)flow, d, c, lr, b1, b2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  return launch_flow_pack(flow, d, c, stream);
}

int launch_flow_clear(float *p, int64_t count, void *stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(flow_clear_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, p, count);
  return (int)hipGetLastError();
}

}  // namespace qmc
