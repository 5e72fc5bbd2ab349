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
#include "qmc_device.h"

namespace qmc {

// One launch per sector dimension D: workgroup blockIdx.x + block_base of the launch's
// global workgroup numbering (workgroups are numbered sector by sector, sectors ordered
// by dimension, so a dimension's workgroups are contiguous).
// The FP64 fast form at d <= 4 is held to 128 registers (four waves per SIMD instead of
// three; a few registers spill): 1% faster on the two-loop workload.
template <int D, int K, int S, bool FAST, bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((D <= 4 && FAST && !F32) ? 4 : 1)))
void qmc_integrate_kernel(LaunchArgs a, int64_t block_base) {
  __shared__ double red[kMaxWaves][kMaxTile * 4][2];
  const BlockWork w = block_work(a, block_base);
  integrate_block<D, K, S, FAST, F32>(a, w.s, w.l_begin, w.tile, w.chunk_id, red);
  __syncthreads();
  block_store(a, w, red);
}

// Combine the workgroup partials of one (sector, shift) in workgroup order: one wave
// per (sector, shift), lanes stride over the sector's chunks, then a TwoSum butterfly.
__global__ __launch_bounds__(64) void qmc_reduce_kernel(LaunchArgs a) {
  if (a.done && *a.done) return;
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
        const int code = (s * a.m + l) * QMC_MAX_ORDERS + (a.cplx ? kk >> 1 : kk);
        atomicMin(a.status, code);
      }
    }
  }
}

// Shift mean and standard error per (sector, order).
__global__ void qmc_stats_kernel(LaunchArgs a) {
  if (a.done && *a.done) return;
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
  const double var = m > 1 ? (ss.s + ss.c) / (double)(m - 1) : 0.0;
  a.mean[idx] = mean;
  a.err[idx] = sqrt(var / (double)m) + (a.f32_bound ? a.f32_bound[idx] : 0.0);
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

template <int D, int S, bool FAST, bool F32>
static hipError_t launch_ds(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  dim3 grid((unsigned)dl.blocks), blk((unsigned)a.block);
  switch (a.K) {
    case 1: hipLaunchKernelGGL((qmc_integrate_kernel<D, 1, S, FAST, F32>), grid, blk, 0, st, a, dl.base); break;
    case 2: hipLaunchKernelGGL((qmc_integrate_kernel<D, 2, S, FAST, F32>), grid, blk, 0, st, a, dl.base); break;
    case 3: hipLaunchKernelGGL((qmc_integrate_kernel<D, 3, S, FAST, F32>), grid, blk, 0, st, a, dl.base); break;
    default: hipLaunchKernelGGL((qmc_integrate_kernel<D, 4, S, FAST, F32>), grid, blk, 0, st, a, dl.base); break;
  }
  return hipGetLastError();
}

// Sectors of the generic shape run one shift per pass (they are the uncommon case).
template <int D>
static hipError_t launch_d(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  if (!dl.fast) return launch_ds<D, 1, false, false>(a, dl, st);
  if (dl.f32) {
    if (a.shifts_per_pass == 1) return launch_ds<D, 1, true, true>(a, dl, st);
    return launch_ds<D, 2, true, true>(a, dl, st);   // FP32 kernels: 1 or 2 shifts per pass
  }
  // FP64 at d >= 7: one shift per pass whatever the shape asks (with two the lattice
  // state, both shifts' points and accumulators overflow the registers: spills and half
  // the occupancy); the sums are the same, shift by shift
  if (D >= 7) return launch_ds<D, 1, true, false>(a, dl, st);
  switch (a.shifts_per_pass) {
    case 1: return launch_ds<D, 1, true, false>(a, dl, st);
    case 4: return launch_ds<D, 4, true, false>(a, dl, st);
    default: return launch_ds<D, 2, true, false>(a, dl, st);
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

int launch_integrate(const LaunchArgs &a, void *stream, const SideStreams *side) {
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (a.ev_start && (e = hipEventRecord((hipEvent_t)a.ev_start, st)) != hipSuccess) return (int)e;
  // The per-dimension launches are independent (disjoint workgroup partials, atomic
  // status): the first runs on the caller's stream, the others round-robin on the side
  // streams, so that the tail of one launch overlaps the others instead of idling CUs.
  int active = 0;
  for (int t = 0; t < a.n_dim_launches; ++t) active += a.dims[t].blocks != 0;
  const int n_side = (side && active > 1) ? side->n : 0;
  if (n_side && (e = hipEventRecord((hipEvent_t)side->fork, st)) != hipSuccess) return (int)e;
  int k = 0, used = 0;
  for (int t = 0; t < a.n_dim_launches; ++t) {
    const DimLaunch &dl = a.dims[t];
    if (dl.blocks == 0) continue;
    hipStream_t ls = st;
    if (n_side && k > 0) {
      const int i = (k - 1) % n_side;
      if (i >= used) {
        if ((e = hipStreamWaitEvent((hipStream_t)side->stream[i], (hipEvent_t)side->fork, 0)) !=
            hipSuccess)
          return (int)e;
        used = i + 1;
      }
      ls = (hipStream_t)side->stream[i];
    }
    ++k;
    if (dl.gen) {
      // plan-specialised kernel of the class (same arguments as qmc_integrate_kernel)
      LaunchArgs args = a;
      int64_t base = dl.base;
      void *params[] = {&args, &base};
      e = hipModuleLaunchKernel((hipFunction_t)dl.gen, (unsigned)dl.blocks, 1, 1, (unsigned)a.block,
                                1, 1, 0, ls, params, nullptr);
    } else {
      e = dl.flow ? (hipError_t)launch_flow_integrate(a, dl, ls)
                  : dl.deform ? (hipError_t)launch_deform(a, dl, ls) : launch_class(a, dl, ls);
    }
    if (e != hipSuccess) return (int)e;
  }
  for (int i = 0; i < used; ++i) {
    if ((e = hipEventRecord((hipEvent_t)side->join[i], (hipStream_t)side->stream[i])) != hipSuccess ||
        (e = hipStreamWaitEvent(st, (hipEvent_t)side->join[i], 0)) != hipSuccess)
      return (int)e;
  }
  if (a.ev_stop && (e = hipEventRecord((hipEvent_t)a.ev_stop, st)) != hipSuccess) return (int)e;
  hipLaunchKernelGGL(qmc_reduce_kernel, dim3((unsigned)(a.n_sectors * a.m)), dim3(64), 0, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  const int nk = a.n_sectors * a.K;
  hipLaunchKernelGGL(qmc_stats_kernel, dim3((unsigned)((nk + 127) / 128)), dim3(128), 0, st, a);
  return (int)hipGetLastError();
}

int launch_reduce_stats(const LaunchArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(qmc_reduce_kernel, dim3((unsigned)(a.n_sectors * a.m)), dim3(64), 0, st, a);
  hipError_t e = hipGetLastError();
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
