// qmc_deform_kernels.hip -- complex integrand on a deformed integration contour.
//
// For kinematics where F changes sign on the unit cube the integral is taken with the
// F - i0 prescription on the contour
//   z_j(x) = x_j - i lambda x_j (1 - x_j) g_j(x),   g = grad F at real x,
// with Jacobian det(dz/dx) and the integrand continued analytically to z.  The
// deformation parameter is chosen from presamples (the paper's library call,
// Sec. 3.1.3).  Per sample, in FP64:
//   lattice point and transform   as on the real contour (shared device helpers)
//   g_j, H_jk                     dense Horner over per-sector derivative tables of F
//   det(dz/dx)                    dz/dx = I - i lambda (D1 + D2 H), D1 = diag((1-2x) g),
//                                 D2 = diag(x(1-x)); with S = D2^(1/2) it is similar to
//                                 the complex symmetric I - i lambda (D1 + S H S), whose
//                                 Hermitian part is I, so Gaussian elimination needs no
//                                 pivoting: a symmetric LDL^T on the lower triangle
//   U(z), F(z)                    nested Horner with complex variables, real coefficients
//   x^p U^a F^b (log F)^m         complex powers; log F = log|F| + i arg F with
//                                 arg F in [-pi, pi) (F - i0); half-integer powers of F
//                                 on the same branch
//   sign check                    Im F(z) > 2^-40 |F(z)| counts as a violation
// The (re, im) parts of every order are accumulated as two real columns, so the
// workgroup partials, the per-sector reduction and the statistics are those of the
// real contour with 2 K columns.
#include "qmc_deform.h"

namespace qmc {

// One workgroup's share of a sector on the deformed contour: the loop structure of
// the real-contour block (one shift per pass), with 2 K accumulator columns.
template <int D, bool F32, int NK>
__device__ __forceinline__ void deform_block(const LaunchArgs &a, int s, int l_begin, int tile,
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
  const double lam = sd->lambda;
  const int grad_off = sd->grad_off, hess_off = sd->hess_off;
  const SectorScalars ss = load_scalars(sd);
  constexpr int KC = 2 * NK;   // (re, im) columns of the NK orders
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
    int64_t it = 0;
#pragma unroll 1
    while (it < n_iter) {
      double part[KC];
#pragma unroll
      for (int c = 0; c < KC; ++c) part[c] = 0.0;
      const int64_t it_end = (n_iter - it < kFold) ? n_iter : it + kFold;
#pragma unroll 1
      for (; it < it_end; ++it, i += B) {
        const cptr<LatticeDev> ltl = launder_uniform(lt);
        const cptr<double> shl = launder_uniform(sh);
        double y[D], x[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const double q = quotient(k[j], n_d, inv_n);
          k[j] = lattice_step(k[j], ltl->ndz[j], n_d);
          asm volatile("" : "+v"(k[j]));
          y[j] = shifted(q, shl[j]);
        }
        const double W = apply_transform<D>(kind, w_scale, y, x);
        C2 f[NK];
        bool bad;
        if (F32) {
          const cptr<float> cl32 = launder_uniform(a.coef32);
          bad = integrand_deform_f32<D, NK>(ss, (cptr<SectorDev>)sd, launder_after_f(cl32, (float)W),
                                        grad_off, hess_off, lam, x, f);
        } else {
          const cptr<double> cl = launder_uniform(a.coef);
          bad = integrand_deform<D, NK>(ss, (cptr<SectorDev>)sd, launder_after(cl, W), grad_off,
                                    hess_off, lam, x, f);
        }
        const bool use = (i < i_end) && (W != 0.0);
        viol += (use && bad) ? 1u : 0u;
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
          part[2 * kk] += use ? W * f[kk].r : 0.0;
          part[2 * kk + 1] += use ? W * f[kk].i : 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < KC; ++c) dd_add(acc[c], part[c]);
    }
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const DD r = wave_reduce(acc[c]);
      if (lane == 0) {
        red[wave][l0 * KC + c][0] = r.s;
        red[wave][l0 * KC + c][1] = r.c;
      }
    }
  }
  // sign-check violations of this workgroup's samples: one vector atomic per wave
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) viol += (uint32_t)__shfl_xor((int)viol, o, 64);
  if (lane == 0 && viol != 0) atomicAdd(a.sign_count + s, (unsigned long long)viol);
}

template <int D, bool F32, int NK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void qmc_deform_kernel(LaunchArgs a, int64_t block_base) {
  __shared__ double red[kMaxWaves][kMaxTile * 4][2];
  const int64_t b = block_base + blockIdx.x;
  const int s = a.order[find_sector(a.block_begin, a.n_sectors, b)];
  const LatticeDev *__restrict__ lt = a.lat + s;
  const int64_t local = b - lt->block_begin;
  const int nch = lt->n_chunks;
  const int tile_id = (int)(local / nch);
  const int64_t chunk_id = local - (int64_t)tile_id * nch;
  const int T = a.shift_tile;
  deform_block<D, F32, NK>(a, s, tile_id * T, T, chunk_id, red);
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
}

__global__ void qmc_clear_u64_kernel(unsigned long long *p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

template <int D, bool F32>
static void launch_deform_k(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  dim3 grid((unsigned)dl.blocks), blk((unsigned)a.block);
  switch (a.K / 2) {
    case 1: hipLaunchKernelGGL((qmc_deform_kernel<D, F32, 1>), grid, blk, 0, st, a, dl.base); break;
    case 2: hipLaunchKernelGGL((qmc_deform_kernel<D, F32, 2>), grid, blk, 0, st, a, dl.base); break;
    case 3: hipLaunchKernelGGL((qmc_deform_kernel<D, F32, 3>), grid, blk, 0, st, a, dl.base); break;
    default: hipLaunchKernelGGL((qmc_deform_kernel<D, F32, 4>), grid, blk, 0, st, a, dl.base); break;
  }
}

template <bool F32>
static void launch_deform_p(const LaunchArgs &a, const DimLaunch &dl, hipStream_t st) {
  switch (dl.d) {
    case 1: launch_deform_k<1, F32>(a, dl, st); break;
    case 2: launch_deform_k<2, F32>(a, dl, st); break;
    case 3: launch_deform_k<3, F32>(a, dl, st); break;
    case 4: launch_deform_k<4, F32>(a, dl, st); break;
    case 5: launch_deform_k<5, F32>(a, dl, st); break;
    case 6: launch_deform_k<6, F32>(a, dl, st); break;
    case 7: launch_deform_k<7, F32>(a, dl, st); break;
    default: launch_deform_k<8, F32>(a, dl, st); break;
  }
}

int launch_deform(const LaunchArgs &a, const DimLaunch &dl, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dl.f32) launch_deform_p<true>(a, dl, st);
  else launch_deform_p<false>(a, dl, st);
  return (int)hipGetLastError();
}

int launch_clear_u64(unsigned long long *p, int64_t count, void *stream) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(qmc_clear_u64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, p, count);
  return (int)hipGetLastError();
}

}  // namespace qmc
