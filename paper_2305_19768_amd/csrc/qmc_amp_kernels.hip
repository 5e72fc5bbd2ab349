// qmc_amp_kernels.hip -- device-resident adaptive evaluation of weighted sums of
// integrals (the batched form of amp_evaluate): a single-workgroup round kernel that
// forms integrals, sums and errors, decides convergence and computes the next lattice
// sizes with the closed form of Sec. 2.1.3 of arXiv:2305.19768 (same reading as the
// host loop), and a persistent integrand kernel that drains the round's work items
// (sector, chunk, shift tile) of every dimension from one atomic counter.  Every kernel
// of a round returns at once when the state says the evaluation is finished, so the
// host can queue several rounds and synchronise once.
#include "qmc_persist.h"

namespace qmc {

// ------------------------------------------------------------ round kernel

constexpr int kRoundThreads = 256;

__device__ __forceinline__ double block_sum_ordered(double v, double *sh) {
  // deterministic: fixed thread -> slot assignment, fixed pairwise tree
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = kRoundThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] = sh[t] + sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Exclusive prefix sum over the workgroup (exact integers); *total gets the sum.
__device__ __forceinline__ int64_t block_scan_excl(int64_t v, int64_t *sh, int64_t *total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kRoundThreads; off <<= 1) {
    const int64_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int64_t incl = sh[t];
  *total = sh[kRoundThreads - 1];
  __syncthreads();
  return incl - v;
}

__device__ __forceinline__ int block_or(int v, int *sh) {
  if (threadIdx.x == 0) *sh = 0;
  __syncthreads();
  if (v) atomicOr(sh, 1);
  __syncthreads();
  const int r = *sh;
  __syncthreads();
  return r;
}

// Lattice record of sector s on table entry l (validity was checked on the host).
__device__ void set_lattice(const AmpArgs &g, int s, int l) {
  LatticeDev &L = g.lat[s];
  const uint64_t n = g.lattice_n[l];
  const uint64_t a = g.lattice_a[l * QMC_MAX_DIM + g.dims[s] - 1] % n;
  L.n = n;
  L.n_d = (double)n;
  L.inv_n = 1.0 / (double)n;
  uint64_t z = 1 % n;
  for (int j = 0; j < QMC_MAX_DIM; ++j) {
    if (j < g.dims[s]) {
      L.z[j] = z;
      L.dz[j] = mulmod((uint64_t)g.block % n, z, n);
      L.ndz[j] = (double)(n - L.dz[j]);
    } else {
      L.z[j] = 0;
      L.dz[j] = 0;
      L.ndz[j] = 0.0;
    }
    z = mulmod(z, a, n);
  }
  L.active = 1;
}

// |C|^2 w_s of the closed form for target (sum tt, order k): the coefficient terms that
// reach order k, each with the variance of the order it multiplies, times n_s^alpha.
__device__ double amp_cw(const AmpArgs &g, int tt, int k, int s, double al) {
  double acc = 0.0;
  for (int q = 0; q < g.P && q <= k; ++q) {
    const double e = g.err[s * g.K + k - q];
    acc += g.c2[(tt * g.NI + g.integral[s]) * g.P + q] * e * e;
  }
  return acc * pow((double)g.lattice_n[g.lidx[s]], al);
}

__global__ __launch_bounds__(kRoundThreads) void qmc_amp_round_kernel(AmpArgs g) {
  AmpState *st = g.state;
  if (st->done) return;
  __shared__ double shd[kRoundThreads];
  __shared__ int64_t shl[kRoundThreads];
  __shared__ int shi;
  const int t = threadIdx.x;
  const int S = g.S, K = g.K, T = g.T, NI = g.NI;

  if (st->rounds > 0) {
    // ---- costs: the ticks of the round just integrated join the running sums; a
    // sector's cost is its ticks per evaluation so far (the prior until it has any)
    for (int s = t; s < S; s += kRoundThreads) {
      if (g.measure_tau) {
        if (g.active[s]) {
          g.tick_sum[s] += (double)g.ticks[s];
          g.eval_sum[s] += (double)g.lattice_n[g.lidx[s]] * (double)g.m;
        }
        if (g.tick_sum[s] > 0.0) g.tau[s] = g.tick_sum[s] / g.eval_sum[s];
      }
      g.ticks[s] = 0;
    }
    __syncthreads();
    // ---- integrals (sum of sectors, variances added) and sums, in a fixed order
    for (int idx = t; idx < NI * K; idx += kRoundThreads) {
      const int c = idx / K, k = idx - c * K;
      double v = 0.0, var = 0.0;
      for (int r = g.int_ptr[c]; r < g.int_ptr[c + 1]; ++r) {   // its sectors, ascending
        const int s = g.int_sec[r];
        v += g.mean[s * K + k];
        var += g.err[s * K + k] * g.err[s * K + k];
      }
      g.I[idx] = v;
      g.VI[idx] = var;
    }
    __syncthreads();
    int unmet_any = 0;
    double eps_max = 0.0;
    for (int idx = t; idx < T * K; idx += kRoundThreads) {
      const int tt = idx / K, k = idx - tt * K;
      double re = 0.0, im = 0.0, vre = 0.0, vim = 0.0;
      for (int i = 0; i < NI; ++i)
        for (int q = 0; q < g.P && q <= k; ++q) {
          const int at = (tt * NI + i) * g.P + q;
          const double cr = g.cre[at], ci = g.cim[at];
          const double v = g.I[i * K + k - q], vv = g.VI[i * K + k - q];
          re += cr * v;
          im += ci * v;
          vre += cr * cr * vv;
          vim += ci * ci * vv;
        }
      g.Are[idx] = re;
      g.Aim[idx] = im;
      g.Vre[idx] = vre;
      g.Vim[idx] = vim;
      const double mag2 = re * re + im * im, var = vre + vim;
      const double eps = mag2 > 0.0 ? sqrt(var / mag2) : (var > 0.0 ? __builtin_inf() : 0.0);
      eps_max = fmax(eps_max, eps);
      const int ok = (eps <= g.epsrel) || (sqrt(var) <= g.epsabs);
      g.unmet[idx] = !ok;
      unmet_any |= !ok;
    }
    const int any = block_or(unmet_any, &shi);
    // max eps over threads (order-independent)
    shd[t] = eps_max;
    __syncthreads();
    for (int w = kRoundThreads / 2; w > 0; w >>= 1) {
      if (t < w) shd[t] = fmax(shd[t], shd[t + w]);
      __syncthreads();
    }
    if (t == 0) st->max_eps = shd[0];
    __syncthreads();
    if (!any) {
      if (t == 0) st->done = 1;
      return;
    }
    if (st->rounds > g.max_rounds) {
      if (t == 0) st->done = 2;
      return;
    }
    // ---- allocation: unmet targets in order, largest request per sector kept
    const int row = st->rounds - 1;   // the costs this allocation uses
    if (g.tau_trace && row < g.trace_rows)
      for (int s = t; s < S; s += kRoundThreads) g.tau_trace[(int64_t)row * S + s] = g.tau[s];
    const double al = g.alpha;
    for (int s = t; s < S; s += kRoundThreads) g.want[s] = (double)g.lattice_n[g.lidx[s]];
    __syncthreads();
    for (int idx = 0; idx < T * K; ++idx) {
      if (!g.unmet[idx]) continue;   // uniform
      const int tt = idx / K, k = idx - tt * K;
      const double mag2 = g.Are[idx] * g.Are[idx] + g.Aim[idx] * g.Aim[idx];
      const double V = fmax(g.epsrel * g.epsrel * mag2, g.epsabs * g.epsabs);
      if (!(V > 0.0)) continue;
      double part = 0.0;
      for (int s = t; s < S; s += kRoundThreads) {
        const double cw = amp_cw(g, tt, k, s, al);
        if (cw > 0.0) part += pow(cw * pow(g.tau[s], al), 1.0 / (al + 1.0));
      }
      const double sum = block_sum_ordered(part, shd);
      if (!(sum > 0.0)) continue;
      const double lam = (1.0 / al) * pow(sum / V, (al + 1.0) / al);
      for (int s = t; s < S; s += kRoundThreads) {
        const double cw = amp_cw(g, tt, k, s, al);
        if (cw > 0.0) g.want[s] = fmax(g.want[s], pow(al * cw * lam / g.tau[s], 1.0 / (al + 1.0)));
      }
      __syncthreads();
    }
    // ---- round up to the table, never shrink
    int act_any = 0, lim_any = 0;
    for (int s = t; s < S; s += kRoundThreads) {
      int l = g.n_lattice - 1;
      bool found = false;
      for (int q = 0; q < g.n_lattice; ++q)
        if ((double)g.lattice_n[q] >= g.want[s]) {
          l = q;
          found = true;
          break;
        }
      if (!found) lim_any = 1;
      if (l < g.lidx[s]) l = g.lidx[s];
      const int act = l != g.lidx[s];
      g.active[s] = act;
      g.lidx[s] = l;
      act_any |= act;
    }
    const int any_act = block_or(act_any, &shi);
    const int lim = block_or(lim_any, &shi);
    if (t == 0 && lim) st->limited = 1;
    if (!any_act) {
      if (t == 0) st->done = 3;
      return;
    }
  } else {
    for (int s = t; s < S; s += kRoundThreads) g.active[s] = 1;   // presample: every sector
    __syncthreads();
  }
  // ---- lattice records of the active sectors, chunking and workgroup table
  double pts = 0.0;
  for (int s = t; s < S; s += kRoundThreads) {
    if (g.active[s]) {
      set_lattice(g, s, g.lidx[s]);
      pts += (double)g.lattice_n[g.lidx[s]];
    } else {
      g.lat[s].active = 0;
      g.lat[s].n_chunks = 0;
    }
  }
  const double total_pts = block_sum_ordered(pts, shd);
  const int tiles = g.m / g.tile;
  const double per_block = (double)kTargetBlocksDevice * g.block;
  int64_t ppt = (int64_t)ceil(total_pts * tiles / per_block);
  if (ppt < 1) ppt = 1;
  const int64_t chunk = ppt * g.block;
  // each thread takes a contiguous run of the workgroup order; an exclusive scan of the
  // runs' workgroup counts places every sector's range
  const int run = (S + kRoundThreads - 1) / kRoundThreads;
  const int q0 = min(S, t * run), q1 = min(S, q0 + run);
  int64_t nb = 0, ev = 0;
  for (int q = q0; q < q1; ++q) {
    const int s = g.order[q];
    if (g.active[s]) {
      const int64_t n = (int64_t)g.lat[s].n;
      nb += (n + chunk - 1) / chunk * tiles;
      ev += n * g.m;
    }
  }
  int64_t total_b, total_ev;
  int64_t b = block_scan_excl(nb, shl, &total_b);
  block_scan_excl(ev, shl, &total_ev);
  for (int q = q0; q < q1; ++q) {
    const int s = g.order[q];
    LatticeDev &L = g.lat[s];
    L.chunk = chunk;
    L.n_chunks = g.active[s] ? (int32_t)((L.n + chunk - 1) / chunk) : 0;
    L.block_begin = b;
    g.block_begin[q] = b;
    if (q == g.n_plain) st->plain_blocks = b;
    b += (int64_t)L.n_chunks * tiles;
  }
  if (t == 0) {
    g.block_begin[S] = total_b;
    st->total_blocks = total_b;
    if (g.n_plain == S) st->plain_blocks = total_b;
    st->work_counter = 0;
    st->flow_counter = 0;
    st->evaluations += total_ev;
    st->rounds += 1;
  }
}

// -------------------------------------------------------- persistent kernel

// Every sector of the fast path without a flow, all dimensions up to DMAX, in one launch
// (the loop: qmc_persist.h).  F32 with FB: sectors without SF_F32OK fall back to the FP64
// form; F32 without FB: every sector of the launch has SF_F32OK, and the FP64 form (whose
// registers would set the occupancy of the whole kernel) is not compiled in.
template <int D, int K, int S, bool F32, bool FB>
__device__ __forceinline__ void run_item(const LaunchArgs &a, int s, int l_begin, int T,
                                         int64_t chunk_id, double (*red)[kMaxTile * 4][2]) {
  if constexpr (F32 && !FB) {
    integrate_block<D, K, S, true, true, false>(a, s, l_begin, T, chunk_id, red);
  } else {
    if (F32 && (a.sectors[s].flags & SF_F32OK))
      integrate_block<D, K, S, true, true, false>(a, s, l_begin, T, chunk_id, red);
    else
      integrate_block<D, K, S, true, false, false>(a, s, l_begin, T, chunk_id, red);
  }
}

// One work item of the table-driven persistent kernel: the sector's dimension picks the
// instantiation.
template <int DMAX, int K, int S, bool F32, bool FB>
struct RunTable {
  __device__ static __forceinline__ void run(const LaunchArgs &a, int s, int l_begin, int T,
                                             int64_t chunk_id, double (*red)[kMaxTile * 4][2]) {
    switch (a.sectors[s].d) {
      case 1: run_item<1, K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
      case 2: if (DMAX >= 2) run_item<(DMAX >= 2 ? 2 : 1), K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
      case 3: if (DMAX >= 3) run_item<(DMAX >= 3 ? 3 : 1), K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
      case 4: if (DMAX >= 4) run_item<(DMAX >= 4 ? 4 : 1), K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
      case 5: if (DMAX >= 5) run_item<(DMAX >= 5 ? 5 : 1), K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
      case 6: if (DMAX >= 6) run_item<(DMAX >= 6 ? 6 : 1), K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
      case 7: if (DMAX >= 7) run_item<(DMAX >= 7 ? 7 : 1), K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
      default: if (DMAX >= 8) run_item<(DMAX >= 8 ? 8 : 1), K, S, F32, FB>(a, s, l_begin, T, chunk_id, red); break;
    }
  }
};

template <int DMAX, int K, int S, bool F32, bool FB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(persistent_waves<DMAX, F32, FB>())))
void qmc_persistent_kernel(LaunchArgs a, AmpState *st) {
  __shared__ double red[kMaxWaves][kMaxTile * 4][2];
  __shared__ int64_t item;
  persistent_loop<K, RunTable<DMAX, K, S, F32, FB>>(a, st, red, item);
}

// ------------------------------------------------------------------ launchers

int launch_amp_round(const AmpArgs &g, void *stream) {
  hipLaunchKernelGGL(qmc_amp_round_kernel, dim3(1), dim3(kRoundThreads), 0, (hipStream_t)stream, g);
  return (int)hipGetLastError();
}

// FP64: one shift per pass (at d = 7, 124 registers instead of 209: twice the waves);
// FP32: two.
template <int DMAX, bool F32, bool FB>
static const void *pk_fn(int K) {
  switch (K) {
    case 1: return (const void *)qmc_persistent_kernel<DMAX, 1, F32 ? 2 : 1, F32, FB>;
    case 2: return (const void *)qmc_persistent_kernel<DMAX, 2, F32 ? 2 : 1, F32, FB>;
    case 3: return (const void *)qmc_persistent_kernel<DMAX, 3, F32 ? 2 : 1, F32, FB>;
    default: return (const void *)qmc_persistent_kernel<DMAX, 4, F32 ? 2 : 1, F32, FB>;
  }
}

template <int DMAX>
static const void *pk_variant(int variant, int K) {
  if (variant == kPersistentF64) return pk_fn<DMAX, false, true>(K);
  if (variant == kPersistentF32Mixed) return pk_fn<DMAX, true, true>(K);
  return pk_fn<DMAX, true, false>(K);
}

static const void *persistent_fn(int d_max, int variant, int K) {
  if (d_max <= 4) return pk_variant<4>(variant, K);
  if (d_max <= 6) return pk_variant<6>(variant, K);
  if (d_max <= 7) return pk_variant<7>(variant, K);
  return pk_variant<8>(variant, K);
}

int launch_persistent(const LaunchArgs &a, AmpState *st, int d_max, int variant, unsigned grid,
                      void *stream) {
  LaunchArgs la = a;
  AmpState *sp = st;
  void *args[] = {&la, &sp};
  return (int)hipLaunchKernel(persistent_fn(d_max, variant, a.K), dim3(grid), dim3(a.block), args,
                              0, (hipStream_t)stream);
}

int persistent_grid(int d_max, int variant, int K, int block, int *grid) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persistent_fn(d_max, variant, K), block, 0);
  if (e != hipSuccess) return (int)e;
  *grid = cus * (per > 0 ? per : 1);
  return 0;
}

}  // namespace qmc
