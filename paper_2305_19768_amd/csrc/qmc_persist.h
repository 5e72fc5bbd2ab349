// qmc_persist.h -- the loop of the batched amplitude form's persistent kernels: each
// workgroup takes the next work item (sector, chunk, shift tile) from the round's atomic
// counter until none is left, integrates it, and writes its compensated partial exactly
// where a per-dimension launch would, so the reduction and its order are unchanged.
// Shared by the library's persistent kernels and the plan-specialised one (compiled at
// run time from the embedded text of this header).  Not part of the C ABI.
#pragma once

#include "qmc_device.h"

namespace qmc {

// The work item is the same for every lane; make that explicit so that the sector's
// tables stay in scalar registers.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// RUN::run(a, s, l_begin, T, chunk_id, red) integrates one work item of sector s into the
// workgroup's reduction buffer red; K: the orders of the launch.
template <int K, class RUN>
__device__ __forceinline__ void persistent_loop(const LaunchArgs &a, AmpState *st,
                                                double (*red)[kMaxTile * 4][2], int64_t &item) {
  if (st->done) return;
  const int64_t total = st->plain_blocks;   // the flow sectors' items follow
  const int T = a.shift_tile;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item = (int64_t)atomicAdd(&st->work_counter, 1u);
    __syncthreads();
    const int64_t b = wave_uniform(item);
    if (b >= total) break;
    const uint64_t t0 = ticks_now();
    const int s = a.order[find_sector(a.block_begin, a.n_sectors, b)];
    const LatticeDev *__restrict__ lt = a.lat + s;
    const int64_t local = b - lt->block_begin;
    const int nch = lt->n_chunks;
    const int tile_id = (int)(local / nch);
    const int64_t chunk_id = local - (int64_t)tile_id * nch;
    RUN::run(a, s, tile_id * T, T, chunk_id, red);
    __syncthreads();
    const int nwaves = blockDim.x >> 6;
    if ((int)threadIdx.x < T * K) {
      DD r{red[0][threadIdx.x][0], red[0][threadIdx.x][1]};
      for (int w = 1; w < nwaves; ++w) r = dd_combine(r, DD{red[w][threadIdx.x][0], red[w][threadIdx.x][1]});
      double *out = a.partial + (b * (T * K) + threadIdx.x) * 2;
      out[0] = r.s;
      out[1] = r.c;
    }
    ticks_add(a, s, t0);
  }
}

// Waves per SIMD asked of the compiler for the persistent kernels: four (128 VGPRs) for
// the pure-FP32 and the FP64 (one shift per pass) forms up to d = 7, which fit with at
// most a few spills; no constraint otherwise (the mixed form and d = 8 need more
// registers).
template <int DMAX, bool F32, bool FB>
constexpr int persistent_waves() {
  return DMAX <= 7 && (!F32 || !FB) ? 4 : 1;
}

}  // namespace qmc
