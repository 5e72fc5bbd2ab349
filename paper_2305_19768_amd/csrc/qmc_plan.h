// qmc_plan.h -- host-side plan object shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qmc_internal.h"

namespace qmc {

extern thread_local std::string g_last_error;
qmc_status fail(qmc_status st, const char *fmt, ...);
qmc_status hip_fail(int e, const char *what);
uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t n);
uint64_t gcd_u64(uint64_t a, uint64_t b);
uint64_t splitmix64(uint64_t seed, uint64_t counter);
size_t align256(size_t v);

constexpr int64_t kTargetBlocks = 16384;   // default workgroups per launch the chunking aims at
constexpr int64_t kTargetBlocksMax = 32768;   // largest target a launch shape may choose
constexpr int32_t kP2MaxCand = 65536;
constexpr size_t kP2PartialDoubles = 1 << 19;   // 4 MiB of P2 partial sums
// Arguments of a P_2 evaluation (n, d, candidates in [1, n)), and the workgroups per
// candidate that fit the partial-sum buffer.
qmc_status p2_check_args(uint64_t n, int32_t d, const uint64_t *cand, int32_t n_cand);
int64_t p2_chunks(uint64_t n, int32_t n_cand);

// A plan-specialised kernel (run-time compiled): a class kernel of launch class (d, f32)
// with spp shifts per pass, or (persistent = 1, d = 0) the batched form's persistent
// kernel for K orders; covering exactly the listed sectors.
struct GenKernel {
  int32_t d, f32, spp;
  int32_t persistent, K;
  void *mod, *fn;                 // hipModule_t, hipFunction_t
  std::vector<int> sectors;
  int32_t grid;                   // persistent: workgroups of the launch (0: not yet known)
};

}  // namespace qmc

struct qmc_plan_s {
  // the plan's host state and the layout of its device workspace
  // problem
  int32_t S = 0, K = 0, M = 0, n_integrals = 0, d_max = 0;
  int32_t cplx = 0;                    // some sector deformed: complex integrands
  int32_t KC = 0;                      // columns per (sector, shift): K, or 2 K if complex
  std::vector<qmc::SectorDev> sec;
  std::vector<double> coef;
  std::vector<float> coef32;           // FP32 copy of coef (same offsets)
  std::vector<double> shifts;          // [S][m][QMC_MAX_DIM]
  std::vector<uint64_t> n_default, a_default;
  std::vector<int32_t> dims;
  std::vector<int32_t> order;          // sectors in workgroup order: by dimension, then index
  int32_t persistent_grid[3] = {0, 0, 0};  // resident workgroups per persistent-kernel variant
  // options
  int32_t m = 0, precision = 0, block = 256, tile = 8, spp = 2;
  uint64_t n_max = 0;
  // workspace layout (byte offsets)
  size_t off_sec = 0, off_coef = 0, off_shift = 0, off_lat = 0, off_begin = 0, off_q = 0,
         off_status = 0, off_partial = 0, off_order = 0, off_mean = 0, off_err = 0, off_coef32 = 0, off_amp = 0, amp_bytes = 0, off_p2cand = 0, off_p2part = 0, off_p2vals = 0,
         off_sign = 0, off_ticks = 0, total = 0;
  bool ticks_on = false;   // record per-sector workgroup ticks (the adaptive loop's costs)
  // FP32 plans: rounding-error bound per (sector, column) from the calibration lattice
  // (fp32_calibrate), with the FP64 estimates there; valid until shifts or flows change
  size_t off_cal = 0, off_bound = 0;
  // bound_off: integrations that need no bound (the calibration itself, the presample
  // choice of the deformation parameters)
  bool cal_valid = false, bound_off = false, bound_in_ws = false;
  std::vector<double> f32_bound, cal_mean;
  int64_t max_blocks = 0;
  int64_t target_blocks = 16384;      // workgroups per launch the chunking aims at
  size_t partial_doubles = 0;         // capacity of the workgroup partial buffer
  char *ws = nullptr;
  size_t ws_bytes = 0;
  // per-call staging
  std::vector<qmc::LatticeDev> lat;
  std::vector<int64_t> begin;
  std::vector<qmc::LatticeDev> lat_uploaded;
  bool lat_valid = false;
  // kernel timing (HIP events around the main kernel of each qmc_integrate)
  bool timing = false;
  std::vector<hipEvent_t> ev;   // pairs: start, stop
  size_t ev_used = 0;
  // side streams of the concurrent per-dimension launches (created when the workspace
  // is bound, on the workspace's device)
  qmc::SideStreams side{};
  // plan-specialised kernels (qmc_specialize)
  std::vector<qmc::GenKernel> gen;
  // status word and sign-check counters of the last qmc_integrate_static call (in the
  // library's static device scratch); NULL after any call that used the workspace
  int32_t *static_status = nullptr;
  unsigned long long *static_sign = nullptr;
  // pinned host image of the batched amplitude form's tables (grown as needed)
  void *amp_host = nullptr;
  size_t amp_host_bytes = 0;
  ~qmc_plan_s() {
    if (amp_host) (void)hipHostFree(amp_host);
    for (qmc::GenKernel &g : gen) (void)hipModuleUnload((hipModule_t)g.mod);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (int i = 0; i < side.n; ++i) {
      (void)hipEventDestroy((hipEvent_t)side.join[i]);
      (void)hipStreamDestroy((hipStream_t)side.stream[i]);
    }
    if (side.fork) (void)hipEventDestroy((hipEvent_t)side.fork);
  }
};


namespace qmc {
// Integrate the sectors with active[s] != 0 (all if active is NULL) on lattices n, a;
// inactive sectors keep their previous Q.  Writes Q to dev_q (or the workspace) and
// the statistics of every sector to dev_mean / dev_err.
// Handle of the plan-specialised kernel of launch class (d, f32) under the plan's
// current launch shape, if one was compiled for exactly the class's current sectors; 0
// otherwise (the table-driven kernel runs).
uint64_t gen_lookup(const qmc_plan_s *p, int d, bool f32);
// The specialised persistent kernel for FP32 (f32) or FP64 and K orders whose sectors are
// exactly `sectors`, or nullptr.
GenKernel *gen_persistent_lookup(qmc_plan_s *p, bool f32, int K, const std::vector<int> &sectors);
// With static_base set, every device region of the call (tables, lattice records,
// workgroup partials, status) is laid out in that buffer of static_cap bytes instead of
// the plan's workspace, and the tables are uploaded on `stream` first.
qmc_status integrate_sectors(qmc_plan_s *p, const uint64_t *n, const uint64_t *a,
                             const uint8_t *active, void *stream, double *dev_q, double *dev_mean,
                             double *dev_err, const uint64_t *zvec = nullptr,
                             char *static_base = nullptr, size_t static_cap = 0);
// FP32 plans: bound the rounding error of the FP32 form per (sector, column) by
// integrating every sector on a small calibration lattice with the FP64 and with the
// FP32 form (same points, same shifts) -- once per plan until its shifts, flows or
// deformation parameters change; synchronizes `stream`.  No-op for FP64 plans.
qmc_status fp32_calibrate(qmc_plan_s *p, void *stream, char *static_base = nullptr,
                          size_t static_cap = 0);
}  // namespace qmc
