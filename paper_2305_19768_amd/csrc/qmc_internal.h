// qmc_internal.h -- device-side records shared by the host planner and the gfx950
// kernels of the lattice QMC library.  Not part of the C ABI.
#pragma once

#ifndef __HIPCC_RTC__
#include <stdint.h>
#endif

#include "qmcamp.h"

namespace qmc {

// Monomial table of one polynomial in the dense nested-Horner layout for total
// degree <= 3 in D variables:
//   P(x) = c0 + sum_j x_j (c_j + sum_{k>=j} x_k (c_jk + sum_{l>=k} c_jkl x_l)),
// stored as c0, then for each j: c_j, then for each k >= j: c_jk followed by the
// c_jkl for l = k .. D-1.  Length C(D+3, 3).
constexpr int dense_len(int D) { return (D + 1) * (D + 2) * (D + 3) / 6; }

constexpr int kMaxTile = 16;    // shifts per workgroup
constexpr int kMaxWaves = 4;    // wavefronts per workgroup
// The same layout truncated to total degree 1 (c0, c_0 .. c_{D-1}; length D + 1): the
// Hessian tables of F in complex plans.
constexpr int dense_len1(int D) { return D + 1; }

enum : int32_t {
  SF_XPOW = 1,      // some x_j has a non-zero exponent
  SF_HALF = 2,      // a half-integer exponent occurs (one square root per sample)
  SF_DEN = 4,       // a negative exponent occurs (one division per sample)
  SF_LOG = 8,       // max_log > 0: log F is needed
  SF_FAST = 16,     // korobov3, no x powers, integer exponents of U and F,
                    // max_log <= n_orders - 1 (log polynomials zero-padded to that degree)
  SF_F32OK = 32,    // SF_FAST and F has non-negative coefficients with a positive constant
                    // term (F >= c0 > 0 on the cube): the FP32 form may evaluate it
  SF_CF32 = 64,     // complex plan in FP32 precision: the polynomial bulk of the deformed
                    // integrand runs in FP32 (deformed at plan time, or no cancellation)
};

// Static per-sector record (plan time).  Read with uniform (scalar) loads.
struct alignas(16) SectorDev {
  int32_t d, transform, u_deg, f_deg;
  int32_t u_off, f_off;            // offsets of the dense tables in the coefficient array
  int32_t flags, max_log;
  int32_t u_num, u_den, f_num, f_den;   // integer parts of the exponents of U and F
  int32_t f_half, n_orders, integral, pad0;  // f_half: +1 numerator, -1 denominator, 0 none
  int32_t x_num[QMC_MAX_DIM];
  int32_t x_den[QMC_MAX_DIM];
  int32_t x_half[QMC_MAX_DIM];     // +1 / -1 / 0 as f_half
  double f_abs;                    // sum of |coefficients| of F (bound of sum |c m(x)| on the cube)
  double w_scale;                  // korobov3: 140^d, the constant of W = 140^d prod (y(1-y))^3
  double logc[QMC_MAX_ORDERS][QMC_MAX_LOG + 1];
  float logc32[QMC_MAX_ORDERS][QMC_MAX_LOG + 1];
  int32_t u_off32, f_off32;        // offsets of the FP32 copies of the dense tables
  int32_t grad_off, hess_off;      // complex plans: D tables dF/dx_j (degree-2 layout), then
                                   // D(D+1)/2 tables d2F/dx_j dx_k, k >= j (degree-1 layout)
  double lambda;                   // complex plans: contour deformation parameter (>= 0)
  uint64_t flow;                   // device address of an attached flow transform, or 0
  int32_t flow_cond, pad1;         // conditioning features of the attached flow
  double cond[QMC_FLOW_MAX_COND];  // their values for this sector
};

// Per-call lattice record of a sector.
struct alignas(16) LatticeDev {
  uint64_t n;
  double n_d;                      // (double) n, exact (n < 2^53)
  double inv_n;                    // RN(1/n)
  int64_t block_begin;             // first workgroup of this sector in the launch
  uint64_t z[QMC_MAX_DIM];         // generating vector
  uint64_t dz[QMC_MAX_DIM];        // (workgroup size * z_j) mod n: lattice stride of a thread
  double ndz[QMC_MAX_DIM];         // n - dz_j as an exact double (the stride step subtracts it)
  int64_t chunk;                   // lattice points per workgroup
  int32_t n_chunks;                // workgroups per shift tile (0 when inactive)
  int32_t active;                  // 0: sector skipped by this launch, its Q is kept
};

// Workgroup partials: per (shift in tile, order): (sum, compensation).
// Status word: first non-finite (sector, shift, order), linearised, or INT32_MAX.

// ---------------------------------------------------------------- launchers
// Workgroups [base, base + blocks) of the launch numbering hold the sectors of dimension
// d and path class `fast` (SF_FAST set or not).
struct DimLaunch {
  int64_t base, blocks;
  int32_t d, fast, f32, deform;   // deform: complex plan (every sector on the deformed path)
  int32_t flow, pad;              // flow: sectors with an attached learned transform
  uint64_t gen;                   // host handle of a plan-specialised kernel for the class, or 0
};

struct LaunchArgs {
  const SectorDev *sectors;
  const double *coef;
  const float *coef32;             // FP32 copy of coef (FP32 integrand form)
  const double *shifts;            // [S][m][QMC_MAX_DIM]
  const LatticeDev *lat;
  const int64_t *block_begin;      // [S+1], in workgroup order (sectors ordered by dimension)
  const int32_t *order;            // [S]: sector index of the s-th sector in workgroup order
  double *partial;                 // [blocks][tile][K][2]
  double *q;                       // [S][m][K] (always written; workspace if caller passes NULL)
  double *mean, *err;              // [S][K]
  int32_t *status;
  int32_t n_sectors, m, K, shift_tile, block, shifts_per_pass;
  int64_t total_blocks;
  int32_t d_max, precision;
  void *ev_start, *ev_stop;        // optional hipEvent_t pair recorded around the main kernel
  const int32_t *done;             // batched form: nonzero once the evaluation finished
  int32_t n_dim_launches;
  int32_t cplx;                    // complex plan: K counts (re, im) columns, K = 2 n_orders
  unsigned long long *sign_count;  // complex plans: [S] sign-check violations
  // adaptive loop: [S] workgroup durations per sector on the 100 MHz constant clock (the
  // measured cost per evaluation), or NULL (not recorded)
  unsigned long long *sector_ticks;
  // FP32 plans: [S][K] bound on the rounding error of each sector's FP32 estimate,
  // added to err by the statistics kernel; NULL: nothing added
  const double *f32_bound;
  DimLaunch dims[4 * QMC_MAX_DIM];
};

struct PointsArgs {
  uint64_t n;
  double n_d, inv_n;
  uint64_t z[QMC_MAX_DIM], dz[QMC_MAX_DIM];
  double ndz[QMC_MAX_DIM];
  double delta[QMC_MAX_DIM];
  int32_t d;
  uint32_t steps;
  uint64_t i0, count;
  double *out;
};

// ------------------------------------------------ batched amplitude evaluation
constexpr int64_t kTargetBlocksDevice = 16384;
constexpr int kAmpMaxSums = 16;
constexpr int kAmpMaxLattice = 256;

struct AmpState {
  int32_t done;          // 0 running, 1 converged, 2 round limit, 3 no lattice can grow
  int32_t rounds;        // integration rounds set up so far (presample included)
  int32_t limited;       // a sector asked for more than the largest lattice
  uint32_t work_counter; // persistent kernel's next work item
  int64_t evaluations;
  int64_t total_blocks;  // work items of the current round
  double max_eps;
  int64_t plain_blocks;  // work items of the sectors without a flow (they come first)
  uint32_t flow_counter; // flow persistent kernel's next work item (after plain_blocks)
  int32_t pad;
};

struct AmpArgs {
  AmpState *state;
  int32_t S, K, T, NI, m, tile, block, n_lattice, max_rounds;
  int32_t P;                       // Laurent terms per coefficient (tables [T][NI][P])
  int32_t n_plain;                 // sectors without a flow: the first n_plain of `order`
  double epsrel, epsabs, alpha;
  const int32_t *integral, *dims, *order;
  const int32_t *int_ptr, *int_sec;   // sectors of integral c: int_sec[int_ptr[c] .. int_ptr[c+1]), ascending
  int32_t *lidx, *active, *unmet;
  double *want;
  double *tau;                     // [S] cost per evaluation the allocation uses
  const double *c2, *cre, *cim;
  // measured costs (Sec. 2.1.3: tau estimated while the evaluation runs): per-round
  // workgroup ticks of each sector (the persistent kernels add, the round kernel drains),
  // their running sums and the evaluations they cover; measure_tau = 0 keeps tau fixed.
  unsigned long long *ticks;
  double *tick_sum, *eval_sum;
  int32_t measure_tau, trace_rows;
  double *tau_trace;               // [trace_rows][S]: tau used by the allocation after each round
  double *I, *VI, *Are, *Aim, *Vre, *Vim;
  const double *mean, *err;
  const uint64_t *lattice_n, *lattice_a;
  LatticeDev *lat;
  int64_t *block_begin;
};

int launch_amp_round(const AmpArgs &g, void *stream);
// Persistent kernel variants: FP64; FP32 with the FP64 form for sectors without
// SF_F32OK; FP32 only (every sector has SF_F32OK).
enum : int { kPersistentF64 = 0, kPersistentF32Mixed = 1, kPersistentF32 = 2 };
int launch_persistent(const LaunchArgs &a, AmpState *st, int d_max, int variant, unsigned grid,
                      void *stream);
int persistent_grid(int d_max, int variant, int K, int block, int *grid);
// The batched form's sectors with an attached flow: work items [plain_blocks,
// total_blocks) of the round, drained like the persistent kernel's.
int launch_persistent_flow(const LaunchArgs &a, AmpState *st, unsigned grid, void *stream);
int persistent_flow_grid(int block, int *grid);

// Returns a hipError_t value (0 = success).
int launch_points(const PointsArgs &pa, unsigned grid, void *stream);
// Side streams on which the per-dimension launches of one integration run beside the
// caller's stream (default priority, non-blocking), with the events that fork them off
// it and join them back.  n = 0: every launch on the caller's stream.
constexpr int kSideStreams = 3;
struct SideStreams {
  int n;
  void *stream[kSideStreams];
  void *fork;
  void *join[kSideStreams];
};
int launch_integrate(const LaunchArgs &a, void *stream, const SideStreams *side = nullptr);
// complex plans: the deformed-contour integrand kernel for one dimension class, and
// the clearing of the per-sector sign-check counters
int launch_deform(const LaunchArgs &a, const DimLaunch &dl, void *stream);
// sectors with an attached flow transform: x = T(periodizing transform(y))
int launch_flow_integrate(const LaunchArgs &a, const DimLaunch &dl, void *stream);
int launch_clear_u64(unsigned long long *p, int64_t count, void *stream);
int launch_status_reset(int32_t *status, void *stream);
int launch_reduce_stats(const LaunchArgs &a, void *stream);
int launch_korobov_p2(uint64_t n, int32_t d, const uint64_t *dev_cand, int32_t n_cand,
                      int32_t chunks, double *dev_partial, double *dev_p2, void *stream);

// Launch shapes compiled into the library: shifts per workgroup (1..16), shifts per
// pass (1, 2, 4; divides the tile), workgroup size (64..256, multiple of 64).
bool tile_supported(int shift_tile, int shifts_per_pass, int block);

}  // namespace qmc
