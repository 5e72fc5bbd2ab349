// qmc_static.hip -- qmc_integrate for callers that cannot allocate device memory.
//
// The plan's device regions of one integration (sector records, coefficient tables,
// shifts, lattice records, workgroup table, workgroup partials, Q, status word) are laid
// out in a file-scope device array instead of a caller-bound workspace.  Each device
// the library runs on holds its own copy of the array until the process ends; the host
// reaches it only through the address hipGetSymbolAddress returns on that device (the
// array's name is a host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <mutex>

#include "qmc_plan.h"

using namespace qmc;

namespace {

static_assert(QMC_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) unsigned char scratch[QMC_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_at[kMaxDevices] = {};   // device address of `scratch`, per device

// Address of the current device's copy of the scratch array, looked up once per device.
qmc_status scratch_address(char **out) {
  int dev = 0;
  int e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(QMC_E_DEVICE, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e ? e : (int)hipErrorInvalidSymbol, "static scratch address");
    g_scratch_at[dev] = (char *)ptr;
  }
  *out = g_scratch_at[dev];
  return QMC_OK;
}

}  // namespace

extern "C" qmc_status qmc_integrate_static(qmc_plan_t p, const uint64_t *n, const uint64_t *a,
                                           void *stream, double *dev_q, double *dev_mean,
                                           double *dev_err) {
  g_last_error.clear();
  if (!p) return fail(QMC_E_INVAL, "NULL plan");
  char *base = nullptr;
  qmc_status st = scratch_address(&base);
  if (st != QMC_OK) return st;
  return integrate_sectors(p, n, a, nullptr, stream, dev_q, dev_mean, dev_err, nullptr, base,
                           (size_t)QMC_STATIC_SCRATCH_BYTES);
}
