// ptap_numeric_noalloc: the numeric phase with no device allocation and no use of the plan's
// workspace for scratch.  The general kernels' device-memory hash tables (rows whose tables do not
// fit in LDS) live in a file-scope device array instead, one per GPU, held until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ptap.h"

namespace {

// Hash-table slots of the array: 4-byte keys then 8-byte values (12 MiB per GPU).
constexpr size_t kScratchSlots = size_t(1) << 20;
constexpr size_t kScratchBytes = kScratchSlots * (sizeof(int) + sizeof(double));
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

// The device address of this GPU's array (looked up once per device, with that device current).
// The array's name is only a host-side stand-in; kernels must be given this address.
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_once[dev], [dev]() {
    void* p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
  });
  *out = g_ptr[dev];
  return g_err[dev];
}

}  // namespace

extern "C" {

// In api.cpp (C linkage, hidden): the numeric phase with the hash tables in the given memory, and
// the number of table slots a plan needs.
ptap_status numeric_with_scratch(ptap_plan* P, const double* A_val, const double* P_val, double* C_val,
                                 int* keys, double* vals, size_t slots, hipStream_t s);
size_t plan_scratch_slots(const ptap_plan* P);

ptap_status ptap_numeric_noalloc(ptap_plan* plan, const double* A_val, const double* P_val,
                                 double* C_val, hipStream_t stream) {
  if (!plan) return PTAP_ERR_INPUT;
  if (plan_scratch_slots(plan) > kScratchSlots) return PTAP_ERR_TOO_LARGE;
  void* base = nullptr;
  const hipError_t e = scratch_address(&base);
  if (e != hipSuccess || !base) return PTAP_ERR_HIP;
  int* keys = static_cast<int*>(base);
  double* vals = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + kScratchSlots * sizeof(int));
  return numeric_with_scratch(plan, A_val, P_val, C_val, keys, vals, kScratchSlots, stream);
}

}  // extern "C"
