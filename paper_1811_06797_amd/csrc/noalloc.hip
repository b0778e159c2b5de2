// Allocation-free form of the raw projected local TT-matvec (eq. KKT_red) for callers that
// cannot allocate device memory: its intermediates live in one fixed device array per GPU.
//
// The array is a file-scope __device__ variable, so every GPU the library runs on holds its
// own copy, at its own address, from the load of the code object until the process ends. In
// host code the variable's name only stands for it; its device address is looked up once per
// device with hipGetSymbolAddress (at context creation, with that device current) and kept in
// a per-device table, which is what the entry point hands to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.hpp"

namespace iga {

long local_matvec_noalloc_len(int r0, int n, int r1, int p, int RM0, int RM1, int RK0, int RK1);
void local_matvec_noalloc_impl(iga_ctx* ctx, int r0, int n, int r1, int p, int RM0, int RM1, int RK0, int RK1,
                               const double* PhiL_M, const double* PhiR_M, const double* PhiL_K,
                               const double* PhiR_K, const double* Mcore, const double* Kcore, double beta,
                               const double* x, double* y, double* ws, long ws_len);

namespace {

constexpr long kScratchDoubles = IGA_NOALLOC_SCRATCH_BYTES / sizeof(double);
static_assert(IGA_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256 bytes");

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the scratch array (the device must be current); idempotent.
void noalloc_scratch_init(int device) {
  require(device >= 0 && device < kMaxDevices, IGA_EINVAL, "noalloc scratch: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  IGA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  require(ptr != nullptr && reinterpret_cast<uintptr_t>(ptr) % 256 == 0, IGA_EHIP,
          "noalloc scratch: bad symbol address");
  g_scratch_ptr[device] = static_cast<double*>(ptr);
}

void local_matvec_noalloc_entry(iga_ctx* ctx, int r0, int n, int r1, int degree, int RM0, int RM1, int RK0,
                                int RK1, const double* PhiL_M, const double* PhiR_M, const double* PhiL_K,
                                const double* PhiR_K, const double* Mcore, const double* Kcore, double beta,
                                const double* x, double* y) {
  double* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) ws = g_scratch_ptr[ctx->device];
  }
  require(ws != nullptr, IGA_EINVAL, "local_matvec_noalloc: scratch of this device not set up (context missing)");
  const long need = local_matvec_noalloc_len(r0, n, r1, degree, RM0, RM1, RK0, RK1);
  require(need <= kScratchDoubles, IGA_EINVAL,
          "local_matvec_noalloc: workspace of " + std::to_string(need * 8) + " bytes exceeds the fixed " +
              std::to_string((long)IGA_NOALLOC_SCRATCH_BYTES) + " bytes");
  local_matvec_noalloc_impl(ctx, r0, n, r1, degree, RM0, RM1, RK0, RK1, PhiL_M, PhiR_M, PhiL_K, PhiR_K, Mcore, Kcore,
                            beta, x, y, ws, kScratchDoubles);
}

}  // namespace iga
