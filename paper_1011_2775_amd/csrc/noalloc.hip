// Library-owned static scratch for the allocation-free entry point
// (wcmg_coarse_solve_noalloc).  Callers that cannot allocate device memory --
// code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc -- still need the work buffers of the persistent coarse solve
// (Krylov bases, reduced vectors, layout staging, partial sums, the grid
// barrier's control block).  They come from one file-scope device array per
// GPU, reserved when the code object is loaded and kept until the process
// ends.
//
// In host code the name `scratch` is a host-side stand-in, not a device
// address: every host use goes through the per-device pointer that
// hipGetSymbolAddress returns (looked up once per device, with that device
// current).  Every call on one GPU shares that GPU's array and finds the
// previous call's contents, so the control block is cleared at every call;
// calls that overlap in time on one GPU race.
#include <mutex>

#include "kernels.h"
#include "runtime.h"

namespace wcmg {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

__global__ void k_zero_words(unsigned* p, size_t nwords) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) fail(WCMG_ENODEV, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) HIPCHK(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    HIPCHK(e);
    if (!p) fail(WCMG_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_ptr[device] = p;
  }
  return g_ptr[device];
}

// bytes must be a multiple of 4 and p 4-byte aligned
void noalloc_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t nw = bytes / 4;
  const int blocks = (int)std::min<size_t>((nw + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, st, reinterpret_cast<unsigned*>(p), nw);
  HIPCHK(hipGetLastError());
}

}  // namespace wcmg
