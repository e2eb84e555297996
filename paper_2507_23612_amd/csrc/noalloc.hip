// Allocation-free entry point: the Rayleigh-Ritz contractions of hcu_gram
// (S = Y^H Y dV, Hs = Y^H HY dV) for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  It needs no
// context: the split-K partial sums and the tile list live in one
// file-scope device array of fixed size, of which each GPU the library runs
// on holds its own copy until the process ends.  Every call on a GPU uses
// that GPU's copy, so calls that overlap on one GPU (several host threads or
// streams) race; each call rewrites every byte it reads, so nothing needs
// clearing between calls.
#include "common.h"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(80) << 20;   // 80 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// device address of `scratch` on each GPU (looked up once, with that GPU
// current; the array's name is only a host-side stand-in)
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

hcu_status scratch_on_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HCU_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HCU_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HCU_OK;
}

}  // namespace

extern "C" hcu_status hcu_gram_noalloc(const void* Y, const void* HY, int ncol, int64_t nd, int64_t ld,
                                       int precision, int is_complex, double dv, double* S, double* Hs,
                                       void* stream) {
  if (!Y || !HY || !S || !Hs) return HCU_INVALID_ARG;
  if (ncol < 1 || nd < 1 || ld < nd || !(dv > 0)) return HCU_INVALID_ARG;
  if (precision != HCU_FP64 && precision != HCU_MIXED) return HCU_INVALID_ARG;
  const bool cp = is_complex != 0;
  if (hcu::gram_scratch_bytes(ncol, nd, cp) > kScratchBytes) return HCU_OOM;
  void* ptr = nullptr;
  const hcu_status s = scratch_on_current_device(&ptr);
  if (s != HCU_OK) return s;
  (void)hipGetLastError();   // start from a clean error state
  hcu::launch_gram_scratch(Y, HY, ncol, ld, nd, dv, precision == HCU_MIXED, cp, ptr, S, Hs, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? HCU_OK : HCU_DEVICE;
}
