// Allocation-free apply (bf_apply_noalloc): the same kernels as bf_apply
// (eq. hybrid_butterfly_mat), with the intermediates placed in a fixed device
// array instead of memory from the stream-ordered pool, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops).
//
// `scratch` below is a host-side stand-in in host code; its device address
// differs per GPU and is looked up once per device with hipGetSymbolAddress
// (with that device current) and used for every kernel argument.
#include <mutex>

#include "factors.h"

namespace bf {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // per device, held until exit
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[64];

// device address of this device's copy of `scratch` (first call on a device
// resolves it; the device must be current)
void* scratch_address(int dev) {
  BF_CHECK(dev >= 0 && dev < 64, BF_ENOTSUP, "bf_apply_noalloc: device index out of range");
  ScratchSlot& sl = g_scratch[dev];
  std::call_once(sl.once, [&sl] {
    void* p = nullptr;
    sl.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (sl.err == hipSuccess) sl.ptr = p;
  });
  BF_CHECK(sl.err == hipSuccess && sl.ptr, BF_EHIP,
           std::string("bf_apply_noalloc: hipGetSymbolAddress(scratch): ") +
               hipGetErrorString(sl.err));
  return sl.ptr;
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

void apply_noalloc(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
                   bf_c64* Y, int64_t ldy, hipStream_t s) {
  int dev = 0;
  BF_HIP(hipGetDevice(&dev));
  BF_CHECK(dev == F->device, BF_EINVAL,
           "bf_apply_noalloc: the factors live on another device than the current one");
  // the fused schedule's intermediates when they fit, else the two ping-pong
  // buffers of the stage-by-stage apply (the second at a 256-byte boundary)
  const size_t staged = apply_scratch_bytes(F, trans, ncols, true);
  BF_CHECK(ncols <= (int64_t)(kScratchBytes / sizeof(bf_c64)) && staged <= kScratchBytes,
           BF_EINVAL,
           "bf_apply_noalloc: " + std::to_string(ncols) + " columns need " +
               std::to_string(staged) + " bytes of scratch, more than the " +
               std::to_string(kScratchBytes) + " bytes available");
  if (ncols == 0) return;
  run_apply(F, trans, X, ldx, ncols, Y, ldy, scratch_address(dev), kScratchBytes, s, false);
}

}  // namespace bf
