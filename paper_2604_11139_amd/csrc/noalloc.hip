// Scratch array of the no-allocation entry point (abi_apply_H_noalloc): its
// work buffers (split-K parts, the coefficients C', the projector part, the
// FFT box batch) are pieces of this array instead of device allocations, for
// callers that cannot allocate (code under graph capture, serving loops).
//
// Each device the library runs on holds its own copy of the array until the
// process ends.  Host code never uses the array's name as an address: the
// device address is looked up once per device with hipGetSymbolAddress (the
// device current) and kept in a table.
#include <mutex>

#include "internal.h"

namespace chebfi {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {nullptr};
std::mutex g_scratch_mu;
}  // namespace

void *scratch_for_device(int dev) {
  CHEBFI_REQUIRE(dev >= 0 && dev < kMaxDevices, ABI_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    CHEBFI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CHEBFI_REQUIRE(p != nullptr, ABI_ERR_DEVICE, "scratch array has no device address");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

size_t scratch_bytes() { return kScratchBytes; }

}  // namespace chebfi
