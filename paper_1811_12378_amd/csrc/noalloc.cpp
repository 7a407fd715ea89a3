// Static scratch memory of the no-allocation entry point (hfci_shifted_solve_noalloc).
//
// `scratch` is a file-scope device array.  Each GPU the library runs on holds its own
// copy, at its own address, from the code object's load until the process ends.  In host
// code the name `scratch` is only a host-side stand-in: a kernel given it would fault.  So
// host code uses the address returned by hipGetSymbolAddress, looked up here once per
// device with that device current (at hfci_ctx_create), never the name itself.
//
// Every call on one GPU shares that GPU's array, and the array keeps whatever the last
// call left there.  The shifted solve initialises every scratch value it reads, so stale
// contents do no harm.  Calls that overlap in time on one GPU (two host threads, or two
// contexts with their own streams) race on the array.
#include <mutex>

#include "internal.h"

namespace hfci {

const size_t kNoAllocScratchBytes = (size_t)64 << 20;  // 64 MiB per device

namespace {

static __device__ __align__(256) unsigned char scratch[(size_t)64 << 20];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Called with `device` current (hfci_ctx_create holds a DeviceGuard for it).
void* noalloc_scratch_for_device(int device) {
  static_assert(sizeof(scratch) == ((size_t)64 << 20), "kNoAllocScratchBytes must be the array's size");
  HFCI_REQUIRE(device >= 0 && device < kMaxDevices, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    HFCI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HFCI_REQUIRE(p != nullptr, "no device address for the static scratch array");
    g_ptr[device] = p;
  }
  return g_ptr[device];
}

}  // namespace hfci
