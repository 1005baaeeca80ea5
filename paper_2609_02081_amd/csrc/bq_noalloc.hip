// Static device workspace of the allocation-free entry point
// (bq_gemm_noalloc): one array per GPU the library runs on, held until the
// process ends.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, looked up once per device
// with that device current (bq_create calls bq::noalloc_scratch), and is the
// only value passed to kernels.
#include <mutex>
#include <vector>

#include "bq.h"
#include "bq_internal.h"

namespace bq {

namespace {

static __device__ __align__(256) unsigned char scratch[BQ_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device index, nullptr until looked up

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr, size_t* bytes) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (!g_scratch_ptr[(size_t)device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[(size_t)device] = p;
  }
  *ptr = g_scratch_ptr[(size_t)device];
  *bytes = BQ_NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

}  // namespace bq
