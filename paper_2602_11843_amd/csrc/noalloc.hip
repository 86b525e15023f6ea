// ns_eval_noalloc: the single-matrix evaluation of ns_eval_ex with every byte
// of device memory it needs beyond A and out taken from a fixed device array,
// for callers that cannot allocate (code under stream capture, serving loops,
// harnesses that forbid allocation).
//
// The array lives in this code object, one copy per GPU, for the life of the
// process.  Its name is only a host-side stand-in for the symbol: its device
// address on each GPU comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is ever handed to a kernel
// or a copy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ns.h"
#include "common.h"

namespace ns {
int eval_fixed(char* ws, size_t ws_bytes, GemmParams* params_host, GemmParams* params_dev,
               size_t params_cap, const void* A, int64_t n, int64_t lda, int64_t k, int method,
               int dtype, void* out, int64_t ldo, hipStream_t s, ns_report* rep);
int fail_status(int status, const char* msg);
}  // namespace ns

namespace {

constexpr size_t kScratchBytes = NS_NOALLOC_SCRATCH_BYTES;
// the last MiB holds the parameter blocks of a call's products, the rest the
// workspace (scalar block and matrices)
constexpr size_t kParamRegion = size_t(1) << 20;
constexpr size_t kParamBlocks = kParamRegion / sizeof(ns::GemmParams);
constexpr size_t kWorkBytes = kScratchBytes - kParamRegion;
static_assert(kWorkBytes % 256 == 0, "parameter region alignment");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;                            // one call at a time on the host side
unsigned char* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device
ns::GemmParams g_params_host[kParamBlocks];  // host staging of the parameter blocks

}  // namespace

extern "C" int ns_eval_noalloc(const void* A, int64_t n, int64_t lda, int64_t k, int method,
                               int dtype, void* out, int64_t ldo, hipStream_t stream,
                               ns_report* rep) {
  try {
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ns::fail_status(NS_ERR_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return ns::fail_status(NS_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
      void* p = nullptr;
      const hipError_t se = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (se != hipSuccess || !p)
        return ns::fail_status(NS_ERR_HIP, "hipGetSymbolAddress of the fixed scratch array failed");
      g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    unsigned char* base = g_scratch[dev];
    return ns::eval_fixed(reinterpret_cast<char*>(base), kWorkBytes, g_params_host,
                          reinterpret_cast<ns::GemmParams*>(base + kWorkBytes), kParamBlocks, A, n,
                          lda, k, method, dtype, out, ldo, stream, rep);
  } catch (...) {
    return ns::fail_status(NS_ERR_HIP, "unexpected C++ exception");
  }
}
