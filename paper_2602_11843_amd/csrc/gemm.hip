// Dense n x n x n products on CDNA4 matrix cores with a fused multi-output
// epilogue.  Every matrix product of the series schedules runs here; the
// linear combinations, identity shifts and running-sum updates of the radix
// kernels are applied in the epilogue, so no O(n^2) elementwise kernel runs
// between products.
//
// Engines
//   FP64: v_mfma_f64_4x4x4f64.  Its four 4x4 blocks are used as four
//         k-slices of one 4x4 output fragment and summed across lanes once
//         per tile (measured on gfx950: this instruction sustains ~57 TFLOP/s
//         against ~44 for the 16x16x4 form).
//   FP32: v_mfma_f32_16x16x4f32.
// Both stage BM x BK and BK x BN tiles through double-buffered LDS with 16-byte
// global loads, one barrier per k-chunk, and order workgroups so that the
// tiles resident on one XCD share rows of X and columns of Y in that XCD's L2.
#include "gemm_device.h"

namespace ns {
namespace {
using namespace dev;

template <class P>
hipError_t launch(const GemmParams& host, const GemmParams* dev, hipStream_t s) {
  if (host.n % P::BM || host.n % P::BN || host.n % P::BK) return hipErrorInvalidValue;
  const int grid = (host.n / P::BM) * (host.n / P::BN);
  const MainArgs a{host.X, host.Y, host.n, host.ld, dev};
  hipLaunchKernelGGL(gemm_kernel<P>, dim3(grid), dim3(P::THREADS), 0, s, a);
  return hipGetLastError();
}

template <class Q>
hipError_t launch_low(const GemmParams& host, const GemmParams* dev, hipStream_t s) {
  if (host.n % Q::BM || host.n % Q::BN || host.n % Q::BK) return hipErrorInvalidValue;
  const int grid = (host.n / Q::BM) * (host.n / Q::BN);
  const MainArgs a{host.X, host.Y, host.n, host.ld, dev};
  hipLaunchKernelGGL(gemm_lowp_kernel<Q>, dim3(grid), dim3(Q::THREADS), 0, s, a);
  return hipGetLastError();
}

// tile choices
using F64Big = PolF64<2, 4, 8, 8, 2>;     // 64 x 128 tile, k-chunk 32, 8 waves
using F64Small = PolF64<2, 2, 4, 4, 1>;   // 32 x 32 tile, k-chunk 16, 4 waves
using F32Big = PolF32<2, 2, 4, 8>;     // 128 x 256 tile, 4 waves
using F32Small = PolF32<2, 2, 2, 2>;   // 64 x 64 tile, 4 waves

constexpr int kBigMin = 2048;          // n from which the large tiles are used

}  // namespace

// below kPanelMin the low-precision engines convert on the way into LDS
using BF3Small = PolLow<2, 2, 1, 1, true>;  // 64 x 64 tile
using H16Small = PolLow<2, 2, 1, 1, false>;

int engine_tile(Engine e, int n) {
  switch (e) {
    case ENG_F64: return n >= kBigMin ? 128 : 32;
    case ENG_F32: return n >= kBigMin ? 256 : 64;
    case ENG_BF16X3:
    case ENG_F16S: return n >= kBigMin ? 256 : 64;
  }
  return 256;
}

hipError_t launch_gemm(Engine e, const GemmParams& host, const GemmParams* dev, hipStream_t s) {
  switch (e) {
    case ENG_F64: return host.n >= kBigMin ? launch<F64Big>(host, dev, s) : launch<F64Small>(host, dev, s);
    case ENG_F32: return host.n >= kBigMin ? launch<F32Big>(host, dev, s) : launch<F32Small>(host, dev, s);
    // at n >= kPanelMin these engines run from panels (launch_gemm_panels)
    case ENG_BF16X3: return panel_path(e, host.n) ? hipErrorInvalidValue : launch_low<BF3Small>(host, dev, s);
    case ENG_F16S: return panel_path(e, host.n) ? hipErrorInvalidValue : launch_low<H16Small>(host, dev, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ns
