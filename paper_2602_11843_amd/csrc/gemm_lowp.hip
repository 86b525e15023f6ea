// Low-precision product engines (split-BF16 and scaled FP16).
#include "common.h"

namespace ns {

int engine_tile_lowp(Engine, int) { return 128; }

hipError_t launch_gemm_lowp(Engine, const GemmParams&, const GemmParams*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace ns
