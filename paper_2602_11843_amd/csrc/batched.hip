// Batched evaluation of many small matrices in one persistent launch.
#include "../../include/ns.h"
#include "common.h"

namespace ns {

int batched_eval(ns_handle*, const void*, const int64_t*, const int32_t*, const int32_t*, int32_t,
                 int64_t, int, int, void*, hipStream_t, ns_report*) {
  return NS_ERR_UNSUPPORTED;
}
int batched_autotune(ns_handle*, const void*, const int64_t*, const int32_t*, const int32_t*,
                     int32_t, int64_t, void*, hipStream_t, int32_t*) {
  return NS_ERR_UNSUPPORTED;
}
void batched_release(ns_handle*) {}

}  // namespace ns
