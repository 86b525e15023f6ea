// O(n^2) helpers around the products: copy-in with zero padding and type
// conversion, copy-out, identity, zero fill, max-abs.  Grid-stride loops over
// 16-byte-aligned rows; none of them runs inside the per-level product chain
// except launch_amax (only for the scaled-FP16 engine's inputs).
#include "common.h"

namespace ns {
namespace {

template <class S, class D>
__global__ void pad_copy_kernel(const S* __restrict__ src, int64_t n, int64_t lda,
                                D* __restrict__ dst, int n_pad) {
  const size_t total = (size_t)n_pad * n_pad;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int64_t r = (int64_t)(i / n_pad), c = (int64_t)(i % n_pad);
    dst[i] = (r < n && c < n) ? (D)src[r * lda + c] : (D)0;
  }
}

template <class S, class D>
__global__ void unpad_copy_kernel(const S* __restrict__ src, int n_pad, D* __restrict__ dst,
                                  int64_t n, int64_t ldo) {
  const size_t total = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int64_t r = (int64_t)(i / n), c = (int64_t)(i % n);
    dst[r * ldo + c] = (D)src[r * (int64_t)n_pad + c];
  }
}

template <class D>
__global__ void identity_kernel(D* __restrict__ dst, int n_pad) {
  const size_t total = (size_t)n_pad * n_pad;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (i / n_pad == i % n_pad) ? (D)1 : (D)0;
}

__global__ void zero_words_kernel(unsigned* __restrict__ p, size_t words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void amax_kernel(const float* __restrict__ x, size_t count, unsigned* amax) {
  float m = 0.f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(x[i]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(amax, __float_as_uint(m));
}

inline int grid_for(size_t total) {
  size_t g = (total + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_pad_copy(const void* src, int src_f64, int64_t n, int64_t lda, void* dst,
                           int dst_f64, int n_pad, hipStream_t s) {
  const int g = grid_for((size_t)n_pad * n_pad);
  if (src_f64 && dst_f64)
    hipLaunchKernelGGL((pad_copy_kernel<double, double>), dim3(g), dim3(256), 0, s,
                       (const double*)src, n, lda, (double*)dst, n_pad);
  else if (src_f64)
    hipLaunchKernelGGL((pad_copy_kernel<double, float>), dim3(g), dim3(256), 0, s,
                       (const double*)src, n, lda, (float*)dst, n_pad);
  else if (dst_f64)
    hipLaunchKernelGGL((pad_copy_kernel<float, double>), dim3(g), dim3(256), 0, s,
                       (const float*)src, n, lda, (double*)dst, n_pad);
  else
    hipLaunchKernelGGL((pad_copy_kernel<float, float>), dim3(g), dim3(256), 0, s,
                       (const float*)src, n, lda, (float*)dst, n_pad);
  return hipGetLastError();
}

hipError_t launch_unpad_copy(const void* src, int src_f64, int n_pad, void* dst, int dst_f64,
                             int64_t n, int64_t ldo, hipStream_t s) {
  const int g = grid_for((size_t)n * n);
  if (src_f64 && dst_f64)
    hipLaunchKernelGGL((unpad_copy_kernel<double, double>), dim3(g), dim3(256), 0, s,
                       (const double*)src, n_pad, (double*)dst, n, ldo);
  else if (src_f64)
    hipLaunchKernelGGL((unpad_copy_kernel<double, float>), dim3(g), dim3(256), 0, s,
                       (const double*)src, n_pad, (float*)dst, n, ldo);
  else if (dst_f64)
    hipLaunchKernelGGL((unpad_copy_kernel<float, double>), dim3(g), dim3(256), 0, s,
                       (const float*)src, n_pad, (double*)dst, n, ldo);
  else
    hipLaunchKernelGGL((unpad_copy_kernel<float, float>), dim3(g), dim3(256), 0, s,
                       (const float*)src, n_pad, (float*)dst, n, ldo);
  return hipGetLastError();
}

hipError_t launch_set_identity(void* dst, int f64, int n_pad, hipStream_t s) {
  const int g = grid_for((size_t)n_pad * n_pad);
  if (f64)
    hipLaunchKernelGGL(identity_kernel<double>, dim3(g), dim3(256), 0, s, (double*)dst, n_pad);
  else
    hipLaunchKernelGGL(identity_kernel<float>, dim3(g), dim3(256), 0, s, (float*)dst, n_pad);
  return hipGetLastError();
}

hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_words_kernel, dim3(grid_for(words)), dim3(256), 0, s, (unsigned*)p, words);
  return hipGetLastError();
}

hipError_t launch_amax(const float* x, size_t count, unsigned* amax, hipStream_t s) {
  hipLaunchKernelGGL(amax_kernel, dim3(grid_for(count)), dim3(256), 0, s, x, count, amax);
  return hipGetLastError();
}

}  // namespace ns
