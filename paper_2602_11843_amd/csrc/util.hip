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

struct FillSet {
  Fill f[kMaxFills];
  int first_block[kMaxFills + 1];   // fill i owns blocks [first_block[i], first_block[i + 1])
  int count;
};

template <class S, class D>
__device__ void pad_range(const Fill& f, size_t i0, size_t step) {
  const S* __restrict__ src = static_cast<const S*>(f.src);
  D* __restrict__ dst = static_cast<D*>(f.dst);
  const size_t total = (size_t)f.n_pad * f.n_pad;
  for (size_t i = i0; i < total; i += step) {
    const int64_t r = (int64_t)(i / f.n_pad), c = (int64_t)(i % f.n_pad);
    dst[i] = (r < f.n && c < f.n) ? (D)src[r * f.lda + c] : (D)0;
  }
}

template <class D>
__device__ void identity_range(const Fill& f, size_t i0, size_t step) {
  D* __restrict__ dst = static_cast<D*>(f.dst);
  const size_t total = (size_t)f.n_pad * f.n_pad;
  for (size_t i = i0; i < total; i += step) dst[i] = (i / f.n_pad == i % f.n_pad) ? (D)1 : (D)0;
}

__global__ void fills_kernel(const FillSet set) {
  int k = 0;
  while (k + 1 < set.count && (int)blockIdx.x >= set.first_block[k + 1]) ++k;
  const Fill& f = set.f[k];
  const int nb = set.first_block[k + 1] - set.first_block[k];
  const size_t i0 = (size_t)(blockIdx.x - set.first_block[k]) * blockDim.x + threadIdx.x;
  const size_t step = (size_t)nb * blockDim.x;
  switch (f.kind) {
    case FILL_ZERO: {
      unsigned* p = static_cast<unsigned*>(f.dst);
      for (size_t i = i0; i < f.bytes / 4; i += step) p[i] = 0u;
      break;
    }
    case FILL_PAD:
      if (f.src_f64 && f.dst_f64) pad_range<double, double>(f, i0, step);
      else if (f.src_f64) pad_range<double, float>(f, i0, step);
      else if (f.dst_f64) pad_range<float, double>(f, i0, step);
      else pad_range<float, float>(f, i0, step);
      break;
    default:
      if (f.dst_f64) identity_range<double>(f, i0, step);
      else identity_range<float>(f, i0, step);
      break;
  }
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

hipError_t launch_fills(const Fill* fills, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxFills) return hipErrorInvalidValue;
  FillSet set{};
  set.count = count;
  int blocks = 0;
  for (int i = 0; i < count; ++i) {
    set.f[i] = fills[i];
    set.first_block[i] = blocks;
    const size_t elems = fills[i].kind == FILL_ZERO ? fills[i].bytes / 4
                                                    : (size_t)fills[i].n_pad * fills[i].n_pad;
    blocks += grid_for(elems);
  }
  set.first_block[count] = blocks;
  hipLaunchKernelGGL(fills_kernel, dim3(blocks), dim3(256), 0, s, set);
  return hipGetLastError();
}

hipError_t launch_amax(const float* x, size_t count, unsigned* amax, hipStream_t s) {
  hipLaunchKernelGGL(amax_kernel, dim3(grid_for(count)), dim3(256), 0, s, x, count, amax);
  return hipGetLastError();
}

}  // namespace ns
