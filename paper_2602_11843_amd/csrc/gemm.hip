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
#include "common.h"

namespace ns {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// workgroup -> output tile.  Workgroups are dispatched round-robin over the 8
// XCDs; XCD x receives the contiguous slice [x T/8, (x+1) T/8) of a grouped
// (GROUP_M rows at a time) tile order, so concurrently running tiles on one
// XCD are neighbours and reuse X row panels / Y column panels from its L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_coords(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n;
  int t = bid;
  if ((T & 7) == 0) t = (bid & 7) * (T >> 3) + (bid >> 3);
  constexpr int G = 8;
  const int per_group = G * tiles_n;
  const int gid = t / per_group;
  const int first = gid * G;
  const int gs = min(tiles_m - first, G);
  const int r = t - gid * per_group;
  tm = first + r % gs;
  tn = r / gs;
}

// ---------------------------------------------------------------------------
// epilogue
// ---------------------------------------------------------------------------
struct EpiState {
  double ssq;
  float amax;
  int bad;
};

__device__ __forceinline__ void epi_element(const GemmParams& p, int row, int col, double v,
                                            EpiState& st) {
  const size_t idx = (size_t)row * p.ld + col;
  double z[kMaxZ];
#pragma unroll
  for (int i = 0; i < kMaxZ; ++i) {
    z[i] = 0.0;
    if (i < p.nz)
      z[i] = p.zf64[i] ? static_cast<const double*>(p.Z[i])[idx]
                       : (double)static_cast<const float*>(p.Z[i])[idx];
  }
  const double idv = (row == col) ? 1.0 : 0.0;
  for (int o = 0; o < p.no; ++o) {
    const EpiOut& e = p.out[o];
    double y = e.a * v + e.id * idv;
#pragma unroll
    for (int i = 0; i < kMaxZ; ++i) y += e.z[i] * z[i];
    if (e.f64) {
      static_cast<double*>(e.ptr)[idx] = y;
    } else {
      const float yf = (float)y;
      static_cast<float*>(e.ptr)[idx] = yf;
      y = (double)yf;
    }
    if (o == 0) {
      st.ssq += y * y;
      if (!isfinite(y)) st.bad = 1;
      st.amax = fmaxf(st.amax, (float)fabs(y));
    }
  }
}

// Reduce the per-thread statistics over the workgroup and publish them with
// one atomic each.  `scratch` is LDS of at least 3 * (THREADS / 64) words
// (the tile buffers are reused; the caller synchronises before the call).
template <int THREADS>
__device__ __forceinline__ void publish_stats(const GemmParams& p, EpiState st, double* scratch) {
  if (!p.sumsq && !p.nonfinite && !p.amax) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    st.ssq += __shfl_xor(st.ssq, off);
    st.amax = fmaxf(st.amax, __shfl_xor(st.amax, off));
    st.bad |= __shfl_xor(st.bad, off);
  }
  constexpr int NW = THREADS / 64;
  if (lane == 0) {
    scratch[wave] = st.ssq;
    scratch[NW + wave] = (double)st.amax;
    scratch[2 * NW + wave] = (double)st.bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, a = 0.0, b = 0.0;
    for (int w = 0; w < NW; ++w) {
      s += scratch[w];
      a = fmax(a, scratch[NW + w]);
      b = fmax(b, scratch[2 * NW + w]);
    }
    if (p.sumsq) atomicAdd(p.sumsq, s);
    if (p.nonfinite && b != 0.0) atomicOr(p.nonfinite, 1);
    if (p.amax) atomicMax(p.amax, __float_as_uint((float)a));
  }
}

// ---------------------------------------------------------------------------
// FP64 policy: v_mfma_f64_4x4x4f64.
// Lane l of the instruction: block b = (l>>2)&3, and
//   A operand  A_b[i][k], i = l&3,  k = l>>4
//   B operand  B_b[k][j], j = l&3,  k = l>>4
//   result     D_b[i][j], i = l>>4, j = l&3
// (decoded on the device).  Block b takes k-slice 4b..4b+3 of a 16-wide
// k-chunk, so one instruction advances a 4x4 output fragment by 16 k.
// ---------------------------------------------------------------------------
template <int NWM_, int NWN_, int NI_, int NJ_>
struct PolF64 {
  using T = double;
  static constexpr int NWM = NWM_, NWN = NWN_, NI = NI_, NJ = NJ_;
  static constexpr int WTM = 4 * NI, WTN = 4 * NJ;
  static constexpr int BM = NWM * WTM, BN = NWN * WTN, BK = 16;
  static constexpr int THREADS = 64 * NWM * NWN;
  static constexpr int APITCH = BK;       // fragment reads are one contiguous 512 B run
  static constexpr int BPITCH = BN + 4;   // 16 k-rows of a fragment spread over banks
  struct Acc {
    double v[NI][NJ];
  };
  static __device__ __forceinline__ void zero(Acc& a) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) a.v[i][j] = 0.0;
  }
  static __device__ __forceinline__ void chunk(const T* __restrict__ As, const T* __restrict__ Bs,
                                               Acc& acc, int wm, int wn, int lane) {
    const int q = lane & 3, kk = 4 * ((lane >> 2) & 3) + (lane >> 4);
    double af[NI], bf[NJ];
#pragma unroll
    for (int i = 0; i < NI; ++i) af[i] = As[(wm * WTM + 4 * i + q) * APITCH + kk];
#pragma unroll
    for (int j = 0; j < NJ; ++j) bf[j] = Bs[kk * BPITCH + wn * WTN + 4 * j + q];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        acc.v[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[i], bf[j], acc.v[i][j], 0, 0, 0);
  }
  template <class F>
  static __device__ __forceinline__ void epilogue(Acc& acc, int lane, int wm, int wn, F&& f) {
    const int i = lane >> 4, b = (lane >> 2) & 3, j = lane & 3;
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
      for (int c = 0; c < NJ; ++c) {
        double x = acc.v[a][c];
        x += __shfl_xor(x, 4);
        x += __shfl_xor(x, 8);
        acc.v[a][c] = x;
      }
    // after the reduction the four block-lanes hold the same sums; block-lane
    // b stores the fragments whose index is b mod 4
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
      for (int c = 0; c < NJ; ++c)
        if (((a * NJ + c) & 3) == b) f(wm * WTM + 4 * a + i, wn * WTN + 4 * c + j, acc.v[a][c]);
  }
};

// ---------------------------------------------------------------------------
// FP32 policy: v_mfma_f32_16x16x4f32.
//   A operand A[i][k], i = l&15, k = l>>4;  B operand B[k][j], j = l&15, k = l>>4
//   result D[4 (l>>4) + r][l&15], r = 0..3
// The 16-wide k-chunk is permuted so that lane group g = l>>4 owns k = 4g..4g+3
// across the four instructions of a chunk: its A values are one 16-byte read.
// ---------------------------------------------------------------------------
template <int NWM_, int NWN_, int NI_, int NJ_>
struct PolF32 {
  using T = float;
  static constexpr int NWM = NWM_, NWN = NWN_, NI = NI_, NJ = NJ_;
  static constexpr int WTM = 16 * NI, WTN = 16 * NJ;
  static constexpr int BM = NWM * WTM, BN = NWN * WTN, BK = 16;
  static constexpr int THREADS = 64 * NWM * NWN;
  static constexpr int APITCH = BK;       // a wave's A reads are one contiguous 1 KB run
  static constexpr int BPITCH = BN + 4;   // the 4 k-rows of a B read land in distinct banks
  struct Acc {
    f4 v[NI][NJ];
  };
  static __device__ __forceinline__ void zero(Acc& a) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) a.v[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  }
  static __device__ __forceinline__ void chunk(const T* __restrict__ As, const T* __restrict__ Bs,
                                               Acc& acc, int wm, int wn, int lane) {
    const int q = lane & 15, g = lane >> 4;
    f4 af[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i)
      af[i] = *reinterpret_cast<const f4*>(&As[(wm * WTM + 16 * i + q) * APITCH + 4 * g]);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float bf[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) bf[j] = Bs[(4 * g + s) * BPITCH + wn * WTN + 16 * j + q];
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc.v[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s], bf[j], acc.v[i][j], 0, 0, 0);
    }
  }
  template <class F>
  static __device__ __forceinline__ void epilogue(Acc& acc, int lane, int wm, int wn, F&& f) {
    const int q = lane & 15, g = lane >> 4;
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
      for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          f(wm * WTM + 16 * a + 4 * g + r, wn * WTN + 16 * c + q, (double)acc.v[a][c][r]);
  }
};

// ---------------------------------------------------------------------------
// the product kernel (shared by the FP64 and FP32 policies)
// ---------------------------------------------------------------------------
template <class P>
struct Loader {
  using T = typename P::T;
  static constexpr int EPV = 16 / sizeof(T);                 // elements per 16-byte vector
  static constexpr int A_VPR = P::BK / EPV, A_VEC = P::BM * A_VPR;
  static constexpr int B_VPR = P::BN / EPV, B_VEC = P::BK * B_VPR;
  static constexpr int NA = (A_VEC + P::THREADS - 1) / P::THREADS;
  static constexpr int NB = (B_VEC + P::THREADS - 1) / P::THREADS;
  static_assert(A_VEC % P::THREADS == 0 && B_VEC % P::THREADS == 0, "tile not divisible");
  uint4 ra[NA], rb[NB];
  __device__ __forceinline__ void load(const T* __restrict__ X, const T* __restrict__ Y, int ld,
                                       int row0, int col0, int k0, int tid) {
#pragma unroll
    for (int it = 0; it < NA; ++it) {
      const int v = tid + it * P::THREADS, r = v / A_VPR, c = v % A_VPR;
      ra[it] = *reinterpret_cast<const uint4*>(X + (size_t)(row0 + r) * ld + k0 + c * EPV);
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int v = tid + it * P::THREADS, r = v / B_VPR, c = v % B_VPR;
      rb[it] = *reinterpret_cast<const uint4*>(Y + (size_t)(k0 + r) * ld + col0 + c * EPV);
    }
  }
  __device__ __forceinline__ void store(T* As, T* Bs, int tid) {
#pragma unroll
    for (int it = 0; it < NA; ++it) {
      const int v = tid + it * P::THREADS, r = v / A_VPR, c = v % A_VPR;
      *reinterpret_cast<uint4*>(&As[r * P::APITCH + c * EPV]) = ra[it];
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int v = tid + it * P::THREADS, r = v / B_VPR, c = v % B_VPR;
      *reinterpret_cast<uint4*>(&Bs[r * P::BPITCH + c * EPV]) = rb[it];
    }
  }
};

template <class P>
__global__ __launch_bounds__(P::THREADS) void gemm_kernel(const GemmParams p) {
  using T = typename P::T;
  constexpr int A_SZ = P::BM * P::APITCH, B_SZ = P::BK * P::BPITCH;
  __shared__ __align__(16) T smem[2 * (A_SZ + B_SZ)];
  // buffer b: A tile at smem + b * A_SZ, B tile at smem + 2 * A_SZ + b * B_SZ

  const int tiles_m = p.n / P::BM, tiles_n = p.n / P::BN;
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int row0 = tm * P::BM, col0 = tn * P::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / P::NWN, wn = wave % P::NWN;
  const T* X = static_cast<const T*>(p.X);
  const T* Y = static_cast<const T*>(p.Y);

  typename P::Acc acc;
  P::zero(acc);
  Loader<P> ld;
  const int nk = p.n / P::BK;
  ld.load(X, Y, p.ld, row0, col0, 0, tid);
  ld.store(smem, smem + 2 * A_SZ, tid);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int cur = kc & 1;
    const bool more = kc + 1 < nk;
    if (more) ld.load(X, Y, p.ld, row0, col0, (kc + 1) * P::BK, tid);
    P::chunk(smem + cur * A_SZ, smem + 2 * A_SZ + cur * B_SZ, acc, wm, wn, lane);
    if (more) ld.store(smem + (cur ^ 1) * A_SZ, smem + 2 * A_SZ + (cur ^ 1) * B_SZ, tid);
    __syncthreads();
  }

  EpiState st{0.0, 0.f, 0};
  P::epilogue(acc, lane, wm, wn,
              [&](int r, int c, double v) { epi_element(p, row0 + r, col0 + c, v, st); });
  publish_stats<P::THREADS>(p, st, reinterpret_cast<double*>(smem));
}

template <class P>
hipError_t launch(const GemmParams& p, hipStream_t s) {
  if (p.n % P::BM || p.n % P::BN || p.n % P::BK) return hipErrorInvalidValue;
  const int grid = (p.n / P::BM) * (p.n / P::BN);
  hipLaunchKernelGGL(gemm_kernel<P>, dim3(grid), dim3(P::THREADS), 0, s, p);
  return hipGetLastError();
}

// tile choices
using F64Big = PolF64<2, 4, 8, 8>;     // 64 x 128 tile, 8 waves
using F64Small = PolF64<2, 2, 4, 4>;   // 32 x 32 tile, 4 waves
using F32Big = PolF32<2, 2, 4, 4>;     // 128 x 128 tile, 4 waves
using F32Small = PolF32<2, 2, 2, 2>;   // 64 x 64 tile, 4 waves

constexpr int kBigMin = 2048;          // n from which the large tiles are used

}  // namespace

hipError_t launch_gemm_lowp(Engine e, const GemmParams& p, hipStream_t s);  // gemm_lowp.hip
int engine_tile_lowp(Engine e, int n);

int engine_tile(Engine e, int n) {
  switch (e) {
    case ENG_F64: return n >= kBigMin ? 128 : 32;
    case ENG_F32: return n >= kBigMin ? 128 : 64;
    default: return engine_tile_lowp(e, n);
  }
}

hipError_t launch_gemm(Engine e, const GemmParams& p, hipStream_t s) {
  switch (e) {
    case ENG_F64: return p.n >= kBigMin ? launch<F64Big>(p, s) : launch<F64Small>(p, s);
    case ENG_F32: return p.n >= kBigMin ? launch<F32Big>(p, s) : launch<F32Small>(p, s);
    default: return launch_gemm_lowp(e, p, s);
  }
}

}  // namespace ns
