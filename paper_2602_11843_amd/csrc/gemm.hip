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

// Load / store VEC consecutive elements of a row-major matrix at idx as
// doubles; `f64` selects the element type.  idx is a multiple of VEC, so the
// accesses are 8-, 16- or 32-byte aligned vectors.
template <int VEC>
__device__ __forceinline__ void load_vec(const void* p, int f64, size_t idx, double (&v)[VEC]) {
  if (f64) {
    const double2* q = reinterpret_cast<const double2*>(static_cast<const double*>(p) + idx);
#pragma unroll
    for (int i = 0; i < VEC / 2; ++i) {
      const double2 t = q[i];
      v[2 * i] = t.x;
      v[2 * i + 1] = t.y;
    }
  } else {
    if constexpr (VEC == 4) {
      const float4 t = *reinterpret_cast<const float4*>(static_cast<const float*>(p) + idx);
      v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
      const float2 t = *reinterpret_cast<const float2*>(static_cast<const float*>(p) + idx);
      v[0] = t.x; v[1] = t.y;
    }
  }
}

template <int VEC>
__device__ __forceinline__ void store_vec(void* p, int f64, size_t idx, double (&v)[VEC]) {
  if (f64) {
    double2* q = reinterpret_cast<double2*>(static_cast<double*>(p) + idx);
#pragma unroll
    for (int i = 0; i < VEC / 2; ++i) q[i] = make_double2(v[2 * i], v[2 * i + 1]);
  } else {
    if constexpr (VEC == 4) {
      *reinterpret_cast<float4*>(static_cast<float*>(p) + idx) =
          make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    } else {
      *reinterpret_cast<float2*>(static_cast<float*>(p) + idx) = make_float2((float)v[0], (float)v[1]);
    }
#pragma unroll
    for (int i = 0; i < VEC; ++i) v[i] = (double)(float)v[i];   // the value actually stored
  }
}

// Apply the affine epilogue to VEC consecutive product values c[] at
// (row, col .. col + VEC - 1).  Every loop has a compile-time trip count so
// the kernel-argument struct is only ever indexed statically.
template <int VEC>
__device__ __forceinline__ void epi_vec(const GemmParams& p, int row, int col, const double (&c)[VEC],
                                        EpiState& st) {
  const size_t idx = (size_t)row * p.ld + col;
  double z[kMaxZ][VEC];
#pragma unroll
  for (int i = 0; i < kMaxZ; ++i) {
    if (i < p.nz) load_vec<VEC>(p.Z[i], p.zf64[i], idx, z[i]);
    else
#pragma unroll
      for (int e = 0; e < VEC; ++e) z[i][e] = 0.0;
  }
#pragma unroll
  for (int o = 0; o < kMaxOut; ++o) {
    if (o >= p.no) break;
    const EpiOut& e = p.out[o];
    double y[VEC];
#pragma unroll
    for (int t = 0; t < VEC; ++t) {
      y[t] = e.a * c[t] + ((row == col + t) ? e.id : 0.0);
#pragma unroll
      for (int i = 0; i < kMaxZ; ++i) y[t] += e.z[i] * z[i][t];
    }
    store_vec<VEC>(e.ptr, e.f64, idx, y);
    if (o == 0) {
#pragma unroll
      for (int t = 0; t < VEC; ++t) {
        st.ssq += y[t] * y[t];
        if (!isfinite(y[t])) st.bad = 1;
        st.amax = fmaxf(st.amax, (float)fabs(y[t]));
      }
    }
  }
}

// Reduce the per-thread statistics over the workgroup and publish them with
// one atomic each.  `scratch` is LDS of at least 3 * (THREADS / 64) doubles;
// the caller synchronises before the call.
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
  // Sum the four k-slices (lanes differing in bits 2-3), then write this
  // wave's WTM x WTN results into the staging tile C (row pitch CPITCH, rows
  // relative to the wave's first row).
  using CT = double;
  static __device__ __forceinline__ void stage(Acc& acc, int lane, int wn, CT* C, int cpitch) {
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
    // the four block-lanes now hold the same sums; block-lane b writes the
    // fragments whose index is b mod 4
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
      for (int c = 0; c < NJ; ++c)
        if (((a * NJ + c) & 3) == b) C[(4 * a + i) * cpitch + wn * WTN + 4 * c + j] = acc.v[a][c];
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
  using CT = float;
  static __device__ __forceinline__ void stage(Acc& acc, int lane, int wn, CT* C, int cpitch) {
    const int q = lane & 15, g = lane >> 4;
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
      for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          C[(16 * a + 4 * g + r) * cpitch + wn * WTN + 16 * c + q] = acc.v[a][c][r];
  }
};

// ---------------------------------------------------------------------------
// the product kernel (shared by the FP64 and FP32 policies)
// ---------------------------------------------------------------------------
// The kernel's own arguments are only what the k-loop needs; the epilogue
// parameters are read from device memory after the loop, so they occupy no
// registers while the matrix cores run.
struct MainArgs {
  const void* X;
  const void* Y;
  int n;
  int ld;
  const GemmParams* epi;
};

template <class P>
__global__ __launch_bounds__(P::THREADS) void gemm_kernel(const MainArgs args) {
  using T = typename P::T;
  using CT = typename P::CT;
  constexpr int A_SZ = P::BM * P::APITCH, B_SZ = P::BK * P::BPITCH;
  constexpr int CPITCH = P::BN + 16 / (int)sizeof(CT);
  constexpr int STAGE_ELEMS = (P::WTM * CPITCH * (int)sizeof(CT) + (int)sizeof(T) - 1) / (int)sizeof(T);
  constexpr int SMEM_ELEMS = 2 * (A_SZ + B_SZ) > STAGE_ELEMS ? 2 * (A_SZ + B_SZ) : STAGE_ELEMS;
  __shared__ __align__(16) T smem[SMEM_ELEMS];
  // buffer b: A tile at smem + b * A_SZ, B tile at smem + 2 * A_SZ + b * B_SZ

  constexpr int EPV = 16 / sizeof(T);                        // elements per 16-byte vector
  constexpr int A_VPR = P::BK / EPV, A_VEC = P::BM * A_VPR;  // vectors per row / per tile
  constexpr int B_VPR = P::BN / EPV, B_VEC = P::BK * B_VPR;
  constexpr int NA = A_VEC / P::THREADS, NB = B_VEC / P::THREADS;
  static_assert(A_VEC % P::THREADS == 0 && B_VEC % P::THREADS == 0, "tile not divisible");

  const int n = args.n, ld = args.ld;
  const int tiles_m = n / P::BM, tiles_n = n / P::BN;
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int row0 = tm * P::BM, col0 = tn * P::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / P::NWN, wn = wave % P::NWN;

  // per-thread global offsets and LDS offsets of its 16-byte vectors
  const T* __restrict__ Xp = static_cast<const T*>(args.X);
  const T* __restrict__ Yp = static_cast<const T*>(args.Y);
  size_t ga[NA], gb[NB];
  int sa[NA], sb[NB];
#pragma unroll
  for (int it = 0; it < NA; ++it) {
    const int v = tid + it * P::THREADS, r = v / A_VPR, c = v % A_VPR;
    ga[it] = (size_t)(row0 + r) * ld + c * EPV;
    sa[it] = r * P::APITCH + c * EPV;
  }
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int v = tid + it * P::THREADS, r = v / B_VPR, c = v % B_VPR;
    gb[it] = (size_t)r * ld + col0 + c * EPV;
    sb[it] = r * P::BPITCH + c * EPV;
  }
  uint4 ra[NA], rb[NB];

  typename P::Acc acc;
  P::zero(acc);
  const int nk = n / P::BK;
#pragma unroll
  for (int it = 0; it < NA; ++it) ra[it] = *reinterpret_cast<const uint4*>(Xp + ga[it]);
#pragma unroll
  for (int it = 0; it < NB; ++it) rb[it] = *reinterpret_cast<const uint4*>(Yp + gb[it]);
#pragma unroll
  for (int it = 0; it < NA; ++it) *reinterpret_cast<uint4*>(smem + sa[it]) = ra[it];
#pragma unroll
  for (int it = 0; it < NB; ++it) *reinterpret_cast<uint4*>(smem + 2 * A_SZ + sb[it]) = rb[it];
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int cur = kc & 1;
    // prefetch the next chunk (the last iteration re-reads its own chunk into
    // the idle buffer, which nothing reads afterwards: no branch, so the
    // prefetch registers stay in registers across the matrix-core work)
    const size_t ka = (size_t)min(kc + 1, nk - 1) * P::BK, kb = ka * ld;
#pragma unroll
    for (int it = 0; it < NA; ++it) ra[it] = *reinterpret_cast<const uint4*>(Xp + ga[it] + ka);
#pragma unroll
    for (int it = 0; it < NB; ++it) rb[it] = *reinterpret_cast<const uint4*>(Yp + gb[it] + kb);
    P::chunk(smem + cur * A_SZ, smem + 2 * A_SZ + cur * B_SZ, acc, wm, wn, lane);
    T* As = smem + (cur ^ 1) * A_SZ;
    T* Bs = smem + 2 * A_SZ + (cur ^ 1) * B_SZ;
#pragma unroll
    for (int it = 0; it < NA; ++it) *reinterpret_cast<uint4*>(As + sa[it]) = ra[it];
#pragma unroll
    for (int it = 0; it < NB; ++it) *reinterpret_cast<uint4*>(Bs + sb[it]) = rb[it];
    __syncthreads();
  }

  // Epilogue in NWM passes: the waves of wave-row `pass` stage their WTM x BN
  // results in LDS, then the whole workgroup applies the affine outputs to
  // those rows with row-contiguous 16-byte vectors (coalesced Z reads and
  // output writes).  The last loop barrier makes smem free for reuse.
  const GemmParams& p = *args.epi;
  constexpr int VEC = 16 / (int)sizeof(CT);          // 2 doubles or 4 floats
  constexpr int VPR = P::BN / VEC;                   // vectors per row
  CT* C = reinterpret_cast<CT*>(smem);
  EpiState st{0.0, 0.f, 0};
#pragma unroll 1
  for (int pass = 0; pass < P::NWM; ++pass) {
    if (wm == pass) P::stage(acc, lane, wn, C, CPITCH);
    __syncthreads();
    for (int v = tid; v < P::WTM * VPR; v += P::THREADS) {
      const int r = v / VPR, cv = (v % VPR) * VEC;
      double c[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) c[e] = (double)C[r * CPITCH + cv + e];
      epi_vec<VEC>(p, row0 + pass * P::WTM + r, col0 + cv, c, st);
    }
    __syncthreads();
  }
  publish_stats<P::THREADS>(p, st, reinterpret_cast<double*>(smem));
}

template <class P>
hipError_t launch(const GemmParams& host, const GemmParams* dev, hipStream_t s) {
  if (host.n % P::BM || host.n % P::BN || host.n % P::BK) return hipErrorInvalidValue;
  const int grid = (host.n / P::BM) * (host.n / P::BN);
  const MainArgs a{host.X, host.Y, host.n, host.ld, dev};
  hipLaunchKernelGGL(gemm_kernel<P>, dim3(grid), dim3(P::THREADS), 0, s, a);
  return hipGetLastError();
}

// tile choices
using F64Big = PolF64<2, 4, 8, 8>;     // 64 x 128 tile, 8 waves
using F64Small = PolF64<2, 2, 4, 4>;   // 32 x 32 tile, 4 waves
using F32Big = PolF32<2, 2, 4, 4>;     // 128 x 128 tile, 4 waves
using F32Small = PolF32<2, 2, 2, 2>;   // 64 x 64 tile, 4 waves

constexpr int kBigMin = 2048;          // n from which the large tiles are used

}  // namespace

hipError_t launch_gemm_lowp(Engine e, const GemmParams& host, const GemmParams* dev,
                            hipStream_t s);  // gemm_lowp.hip
int engine_tile_lowp(Engine e, int n);

int engine_tile(Engine e, int n) {
  switch (e) {
    case ENG_F64: return n >= kBigMin ? 128 : 32;
    case ENG_F32: return n >= kBigMin ? 128 : 64;
    default: return engine_tile_lowp(e, n);
  }
}

hipError_t launch_gemm(Engine e, const GemmParams& host, const GemmParams* dev, hipStream_t s) {
  switch (e) {
    case ENG_F64: return host.n >= kBigMin ? launch<F64Big>(host, dev, s) : launch<F64Small>(host, dev, s);
    case ENG_F32: return host.n >= kBigMin ? launch<F32Big>(host, dev, s) : launch<F32Small>(host, dev, s);
    default: return launch_gemm_lowp(e, host, dev, s);
  }
}

}  // namespace ns
