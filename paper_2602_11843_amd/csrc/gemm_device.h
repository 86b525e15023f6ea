// Device code shared by the single-matrix product launches (gemm.hip) and
// the batched persistent kernel (batched.hip): tile order, the MFMA tile
// policies, the LDS-staged fused epilogue and the low-precision kernels.
#pragma once

#include <type_traits>

#include "common.h"

namespace ns {
namespace dev {


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
// Per-thread epilogue statistics; the AMAXO form also tracks every output's
// max-abs (scaled-FP16 products only, so the other kernels carry no extra state).
template <bool AMAXO>
struct EpiStateT {
  double ssq;
  float amax;
  int bad;
};
template <>
struct EpiStateT<true> {
  double ssq;
  float amax;
  int bad;
  float oamax[kMaxOut];
};
using EpiState = EpiStateT<false>;

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
__device__ __forceinline__ void epi_load(const GemmParams& p, size_t idx, double (&z)[kMaxZ][VEC]) {
#pragma unroll
  for (int i = 0; i < kMaxZ; ++i) {
    if (i < p.nz) load_vec<VEC>(p.Z[i], p.zf64[i], idx, z[i]);
    else
#pragma unroll
      for (int e = 0; e < VEC; ++e) z[i][e] = 0.0;
  }
}

template <int VEC, bool AMAXO>
__device__ __forceinline__ void epi_apply(const GemmParams& p, int row, int col, size_t idx,
                                          const double (&c)[VEC], const double (&z)[kMaxZ][VEC],
                                          EpiStateT<AMAXO>& st) {
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
    if constexpr (AMAXO) {
#pragma unroll
      for (int t = 0; t < VEC; ++t) st.oamax[o] = fmaxf(st.oamax[o], (float)fabs(y[t]));
    }
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

template <int VEC, bool AMAXO = false>
__device__ __forceinline__ void epi_vec(const GemmParams& p, int row, int col, const double (&c)[VEC],
                                        EpiStateT<AMAXO>& st) {
  const size_t idx = (size_t)row * p.ld + col;
  double z[kMaxZ][VEC];
  epi_load<VEC>(p, idx, z);
  epi_apply<VEC, AMAXO>(p, row, col, idx, c, z, st);
}

// Two vectors of the general (mixed-type) epilogue, loads first.
template <int VEC, bool AMAXO = false>
__device__ __forceinline__ void epi_vec_pair(const GemmParams& p, int row0, int col0,
                                             const double (&c0)[VEC], int row1, int col1,
                                             const double (&c1)[VEC], EpiStateT<AMAXO>& st) {
  const size_t i0 = (size_t)row0 * p.ld + col0, i1 = (size_t)row1 * p.ld + col1;
  double z0[kMaxZ][VEC], z1[kMaxZ][VEC];
  epi_load<VEC>(p, i0, z0);
  epi_load<VEC>(p, i1, z1);
  epi_apply<VEC, AMAXO>(p, row0, col0, i0, c0, z0, st);
  epi_apply<VEC, AMAXO>(p, row1, col1, i1, c1, z1, st);
}

// The same epilogue when every Z input and every output is FP32: float
// arithmetic, no per-element type branches (fewer registers; used by the FP32
// engine whenever a product's inputs and outputs are all FP32, and always by
// the batched kernel, so both produce identical bits).  Split into the Z loads
// and the arithmetic + stores, so that a caller can issue the loads of two
// vectors before the stores of the first (epi_vec_f32_pair): a store to an
// output may alias a Z input at the same element, which keeps the compiler from
// moving the next vector's loads above it, and one load at a time leaves the
// epilogue waiting on memory latency.
__device__ __forceinline__ void epi_load_f32(const GemmParams& p, size_t idx, float (&z)[kMaxZ][4]) {
#pragma unroll
  for (int i = 0; i < kMaxZ; ++i) {
    if (i < p.nz) {
      const float4 t = *reinterpret_cast<const float4*>(static_cast<const float*>(p.Z[i]) + idx);
      z[i][0] = t.x; z[i][1] = t.y; z[i][2] = t.z; z[i][3] = t.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) z[i][e] = 0.f;
    }
  }
}

template <bool AMAXO>
__device__ __forceinline__ void epi_apply_f32(const GemmParams& p, int row, int col, size_t idx,
                                              const double (&c)[4], const float (&z)[kMaxZ][4],
                                              EpiStateT<AMAXO>& st) {
  constexpr int VEC = 4;
#pragma unroll
  for (int o = 0; o < kMaxOut; ++o) {
    if (o >= p.no) break;
    const EpiOut& e = p.out[o];
    const float a = (float)e.a, id = (float)e.id;
    float zc[kMaxZ];
#pragma unroll
    for (int i = 0; i < kMaxZ; ++i) zc[i] = (float)e.z[i];
    float y[VEC];
#pragma unroll
    for (int t = 0; t < VEC; ++t) {
      y[t] = a * (float)c[t] + ((row == col + t) ? id : 0.f);
#pragma unroll
      for (int i = 0; i < kMaxZ; ++i) y[t] += zc[i] * z[i][t];
    }
    *reinterpret_cast<float4*>(static_cast<float*>(e.ptr) + idx) = make_float4(y[0], y[1], y[2], y[3]);
    if constexpr (AMAXO) {
#pragma unroll
      for (int t = 0; t < VEC; ++t) st.oamax[o] = fmaxf(st.oamax[o], fabsf(y[t]));
    }
    if (o == 0) {
#pragma unroll
      for (int t = 0; t < VEC; ++t) {
        st.ssq += (double)y[t] * (double)y[t];
        if (!isfinite(y[t])) st.bad = 1;
        st.amax = fmaxf(st.amax, fabsf(y[t]));
      }
    }
  }
}

template <int VEC, bool AMAXO = false>
__device__ __forceinline__ void epi_vec_f32(const GemmParams& p, int row, int col,
                                            const double (&c)[VEC], EpiStateT<AMAXO>& st) {
  static_assert(VEC == 4, "float epilogue works on float4 vectors");
  const size_t idx = (size_t)row * p.ld + col;
  float z[kMaxZ][4];
  epi_load_f32(p, idx, z);
  epi_apply_f32<AMAXO>(p, row, col, idx, c, z, st);
}

// Two vectors: both vectors' Z loads first, then the arithmetic and stores.
template <bool AMAXO = false>
__device__ __forceinline__ void epi_vec_f32_pair(const GemmParams& p, int row0, int col0,
                                                 const double (&c0)[4], int row1, int col1,
                                                 const double (&c1)[4], EpiStateT<AMAXO>& st) {
  const size_t i0 = (size_t)row0 * p.ld + col0, i1 = (size_t)row1 * p.ld + col1;
  float z0[kMaxZ][4], z1[kMaxZ][4];
  epi_load_f32(p, i0, z0);
  epi_load_f32(p, i1, z1);
  epi_apply_f32<AMAXO>(p, row0, col0, i0, c0, z0, st);
  epi_apply_f32<AMAXO>(p, row1, col1, i1, c1, z1, st);
}

// true if every Z input and output of the block is FP32
__device__ __forceinline__ bool all_f32(const GemmParams& p) {
  bool f = true;
#pragma unroll
  for (int i = 0; i < kMaxZ; ++i)
    if (i < p.nz && p.zf64[i]) f = false;
#pragma unroll
  for (int o = 0; o < kMaxOut; ++o)
    if (o < p.no && p.out[o].f64) f = false;
  return f;
}

// Reduce the per-thread statistics over the workgroup and publish them with
// one atomic each.  `scratch` is LDS of at least (3 + kMaxOut) * (THREADS / 64)
// doubles; the caller synchronises before the call.  AMAXO also publishes the
// per-output max-abs to EpiOut::amax.
template <int THREADS, bool AMAXO = false>
__device__ __forceinline__ void publish_stats(const GemmParams& p, EpiStateT<AMAXO> st, double* scratch) {
  if (!AMAXO && !p.sumsq && !p.nonfinite && !p.amax) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    st.ssq += __shfl_xor(st.ssq, off);
    st.amax = fmaxf(st.amax, __shfl_xor(st.amax, off));
    st.bad |= __shfl_xor(st.bad, off);
    if constexpr (AMAXO) {
#pragma unroll
      for (int o = 0; o < kMaxOut; ++o) st.oamax[o] = fmaxf(st.oamax[o], __shfl_xor(st.oamax[o], off));
    }
  }
  constexpr int NW = THREADS / 64;
  if (lane == 0) {
    scratch[wave] = st.ssq;
    scratch[NW + wave] = (double)st.amax;
    scratch[2 * NW + wave] = (double)st.bad;
    if constexpr (AMAXO) {
#pragma unroll
      for (int o = 0; o < kMaxOut; ++o) scratch[(3 + o) * NW + wave] = (double)st.oamax[o];
    }
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
    if constexpr (AMAXO) {
      for (int o = 0; o < kMaxOut; ++o) {
        if (o >= p.no || !p.out[o].amax) continue;
        double m = 0.0;
        for (int w = 0; w < NW; ++w) m = fmax(m, scratch[(3 + o) * NW + w]);
        atomicMax(p.out[o].amax, __float_as_uint((float)m));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 policy on v_mfma_f64_16x16x4f64: one instruction is a 16x16 output
// fragment times a 4-deep k-slice (1024 FMAs, 64 matrix-core cycles).
//   A operand A[i][k], i = l&15, k = l>>4;  B operand B[k][j], j = l&15, k = l>>4
//   result D[4 r + (l>>4)][l&15], r = 0..3 (decoded on the device: rows are
//   interleaved, unlike the FP32 16x16x4 form's D[4 (l>>4) + r][l&15])
// As in the FP32 policy the 16-wide k-chunk is permuted: lane group g = l>>4
// owns k = 4g..4g+3 across the four instructions of a chunk, so its A values
// are one 32-byte run of the row.  X-tile rows are 128 bytes; 16-byte chunk c
// of row r is stored at chunk c ^ (r & 7), so the eight rows a 16-byte read
// serves at once fall on distinct banks.
// ---------------------------------------------------------------------------
template <int NWM_, int NWN_, int NI_, int NJ_, int MINB_ = 2>
struct PolF64M16 {
  using T = double;
  static constexpr int NWM = NWM_, NWN = NWN_, NI = NI_, NJ = NJ_;
  // workgroups per CU the register allocation must allow: capped at two, the
  // compiler keeps the accumulators in VGPRs (measured: 2.07 ms per n = 4096
  // product; uncapped it moves them to AGPRs and takes 2.73 ms)
  static constexpr int MINB = MINB_;
  static constexpr int WTM = 16 * NI, WTN = 16 * NJ;
  static constexpr int BM = NWM * WTM, BN = NWN * WTN, BK = 16;
  static constexpr int THREADS = 64 * NWM * NWN;
  static constexpr int APITCH = BK;
  static constexpr int BPITCH = BN + 2;
  static constexpr int EPI_PASSES = NWM;  // stage one wave-row at a time (bounds the LDS)
  static constexpr int DMA_STAGES = 2;
  static __device__ __forceinline__ int a_swz(int r) { return r & 7; }
  static __device__ __forceinline__ int b_swz(int) { return 0; }
  struct Acc {
    d4 v[NI][NJ];
  };
  static __device__ __forceinline__ void zero(Acc& a) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) a.v[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  }
  static __device__ __forceinline__ void chunk(const T* __restrict__ As, const T* __restrict__ Bs,
                                               Acc& acc, int wm, int wn, int lane) {
    const int q = lane & 15, g = lane >> 4;
    double af[NI][4];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int row = wm * WTM + 16 * i + q;
      const double2 t0 = *reinterpret_cast<const double2*>(&As[row * APITCH + ((2 * g) ^ a_swz(row)) * 2]);
      const double2 t1 = *reinterpret_cast<const double2*>(&As[row * APITCH + ((2 * g + 1) ^ a_swz(row)) * 2]);
      af[i][0] = t0.x;
      af[i][1] = t0.y;
      af[i][2] = t1.x;
      af[i][3] = t1.y;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double bf[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) bf[j] = Bs[(4 * g + s) * BPITCH + wn * WTN + 16 * j + q];
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc.v[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][s], bf[j], acc.v[i][j], 0, 0, 0);
    }
  }
  using CT = double;
  static __device__ __forceinline__ void stage(Acc& acc, int lane, int wn, CT* C, int cpitch) {
    const int q = lane & 15, g = lane >> 4;
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
      for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          C[(16 * a + 4 * r + g) * cpitch + wn * WTN + 16 * c + q] = acc.v[a][c][r];
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
  static constexpr int MINB = 1;
  static constexpr int APITCH = BK;       // a wave's A reads are one contiguous 1 KB run
  static constexpr int BPITCH = BN + 4;   // the 4 k-rows of a B read land in distinct banks
  static constexpr int EPI_PASSES = NWM;  // stage one wave-row at a time (bounds the LDS)
  static constexpr int DMA_STAGES = 2;    // LDS buffers of the direct-to-LDS k-loop
  static __device__ __forceinline__ int a_swz(int) { return 0; }   // no LDS swizzle
  static __device__ __forceinline__ int b_swz(int) { return 0; }
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
  // An optional second, independent product of the same shape in the same
  // grid: blocks [tiles, 2 tiles) compute X2 Y2 with epilogue epi2.  tiles is
  // the grid of one product (== gridDim.x for a single product).
  const void* X2;
  const void* Y2;
  const GemmParams* epi2;
  int tiles;
};

// The operands of this workgroup's product and its tile index within that
// product (wave-uniform: a scalar select at kernel start).
struct Which {
  const void* X;
  const void* Y;
  const GemmParams* epi;
  int bid;
};
__device__ __forceinline__ Which which_product(const MainArgs& a) {
  const int b = blockIdx.x;
  if (b >= a.tiles) return Which{a.X2, a.Y2, a.epi2, b - a.tiles};
  return Which{a.X, a.Y, a.epi, b};
}

template <class P>
struct DmaShape {
  using T = typename P::T;
  static constexpr int NW = P::THREADS / 64;
  static constexpr int A_BYTES = P::BM * P::BK * (int)sizeof(T);
  static constexpr int A_INS = A_BYTES / 1024;                 // wave instructions per X tile
  static constexpr bool OK = P::BN * (int)sizeof(T) == 1024 && P::APITCH == P::BK &&
                             A_BYTES % 1024 == 0 && A_INS % NW == 0 && P::BK % NW == 0;
};

// LDS elements (of P::T) a tile needs: two k-chunk stages, or one wave-row
// of FP32/FP64 results for the epilogue, whichever is larger.
template <class P>
constexpr int tile_smem_elems() {
  using T = typename P::T;
  using CT = typename P::CT;
  constexpr int A_SZ = P::BM * P::APITCH, B_SZ = P::BK * P::BPITCH;
  constexpr int CPITCH = P::BN + 16 / (int)sizeof(CT);
  constexpr int STAGE = (P::BM / P::EPI_PASSES * CPITCH * (int)sizeof(CT) + (int)sizeof(T) - 1) /
                        (int)sizeof(T);
  constexpr int LOOP = (DmaShape<P>::OK ? P::DMA_STAGES : 2) * (A_SZ + B_SZ);
  return LOOP > STAGE ? LOOP : STAGE;
}

// acc += X[row0:row0+BM, :K] Y[:K, col0:col0+BN] with double-buffered LDS
// staging of 16-byte vectors and one barrier per k-chunk.  Leaves smem free.
template <class P>
__device__ __forceinline__ void tile_mainloop(const typename P::T* __restrict__ Xp,
                                              const typename P::T* __restrict__ Yp, int ld, int K,
                                              int row0, int col0, typename P::T* smem,
                                              typename P::Acc& acc) {
  using T = typename P::T;
  constexpr int A_SZ = P::BM * P::APITCH, B_SZ = P::BK * P::BPITCH;
  // buffer b: A tile at smem + b * A_SZ, B tile at smem + 2 * A_SZ + b * B_SZ
  constexpr int EPV = 16 / sizeof(T);                        // elements per 16-byte vector
  constexpr int A_VPR = P::BK / EPV, A_VEC = P::BM * A_VPR;  // vectors per row / per tile
  constexpr int B_VPR = P::BN / EPV, B_VEC = P::BK * B_VPR;
  constexpr int NA = A_VEC / P::THREADS, NB = B_VEC / P::THREADS;
  static_assert(A_VEC % P::THREADS == 0 && B_VEC % P::THREADS == 0, "tile not divisible");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / P::NWN, wn = wave % P::NWN;

  size_t ga[NA], gb[NB];
  int sa[NA], sb[NB];
#pragma unroll
  for (int it = 0; it < NA; ++it) {
    const int v = tid + it * P::THREADS, r = v / A_VPR, c = v % A_VPR;
    ga[it] = (size_t)(row0 + r) * ld + c * EPV;
    sa[it] = r * P::APITCH + (c ^ P::a_swz(r)) * EPV;     // the policy's LDS swizzle
  }
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int v = tid + it * P::THREADS, r = v / B_VPR, c = v % B_VPR;
    gb[it] = (size_t)r * ld + col0 + c * EPV;
    sb[it] = r * P::BPITCH + (c ^ P::b_swz(r)) * EPV;
  }
  uint4 ra[NA], rb[NB];
  const int nk = K / P::BK;
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
}

// Direct-to-LDS variant of the k-loop for tiles whose Y-tile rows are exactly
// 1 KB and whose X tile is unpadded: every 16-byte vector goes from global
// memory straight into LDS (global_load_lds_dwordx4 writes lane l's 16 bytes
// at a wave-uniform LDS address + 16 l), so a wave instruction fills one
// contiguous 1 KB run.  The next chunk streams into the idle buffer while the
// matrix cores work on the current one, with no staging registers.
template <class P>
struct DmaPlan {
  using T = typename P::T;
  using D = DmaShape<P>;
  static constexpr int NA = D::A_INS / D::NW, NB = P::BK / D::NW;
  uint32_t a_off[NA];         // element offsets of this lane's vectors, chunk 0
  uint32_t b_off[NB];
  int a_lds[NA], b_lds[NB];   // wave-uniform LDS element offsets within a buffer
  __device__ __forceinline__ void init(int ld, int row0, int col0) {
    constexpr int EPV = 16 / (int)sizeof(T);
    constexpr int ROW_VEC = P::BK / EPV;               // 16-byte vectors per X-tile row
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int ins = wave + i * D::NW;                // this instruction's 1 KB run of the X tile
      // LDS chunk v % ROW_VEC of row r holds global chunk (v % ROW_VEC) ^ a_swz(r)
      const int v = ins * 64 + lane, r = v / ROW_VEC, c = ((v % ROW_VEC) ^ P::a_swz(r)) * EPV;
      // element offsets stay below n^2 <= 2^32 (n <= 65536): unsigned 32-bit
      // arithmetic is exact, where signed int would overflow past n = 46340
      a_off[i] = (uint32_t)(row0 + r) * (uint32_t)ld + (uint32_t)c;
      a_lds[i] = ins * (1024 / (int)sizeof(T));
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int r = wave + i * D::NW;                  // one Y-tile row per instruction
      b_off[i] = (uint32_t)r * (uint32_t)ld + (uint32_t)(col0 + (lane ^ P::b_swz(r)) * EPV);
      b_lds[i] = r * P::BPITCH;
    }
  }
  // issue the loads of k-chunk kc into the LDS buffers As / Bs
  __device__ __forceinline__ void issue(const T* __restrict__ Xp, const T* __restrict__ Yp, int ld,
                                        int kc, T* As, T* Bs) const {
    const T* xa = Xp + (size_t)kc * P::BK;
    const T* yb = Yp + (size_t)kc * P::BK * ld;
#pragma unroll
    for (int i = 0; i < NA; ++i)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(xa + a_off[i]),
                                       (__attribute__((address_space(3))) void*)(As + a_lds[i]), 16, 0, 0);
#pragma unroll
    for (int i = 0; i < NB; ++i)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(yb + b_off[i]),
                                       (__attribute__((address_space(3))) void*)(Bs + b_lds[i]), 16, 0, 0);
  }
};

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding:
// vmcnt in bits 3:0, expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 16, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

template <class P>
__device__ __forceinline__ void tile_mainloop_dma(const typename P::T* __restrict__ Xp,
                                                  const typename P::T* __restrict__ Yp, int ld, int K,
                                                  int row0, int col0, typename P::T* smem,
                                                  typename P::Acc& acc) {
  constexpr int A_SZ = P::BM * P::APITCH, B_SZ = P::BK * P::BPITCH;
  constexpr int S = P::DMA_STAGES;
  constexpr int PER_CHUNK = DmaPlan<P>::NA + DmaPlan<P>::NB;   // this wave's loads per chunk
  static_assert(S == 2 || S == 3, "two or three LDS stages");
  // every load instruction copies one whole 1 KB Y-tile row: any other tile
  // shape would read past the matrix and write past the LDS buffers
  static_assert(DmaShape<P>::OK, "tile shape unsupported by the direct-to-LDS k-loop");
  // buffer b: X tile at smem + b * A_SZ, Y tile at smem + S * A_SZ + b * B_SZ
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / P::NWN, wn = wave % P::NWN;
  const int nk = K / P::BK;
  DmaPlan<P> plan;
  plan.init(ld, row0, col0);
  for (int c = 0; c < S - 1 && c < nk; ++c)
    plan.issue(Xp, Yp, ld, c, smem + c * A_SZ, smem + S * A_SZ + c * B_SZ);
  if constexpr (S == 3) {
    if (nk > 1) wait_vmcnt<PER_CHUNK>();   // chunk 0 landed, chunk 1 may still fly
    else wait_vmcnt<0>();
  } else {
    wait_vmcnt<0>();
  }
  __syncthreads();
  int cur = 0;
  for (int kc = 0; kc < nk; ++kc) {
    // the buffer of chunk kc + S - 1 was last read in iteration kc - 1, which
    // every wave has finished (barrier at its end)
    const int nxt = kc + S - 1;
    const int nb = cur + S - 1 >= S ? cur - 1 : cur + S - 1;
    if (nxt < nk) plan.issue(Xp, Yp, ld, nxt, smem + nb * A_SZ, smem + S * A_SZ + nb * B_SZ);
    P::chunk(smem + cur * A_SZ, smem + S * A_SZ + cur * B_SZ, acc, wm, wn, lane);
    // chunk kc + 1 must be in LDS before the barrier; newer loads may stay in flight
    if (S == 3 && nxt < nk) wait_vmcnt<PER_CHUNK>();
    else wait_vmcnt<0>();
    __syncthreads();
    cur = cur + 1 == S ? 0 : cur + 1;
  }
}

// Epilogue of one tile in EPI_PASSES passes: the waves whose rows fall in the
// pass stage their results in LDS, then the whole workgroup applies the
// affine outputs to those rows with row-contiguous 16-byte vectors (coalesced
// Z reads and output writes).  smem must be free on entry (the k-loops leave
// it so) and is free again on exit.
template <class P, bool F32 = false>
__device__ __forceinline__ void tile_epilogue(typename P::Acc& acc, const GemmParams& p, int row0,
                                              int col0, typename P::T* smem, EpiState& st) {
  using CT = typename P::CT;
  constexpr int CPITCH = P::BN + 16 / (int)sizeof(CT);
  constexpr int VEC = 16 / (int)sizeof(CT);          // 2 doubles or 4 floats
  constexpr int VPR = P::BN / VEC;                   // vectors per row
  constexpr int WROWS = P::NWM / P::EPI_PASSES;      // wave-rows per pass
  constexpr int PROWS = WROWS * P::WTM;              // tile rows per pass
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / P::NWN, wn = wave % P::NWN;
  CT* C = reinterpret_cast<CT*>(smem);
#pragma unroll 1
  for (int pass = 0; pass < P::EPI_PASSES; ++pass) {
    if (wm / WROWS == pass) P::stage(acc, lane, wn, C + (wm % WROWS) * P::WTM * CPITCH, CPITCH);
    __syncthreads();
    if constexpr (F32) {
      // two vectors per step (their Z loads ahead of their stores)
      for (int v = tid; v < PROWS * VPR; v += 2 * P::THREADS) {
        const int r = v / VPR, cv = (v % VPR) * VEC;
        double c[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) c[e] = (double)C[r * CPITCH + cv + e];
        const int v2 = v + P::THREADS;
        if (v2 < PROWS * VPR) {
          const int r2 = v2 / VPR, cv2 = (v2 % VPR) * VEC;
          double c2[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) c2[e] = (double)C[r2 * CPITCH + cv2 + e];
          epi_vec_f32_pair(p, row0 + pass * PROWS + r, col0 + cv, c, row0 + pass * PROWS + r2,
                           col0 + cv2, c2, st);
        } else {
          epi_vec_f32<VEC>(p, row0 + pass * PROWS + r, col0 + cv, c, st);
        }
      }
    } else {
      for (int v = tid; v < PROWS * VPR; v += 2 * P::THREADS) {
        const int r = v / VPR, cv = (v % VPR) * VEC;
        double c[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) c[e] = (double)C[r * CPITCH + cv + e];
        const int v2 = v + P::THREADS;
        if (v2 < PROWS * VPR) {
          const int r2 = v2 / VPR, cv2 = (v2 % VPR) * VEC;
          double c2[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) c2[e] = (double)C[r2 * CPITCH + cv2 + e];
          epi_vec_pair<VEC>(p, row0 + pass * PROWS + r, col0 + cv, c, row0 + pass * PROWS + r2,
                            col0 + cv2, c2, st);
        } else {
          epi_vec<VEC>(p, row0 + pass * PROWS + r, col0 + cv, c, st);
        }
      }
    }
    __syncthreads();
  }
}

template <class P>
__global__ __launch_bounds__(P::THREADS, P::MINB) void gemm_kernel(const MainArgs args) {
  using T = typename P::T;
  __shared__ __align__(16) T smem[tile_smem_elems<P>()];
  const int tiles_m = args.n / P::BM, tiles_n = args.n / P::BN;
  const Which w = which_product(args);
  int tm, tn;
  tile_coords(w.bid, tiles_m, tiles_n, tm, tn);
  const int row0 = tm * P::BM, col0 = tn * P::BN;
  typename P::Acc acc;
  P::zero(acc);
  if constexpr (DmaShape<P>::OK)
    tile_mainloop_dma<P>(static_cast<const T*>(w.X), static_cast<const T*>(w.Y), args.ld,
                         args.n, row0, col0, smem, acc);
  else
    tile_mainloop<P>(static_cast<const T*>(w.X), static_cast<const T*>(w.Y), args.ld, args.n,
                     row0, col0, smem, acc);
  // the epilogue parameters are read from device memory only now, so they
  // occupy no registers while the matrix cores run
  const GemmParams& p = *w.epi;
  EpiState st{0.0, 0.f, 0};
  if constexpr (std::is_same<typename P::CT, float>::value) {
    if (all_f32(p)) tile_epilogue<P, true>(acc, p, row0, col0, smem, st);
    else tile_epilogue<P, false>(acc, p, row0, col0, smem, st);
  } else {
    tile_epilogue<P, false>(acc, p, row0, col0, smem, st);
  }
  publish_stats<P::THREADS>(p, st, reinterpret_cast<double*>(smem));
}

// ---------------------------------------------------------------------------
// Low-precision engines: FP32 operands in HBM, 16-bit MFMA inside.
//   split-BF16: x = x_hi + x_lo with x_hi = bf16(x), x_lo = bf16(x - x_hi)
//               (round to nearest even); X Y ~ Xh Yh + Xh Yl + Xl Yh, three
//               v_mfma_f32_32x32x16_bf16 per fragment pair, FP32 accumulate.
//               BF16 has FP32's exponent range, so no operand scaling is used.
//   scaled FP16: x -> fp16(x * 2^sx) with 2^sx putting max|X| in [2^14, 2^15);
//               one v_mfma_f32_32x32x16_f16 per fragment pair; the product is
//               multiplied by 2^-(sx+sy) (exact) before the epilogue.
// The conversion happens between the global load and the LDS store, so HBM
// and L2 only ever see FP32.  v_mfma_f32_32x32x16_{bf16,f16} lanes:
//   A[i][k]: i = l&31, k = 8 (l>>5) + e;  B[k][j]: j = l&31, k = 8 (l>>5) + e
//   D[8 (r>>2) + 4 (l>>5) + (r&3)][l&31], r = 0..15
// Both operands are stored k-contiguous in LDS ([row][k] for X, [col][k] for
// Y) so each lane's eight k values are one 16-byte read.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <int NWM_, int NWN_, int NI_, int NJ_, bool SPLIT_>
struct PolLow {
  static constexpr bool SPLIT = SPLIT_;
  static constexpr int NWM = NWM_, NWN = NWN_, NI = NI_, NJ = NJ_;
  static constexpr int WTM = 32 * NI, WTN = 32 * NJ;
  static constexpr int BM = NWM * WTM, BN = NWN * WTN, BK = 32;
  static constexpr int THREADS = 64 * NWM * NWN;
  static constexpr int PLANES = SPLIT ? 2 : 1;
  static constexpr int KP = BK + 8;                 // LDS row pitch, 16-bit elements
  static constexpr int A_ELEMS = PLANES * BM * KP, B_ELEMS = PLANES * BN * KP;
  using CT = float;
};

// 2^e for e in [-126, 127] (a normal float)
__device__ __forceinline__ float pow2f(int e) { return __int_as_float((e + 127) << 23); }

// Exponent e with 2^e <= x < 2^(e+1) for the max-abs float bits (0 -> 0),
// raised to at least kMinScaleExp.  An operand whose max-abs lies below
// 2^kMinScaleExp (FP32 denormals included) is scaled as if it were
// 2^kMinScaleExp: the operand scale 2^(14 - e) then stays at most 2^114, a
// normal float, and the operand's entries land below 2^14 in FP16 (tiny ones
// underflow there, as they would in any 16-bit format).  The largest e is 128
// (an Inf or NaN max-abs), giving the normal scale 2^-114.
constexpr int kMinScaleExp = -100;
__device__ __forceinline__ int amax_exponent(const unsigned* amax) {
  if (!amax) return 0;
  const unsigned b = *amax;
  const int e = b ? (int)((b >> 23) & 0xff) - 127 : 0;
  return e < kMinScaleExp ? kMinScaleExp : e;
}

// The product of two operands scaled by 2^(14 - ex) and 2^(14 - ey) is
// unscaled by 2^(ex + ey - 28), applied with ldexp: ex + ey - 28 may fall
// outside the normal exponent range (down to -228), where a formed power of two
// would be wrong; ldexp rounds a result below FP32's range to a denormal or 0.
__device__ __forceinline__ int unscale_exponent(const unsigned* xamax, const unsigned* yamax) {
  return amax_exponent(xamax) + amax_exponent(yamax) - 28;
}

// split 8 floats into bf16 hi / lo (or scaled fp16 in `hi`)
template <bool SPLIT>
__device__ __forceinline__ void convert8(const float (&x)[8], float scale, u16x8& hi, u16x8& lo) {
  if constexpr (SPLIT) {
    bf16x8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 t = (__bf16)x[e];
      h[e] = t;
      l[e] = (__bf16)(x[e] - (float)t);
    }
    hi = __builtin_bit_cast(u16x8, h);
    lo = __builtin_bit_cast(u16x8, l);
  } else {
    f16x8 h;
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = (_Float16)(x[e] * scale);
    hi = __builtin_bit_cast(u16x8, h);
    lo = hi;
  }
}

template <class Q>
__global__ __launch_bounds__(Q::THREADS) void gemm_lowp_kernel(const MainArgs args) {
  constexpr int STAGE_ELEMS = 2 * (Q::A_ELEMS + Q::B_ELEMS);                 // 16-bit
  constexpr int CPITCH = Q::BN + 4;
  constexpr int EPI_ELEMS = (Q::WTM * CPITCH * 4 + 1) / 2;
  constexpr int SMEM = STAGE_ELEMS > EPI_ELEMS ? STAGE_ELEMS : EPI_ELEMS;
  __shared__ __align__(16) unsigned short smem[SMEM];
  // stage b: A planes at b * A_ELEMS, B planes at 2 * A_ELEMS + b * B_ELEMS

  // loader items: A item = (row, k-group of 8), B item = (col, k-group of 8)
  constexpr int KG = Q::BK / 8;
  constexpr int NA = Q::BM * KG / Q::THREADS, NB = Q::BN * KG / Q::THREADS;
  static_assert((Q::BM * KG) % Q::THREADS == 0 && (Q::BN * KG) % Q::THREADS == 0, "loader");

  const int n = args.n, ld = args.ld;
  const int tiles_m = n / Q::BM, tiles_n = n / Q::BN;
  const Which w = which_product(args);
  int tm, tn;
  tile_coords(w.bid, tiles_m, tiles_n, tm, tn);
  const int row0 = tm * Q::BM, col0 = tn * Q::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / Q::NWN, wn = wave % Q::NWN;
  const float* __restrict__ Xp = static_cast<const float*>(w.X);
  const float* __restrict__ Yp = static_cast<const float*>(w.Y);

  float sx = 1.f, sy = 1.f;
  int ush = 0;
  if constexpr (!Q::SPLIT) {
    const int ex = amax_exponent(w.epi->xamax), ey = amax_exponent(w.epi->yamax);
    sx = pow2f(14 - ex);
    sy = pow2f(14 - ey);
    ush = ex + ey - 28;
  }

  // A items: consecutive threads take consecutive k-groups of a row (row-contiguous
  // 32-byte global reads); B items: consecutive threads take consecutive columns
  // (each of the eight k rows is a 256-byte coalesced read per wave)
  size_t ga[NA], gb[NB];
  int la[NA], lb[NB];
#pragma unroll
  for (int it = 0; it < NA; ++it) {
    const int v = tid + it * Q::THREADS, r = v / KG, g = v % KG;
    ga[it] = (size_t)(row0 + r) * ld + 8 * g;
    la[it] = r * Q::KP + 8 * g;
  }
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int v = tid + it * Q::THREADS, c = v % Q::BN, g = v / Q::BN;
    gb[it] = (size_t)(8 * g) * ld + col0 + c;
    lb[it] = c * Q::KP + 8 * g;
  }
  float ra[NA][8], rb[NB][8];

  auto gload = [&](int kc) {
    const size_t ka = (size_t)kc * Q::BK, kb = ka * ld;
#pragma unroll
    for (int it = 0; it < NA; ++it) {
      const float4 u = *reinterpret_cast<const float4*>(Xp + ga[it] + ka);
      const float4 w = *reinterpret_cast<const float4*>(Xp + ga[it] + ka + 4);
      ra[it][0] = u.x; ra[it][1] = u.y; ra[it][2] = u.z; ra[it][3] = u.w;
      ra[it][4] = w.x; ra[it][5] = w.y; ra[it][6] = w.z; ra[it][7] = w.w;
    }
#pragma unroll
    for (int it = 0; it < NB; ++it)
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[it][e] = Yp[gb[it] + kb + (size_t)e * ld];
  };
  auto lstore = [&](int stage) {
    unsigned short* As = smem + stage * Q::A_ELEMS;
    unsigned short* Bs = smem + 2 * Q::A_ELEMS + stage * Q::B_ELEMS;
#pragma unroll
    for (int it = 0; it < NA; ++it) {
      u16x8 h, l;
      convert8<Q::SPLIT>(ra[it], sx, h, l);
      *reinterpret_cast<u16x8*>(As + la[it]) = h;
      if constexpr (Q::SPLIT) *reinterpret_cast<u16x8*>(As + Q::BM * Q::KP + la[it]) = l;
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      u16x8 h, l;
      convert8<Q::SPLIT>(rb[it], sy, h, l);
      *reinterpret_cast<u16x8*>(Bs + lb[it]) = h;
      if constexpr (Q::SPLIT) *reinterpret_cast<u16x8*>(Bs + Q::BN * Q::KP + lb[it]) = l;
    }
  };

  f32x16 acc[Q::NI][Q::NJ];
#pragma unroll
  for (int i = 0; i < Q::NI; ++i)
#pragma unroll
    for (int j = 0; j < Q::NJ; ++j) acc[i][j] = f32x16{};

  const int nk = n / Q::BK;
  gload(0);
  lstore(0);
  __syncthreads();
  const int fr = lane & 31, fk = 8 * (lane >> 5);
  for (int kc = 0; kc < nk; ++kc) {
    const int cur = kc & 1;
    gload(min(kc + 1, nk - 1));     // unconditional prefetch (see the FP64/FP32 kernel)
    const unsigned short* As = smem + cur * Q::A_ELEMS;
    const unsigned short* Bs = smem + 2 * Q::A_ELEMS + cur * Q::B_ELEMS;
#pragma unroll
    for (int ks = 0; ks < Q::BK / 16; ++ks) {
      u16x8 ah[Q::NI], al[Q::NI], bh[Q::NJ], bl[Q::NJ];
#pragma unroll
      for (int i = 0; i < Q::NI; ++i) {
        const int off = (wm * Q::WTM + 32 * i + fr) * Q::KP + 16 * ks + fk;
        ah[i] = *reinterpret_cast<const u16x8*>(As + off);
        if constexpr (Q::SPLIT) al[i] = *reinterpret_cast<const u16x8*>(As + Q::BM * Q::KP + off);
      }
#pragma unroll
      for (int j = 0; j < Q::NJ; ++j) {
        const int off = (wn * Q::WTN + 32 * j + fr) * Q::KP + 16 * ks + fk;
        bh[j] = *reinterpret_cast<const u16x8*>(Bs + off);
        if constexpr (Q::SPLIT) bl[j] = *reinterpret_cast<const u16x8*>(Bs + Q::BN * Q::KP + off);
      }
#pragma unroll
      for (int i = 0; i < Q::NI; ++i)
#pragma unroll
        for (int j = 0; j < Q::NJ; ++j) {
          if constexpr (Q::SPLIT) {
            const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah[i]), Al = __builtin_bit_cast(bf16x8, al[i]);
            const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[j]), Bl = __builtin_bit_cast(bf16x8, bl[j]);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bh, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bl, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bh, acc[i][j], 0, 0, 0);
          } else {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, ah[i]),
                                                              __builtin_bit_cast(f16x8, bh[j]),
                                                              acc[i][j], 0, 0, 0);
          }
        }
    }
    lstore(cur ^ 1);
    __syncthreads();
  }

  // epilogue: stage FP32 results per wave-row pass, apply the affine outputs
  const GemmParams& p = *w.epi;
  float* C = reinterpret_cast<float*>(smem);
  constexpr int VEC = 4, VPR = Q::BN / VEC;
  EpiStateT<!Q::SPLIT> st{};
#pragma unroll 1
  for (int pass = 0; pass < Q::NWM; ++pass) {
    if (wm == pass) {
#pragma unroll
      for (int i = 0; i < Q::NI; ++i)
#pragma unroll
        for (int j = 0; j < Q::NJ; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            C[(32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * CPITCH + wn * Q::WTN + 32 * j + (lane & 31)] =
                ldexpf(acc[i][j][r], ush);
    }
    __syncthreads();
    for (int v = tid; v < Q::WTM * VPR; v += Q::THREADS) {
      const int r = v / VPR, cv = (v % VPR) * VEC;
      double c[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) c[e] = (double)C[r * CPITCH + cv + e];
      epi_vec<VEC, !Q::SPLIT>(p, row0 + pass * Q::WTM + r, col0 + cv, c, st);
    }
    __syncthreads();
  }
  publish_stats<Q::THREADS, !Q::SPLIT>(p, st, reinterpret_cast<double*>(smem));
}

}  // namespace dev
}  // namespace ns
