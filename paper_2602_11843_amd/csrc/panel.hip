// Low-precision products at large n from pre-split 16-bit panels.
//
// The split-BF16 and scaled-FP16 forms (FP32 operands in HBM, 16-bit MFMA
// inside) first rewrite each operand once into 16-bit planes, then run a
// product kernel whose k-loop is nothing but direct-to-LDS loads, 16-byte LDS
// reads and MFMAs.  Converting in the k-loop instead would redo the split of
// every X row panel once per output-tile column (n / BN times); here it is
// done once per operand, by a pass bound by HBM bandwidth.
//
// Planes
//   split-BF16:  x_hi = bf16_rne(x), x_lo = bf16_rne(x - x_hi); X Y is taken
//                as Xh Yh + Xh Yl + Xl Yh with FP32 accumulation.
//   scaled FP16: x_h = fp16_rne(x 2^sx), 2^sx placing max|X| in [2^14, 2^15);
//                the product is multiplied by 2^-(sx+sy) (exact) before the
//                epilogue.
//
// Panel layout of an operand M (n x n, n a multiple of 64): the product needs
// M[r][k] for output row r (X: M = X; Y: M = Y^T, r the output column) with k
// contiguous.  M is cut into 16 x 32 blocks of 1 KB; block (rb, kb) starts at
// element (kb (n/16) + rb) 512, so the BM x 32 k-slab that a workgroup loads
// per k-chunk is BM/16 consecutive KB.  Inside a block, row rr's 16-byte
// chunk c (k = 8c .. 8c+7) sits at rr 32 + 8 (c ^ swz(rr)) with
// swz(rr) = ((rr >> 1) ^ (rr >> 3)) & 3: the sixteen (or eight) lanes that
// one LDS cycle serves for an MFMA fragment read -- consecutive rows, one
// chunk -- then hit distinct banks on a 64-bank and on a 32-bank LDS.
// Plane p of a split operand starts at element p n^2.
//
// Fragment-major layout (the Y operand of the scaled-FP16 product, which its
// waves load straight into registers): one 1 KB unit per (32-row group g,
// 32-deep slab kb, 16-deep step ks), unit ((kb (n/32) + g) 2 + ks) at element
// 512 times that index; lane l's 16 bytes at 8 l hold row 32 g + (l & 31),
// k = 32 kb + 16 ks + 8 (l >> 5) .. + 7 -- exactly the B operand of one
// v_mfma_f32_32x32x16_f16, so one wave load is 1 KB contiguous.
#include "ydirect.h"

namespace ns {
namespace dev {
namespace {

__device__ __forceinline__ int swz(int rr) { return ((rr >> 1) ^ (rr >> 3)) & 3; }

// ---------------------------------------------------------------------------
// FP32 matrix -> 16-bit panels.  One workgroup per 64 x 64 region of M: the
// source is read with row-contiguous 16-byte loads (rows of X, or rows of Y
// for the transposed Y^T), staged in LDS as M[r][k], then every 64 threads
// write one 1 KB block contiguously.
// ---------------------------------------------------------------------------
template <bool SPLIT, bool FRAG>
__global__ __launch_bounds__(256) void to_panels_kernel(const float* __restrict__ src, int n, int ld,
                                                        int transpose, uint16_t* __restrict__ dst,
                                                        const unsigned* __restrict__ amax) {
  static_assert(!(SPLIT && FRAG), "the fragment-major layout holds one fp16 plane");
  __shared__ float t[64][65];
  const int r0 = 64 * blockIdx.y, k0 = 64 * blockIdx.x, tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = tid + 256 * i, a = v >> 4, c4 = (v & 15) * 4;
    if (!transpose) {
      const float4 x = *reinterpret_cast<const float4*>(src + (size_t)(r0 + a) * ld + k0 + c4);
      t[a][c4] = x.x; t[a][c4 + 1] = x.y; t[a][c4 + 2] = x.z; t[a][c4 + 3] = x.w;
    } else {   // src row k0 + a holds M[r0 + c4 ..][k0 + a]
      const float4 x = *reinterpret_cast<const float4*>(src + (size_t)(k0 + a) * ld + r0 + c4);
      t[c4][a] = x.x; t[c4 + 1][a] = x.y; t[c4 + 2][a] = x.z; t[c4 + 3][a] = x.w;
    }
  }
  float scale = 1.f;
  if constexpr (!SPLIT) scale = pow2f(14 - amax_exponent(amax));
  __syncthreads();
  if constexpr (FRAG) {
    // eight 1 KB units per region: (row group, slab, step) = (f & 1, (f >> 1) & 1, f >> 2)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int u = tid + 256 * i, f = u >> 6, l = u & 63;
      const int gl = f & 1, kbl = (f >> 1) & 1, ks = f >> 2;
      const int r = 32 * gl + (l & 31), kk = 32 * kbl + 16 * ks + 8 * (l >> 5);
      const size_t unit = ((size_t)(k0 / 32 + kbl) * (n / 32) + (r0 / 32 + gl)) * 2 + ks;
      f16x8 h;
#pragma unroll
      for (int e = 0; e < 8; ++e) h[e] = (_Float16)(t[r][kk + e] * scale);
      *reinterpret_cast<f16x8*>(dst + unit * 512 + 8 * l) = h;
    }
    return;
  }
  const size_t plane = (size_t)n * n;
  const size_t nb16 = (size_t)(n / 16);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int q = tid + 256 * i;                  // chunk of the region: 8 blocks x 64
    const int blk = q >> 6, pos = q & 63;
    const int rbl = blk & 3, kbl = blk >> 2;
    const int rr = pos >> 2, pc = pos & 3, c = pc ^ swz(rr);
    const int r = 16 * rbl + rr, kk = 32 * kbl + 8 * c;
    const size_t off = ((size_t)(k0 / 32 + kbl) * nb16 + (r0 / 16 + rbl)) * 512 + 8 * pos;
    if constexpr (SPLIT) {
      bf16x8 h, l;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = t[r][kk + e];
        const __bf16 hb = (__bf16)x;
        h[e] = hb;
        l[e] = (__bf16)(x - (float)hb);
      }
      *reinterpret_cast<bf16x8*>(dst + off) = h;
      *reinterpret_cast<bf16x8*>(dst + plane + off) = l;
    } else {
      f16x8 h;
#pragma unroll
      for (int e = 0; e < 8; ++e) h[e] = (_Float16)(t[r][kk + e] * scale);
      *reinterpret_cast<f16x8*>(dst + off) = h;
    }
  }
}

// ---------------------------------------------------------------------------
// Product from panels.  NWM x NWN waves, each owning NI x NJ fragments of
// v_mfma_f32_32x32x16_{bf16,f16}; k-chunk 32 KSLAB (two MFMA k-steps per
// 32-slab), STAGES LDS stages (prefetch distance STAGES - 1).  The epilogue
// stages EFR fragment-rows (32 EFR output rows) per pass.  Stage layout
// (16-bit elements), per slab: the X
// planes' BM/16 blocks, then the Y planes' BN/16 blocks -- the same bytes, in
// the same order, as the global slabs, so every wave instruction of the
// loader copies one 1 KB block.
// ---------------------------------------------------------------------------
// YDIR: Y fragments are loaded by each wave straight from fragment-major
// panels into a ring of D chunks of registers and only X goes through LDS
// (three stages); one fp16 plane, 32-deep chunks.
template <int NWM_, int NWN_, int NI_, int NJ_, bool SPLIT_, int KSLAB_, int STAGES_, int EFR_,
          int MINB_ = 1, bool EPI2_ = true, bool YDIR_ = false, int D_ = 4>
struct PolPanel {
  static constexpr bool YDIR = YDIR_;
  static constexpr int D = D_;
  static_assert(!YDIR || (!SPLIT_ && KSLAB_ == 1 && D_ >= 3), "direct Y: one plane, 32-deep chunks, ring of 3+");
  static constexpr bool EPI2 = EPI2_;     // FP32 epilogue: two vectors per step
  static constexpr int MINB = MINB_;                          // workgroups per CU to fit
  static constexpr bool SPLIT = SPLIT_;
  static constexpr int NWM = NWM_, NWN = NWN_, NI = NI_, NJ = NJ_, KSLAB = KSLAB_;
  static constexpr int STAGES = STAGES_, EFR = EFR_;
  static_assert(STAGES == 2 || STAGES == 3, "two or three LDS stages");
  static_assert(NI % EFR == 0, "epilogue passes");
  static constexpr int WTM = 32 * NI, WTN = 32 * NJ;
  static constexpr int BM = NWM * WTM, BN = NWN * WTN, BK = 32 * KSLAB;
  static constexpr int THREADS = 64 * NWM * NWN, NW = THREADS / 64;
  static constexpr int PLANES = SPLIT ? 2 : 1;
  static constexpr int A_BLK = PLANES * BM / 16, B_BLK = PLANES * BN / 16;   // 1 KB blocks
  static constexpr int A_EL = A_BLK * 512, SLAB_EL = (A_BLK + B_BLK) * 512;
  static constexpr int STAGE_EL = KSLAB * SLAB_EL;
  static constexpr int PER_WAVE = KSLAB * (A_BLK + B_BLK) / NW;
  static_assert((KSLAB * (A_BLK + B_BLK)) % NW == 0, "loader blocks per wave");
  static constexpr int KL_EL = YDIR ? 3 * (BM / 16) * 512 : STAGES * STAGE_EL;   // direct Y: three X chunks
  static constexpr int CPITCH = BN + 4;                       // epilogue staging, floats
  static constexpr int EPI_EL = 32 * EFR * CPITCH * 2;       // one pass, in 16-bit units
  static constexpr int SMEM_EL = KL_EL > EPI_EL ? KL_EL : EPI_EL;
};


template <class Q>
__global__ __launch_bounds__(Q::THREADS, Q::MINB) void gemm_panel_kernel(const MainArgs args) {
  __shared__ __align__(16) uint16_t smem[Q::SMEM_EL];
  const int n = args.n;
  const int tiles_m = n / Q::BM, tiles_n = n / Q::BN;
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int row0 = tm * Q::BM, col0 = tn * Q::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / Q::NWN, wn = wave % Q::NWN;
  const uint16_t* __restrict__ Xp = static_cast<const uint16_t*>(args.X);
  const uint16_t* __restrict__ Yp = static_cast<const uint16_t*>(args.Y);

  f32x16 acc[Q::NI][Q::NJ];
#pragma unroll
  for (int i = 0; i < Q::NI; ++i)
#pragma unroll
    for (int j = 0; j < Q::NJ; ++j) acc[i][j] = f32x16{};

  if constexpr (Q::YDIR) {
    const size_t chunk_el = (size_t)n * 32, yslab = (size_t)(n / 32) * 1024;
    const uint16_t* ybase = Yp + (size_t)((col0 + wn * Q::WTN) / 32) * 1024 + 8 * lane;
    kloop_ydirect<Q>([=](int c) { return Xp + (size_t)c * chunk_el; },
                     [=](int c) { return ybase + (size_t)c * yslab; }, n / 32, row0, lane, wave, wm,
                     smem, acc, [](f32x16& a, const u16x8& x, const u16x8& y) {
                       a = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, x),
                                                                  __builtin_bit_cast(f16x8, y), a, 0, 0, 0);
                     });
  } else {
  const size_t plane = (size_t)n * n;
  const size_t chunk_el = (size_t)n * Q::BK;      // one k-chunk: KSLAB slabs of n/16 blocks

  // loader: this wave's blocks; element offsets within a k-slab (plane
  // included) and LDS offsets within a stage, both per lane
  uint32_t goff[Q::PER_WAVE];
  const uint16_t* gsrc[Q::PER_WAVE];
  int loff[Q::PER_WAVE];
#pragma unroll
  for (int i = 0; i < Q::PER_WAVE; ++i) {
    const int b = wave + i * Q::NW;
    const int slab = b / (Q::A_BLK + Q::B_BLK), bs = b % (Q::A_BLK + Q::B_BLK);
    if (bs < Q::A_BLK) {
      const int p = bs / (Q::BM / 16), rb = bs % (Q::BM / 16);
      gsrc[i] = Xp + (size_t)p * plane;
      goff[i] = (uint32_t)(slab * n * 32 + (row0 / 16 + rb) * 512 + 8 * lane);
    } else {
      const int bb = bs - Q::A_BLK;
      const int p = bb / (Q::BN / 16), cb = bb % (Q::BN / 16);
      gsrc[i] = Yp + (size_t)p * plane;
      goff[i] = (uint32_t)(slab * n * 32 + (col0 / 16 + cb) * 512 + 8 * lane);
    }
    loff[i] = b * 512;
  }
  auto issue = [&](int kc, int stage) {
    const size_t kofs = (size_t)kc * chunk_el;
#pragma unroll
    for (int i = 0; i < Q::PER_WAVE; ++i)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(gsrc[i] + kofs + goff[i]),
          (__attribute__((address_space(3))) void*)(smem + stage * Q::STAGE_EL + loff[i]), 16, 0, 0);
  };

  // fragment reads: lane l takes row (l & 31) of a 32-row fragment and chunk
  // 2 ks + (l >> 5); the row's block and swizzle depend on the lane only
  const int fr = lane & 31, rr = fr & 15;
  const int lrow = (fr >> 4) * 512 + rr * 32;
  const int cofs0 = 8 * ((lane >> 5) ^ swz(rr));           // ks = 0
  const int cofs1 = 8 * ((2 + (lane >> 5)) ^ swz(rr));     // ks = 1

  const int nk = n / Q::BK;
  constexpr int S = Q::STAGES;
  issue(0, 0);
  if constexpr (S == 3) {
    if (nk > 1) {
      issue(1, 1);
      wait_vmcnt<Q::PER_WAVE>();     // chunk 0 landed, chunk 1 may still fly
    } else {
      wait_vmcnt<0>();
    }
  } else {
    wait_vmcnt<0>();
  }
  __syncthreads();
  int cur = 0;
  for (int kc = 0; kc < nk; ++kc) {
    // the stage of chunk kc + S - 1 was last read in iteration kc - 1, which
    // every wave has finished (barrier at its end)
    const int nxt = kc + S - 1;
    if (nxt < nk) issue(nxt, cur == 0 ? S - 1 : cur - 1);
#pragma unroll
    for (int kk = 0; kk < 2 * Q::KSLAB; ++kk) {
      const int ks = kk & 1;
      const uint16_t* As = smem + cur * Q::STAGE_EL + (kk >> 1) * Q::SLAB_EL;
      const uint16_t* Bs = As + Q::A_EL;
      const int co = ks ? cofs1 : cofs0;
      u16x8 ah[Q::NI], al[Q::NI], bh[Q::NJ], bl[Q::NJ];
#pragma unroll
      for (int i = 0; i < Q::NI; ++i) {
        const int off = (wm * Q::WTM / 16 + 2 * i) * 512 + lrow + co;
        ah[i] = *reinterpret_cast<const u16x8*>(As + off);
        if constexpr (Q::SPLIT) al[i] = *reinterpret_cast<const u16x8*>(As + Q::BM * 32 + off);
      }
#pragma unroll
      for (int j = 0; j < Q::NJ; ++j) {
        const int off = (wn * Q::WTN / 16 + 2 * j) * 512 + lrow + co;
        bh[j] = *reinterpret_cast<const u16x8*>(Bs + off);
        if constexpr (Q::SPLIT) bl[j] = *reinterpret_cast<const u16x8*>(Bs + Q::BN * 32 + off);
      }
      if constexpr (Q::SPLIT) {
        // the three partial products in turn over all fragments, so that
        // consecutive MFMAs never wait on each other's accumulator
#pragma unroll
        for (int i = 0; i < Q::NI; ++i)
#pragma unroll
          for (int j = 0; j < Q::NJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al[i]),
                                                                __builtin_bit_cast(bf16x8, bh[j]),
                                                                acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < Q::NI; ++i)
#pragma unroll
          for (int j = 0; j < Q::NJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                                __builtin_bit_cast(bf16x8, bl[j]),
                                                                acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < Q::NI; ++i)
#pragma unroll
          for (int j = 0; j < Q::NJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                                __builtin_bit_cast(bf16x8, bh[j]),
                                                                acc[i][j], 0, 0, 0);
      } else {
#pragma unroll
        for (int i = 0; i < Q::NI; ++i)
#pragma unroll
          for (int j = 0; j < Q::NJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, ah[i]),
                                                               __builtin_bit_cast(f16x8, bh[j]),
                                                               acc[i][j], 0, 0, 0);
      }
    }
    // chunk kc + 1 must be in LDS, and every wave done with chunk kc, before
    // the next iteration overwrites this stage; newer loads may stay in flight
    if constexpr (S == 3) {
      if (nxt < nk) wait_vmcnt<Q::PER_WAVE>();
      else wait_vmcnt<0>();
    } else {
      wait_vmcnt<0>();
    }
    __syncthreads();
    cur = cur + 1 == S ? 0 : cur + 1;
  }
  }   // LDS k-loop

  // epilogue: stage EFR fragment-rows of FP32 results at a time, then apply
  // the affine outputs with row-contiguous 16-byte vectors
  const GemmParams& p = *args.epi;
  int ush = 0;
  if constexpr (!Q::SPLIT) ush = unscale_exponent(p.xamax, p.yamax);
  const bool f32_out = all_f32(p);
  float* C = reinterpret_cast<float*>(smem);
  constexpr int VEC = 4, VPR = Q::BN / VEC;
  EpiStateT<!Q::SPLIT> st{};
  constexpr int PPW = Q::NI / Q::EFR;                // passes per wave-row
  constexpr int PROWS = 32 * Q::EFR;
#pragma unroll 1
  for (int pass = 0; pass < Q::NWM * PPW; ++pass) {
    const int pw = pass / PPW, pi = pass % PPW;
    if (wm == pw) {
#pragma unroll
      for (int i = 0; i < Q::NI; ++i) {
        if (i / Q::EFR != pi) continue;
#pragma unroll
        for (int j = 0; j < Q::NJ; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            C[(32 * (i % Q::EFR) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * Q::CPITCH + wn * Q::WTN +
              32 * j + (lane & 31)] = ldexpf(acc[i][j][r], ush);
      }
    }
    __syncthreads();
    const int grow = row0 + pw * Q::WTM + pi * PROWS;
    if (Q::EPI2 && f32_out) {
      // two vectors per step (their Z loads ahead of their stores)
      for (int v = tid; v < PROWS * VPR; v += 2 * Q::THREADS) {
        const int r = v / VPR, cv = (v % VPR) * VEC;
        double c[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) c[e] = (double)C[r * Q::CPITCH + cv + e];
        const int v2 = v + Q::THREADS;
        if (v2 < PROWS * VPR) {
          const int r2 = v2 / VPR, cv2 = (v2 % VPR) * VEC;
          double c2[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) c2[e] = (double)C[r2 * Q::CPITCH + cv2 + e];
          epi_vec_f32_pair<!Q::SPLIT>(p, grow + r, col0 + cv, c, grow + r2, col0 + cv2, c2, st);
        } else {
          epi_vec_f32<VEC, !Q::SPLIT>(p, grow + r, col0 + cv, c, st);
        }
      }
    } else {
      for (int v = tid; v < PROWS * VPR; v += Q::THREADS) {
        const int r = v / VPR, cv = (v % VPR) * VEC;
        double c[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) c[e] = (double)C[r * Q::CPITCH + cv + e];
        if (f32_out) epi_vec_f32<VEC, !Q::SPLIT>(p, grow + r, col0 + cv, c, st);
        else epi_vec<VEC, !Q::SPLIT>(p, grow + r, col0 + cv, c, st);
      }
    }
    __syncthreads();
  }
  publish_stats<Q::THREADS, !Q::SPLIT>(p, st, reinterpret_cast<double*>(smem));
}

// split-BF16: 256 x 256 tile, 8 waves of 128 x 64, both operands through LDS,
// one workgroup per CU; 64-row epilogue passes
using BF3Panel = PolPanel<2, 4, 4, 2, true, 1, 2, 2>;
// scaled FP16: 128 x 256 tile, 4 waves of 128 x 64, Y in registers, two
// workgroups per CU (one's epilogue runs beside the other's k-loop)
using H16Panel = PolPanel<1, 4, 4, 2, false, 1, 2, 2, 2, true, true, 4>;

template <class Q>
hipError_t launch_panel(const GemmParams& host, const GemmParams* dev, hipStream_t s) {
  if (host.n % Q::BM || host.n % Q::BN || host.ld != host.n) return hipErrorInvalidValue;
  if (Q::YDIR && ((host.n / 32) % Q::D || host.n / 32 < Q::D)) return hipErrorInvalidValue;
  const int grid = (host.n / Q::BM) * (host.n / Q::BN);
  const MainArgs a{host.X, host.Y, host.n, host.ld, dev, nullptr, nullptr, nullptr, grid};
  hipLaunchKernelGGL(gemm_panel_kernel<Q>, dim3(grid), dim3(Q::THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace
}  // namespace dev

bool panel_path(Engine e, int n) {
  return (e == ENG_BF16X3 || e == ENG_F16S) && n >= panel_min(e) && n % 256 == 0;
}

size_t panel_bytes(Engine e, int n) {
  return (size_t)(e == ENG_BF16X3 ? 2 : 1) * n * n * sizeof(uint16_t);
}

hipError_t launch_to_panels(Engine e, const float* src, int n, int ld, int transpose, void* dst,
                            const unsigned* amax, hipStream_t s) {
  if (n % 64 || ld < n) return hipErrorInvalidValue;
  const dim3 grid(n / 64, n / 64);
  if (e == ENG_BF16X3)
    hipLaunchKernelGGL((dev::to_panels_kernel<true, false>), grid, dim3(256), 0, s, src, n, ld,
                       transpose, static_cast<uint16_t*>(dst), amax);
  else if (e == ENG_F16S && transpose)     // the FP16 product loads Y fragment-major
    hipLaunchKernelGGL((dev::to_panels_kernel<false, true>), grid, dim3(256), 0, s, src, n, ld,
                       transpose, static_cast<uint16_t*>(dst), amax);
  else if (e == ENG_F16S)
    hipLaunchKernelGGL((dev::to_panels_kernel<false, false>), grid, dim3(256), 0, s, src, n, ld,
                       transpose, static_cast<uint16_t*>(dst), amax);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gemm_panels(Engine e, const GemmParams& host, const GemmParams* dev, hipStream_t s) {
  switch (e) {
    case ENG_BF16X3: return dev::launch_panel<dev::BF3Panel>(host, dev, s);
    case ENG_F16S: return dev::launch_panel<dev::H16Panel>(host, dev, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ns
