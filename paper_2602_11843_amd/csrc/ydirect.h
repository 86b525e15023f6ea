// k-loop of the 16-bit and int8 panel products with the Y operand in
// registers: each wave loads its Y fragments straight from fragment-major
// panels into a ring of D k-chunks of registers, and only X goes through LDS
// (direct-to-LDS copies, three stages).  Included by panel.hip (scaled FP16)
// and ozaki.hip (int8 digit slices).
//
// Units are 16-bit elements.  A k-chunk is one 32-unit slab: two MFMA steps of
// 16 units (16 fp16, or 32 int8, per row).  X chunk c is BM/16 blocks of 1 KB
// (16 rows x 32 units, rows swizzled as in the panel layout); Y chunk c holds,
// for this wave, NJ fragment groups of two 1 KB units (one per step), each unit
// the B operand of one MFMA, lane l's 16 bytes at 8 l.
#pragma once

#include <type_traits>
#include <utility>

#include "gemm_device.h"

namespace ns {
namespace dev {

// s_waitcnt vmcnt(N) lgkmcnt(0) (gfx9 encoding: vmcnt bits 3:0 and 15:14,
// expcnt 6:4 left at its maximum, lgkmcnt 11:8 zero)
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0070);
}

// Workgroup barrier without a memory fence.  The fence of __syncthreads would
// wait for every outstanding load, the register ring's included; the k-loop
// waits for the LDS traffic and the X chunk it needs itself, and the empty asm
// statements keep the compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void bare_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// f(integral_constant<int, U>) for U = 0, 1, ... in order (ring slots must be
// compile-time indices to stay in registers)
template <class F, int... U>
__device__ __forceinline__ void unroll_seq(F&& f, std::integer_sequence<int, U...>) {
  (f(std::integral_constant<int, U>{}), ...);
}

// Re-defines ring registers whose loads the waits have completed, so that the
// compiler carries no pending load for them over the loop's back edge (it
// would otherwise wait for every load at the head of the loop).
template <int A, int B>
__device__ __forceinline__ void settle(u16x8 (&r)[A][B]) {
#pragma unroll
  for (int a = 0; a < A; ++a)
#pragma unroll
    for (int b = 0; b < B; ++b) asm volatile("" : "+v"(r[a][b]));
}

// The panel layout's 16-byte chunk swizzle within a 1 KB block row.
__device__ __forceinline__ int ydir_swz(int rr) { return ((rr >> 1) ^ (rr >> 3)) & 3; }

// One output tile's k-loop over nk chunks (nk a multiple of Q::D, at least
// Q::D; the launchers check).  X chunk c + 2 is copied into LDS while chunk c
// is multiplied, and Y chunk c + D is loaded into the ring slot chunk c has
// just used.  At the end of iteration c every load up to X chunk c + 1 has
// landed (the newest two Y chunks and X chunk c + 2 may fly), so a Y chunk
// has two iterations to arrive.
//   xchunk(c): X chunk c's first block (block b of the tile at + (row0/16 + b) 512)
//   ychunk(c): this wave's Y chunk c (fragment group j at + 1024 j, step ks at + 512 ks)
//   mma(acc, a, b): one MFMA step on 16-byte operands
// Q: NW waves, NI x NJ fragments of 32 x 32 per wave (WTM = 32 NI rows), BM rows, ring depth D.
template <class Q, class Acc, class XChunk, class YChunk, class Mma>
__device__ __forceinline__ void kloop_ydirect(XChunk xchunk, YChunk ychunk, int nk, int row0,
                                              int lane, int wave, int wm, uint16_t* smem,
                                              Acc (&acc)[Q::NI][Q::NJ], Mma mma) {
  constexpr int D = Q::D, NJ = Q::NJ, NI = Q::NI;
  constexpr int XBLK = Q::BM / 16, STAGE = XBLK * 512, PW = XBLK / Q::NW, YOPS = 2 * NJ;
  static_assert(XBLK % Q::NW == 0, "X loader blocks per wave");
  static_assert(D >= 3, "a ring slot is settled one chunk after its reload");
  static_assert(2 * YOPS + PW < 64 && (D - 1) * YOPS < 64, "vmcnt range");
  uint32_t goff[PW];
  int loff[PW];
#pragma unroll
  for (int i = 0; i < PW; ++i) {
    const int b = wave + i * Q::NW;
    goff[i] = (uint32_t)((row0 / 16 + b) * 512 + 8 * lane);
    loff[i] = b * 512;
  }
  auto issue = [&](int c, int stage) {
    const uint16_t* src = xchunk(c);
#pragma unroll
    for (int i = 0; i < PW; ++i)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(src + goff[i]),
          (__attribute__((address_space(3))) void*)(smem + stage * STAGE + loff[i]), 16, 0, 0);
  };
  auto yload = [&](int c, u16x8 (&dst)[2][NJ]) {
    const uint16_t* src = ychunk(c);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int j = 0; j < NJ; ++j) dst[ks][j] = *reinterpret_cast<const u16x8*>(src + j * 1024 + ks * 512);
  };
  // X fragment reads as in the LDS k-loops: lane l takes row (l & 31) of a
  // 32-row fragment and 16-byte chunk 2 ks + (l >> 5)
  const int fr = lane & 31, rr = fr & 15;
  const int lrow = (fr >> 4) * 512 + rr * 32;
  const int cofs0 = 8 * ((lane >> 5) ^ ydir_swz(rr));
  const int cofs1 = 8 * ((2 + (lane >> 5)) ^ ydir_swz(rr));
  u16x8 yb[D][2][NJ];
  issue(0, 0);
  issue(1, 1);
#pragma unroll
  for (int c = 0; c < D; ++c) yload(c, yb[c]);
  wait_vm_lgkm0<(D - 1) * YOPS>();          // X chunks 0 and 1 and ring slot 0 landed
  settle(yb[0]);
  bare_barrier();
  int cur = 0;
  auto step = [&](int k, u16x8 (&ybu)[2][NJ], auto steady) {
    constexpr bool ST = decltype(steady)::value;
    if (ST || k + 2 < nk) issue(k + 2, cur == 0 ? 2 : cur - 1);
    const uint16_t* As = smem + cur * STAGE;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int co = ks ? cofs1 : cofs0;
      u16x8 ah[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i)
        ah[i] = *reinterpret_cast<const u16x8*>(As + (wm * Q::WTM / 16 + 2 * i) * 512 + lrow + co);
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) mma(acc[i][j], ah[i], ybu[ks][j]);
    }
    if constexpr (ST) {
      yload(k + D, ybu);
      wait_vm_lgkm0<2 * YOPS + PW>();
    } else {
      wait_vm_lgkm0<0>();
    }
    bare_barrier();
    cur = cur == 2 ? 0 : cur + 1;
  };
  int kc = 0;
  for (; kc + 2 * D <= nk; kc += D) {
    unroll_seq([&](auto u) { step(kc + u, yb[u], std::true_type{}); },
               std::make_integer_sequence<int, D>{});
    settle(yb[0]);
  }
  unroll_seq([&](auto u) { step(kc + u, yb[u], std::false_type{}); },   // the last D chunks
             std::make_integer_sequence<int, D>{});
}

}  // namespace dev
}  // namespace ns
