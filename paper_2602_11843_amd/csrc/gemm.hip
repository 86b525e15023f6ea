// Dense n x n x n products on CDNA4 matrix cores with a fused multi-output
// epilogue.  Every matrix product of the series schedules runs here; the
// linear combinations, identity shifts and running-sum updates of the radix
// kernels are applied in the epilogue, so no O(n^2) elementwise kernel runs
// between products.
//
// Engines
//   FP64: v_mfma_f64_16x16x4f64: 128 x 128 tiles from n = 2048 (four waves
//         of 64 x 64, two workgroups per CU), 32 x 32 tiles below (four waves
//         of 16 x 16, four workgroups per CU), except the split-K kernel for
//         padded n in [160, 256].  v_mfma_f64_4x4x4f64 (its four 4x4 blocks
//         as four k-slices of one fragment) serves the split-K kernel.
//   FP32: v_mfma_f32_16x16x4f32.
// Both stage BM x BK and BK x BN tiles through double-buffered LDS with 16-byte
// global loads, one barrier per k-chunk, and order workgroups so that the
// tiles resident on one XCD share rows of X and columns of Y in that XCD's L2.
// The exception is FP64 at padded n in [160, 256], where a product is
// latency-bound: gemm_f64_splitk_kernel below splits k over the waves and
// loads its operands straight into registers.
#include "gemm_device.h"

namespace ns {
namespace {
using namespace dev;

// Kernel arguments of one product (host2 == nullptr) or of two independent
// products of the same shape in one grid of 2 `tiles` workgroups.
MainArgs main_args(const GemmParams& host, const GemmParams* dev, const GemmParams* host2,
                   const GemmParams* dev2, int tiles) {
  MainArgs a{host.X, host.Y, host.n, host.ld, dev, nullptr, nullptr, nullptr, tiles};
  if (host2) {
    a.X2 = host2->X;
    a.Y2 = host2->Y;
    a.epi2 = dev2;
  }
  return a;
}

bool pair_ok(const GemmParams& host, const GemmParams* host2) {
  return !host2 || (host2->n == host.n && host2->ld == host.ld);
}

template <class P>
hipError_t launch(const GemmParams& host, const GemmParams* dev, hipStream_t s,
                  const GemmParams* host2, const GemmParams* dev2) {
  if (host.n % P::BM || host.n % P::BN || host.n % P::BK || !pair_ok(host, host2))
    return hipErrorInvalidValue;
  const int tiles = (host.n / P::BM) * (host.n / P::BN);
  const MainArgs a = main_args(host, dev, host2, dev2, tiles);
  hipLaunchKernelGGL(gemm_kernel<P>, dim3(host2 ? 2 * tiles : tiles), dim3(P::THREADS), 0, s, a);
  return hipGetLastError();
}

template <class Q>
hipError_t launch_low(const GemmParams& host, const GemmParams* dev, hipStream_t s,
                      const GemmParams* host2, const GemmParams* dev2) {
  if (host.n % Q::BM || host.n % Q::BN || host.n % Q::BK || !pair_ok(host, host2))
    return hipErrorInvalidValue;
  const int tiles = (host.n / Q::BM) * (host.n / Q::BN);
  const MainArgs a = main_args(host, dev, host2, dev2, tiles);
  hipLaunchKernelGGL(gemm_lowp_kernel<Q>, dim3(host2 ? 2 * tiles : tiles), dim3(Q::THREADS), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Latency-bound FP64 sizes (kSplitKMin <= n <= kSplitKMax): a 16 x 16 output
// tile per workgroup, so that n = 256 gives 256 workgroups (the 32 x 32 tile
// gives 64), with the k range split over the four waves: wave w takes the
// 16-wide k-chunks w, w + 4, ... and loads its operands straight from global
// memory into the v_mfma_f64_4x4x4f64 operand layout, SK_CB chunks per batch
// with the next batch in flight.  A chunk is 16 MFMAs per wave, far less than
// a load's latency, so an LDS-staged k-loop waits on memory once per chunk;
// here a wave waits about once per batch.  The four partial tiles are summed
// in LDS in wave order before the shared epilogue.  (Above n = 256 the 16 x 16
// tiles re-read X and Y too often: 1.7x slower than 32 x 32 at n = 384.)
// v_mfma_f64_4x4x4f64 lanes (decoded on the device): block b = (l >> 2) & 3
// holds A_b[i][k] at i = l & 3, k = l >> 4 and B_b[k][j] at j = l & 3; its
// result D_b[i][j] sits at i = l >> 4, j = l & 3.  Here the four blocks take
// four disjoint k-slices (k = 4 b + (l >> 4) within a 16-wide chunk) of one
// 4x4 output fragment, and their partial sums are added across lanes.
// ---------------------------------------------------------------------------
constexpr int SK_TILE = 16, SK_WAVES = 4, SK_CB = 4;
constexpr int kSplitKMin = 160, kSplitKMax = 256;

__global__ __launch_bounds__(64 * SK_WAVES, 2) void gemm_f64_splitk_kernel(const MainArgs args) {
  __shared__ double part[SK_WAVES][SK_TILE][SK_TILE + 2];
  __shared__ double stats[(3 + kMaxOut) * SK_WAVES];
  const int tiles = args.n / SK_TILE;
  const Which wp = which_product(args);
  int tm, tn;
  tile_coords(wp.bid, tiles, tiles, tm, tn);
  const int row0 = tm * SK_TILE, col0 = tn * SK_TILE, ld = args.ld;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane & 3, kk = 4 * ((lane >> 2) & 3) + (lane >> 4);
  const double* __restrict__ X = static_cast<const double*>(wp.X) + (size_t)(row0 + q) * ld + kk;
  const double* __restrict__ Y = static_cast<const double*>(wp.Y) + (size_t)kk * ld + col0 + q;
  const int nk = args.n / 16;
  const int mine = nk > w ? (nk - w + SK_WAVES - 1) / SK_WAVES : 0;   // this wave's chunks
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  // operands of batch bt; slots past the wave's last chunk re-read that chunk
  // and are not multiplied
  auto load = [&](int bt, double (&a)[SK_CB][4], double (&b)[SK_CB][4]) {
#pragma unroll
    for (int j = 0; j < SK_CB; ++j) {
      const int c = w + SK_WAVES * min(bt * SK_CB + j, mine - 1);
      const size_t k = (size_t)16 * c;
#pragma unroll
      for (int f = 0; f < 4; ++f) a[j][f] = X[(size_t)4 * f * ld + k];
#pragma unroll
      for (int f = 0; f < 4; ++f) b[j][f] = Y[k * ld + 4 * f];
    }
  };
  if (mine > 0) {
    const int nb = (mine + SK_CB - 1) / SK_CB;
    double a0[SK_CB][4], b0[SK_CB][4];
    load(0, a0, b0);
    for (int bt = 0; bt < nb; ++bt) {
      double a1[SK_CB][4], b1[SK_CB][4];
      load(min(bt + 1, nb - 1), a1, b1);
#pragma unroll
      for (int j = 0; j < SK_CB; ++j) {
        if (bt * SK_CB + j >= mine) break;        // wave-uniform
#pragma unroll
        for (int fi = 0; fi < 4; ++fi)
#pragma unroll
          for (int fj = 0; fj < 4; ++fj)
            acc[fi][fj] = __builtin_amdgcn_mfma_f64_4x4x4f64(a0[j][fi], b0[j][fj], acc[fi][fj], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < SK_CB; ++j)
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          a0[j][f] = a1[j][f];
          b0[j][f] = b1[j][f];
        }
    }
  }
  // sum the four k-slices of each fragment; block-lane b then writes the
  // fragments whose index is b mod 4 (result lane: row l >> 4, column l & 3)
  const int bb = (lane >> 2) & 3, ri = lane >> 4, cj = lane & 3;
#pragma unroll
  for (int fi = 0; fi < 4; ++fi)
#pragma unroll
    for (int fj = 0; fj < 4; ++fj) {
      double x = acc[fi][fj];
      x += __shfl_xor(x, 4);
      x += __shfl_xor(x, 8);
      if (((fi * 4 + fj) & 3) == bb) part[w][4 * fi + ri][4 * fj + cj] = x;
    }
  __syncthreads();
  const GemmParams& p = *wp.epi;
  EpiState st{0.0, 0.f, 0};
  if (threadIdx.x < SK_TILE * SK_TILE / 2) {
    const int r = threadIdx.x / (SK_TILE / 2), cv = (threadIdx.x % (SK_TILE / 2)) * 2;
    double c[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      double v = part[0][r][cv + e];
#pragma unroll
      for (int ww = 1; ww < SK_WAVES; ++ww) v += part[ww][r][cv + e];
      c[e] = v;
    }
    epi_vec<2>(p, row0 + r, col0 + cv, c, st);
  }
  publish_stats<64 * SK_WAVES>(p, st, stats);
}

hipError_t launch_splitk(const GemmParams& host, const GemmParams* dev, hipStream_t s,
                         const GemmParams* host2, const GemmParams* dev2) {
  if (host.n % 32 || host.n > kSplitKMax || !pair_ok(host, host2)) return hipErrorInvalidValue;
  const int t = host.n / SK_TILE;
  const MainArgs a = main_args(host, dev, host2, dev2, t * t);
  hipLaunchKernelGGL(gemm_f64_splitk_kernel, dim3(host2 ? 2 * t * t : t * t), dim3(64 * SK_WAVES), 0,
                     s, a);
  return hipGetLastError();
}

// tile choices
using F64Big = PolF64M16<2, 2, 4, 4>;    // 128 x 128 tile, 16x16x4 MFMA, 4 waves, two per CU
using F64Small = PolF64M16<2, 2, 1, 1, 4>;   // 32 x 32 tile, 16x16x4 MFMA, 4 waves, four per CU
using F32Big = PolF32<2, 2, 4, 8>;     // 128 x 256 tile, 4 waves
using F32Small = PolF32<2, 2, 2, 2>;   // 64 x 64 tile, 4 waves

constexpr int kBigMin = 2048;          // n from which the large tiles are used
// FP32 keeps the 64 x 64 tile up to n = 4096: below it the 128 x 256 tile
// leaves CUs idle (128 workgroups at n = 2048).  Measured per product, one
// output: n = 2048 0.175 against 0.287 ms, 3072 0.560 against 0.759 ms,
// even at 2560 and 3584, and 1.21 against 1.02 ms at 4096.
constexpr int kBigMinF32 = 4096;

}  // namespace

// below panel_min the low-precision engines convert on the way into LDS
using BF3Small = PolLow<2, 2, 1, 1, true>;  // 64 x 64 tile
using H16Small = PolLow<2, 2, 1, 1, false>;

int engine_tile(Engine e, int n) {
  switch (e) {
    case ENG_F64: return n >= kBigMin ? 128 : 32;
    case ENG_F32: return n >= kBigMinF32 ? 256 : 64;
    case ENG_BF16X3:
    case ENG_F16S: return n >= panel_min(e) ? 256 : 64;
  }
  return 256;
}

hipError_t launch_gemm(Engine e, const GemmParams& host, const GemmParams* dev, hipStream_t s,
                       const GemmParams* host2, const GemmParams* dev2) {
  switch (e) {
    case ENG_F64:
      if (host.n >= kBigMin) return launch<F64Big>(host, dev, s, host2, dev2);
      if (host.n >= kSplitKMin && host.n <= kSplitKMax) return launch_splitk(host, dev, s, host2, dev2);
      return launch<F64Small>(host, dev, s, host2, dev2);
    case ENG_F32:
      return host.n >= kBigMinF32 ? launch<F32Big>(host, dev, s, host2, dev2)
                                  : launch<F32Small>(host, dev, s, host2, dev2);
    // from panel_min these engines run from panels (launch_gemm_panels)
    case ENG_BF16X3:
      return panel_path(e, host.n) ? hipErrorInvalidValue : launch_low<BF3Small>(host, dev, s, host2, dev2);
    case ENG_F16S:
      return panel_path(e, host.n) ? hipErrorInvalidValue : launch_low<H16Small>(host, dev, s, host2, dev2);
  }
  return hipErrorInvalidValue;
}

int gemm_grid(Engine e, int n) {
  switch (e) {
    case ENG_F64:
      if (n >= kBigMin) return (n / F64Big::BM) * (n / F64Big::BN);
      if (n >= kSplitKMin && n <= kSplitKMax) return (n / SK_TILE) * (n / SK_TILE);
      return (n / F64Small::BM) * (n / F64Small::BN);
    case ENG_F32:
      return n >= kBigMinF32 ? (n / F32Big::BM) * (n / F32Big::BN) : (n / F32Small::BM) * (n / F32Small::BN);
    case ENG_BF16X3:
    case ENG_F16S:
      return panel_path(e, n) ? (n / 256) * (n / 256) : (n / BF3Small::BM) * (n / BF3Small::BN);
  }
  return 0;
}

}  // namespace ns
