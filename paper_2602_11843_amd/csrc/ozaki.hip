// FP64 products emulated from int8 slices with exact integer accumulation
// (Ozaki's error-free splitting), for the residual product A Y of
// R = I - (I - A) Y (Sec. 5.3, eq. (8)) in the FP64-accumulating precision
// forms.
//
// Splitting.  Each row i of X gets the exponent e_i with max_j |X_ij| < 2^e_i;
// x = X_ij 2^-e_i lies in (-1, 1) and is cut into s signed 7-bit digits by
//   t = 128 x,  d = trunc(t) in [-127, 127],  x <- t - d       (all exact),
// so X_ij = 2^e_i (sum_p d_p 2^-7p + r 2^-7s), |r| < 1.  Y is cut the same way
// by columns (exponents f_j).  Then
//   (X Y)_ij ~ 2^(e_i + f_j) sum_{p + q <= s + 1} 2^-7(p+q) (D_p E_q)_ij,
// every D_p E_q an int8 product with int32 accumulation.  The pairs of one
// diagonal d = p + q share their scale, so one diagonal is ONE int8 product
// over the k-concatenation of its d - 1 slice pairs; the longest (d = s + 1)
// sums s n products of two digits, exact while s n 127^2 < 2^31 (n up to
// 16384 for s = 8).  The dropped pairs and the digit remainders bound the
// error by about n 2^(e_i + f_j) (s + 1) 2^-7s.
//
// Layout.  The digits of plane p (p = 0..s-1) form a panel of the n x n int8
// matrix M (X by rows; Y^T, i.e. Y by columns).  X's planes have the byte
// layout of the 16-bit panels of an n x n/2 matrix: 16 x 64-byte blocks of
// 1 KB, block (rb, kb) at byte (kb (n/16) + rb) 1024, row rr's 16-byte chunk c
// at rr 64 + 16 (c ^ swz(rr)).  Y's planes are fragment-major: one 1 KB unit
// per (32-row group g, 64-byte slab kb, 32-byte step ks), unit
// (kb (n/32) + g) 2 + ks, lane l's 16 bytes at 16 l holding row 32 g + (l & 31),
// k = 64 kb + 32 ks + 16 (l >> 5) .. + 15 -- one MFMA B operand.  So the product
// kernel's X loader and fragment reads are the 16-bit panel kernel's, in
// 16-bit units, and its waves load Y straight into registers (ydirect.h).
//
// Product.  One launch per diagonal, d = s + 1 down to 2, each over K = (d - 1) n:
// k-chunk c reads X plane j = c / (n/64) and Y plane d - 2 - j.  The launch of
// the last diagonal adds the FP64 partial sum of the earlier ones, scales by
// 2^(e_i + f_j) and applies the product's affine epilogue; the others write
// their partial sum (FP64) to an accumulator matrix.
//
// Residue form (NS_RESID_CRT).  X_ij = 2^e_i x with |x| < 1 becomes the integer
// X'_ij = rint(2^B x), |X'| <= 2^B (B = kCrtBits), and Y'_ij likewise by
// columns, so X Y ~ 2^(e_i + f_j - 2B) X'Y' with an error of about
// n 2^(e_i + f_j - B), the int8 form's bound at s = 7.  X'Y' is an exact
// integer with |X'Y'| <= n 2^2B.  For pairwise-coprime moduli m_1..m_N <= 256
// with product M > 4 n 2^2B, the residues of X' and Y' modulo m_l fit int8
// (symmetric range), one int8 product per modulus gives X'Y' mod m_l exactly
// (int32 sums of n products of at most 2^14), and the Chinese remainder
// theorem rebuilds X'Y' = sum_l M_l t_l - q M (M_l = M / m_l, t_l = (X'Y' mod
// m_l) (M_l^-1 mod m_l) mod m_l, q the nearest integer to that sum over M)
// with FP64 limbs of 32 bits, every step exact until the final conversion.
// N = 14 products at n = 8192 where the int8 form at s = 7 takes 28.
#include "ydirect.h"

namespace ns {
namespace dev {
namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef unsigned long long u64;

__device__ __forceinline__ int swz8(int rr) { return ((rr >> 1) ^ (rr >> 3)) & 3; }

// smallest e with max < 2^e for the bits of a non-negative double max (0 for 0)
__device__ __forceinline__ int exp_above(u64 bits) {
  if (bits == 0) return 0;
  const int ef = (int)((bits >> 52) & 0x7ff);
  return ef == 0 ? -1022 : ef - 1022;
}
__device__ __forceinline__ bool max_finite(u64 bits) { return ((bits >> 52) & 0x7ff) != 0x7ff; }

// Row and/or column max-abs of an n x n FP64 matrix, as the bits of
// non-negative doubles, atomically into zeroed arrays.  Block: 64 rows x 256
// columns, one column per thread.  NaN entries are recorded as Inf.
__global__ __launch_bounds__(256) void maxabs_rc_kernel(const double* __restrict__ src, int n,
                                                        u64* __restrict__ rowmax,
                                                        u64* __restrict__ colmax) {
  __shared__ double wred[4][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = blockIdx.x * 256 + tid, r0 = blockIdx.y * 64;
  double cm = 0.0;
  for (int r = 0; r < 64; ++r) {
    double v = fabs(src[(size_t)(r0 + r) * n + c]);
    if (v != v) v = INFINITY;
    cm = fmax(cm, v);
    if (rowmax) {
      double m = v;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
      if (lane == 0) wred[wave][r] = m;
    }
  }
  if (colmax) atomicMax(&colmax[c], (u64)__double_as_longlong(cm));
  if (rowmax) {
    __syncthreads();
    if (tid < 64) {
      const double m = fmax(fmax(wred[0][tid], wred[1][tid]), fmax(wred[2][tid], wred[3][tid]));
      atomicMax(&rowmax[r0 + tid], (u64)__double_as_longlong(m));
    }
  }
}

// Moduli of the residue form, as the slicing kernel takes them.
struct CrtMods {
  int n;
  double m[kMaxCrtModuli];
  double inv[kMaxCrtModuli];    // 1 / m, rounded
};

// int8 residue of the integer x (|x| < 2^53) modulo m, in the symmetric range
// (r - m for r > 127: at least -128 for m = 256, -127 for odd m)
__device__ __forceinline__ unsigned residue8(double x, double m, double inv) {
  const double q = floor(x * inv);
  double r = fma(-q, m, x);                   // exact: an integer below 2 m in magnitude
  if (r < 0.0) r += m;
  else if (r >= m) r -= m;
  int ri = (int)r;
  if (ri > 127) ri -= (int)m;
  return (unsigned)ri & 0xffu;
}

// The s digit planes of an n x n FP64 matrix (transpose = 0: M = src by rows;
// 1: M = src^T, i.e. by columns), with the exponent of M's row r from mx[r];
// with CRT, the cm.n residue planes of its rows scaled to integers instead.
// One workgroup per 64 x 64 region of M, staged in LDS as M[r][k]; each thread
// then writes one 16-byte chunk of every plane.
template <bool CRT>
__global__ __launch_bounds__(256) void slices_kernel(const double* __restrict__ src, int n,
                                                     int transpose, const u64* __restrict__ mx,
                                                     int s, int8_t* __restrict__ dst, CrtMods cm) {
  __shared__ double t[64][65];
  const int r0 = 64 * blockIdx.y, k0 = 64 * blockIdx.x, tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int v = tid + 256 * i, a = v >> 5, c2 = (v & 31) * 2;
    if (!transpose) {
      const double2 x = *reinterpret_cast<const double2*>(src + (size_t)(r0 + a) * n + k0 + c2);
      t[a][c2] = x.x;
      t[a][c2 + 1] = x.y;
    } else {   // src row k0 + a holds M[r0 + c2 ..][k0 + a]
      const double2 x = *reinterpret_cast<const double2*>(src + (size_t)(k0 + a) * n + r0 + c2);
      t[c2][a] = x.x;
      t[c2 + 1][a] = x.y;
    }
  }
  __syncthreads();
  // each thread: 16 consecutive k of one row of M, written as one 16-byte
  // chunk per plane -- by rows (X) one chunk of the swizzled blocks, by
  // columns (Y) one lane's share of a fragment-major unit
  int r, kk;
  size_t off;
  if (!transpose) {
    const int blk = tid >> 6, pos = tid & 63, rr = pos >> 2, pc = pos & 3;
    r = 16 * blk + rr;
    kk = 16 * (pc ^ swz8(rr));
    off = ((size_t)(k0 / 64) * (n / 16) + (r0 / 16 + blk)) * 1024 + 16 * pos;
  } else {
    const int u = tid >> 6, l = tid & 63, gl = u & 1, ks = u >> 1;
    r = 32 * gl + (l & 31);
    kk = 32 * ks + 16 * (l >> 5);
    off = (((size_t)(k0 / 64) * (n / 32) + (r0 / 32 + gl)) * 2 + ks) * 1024 + 16 * l;
  }
  const int e = exp_above(mx[r0 + r]);
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const double v = ldexp(t[r][kk + i], -e);
    x[i] = (v == v && fabs(v) < 1.0) ? v : 0.0;   // non-finite rows are flagged by the product
  }
  const size_t plane = (size_t)n * n;
  if constexpr (CRT) {
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = rint(ldexp(x[i], kCrtBits));   // |x| <= 2^B, an integer
    for (int p = 0; p < cm.n; ++p) {
      i32x4 w;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        unsigned b = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) b |= residue8(x[4 * q + i], cm.m[p], cm.inv[p]) << (8 * i);
        w[q] = (int)b;
      }
      *reinterpret_cast<i32x4*>(dst + p * plane + off) = w;
    }
    return;
  }
  for (int p = 0; p < s; ++p) {
    i32x4 w;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      unsigned b = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double tt = 128.0 * x[4 * q + i];
        const double d = trunc(tt);
        x[4 * q + i] = tt - d;
        b |= ((unsigned)(int)d & 0xffu) << (8 * i);
      }
      w[q] = (int)b;
    }
    *reinterpret_cast<i32x4*>(dst + p * plane + off) = w;
  }
}

// One diagonal of the emulated product.
struct I8Args {
  const uint16_t* X;        // digit planes of X (rows), viewed as 16-bit panels
  const uint16_t* Y;        // digit planes of Y (columns)
  int n;                    // padded n, a multiple of 256
  int d;                    // diagonal p + q (2 .. s + 1)
  int first, last;          // first: no partial sum to add; last: apply the epilogue
  double* acc;              // FP64 partial sums, n x n
  const u64* rowmax;        // X row max-abs bits
  const u64* colmax;        // Y column max-abs bits
  const GemmParams* epi;    // the product's epilogue (device), read by the last launch
  // residue form: with tout set, the launch writes t = (P mod m) y mod m of its
  // int32 product P as bytes to tout (row-major n x n) and nothing else
  int crt_m = 0, crt_y = 0;
  uint8_t* tout = nullptr;
};

// 128 x 256 tile, 4 waves of 128 x 64 (4 x 2 fragments of
// v_mfma_i32_32x32x32_i8), k-chunk 64 int8 (two MFMA steps), X through LDS
// (three stages of 8 KB), Y in a ring of D chunks of registers; two
// workgroups per CU, so one's epilogue (FP64 partial sums) runs beside the
// other's k-loop.
struct PolI8 {
  static constexpr int NWM = 1, NWN = 4, NI = 4, NJ = 2, D = 4, MINB = 2;
  static constexpr int WTM = 32 * NI, WTN = 32 * NJ;
  static constexpr int BM = NWM * WTM, BN = NWN * WTN;
  static constexpr int THREADS = 64 * NWM * NWN, NW = THREADS / 64;
  static constexpr int EFR = 2;                      // fragment-rows per epilogue pass
  static constexpr int CPITCH = BN + 4;              // epilogue staging, int32
  static constexpr int EPI_EL = 32 * EFR * CPITCH * 2;
  static constexpr int KL_EL = 3 * (BM / 16) * 512;
  static constexpr int SMEM_EL = KL_EL > EPI_EL ? KL_EL : EPI_EL;
};

template <class Q>
__global__ __launch_bounds__(Q::THREADS, Q::MINB) void gemm_i8_kernel(const I8Args args) {
  __shared__ __align__(16) uint16_t smem[Q::SMEM_EL];
  const int n = args.n;
  const int tiles_m = n / Q::BM, tiles_n = n / Q::BN;
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int row0 = tm * Q::BM, col0 = tn * Q::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / Q::NWN, wn = wave % Q::NWN;
  const size_t plane16 = (size_t)n * n / 2;          // one digit plane, 16-bit units
  const size_t chunk_el = (size_t)n * 32;            // one 64-byte slab of X's row blocks
  const size_t yslab = (size_t)(n / 32) * 1024;      // one slab of Y's fragment units
  const int nkp = n / 64;                            // k-chunks per plane
  const int nk = (args.d - 1) * nkp;
  const uint16_t* const X = args.X;
  const uint16_t* const Yw = args.Y + (size_t)((col0 + wn * Q::WTN) / 32) * 1024 + 8 * lane;
  const int d2 = args.d - 2;

  i32x16 acc[Q::NI][Q::NJ];
#pragma unroll
  for (int i = 0; i < Q::NI; ++i)
#pragma unroll
    for (int j = 0; j < Q::NJ; ++j) acc[i][j] = i32x16{};

  // chunk c: X plane j = c / nkp with Y plane d - 2 - j, slab c - j nkp of both
  kloop_ydirect<Q>(
      [=](int c) {
        const int j = c / nkp;
        return X + (size_t)j * plane16 + (size_t)(c - j * nkp) * chunk_el;
      },
      [=](int c) {
        const int j = c / nkp;
        return Yw + (size_t)(d2 - j) * plane16 + (size_t)(c - j * nkp) * yslab;
      },
      nk, row0, lane, wave, wm, smem, acc, [](i32x16& a, const u16x8& x, const u16x8& y) {
        a = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i32x4, x), __builtin_bit_cast(i32x4, y), a,
                                                  0, 0, 0);
      });

  // epilogue: stage EFR fragment-rows of int32 results at a time; each thread
  // then handles row-contiguous vectors of 4
  int* C = reinterpret_cast<int*>(smem);
  constexpr int VEC = 4, VPR = Q::BN / VEC;
  constexpr int PPW = Q::NI / Q::EFR, PROWS = 32 * Q::EFR;
  const double dscale = ldexp(1.0, -7 * args.d);
  EpiState st{0.0, 0.f, 0};
  const GemmParams* p = args.last ? args.epi : nullptr;
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
              32 * j + (lane & 31)] = acc[i][j][r];
      }
    }
    __syncthreads();
    const int grow = row0 + pw * Q::WTM + pi * PROWS;
    for (int v = tid; v < PROWS * VPR; v += Q::THREADS) {
      const int r = v / VPR, cv = (v % VPR) * VEC;
      const int row = grow + r, col = col0 + cv;
      const size_t idx = (size_t)row * n + col;
      if (args.tout) {
        unsigned w = 0;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          int rm = C[r * Q::CPITCH + cv + e] % args.crt_m;
          if (rm < 0) rm += args.crt_m;
          w |= (unsigned)((rm * args.crt_y) % args.crt_m) << (8 * e);
        }
        *reinterpret_cast<unsigned*>(args.tout + idx) = w;
        continue;
      }
      double c[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) c[e] = (double)C[r * Q::CPITCH + cv + e] * dscale;
      if (!args.first) {
        const double2 a0 = *reinterpret_cast<const double2*>(args.acc + idx);
        const double2 a1 = *reinterpret_cast<const double2*>(args.acc + idx + 2);
        c[0] += a0.x; c[1] += a0.y; c[2] += a1.x; c[3] += a1.y;
      }
      if (!args.last) {
        *reinterpret_cast<double2*>(args.acc + idx) = make_double2(c[0], c[1]);
        *reinterpret_cast<double2*>(args.acc + idx + 2) = make_double2(c[2], c[3]);
        continue;
      }
      const u64 rb = args.rowmax[row];
      const int er = exp_above(rb);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const u64 cb = args.colmax[col + e];
        c[e] = (max_finite(rb) && max_finite(cb)) ? ldexp(c[e], er + exp_above(cb)) : NAN;
      }
      epi_vec<VEC>(*p, row, col, c, st);
    }
    __syncthreads();
  }
  if (args.last) publish_stats<Q::THREADS>(*p, st, reinterpret_cast<double*>(smem));
}

// Chinese-remainder constants of one padded n.
struct CrtConsts {
  int n;                          // moduli
  double ml[kMaxCrtModuli][4];    // M / m_l in 32-bit limbs, low first
  double mm[4];                   // M in 32-bit limbs
  double inv_md;                  // 1 / M, rounded
};

// Rebuild X'Y' from its reduced residues t_l, scale by 2^(e_i + f_j - 2B) and
// apply the product's epilogue: four consecutive elements of one row per
// thread, 1024 columns per workgroup.
__global__ __launch_bounds__(256) void crt_combine_kernel(const uint8_t* __restrict__ t, int n,
                                                          CrtConsts cc, const u64* __restrict__ rowmax,
                                                          const u64* __restrict__ colmax,
                                                          const GemmParams* __restrict__ epi) {
  __shared__ double scratch[(3 + kMaxOut) * 4];
  const int bpr = (n + 1023) / 1024;
  const int row = blockIdx.x / bpr, col = (blockIdx.x % bpr) * 1024 + 4 * threadIdx.x;
  constexpr double TWO32 = 4294967296.0, INV32 = 1.0 / 4294967296.0;
  EpiState st{0.0, 0.f, 0};
  if (col < n) {
    const size_t idx = (size_t)row * n + col;
    const size_t plane = (size_t)n * n;
    // every plane's word is loaded before the first is used, so the loads
    // overlap instead of each waiting for the previous one
    unsigned w[kMaxCrtModuli];
#pragma unroll
    for (int l = 0; l < kMaxCrtModuli; ++l)
      w[l] = l < cc.n ? *reinterpret_cast<const unsigned*>(t + l * plane + idx) : 0u;
    const u64 rb = rowmax[row];
    u64 cb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) cb[e] = colmax[col + e];
    double L[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int j = 0; j < 4; ++j) L[e][j] = 0.0;
#pragma unroll
    for (int l = 0; l < kMaxCrtModuli; ++l) {
      if (l >= cc.n) break;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double te = (double)((w[l] >> (8 * e)) & 0xffu);
#pragma unroll
        for (int j = 0; j < 4; ++j) L[e][j] = fma(te, cc.ml[l][j], L[e][j]);   // < 2^44: exact
      }
    }
    const int er = exp_above(rb);
    double c[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double* v = L[e];
#pragma unroll
      for (int j = 0; j < 3; ++j) {            // limbs into [0, 2^32)
        const double cr = floor(v[j] * INV32);
        v[j] = fma(-cr, TWO32, v[j]);
        v[j + 1] += cr;
      }
      const double sd = ((v[3] * TWO32 + v[2]) * TWO32 + v[1]) * TWO32 + v[0];
      const double q = rint(sd * cc.inv_md);   // the sum is within M / 4 of q M
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = fma(-q, cc.mm[j], v[j]);
      double sg = 1.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double cr = floor(v[j] * INV32);
        v[j] = fma(-cr, TWO32, v[j]);
        v[j + 1] += cr;
      }
      if (v[3] < 0.0) {                        // negative: take the magnitude's limbs
        sg = -1.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = -v[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double cr = floor(v[j] * INV32);
          v[j] = fma(-cr, TWO32, v[j]);
          v[j + 1] += cr;
        }
      }
      const double z = sg * (((v[3] * TWO32 + v[2]) * TWO32 + v[1]) * TWO32 + v[0]);
      c[e] = (max_finite(rb) && max_finite(cb[e])) ? ldexp(z, er + exp_above(cb[e]) - 2 * kCrtBits)
                                                   : NAN;
    }
    epi_vec<4>(*epi, row, col, c, st);
  }
  publish_stats<256>(*epi, st, scratch);
}

}  // namespace
}  // namespace dev

int i8_tile() { return dev::PolI8::BN; }    // BN = 256 is a multiple of BM = 128

hipError_t launch_maxabs_rc(const double* src, int n, unsigned long long* rowmax,
                            unsigned long long* colmax, hipStream_t s) {
  if (n % 256 || (!rowmax && !colmax)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dev::maxabs_rc_kernel, dim3(n / 256, n / 64), dim3(256), 0, s, src, n, rowmax,
                     colmax);
  return hipGetLastError();
}

hipError_t launch_i8_slices(const double* src, int n, int transpose, const unsigned long long* mx,
                            int slices, void* dst, hipStream_t s) {
  if (n % 64 || slices < 1 || slices > kMaxI8Slices) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dev::slices_kernel<false>, dim3(n / 64, n / 64), dim3(256), 0, s, src, n, transpose,
                     mx, slices, static_cast<int8_t*>(dst), dev::CrtMods{});
  return hipGetLastError();
}

hipError_t launch_gemm_i8(const void* xs, const void* ys, int n, int slices, double* acc,
                          const unsigned long long* rowmax, const unsigned long long* colmax,
                          const GemmParams* epi, hipStream_t s) {
  using Q = dev::PolI8;
  if (n % Q::BM || n % Q::BN || slices < 1 || slices > kMaxI8Slices) return hipErrorInvalidValue;
  if ((n / 64) % Q::D) return hipErrorInvalidValue;   // k-chunks per plane: a whole number of ring turns
  const int grid = (n / Q::BM) * (n / Q::BN);
  for (int d = slices + 1; d >= 2; --d) {
    const dev::I8Args a{static_cast<const uint16_t*>(xs), static_cast<const uint16_t*>(ys), n, d,
                        d == slices + 1, d == 2, acc, rowmax, colmax, epi};
    hipLaunchKernelGGL(dev::gemm_i8_kernel<Q>, dim3(grid), dim3(Q::THREADS), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {

// Pairwise-coprime moduli, largest first (256 = 2^8; 255 = 3 5 17;
// 253 = 11 23; 247 = 13 19; 217 = 7 31; the others prime).
constexpr int kCrtModuli[kMaxCrtModuli] = {256, 255, 253, 251, 247, 241, 239, 233,
                                           229, 227, 223, 217, 211, 199, 197, 193};
typedef unsigned __int128 u128;

// (a^-1) mod m for gcd(a, m) = 1
int inverse_mod(int a, int m) {
  int r0 = m, r1 = a % m, s0 = 0, s1 = 1;
  while (r1) {
    const int q = r0 / r1, r2 = r0 - q * r1, s2 = s0 - q * s1;
    r0 = r1; r1 = r2; s0 = s1; s1 = s2;
  }
  return ((s0 % m) + m) % m;
}

void limbs(u128 v, double (&out)[4]) {
  for (int j = 0; j < 4; ++j) {
    out[j] = (double)(unsigned long long)(v & 0xffffffffu);
    v >>= 32;
  }
}

}  // namespace

int crt_moduli(int n) {
  const u128 need = (u128)n << (2 * kCrtBits + 2);
  u128 M = 1;
  for (int l = 0; l < kMaxCrtModuli; ++l) {
    M *= (u128)kCrtModuli[l];
    if (M > need) return l + 1;
  }
  return 0;   // n too large for the table
}

hipError_t launch_crt_slices(const double* src, int n, int transpose, const unsigned long long* mx,
                             void* dst, hipStream_t s) {
  const int N = crt_moduli(n);
  if (n % 64 || N == 0) return hipErrorInvalidValue;
  dev::CrtMods cm{};
  cm.n = N;
  for (int l = 0; l < N; ++l) {
    cm.m[l] = kCrtModuli[l];
    cm.inv[l] = 1.0 / kCrtModuli[l];
  }
  hipLaunchKernelGGL(dev::slices_kernel<true>, dim3(n / 64, n / 64), dim3(256), 0, s, src, n, transpose,
                     mx, N, static_cast<int8_t*>(dst), cm);
  return hipGetLastError();
}

hipError_t launch_gemm_crt(const void* xs, const void* ys, int n, void* tplanes,
                           const unsigned long long* rowmax, const unsigned long long* colmax,
                           const GemmParams* epi, hipStream_t s) {
  using Q = dev::PolI8;
  const int N = crt_moduli(n);
  if (n % Q::BM || n % Q::BN || N == 0) return hipErrorInvalidValue;
  if ((n / 64) % Q::D) return hipErrorInvalidValue;
  if ((long long)n * 128 * 128 >= (1LL << 31)) return hipErrorInvalidValue;   // int32 sums
  u128 M = 1;
  for (int l = 0; l < N; ++l) M *= (u128)kCrtModuli[l];
  dev::CrtConsts cc{};
  cc.n = N;
  limbs(M, cc.mm);
  cc.inv_md = 1.0 / (double)M;
  const size_t plane = (size_t)n * n;   // bytes of one residue plane
  const int grid = (n / Q::BM) * (n / Q::BN);
  for (int l = 0; l < N; ++l) {
    const int m = kCrtModuli[l];
    const u128 Ml = M / (u128)m;
    limbs(Ml, cc.ml[l]);
    dev::I8Args a{static_cast<const uint16_t*>(xs) + l * plane / 2,
                  static_cast<const uint16_t*>(ys) + l * plane / 2, n, 2, 1, 0, nullptr, rowmax,
                  colmax, nullptr};
    a.crt_m = m;
    a.crt_y = inverse_mod((int)(Ml % (u128)m), m);
    a.tout = static_cast<uint8_t*>(tplanes) + l * plane;
    hipLaunchKernelGGL(dev::gemm_i8_kernel<Q>, dim3(grid), dim3(Q::THREADS), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int bpr = (n + 1023) / 1024;
  hipLaunchKernelGGL(dev::crt_combine_kernel, dim3(n * bpr), dim3(256), 0, s,
                     static_cast<const uint8_t*>(tplanes), n, cc, rowmax, colmax, epi);
  return hipGetLastError();
}

}  // namespace ns
