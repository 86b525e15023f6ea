// Internal declarations shared by the host scheduler and the HIP kernels.
// Not part of the public ABI (include/ns.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ns {

constexpr int kMaxZ = 3;     // epilogue inputs per product
constexpr int kMaxOut = 6;   // epilogue outputs per product

// One epilogue output:  out = a * (X Y) + sum_i z[i] * Z_i + id * I
struct EpiOut {
  void* ptr;
  int f64;                   // element type of ptr: 1 double, 0 float
  double a;
  double z[kMaxZ];
  double id;
  unsigned* amax;            // scaled-FP16 products: atomicMax of |out| as float bits, or null
};

// Operand storage / arithmetic of a product launch.
enum Engine : int {
  ENG_F64 = 0,        // double operands, FP64 MFMA (16x16x4; 4x4x4 in the split-K kernel)
  ENG_F32 = 1,        // float operands, FP32 MFMA 16x16x4
  ENG_BF16X3 = 2,     // float operands split to bf16 hi/lo, 3 BF16 MFMA products
  ENG_F16S = 3,       // float operands scaled by 2^-e and rounded to fp16, 1 FP16 MFMA product
  ENG_I8 = 4,         // double operands cut into int8 digit slices, int8 MFMA products with
                      // exact int32 accumulation, summed in FP64 (ozaki.hip)
};

// Parameters of one n x n x n product C = X Y with a fused multi-output
// epilogue.  All buffers are row-major with leading dimension ld (= the
// internal, tile-padded n).
struct GemmParams {
  const void* X;
  const void* Y;
  int n;                      // padded dimension (multiple of the tile size)
  int ld;
  int nz;
  const void* Z[kMaxZ];
  int zf64[kMaxZ];
  int no;
  EpiOut out[kMaxOut];
  double* sumsq;              // if non-null: += sum of squares of output 0
  int* nonfinite;             // if non-null: set to 1 if any output 0 entry is Inf/NaN
  unsigned* amax;             // if non-null: atomicMax of |output 0| as float bits (the scaled-FP16
                              // products use the per-output EpiOut::amax instead)
  const unsigned* xamax;      // low-precision engines: max-abs of X (float bits) for scaling
  const unsigned* yamax;      // ... of Y
};

// Tile-size requirement of each engine for a given n (the padded n must be a
// multiple of it).  Small n use smaller tiles.
int engine_tile(Engine e, int n);

// Launch one product on `stream`.  `host` is the parameter block on the host
// (for the grid), `dev` the same block already in device memory (the kernel
// reads the epilogue part from there).  With host2 / dev2 a second product of
// the same n and engine, independent of the first (neither reads what the other
// writes), runs in the same grid.  Not for the 16-bit engines' panel path.
// Returns hipSuccess or the launch error.
hipError_t launch_gemm(Engine e, const GemmParams& host, const GemmParams* dev, hipStream_t stream,
                       const GemmParams* host2 = nullptr, const GemmParams* dev2 = nullptr);
// Workgroups of one product's grid on engine e at padded n.
int gemm_grid(Engine e, int n);

// Low-precision products at large n (panel.hip): each operand is first
// rewritten into 16-bit panels (bf16 hi/lo planes, or one scaled fp16 plane),
// X by rows and Y by columns, then multiplied from the panels.
// n from which each 16-bit engine multiplies from panels (and pads to a
// multiple of 256); below it the operands are converted in the k-loop of a
// 64 x 64 tile, which keeps more CUs busy.  Measured on radix-9, k = 81
// (panels against in-loop conversion, whole call): split-BF16 (256 x 256
// tiles) 1.93 against 1.03 ms at n = 2048, 2.39 against 1.96 at 2560, 2.89
// against 2.88 at 3072; scaled FP16 (128 x 256 tiles, two per CU) 1.00
// against 0.73 ms at 1536, 1.04 against 1.18 at 1792, 1.10 against 1.34 at
// 2048.
constexpr int kPanelMinBF16X3 = 3072, kPanelMinF16S = 1792;
inline int panel_min(Engine e) { return e == ENG_BF16X3 ? kPanelMinBF16X3 : kPanelMinF16S; }
bool panel_path(Engine e, int n);
size_t panel_bytes(Engine e, int n);      // bytes of one operand's panels
// dst <- panels of src (n x n, ld; row-major FP32).  transpose = 0 lays out the
// rows of src (an X operand), 1 its columns (a Y operand).  amax: the max-abs
// slot of src for the FP16 scale (scaled FP16 only).
hipError_t launch_to_panels(Engine e, const float* src, int n, int ld, int transpose, void* dst,
                            const unsigned* amax, hipStream_t s);
// host.X / host.Y point at the panels of X (rows) and Y (columns).
hipError_t launch_gemm_panels(Engine e, const GemmParams& host, const GemmParams* dev, hipStream_t s);

// FP64 products emulated from int8 slices (ozaki.hip).  The product kernel's
// tile (the padded n must be a multiple of it); the slice count is at most
// kMaxI8Slices.
constexpr int kMaxI8Slices = 8;
int i8_tile();
// Row max-abs (rowmax, may be null) and column max-abs (colmax, may be null)
// of an n x n FP64 matrix, as the bits of non-negative doubles, atomically into
// arrays the caller has zeroed.  n a multiple of 256.
hipError_t launch_maxabs_rc(const double* src, int n, unsigned long long* rowmax,
                            unsigned long long* colmax, hipStream_t s);
// The `slices` int8 digit planes (slices n^2 bytes) of src by rows
// (transpose = 0, mx = row max-abs) or by columns (1, mx = column max-abs).
hipError_t launch_i8_slices(const double* src, int n, int transpose, const unsigned long long* mx,
                            int slices, void* dst, hipStream_t s);
// X Y from the digit planes xs (of X, by rows) and ys (of Y, by columns): one
// launch per diagonal of slice pairs, the partial sums in acc (n x n FP64),
// the last launch applying the epilogue epi (device copy).
hipError_t launch_gemm_i8(const void* xs, const void* ys, int n, int slices, double* acc,
                          const unsigned long long* rowmax, const unsigned long long* colmax,
                          const GemmParams* epi, hipStream_t s);

// The same product through residues (ozaki.hip, the NS_RESID_CRT form): X
// and Y are scaled by rows / columns to integers of at most kCrtBits bits,
// reduced modulo crt_moduli(n) pairwise-coprime moduli m <= 256 into int8
// planes, multiplied exactly per modulus on int8 MFMA, and the integer
// product is rebuilt by the Chinese remainder theorem.
constexpr int kCrtBits = 46;
constexpr int kMaxCrtModuli = 16;
// number of moduli for padded n (their product exceeds n 2^(2 kCrtBits + 2))
int crt_moduli(int n);
// residue planes (crt_moduli(n) n^2 bytes) of src by rows (transpose = 0) or
// columns (1), exponents from mx
hipError_t launch_crt_slices(const double* src, int n, int transpose, const unsigned long long* mx,
                             void* dst, hipStream_t s);
// X Y from the residue planes; tplanes (crt_moduli(n) n^2 bytes) holds each
// modulus' reduced product until the combining launch applies epi
hipError_t launch_gemm_crt(const void* xs, const void* ys, int n, void* tplanes,
                           const unsigned long long* rowmax, const unsigned long long* colmax,
                           const GemmParams* epi, hipStream_t s);

// Elementwise helpers (util.hip).
// dst (padded n_pad x n_pad, ld n_pad) <- src (n x n, lda) converted; the
// padding is zero.  *_f64 flags give element types.
hipError_t launch_pad_copy(const void* src, int src_f64, int64_t n, int64_t lda,
                           void* dst, int dst_f64, int n_pad, hipStream_t s);
// dst (n x n, ldo) <- top-left n x n block of src (ld n_pad).
hipError_t launch_unpad_copy(const void* src, int src_f64, int n_pad, void* dst, int dst_f64,
                             int64_t n, int64_t ldo, hipStream_t s);
// dst <- identity (padded), element type by flag.
hipError_t launch_set_identity(void* dst, int f64, int n_pad, hipStream_t s);
// Fill `count` doubles / ints / unsigned with zero (a kernel, not a memset).
hipError_t launch_zero_words(void* p, size_t bytes, hipStream_t s);
// max-abs of a float matrix into *amax (float bits), atomically.
hipError_t launch_amax(const float* x, size_t count, unsigned* amax, hipStream_t s);

// Up to kMaxFills independent fills in ONE launch (the grid is split between
// them): the scalar-block reset, copies-in and identities that start a call
// write distinct buffers and read only the caller's A.
enum FillKind : int { FILL_ZERO = 0, FILL_PAD, FILL_IDENTITY };
struct Fill {
  int kind;                 // FillKind
  int src_f64, dst_f64;     // element types (PAD: both; IDENTITY: dst)
  int n_pad;                // PAD / IDENTITY: padded dimension
  int64_t n, lda;           // PAD: the caller's n and leading dimension
  const void* src;          // PAD source
  void* dst;
  size_t bytes;             // ZERO: bytes to clear (a multiple of 4)
};
constexpr int kMaxFills = 4;
hipError_t launch_fills(const Fill* fills, int count, hipStream_t s);


// Makes a handle's device current for the guard's lifetime and restores the
// caller's device afterwards: an entry point never changes the calling
// thread's current device.  err holds the first failing runtime call.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int device) {
    int cur = -1;
    err = hipGetDevice(&cur);
    if (err == hipSuccess && cur != device) {
      err = hipSetDevice(device);
      if (err == hipSuccess) prev = cur;
    }
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
};

}  // namespace ns
