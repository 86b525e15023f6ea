/*
 * ns.h - C ABI of libns: truncated Neumann series S_k(A) = I + A + ... + A^(k-1)
 * by low-product radix kernels, evaluated with hand-written MFMA kernels on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (eq. (1) of the paper, "Fast Evaluation of Truncated Neumann
 * Series by Low-Product Radix Kernels"): given a dense real n x n matrix A
 * with spectral radius below one and a series length k >= 1, produce S_k(A),
 * counting cost in n x n x n matrix products (Sec. 2, eq. (3)).
 *
 * Conventions shared by every entry point
 *   - Matrices are dense, row-major, leading dimension >= n.  Because S_k(A)
 *     is a polynomial in A, S_k(A^T) = S_k(A)^T: column-major callers get the
 *     right answer as long as A and out use the same convention.
 *   - A and out are DEVICE pointers on the handle's device.  The caller owns
 *     them; out must not overlap A.  The library never frees caller memory.
 *   - Work is enqueued on the given HIP stream and is asynchronous unless a
 *     report is requested (then the call waits for the stream once, at the end,
 *     to fill the report).
 *   - Every function returns an int status: NS_OK (0) or a negative NS_ERR_*.
 *     No C++ exception crosses this boundary.  After an error,
 *     ns_last_error() returns a message for the calling thread.
 *   - Divergence or Inf/NaN in the result is not an error: it is reported in
 *     ns_report.nonfinite and in the growth of ns_report.level_norm.
 *   - k is rounded up to k_eff, the smallest pure power of the method's radix
 *     (the paper evaluates pure powers k = m^t only, Sec. 6); k_eff is
 *     reported.  NS_NAIVE and NS_MIXED use k itself.  k = 1 gives I with no
 *     product.
 *   - One handle per host thread; calls that share a handle must not overlap
 *     (ns_eval, whose default handle every thread shares, serialises its
 *     callers itself).  Consecutive calls on one handle may use different
 *     streams: each call waits for the previous one on that handle.
 *   - A call makes the handle's device current while it runs and restores the
 *     calling thread's current device before returning.
 */
#ifndef NS_H
#define NS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- methods ---------------------------------------------------------- */
enum ns_method {
  /* Naive evaluation in Horner form, S <- I + A S, k - 1 products (Sec. 2.1). */
  NS_NAIVE = 0,
  /* Binary splitting: per level S <- S (I + P), P <- P P; 2 ceil(log2 k)
     products (Sec. 2.1; Sec. 6 setup). */
  NS_BINARY = 1,
  /* Exact radix-9 kernel of Theorem 3.1 in the telescoping update of
     Sec. 2.2 (block concatenation eq. (2), telescoping identity):
     5 ceil(log9 k) products. */
  NS_RADIX9 = 2,
  /* Approximate radix-15 kernel (Sec. 4.1 eq. (4)-(5), coefficients App. B
     polished to an exact prefix) inside the general radix-kernel iteration
     of Sec. 5.3 eq. (8): Y <- Y f(R), R <- I - (I - A) Y.
     6 ceil(log15 k) products.  The result is the iterate Y_t, which equals
     S_k up to (A^k - E^[t](A))(I - A)^{-1} (Lemma 5.9). */
  NS_RADIX15 = 3,
  /* The exact radix-9 kernel run through the same residual iteration
     (Sec. 5.5, exact radix-m special case): 5 ceil(log9 k) products. */
  NS_RADIX9_RESID = 4,
  /* Gustafsson's quinary kernel (Sec. 2.3) in the telescoping update:
     4 ceil(log5 k) products. */
  NS_QUINARY = 5,
  /* Ternary splitting (Sec. 2.1): 3 ceil(log3 k) products. */
  NS_TERNARY = 6,
  /* Hensel lifting, the m = 2 case of the framework (Sec. 5.5):
     Y <- Y (I + R), R <- I - (I - A) Y; 2 ceil(log2 k) products. */
  NS_HENSEL = 7,
  /* Exact S_k for any k, no round-up: the cheapest sequence of exact radix
     updates (S_n, A^n) -> (S_mn, A^mn) (Sec. 2.2, kernels m = 2, 3, 5 and
     the radix-9 kernel of Theorem 3.1, mu_m + 2 products each) and additive
     steps S_{n+1} = S_n + A^n, A^{n+1} = A A^n (the split of the series at
     n, one product).  A final additive step is fused into the previous
     product's epilogue at no cost.  Ties between plans of equal cost go, in
     order, to the additive chain from 1, then m = 9, 5, 3, 2 as the last
     radix update.  levels counts the radix updates. */
  NS_MIXED = 8,
  /* NS_RADIX15 with a contraction-aware coefficient table: another point of
     the prefix-exact set of Sec. 4.2, whose error map E(z) = z^15 (c0 + c1 z
     + c2 z^2) (Definition 5.2) has c0, c1, c2 > 0 and hence |E(z)| <= |z|^15
     on the unit disk, so the iteration of eq. (8) converges for every A with
     spectral radius below 1 (the App. B table has c1 < 0 and diverges near
     eigenvalue -0.99).  See ns_radix15c_coeffs.  6 ceil(log15 k) products. */
  NS_RADIX15C = 9
};

/* ---- compute precision ------------------------------------------------ */
enum ns_dtype {
  /* A and out FP64; every product on FP64 MFMA. */
  NS_F64 = 0,
  /* A and out FP32; every product on FP32 MFMA, all state in FP32. */
  NS_F32 = 1,
  /* A and out FP64.  Products as three BF16 MFMA products
     x_hi*y_hi + x_hi*y_lo + x_lo*y_hi (x_hi = bf16(x), x_lo = bf16(x - x_hi),
     round to nearest even) with FP32 accumulation.  The running sum S (or Y)
     is accumulated in FP64 as S <- S + S (T - I); residual methods compute
     R = I - (I - A) Y as an FP64 product. */
  NS_SPLIT_BF16 = 2,
  /* As NS_SPLIT_BF16 but each product is one FP16 MFMA product of operands
     scaled by a power of two derived from their max-abs, unscaled exactly in
     the FP32 epilogue. */
  NS_F16_SCALED = 3,
  /* As NS_SPLIT_BF16 but each product is an FP32 MFMA product. */
  NS_F32_ACC64 = 4
};

/* Residual-product modifiers, OR-ed into the dtype of a residual method
   (NS_RADIX15, NS_RADIX15C, NS_RADIX9_RESID, NS_HENSEL) in one of the
   FP64-accumulating forms (NS_SPLIT_BF16, NS_F16_SCALED, NS_F32_ACC64).  They
   change only how the product A Y of the residual R = I - (I - A) Y of
   eq. (8) (Sec. 5.3) is computed; without one it is an FP64 MFMA product at
   every level.  Any other combination is NS_ERR_UNSUPPORTED.
     NS_RESID_LAST: the exact (FP64, or emulated with NS_RESID_INT8 or
       NS_RESID_CRT) residual only at the last two levels -- the residual the
       final update uses and the reported final one; the earlier ones are
       products of the working precision, whose error the next exact
       residual sees and the update after it removes (Lemma 5.9:
       R_(n+1) = E(R_n) for the true residual of each iterate).
     NS_RESID_INT8(s): the residual product emulated from s int8 slices per
       operand (1 <= s <= 8; s = 0 means 7): X = A by rows and Y by columns are
       cut into signed 7-bit digits under a per-row / per-column power of two;
       the s (s + 1) / 2 digit products with p + q <= s + 1 run on int8 MFMA
       with exact int32 accumulation and are summed in FP64.  Error about
       n 2^(e_i + f_j) (s + 1) 2^(-7 s), e_i and f_j the row and column
       exponents.  The padded n is a multiple of 256; s n 127^2 must stay
       below 2^31 (NS_ERR_RANGE otherwise).
     NS_RESID_CRT: the residual product emulated through residues: A's rows
       and Y's columns are scaled by powers of two to integers of at most 46
       bits, reduced modulo N pairwise-coprime moduli m <= 256 (N = 13 for
       padded n = 256, 14 from 512 to 65536) into int8, multiplied exactly
       per modulus on int8 MFMA, and the exact integer product is rebuilt
       with the Chinese remainder theorem in FP64 limbs.  Error about
       n 2^(e_i + f_j - 46), the bound of NS_RESID_INT8 with s = 7, from N
       products where that form takes 28 (Ozaki's scheme with integer moduli).
       Excludes NS_RESID_INT8; n 2^14 must stay below 2^31. */
#define NS_RESID_LAST 0x100
#define NS_RESID_INT8(s) (0x200 | ((s) << 12))
#define NS_RESID_CRT 0x400

/* ---- status ----------------------------------------------------------- */
enum ns_status {
  NS_OK = 0,
  NS_ERR_ARG = -1,          /* null pointer, n <= 0, k < 1, ld < n, overlap,
                               unknown method or dtype, batch < 0 */
  NS_ERR_UNSUPPORTED = -2,  /* valid but not provided (e.g. NS_NAIVE with a
                               split dtype, batched with n > 256) */
  NS_ERR_NOMEM = -3,        /* device workspace allocation failed */
  NS_ERR_HIP = -4,          /* a HIP runtime call failed; see ns_last_error */
  NS_ERR_RANGE = -5         /* k or n too large for the internal limits */
};

#define NS_MAX_LEVELS 64

/* Per-call report (Sec. 6 metrics).  Filled when a non-null pointer is
   passed; costs one stream synchronisation. */
typedef struct ns_report {
  int64_t k_eff;            /* series length actually evaluated */
  int32_t levels;           /* radix levels (NS_NAIVE: k - 1 steps) */
  int32_t gemms_performed;  /* n x n x n products launched */
  int32_t gemms_formula;    /* the paper's count for the method at k_eff */
  int32_t nonfinite;        /* 1 if any product wrote Inf or NaN */
  int32_t n_internal;       /* internal (tile-padded) dimension */
  int32_t method, dtype;
  /* After level i: ||A^(m^(i+1))||_F for the telescoping methods (the power
     the next level uses), ||R_(i+1)||_F for the residual methods.  FP64
     accumulation.  Unused entries are 0. */
  double level_norm[NS_MAX_LEVELS];
  /* Radix-15 kernel in use (0 for exact kernels):
     max_{j<=14} |[f]_j - 1| and the spillover coefficients [f]_15, [f]_16. */
  double kernel_prefix_err, spill15, spill16;
  /* Kernel launches that carried the products: two independent products of
     a level (binary splitting's S (I + P) and P P, a telescoping level's sum
     and power updates, Sec. 2.1-2.2) share one launch when the matrix is small
     enough that one product leaves the GPU under-filled, so this is the
     length of the call's critical path in products. */
  int32_t product_launches;
  int32_t reserved;
} ns_report;

typedef struct ns_handle ns_handle;

/* Create a handle bound to HIP device `device` (workspace pool, tile choices
   and graph cache live in the handle).  *h is set to NULL on failure. */
int ns_create(ns_handle** h, int device);
/* Release the handle's device memory and graphs.  Null is accepted. */
int ns_destroy(ns_handle* h);

/* Host-only planning: k_eff, number of levels and the product count of the
   literal schedule (Sec. 2.1-2.2 cost model, Sec. 5.4 eq. (9), Table 2).
   Any output pointer may be null. */
int ns_plan(int64_t k, int method, int64_t* k_eff, int32_t* levels, int32_t* gemms);

/* Device workspace a call with these arguments allocates (bytes). */
int ns_workspace_bytes(int64_t n, int method, int dtype, size_t* bytes);

/* S_k(A) with a per-device default handle on the null stream; lda = ldo = n.
   Element type of A and out: double for NS_F64 and the mixed forms,
   float for NS_F32.  Calls from several host threads are serialised on the
   host (they share the default handle) and run in order on the null stream. */
int ns_eval(const void* A, int64_t n, int64_t k, int method, int dtype, void* out);

/* Full form.  lda, ldo: leading dimensions (>= n).  stream may be 0.
   rep may be null. */
int ns_eval_ex(ns_handle* h, const void* A, int64_t n, int64_t lda, int64_t k,
               int method, int dtype, void* out, int64_t ldo,
               hipStream_t stream, ns_report* rep);

/* Batched S_k over `batch` independent small matrices (Sec. 1 applications,
   e.g. MIMO detection), all in ONE persistent kernel launch replayed from a
   cached HIP graph.
     A_packed, out_packed: device buffers; matrix i is row-major n_i x n_i,
       lda = n_i, starting at element offset off_dev[i] in both buffers.
     off_dev (int64, device): per-matrix element offset.
     n_host (int32, host): per-matrix n.  The library validates these, and
       uploads its own copy with the work queue; the kernel reads n only from
       there.
     n_dev (int32, device): not read (the device copy of n of earlier
       versions of this interface); may be null.
   Supported: method NS_RADIX9 or NS_BINARY or NS_NAIVE, dtype NS_F32 (float
   buffers), 1 <= n_i <= 256.  The graph cache is keyed on the
   buffers, the per-matrix n, k, method and dtype: a call with new pointers or
   new n captures a new graph.  The handle keeps at most 16 graphs (the oldest is dropped
   after a device synchronisation), and drops them all when a call or the
   autotuner needs a larger workspace.  rep (nullable) aggregates: level_norm holds the sum over
   matrices of squared norms' square root per level, nonfinite is the OR. */
int ns_eval_batched(ns_handle* h, const void* A_packed, const int64_t* off_dev,
                    const int32_t* n_dev, const int32_t* n_host, int32_t batch,
                    int64_t k, int method, int dtype, void* out_packed,
                    hipStream_t stream, ns_report* rep);

/* For callers that cannot allocate (code under HIP stream capture, tight
   serving loops, harnesses that forbid device allocation): the same
   evaluation as ns_eval_ex, with the same arguments apart from the handle,
   on the current device.  It allocates nothing: the workspace and the
   products' parameter blocks come from a fixed device array of
   NS_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
   until the process ends; the caller still provides A and out.
     - Fits when ns_workspace_bytes(n, method, dtype) is at most
       NS_NOALLOC_SCRATCH_BYTES - 1 MiB (e.g. n <= 960 for NS_F64 radix-9,
       n <= 1344 for NS_F32 radix-9) and the call has at most 1 MiB of product
       parameter blocks (about 2000 products); otherwise NS_ERR_RANGE, and
       nothing is enqueued.
     - Every call of the process on a GPU shares that GPU's array, which
       keeps the last call's contents (each call clears what must start at
       zero).  Calls that overlap on one GPU (e.g. on two streams) race on the
       array: the caller must order them (one stream does).  Host threads are
       serialised while a call is enqueued.
     - The parameter blocks go up from host memory that is not pinned, so the
       host waits for that copy, i.e. for the stream's earlier work.
     - No product timing and no handle state; rep (nullable) as in
       ns_eval_ex. */
#define NS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ns_eval_noalloc(const void* A, int64_t n, int64_t lda, int64_t k, int method, int dtype,
                    void* out, int64_t ldo, hipStream_t stream, ns_report* rep);

/* Reference path for the batched form: the same matrices evaluated one at a
   time with the per-matrix single-GEMM kernels (one launch per product, no
   graph).  Same arguments and result layout as ns_eval_batched; off_host is
   the host copy of the offsets. */
int ns_eval_batched_loop(ns_handle* h, const void* A_packed, const int64_t* off_host,
                         const int32_t* n_host, int32_t batch, int64_t k, int method,
                         int dtype, void* out_packed, hipStream_t stream);

/* Time every candidate configuration of the batched kernel (tile shapes and
   resident workgroups per CU) on this batch, radix-9, and keep the fastest
   for batches with the same histogram of n, in the handle (and in the JSON
   file named by the NS_TUNE_CACHE environment variable, if set); later
   ns_eval_batched calls on such batches use it.  Same buffer arguments as
   ns_eval_batched; the contents of out_packed are overwritten.  Returns the
   number of configurations timed in *n_timed. */
int ns_autotune_batched(ns_handle* h, const void* A_packed, const int64_t* off_dev,
                        const int32_t* n_dev, const int32_t* n_host, int32_t batch,
                        int64_t k, void* out_packed, hipStream_t stream,
                        int32_t* n_timed);

/* The radix-15 coefficient table the library uses, in the order
   L2[I,B,P1] R2[..] L3[I,B,P1,P2] R3[..] L4[I,B,P1,P2,P3] R4[..] g1..g4
   (Sec. 4.1 eq. (4)-(5)); derived at load time from the App. B digits by the
   library's own minimum-norm Gauss-Newton.  Outputs may be null except c28. */
int ns_radix15_coeffs(double c28[28], double* prefix_err, double* spill15, double* spill16);

/* The contraction-aware table of NS_RADIX15C, same order and outputs: its
   six-decimal start point (a minimum-norm point of the prefix-exact set with
   c0, c1, c2 >= 0.12) polished by the same Gauss-Newton. */
int ns_radix15c_coeffs(double c28[28], double* prefix_err, double* spill15, double* spill16);

/* Per-product timing for roofline measurement: when enabled, every product
   launch issued by ns_eval_ex on this handle is bracketed by HIP events on the
   call's stream.  ns_product_timing returns the number of timed launches, the
   summed kernel time in ms and the summed algorithmic flops (2 n^3 each,
   unpadded n) since the last reset, waiting for the events first. */
int ns_set_product_timing(ns_handle* h, int enable);
int ns_product_timing(ns_handle* h, int32_t* count, double* total_ms, double* total_flops,
                      int reset);
/* The same sums over the timed launches of one product engine only, named by
   the dtype that uses it: NS_F64 (FP64 products, including the FP64 residual
   products of the mixed forms), NS_F32 (FP32 products, including those of
   NS_F32_ACC64), NS_SPLIT_BF16, NS_F16_SCALED, or NS_RESID_INT8(0) for the
   int8-emulated residual products of either form (one timed record per
   product, covering all its diagonal launches, or all its per-modulus
   launches and the combining pass).  Resets nothing. */
int ns_product_timing_dtype(ns_handle* h, int dtype, int32_t* count, double* total_ms,
                            double* total_flops);

/* The timed launches one by one, in launch order, since the last reset: up to
   cap entries of kernel milliseconds (ms) and product engine (engine: the
   dtype naming it, as for ns_product_timing_dtype; either array may be
   null).  *count receives the number of timed launches (which may exceed
   cap).  Per-level time splits of a call are sums over its launches. */
int ns_product_timing_launches(ns_handle* h, int32_t cap, float* ms, int32_t* engine,
                               int32_t* count);

const char* ns_status_string(int status);
const char* ns_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NS_H */
