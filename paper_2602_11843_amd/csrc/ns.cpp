// libns host side: argument checking, workspace, the series schedules and the
// C ABI of include/ns.h.
//
// Every schedule below is a sequence of n x n x n products issued to the
// engines of gemm.hip; each product carries the linear combinations the
// paper's circuit needs next as extra epilogue outputs, so the only device
// work between products is the products themselves.
//
// Schedules use the "increment" form of the updates, algebraically identical
// to the paper's and better conditioned in low precision:
//   S_{mn} = S_n T            ->  S += S (T - I)
//   A^{mn} = I - T + T A^n    ->  B  = B - (T - I) + (T - I) B
//   Y_{n+1} = Y_n f(R_n)      ->  Y += Y (f(R) - I)
//   R_{n+1} = I - (I - A) Y   ->  R  = I - Y + A Y
// so T - I (or f(R) - I) is formed instead of T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <unordered_map>
#include <vector>

#include "../../include/ns.h"
#include "common.h"

namespace ns {
Engine work_engine_of(int dtype);
bool radix15_table(double c[28], double* prefix_err, double* s15, double* s16);
bool radix15c_table(double c[28], double* prefix_err, double* s15, double* s16);
int batched_eval(ns_handle* h, const void* A_packed, const int64_t* off_dev, const int32_t* n_dev,
                 const int32_t* n_host, int32_t batch, int64_t k, int method, int dtype,
                 void* out_packed, hipStream_t stream, ns_report* rep);
int batched_autotune(ns_handle* h, const void* A_packed, const int64_t* off_dev,
                     const int32_t* n_dev, const int32_t* n_host, int32_t batch, int64_t k,
                     void* out_packed, hipStream_t stream, int32_t* n_timed);
void batched_release(ns_handle* h);
}  // namespace ns

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {
thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

#define NS_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(NS_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                               \
  } while (0)
}  // namespace

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct ns_handle {
  int device = 0;
  void* ws = nullptr;            // workspace arena
  size_t ws_bytes = 0;
  // timing of product launches: one record per launch, its events reused
  struct Timed {
    hipEvent_t e0, e1;
    int engine;
    double flops;      // algorithmic: 2 n^3 (unpadded n) per product of the launch
  };
  bool timing = false;
  std::vector<Timed> ev;
  size_t ev_used = 0;
  // product parameter blocks: staged in pinned host memory and uploaded with
  // one copy per call, into a ring of kParamSlots slots (params_cap blocks
  // each, host and device).  A call takes the next slot; its event marks when
  // that slot's upload has finished, so the host waits only when it is a whole
  // ring of calls ahead of the device.
  static constexpr int kParamSlots = 4;
  ns::GemmParams* params_host = nullptr;   // kParamSlots * params_cap
  ns::GemmParams* params_dev = nullptr;
  size_t params_cap = 0;
  hipEvent_t params_free[kParamSlots] = {};
  unsigned params_next = 0;
  int64_t product_launches = 0;            // of the last call (a pair counts once)
  // recorded after each call's last operation; the next call's stream waits on
  // it, so calls on different streams never share the workspace concurrently
  hipEvent_t call_done = nullptr;
  // batched state (owned by batched.hip)
  void* batched = nullptr;
};

namespace ns {
namespace {

constexpr int kScalarBytes = 64 * 1024;   // norms, flags and max-abs slots
// Two independent products share one launch when one product's grid has at
// most this many workgroups (2 per CU): below it a single product leaves CUs
// idle or runs a short tail, and the pair halves the launches on the critical
// path (binary splitting's S P and P P, a telescoping level's S (T - I) and
// (T - I) B).  Larger grids fill the chip on their own and keep one launch
// per product.
constexpr int kPairMaxGrid = 512;
constexpr int kAmaxSlots = 8192;

struct Scalars {                          // layout of the scalar block in device memory
  double level_sumsq[NS_MAX_LEVELS];
  int nonfinite;
  int pad;
  unsigned amax[kAmaxSlots];
};
static_assert(sizeof(Scalars) <= kScalarBytes, "scalar block too small");

// A dtype argument is a base precision (low byte) plus residual-product
// modifiers (NS_RESID_LAST, NS_RESID_INT8(s), NS_RESID_CRT).
constexpr int kBaseMask = 0xff, kResidInt8 = 0x200, kSliceShift = 12;
constexpr int kModifierBits = NS_RESID_LAST | kResidInt8 | NS_RESID_CRT | (0xf << kSliceShift);
int base_of(int dtype) { return dtype & kBaseMask; }
bool resid_last(int dtype) { return (dtype & NS_RESID_LAST) != 0; }
bool resid_crt(int dtype) { return (dtype & NS_RESID_CRT) != 0; }
// slices of the int8-emulated residual product, 0 without the modifier
int resid_slices(int dtype) {
  if (!(dtype & kResidInt8)) return 0;
  const int sl = (dtype >> kSliceShift) & 0xf;
  return sl ? sl : 7;
}
bool is_mixed(int dtype) {
  const int b = base_of(dtype);
  return b == NS_SPLIT_BF16 || b == NS_F16_SCALED || b == NS_F32_ACC64;
}
bool is_residual(int method) {
  return method == NS_RADIX15 || method == NS_RADIX15C || method == NS_RADIX9_RESID ||
         method == NS_HENSEL;
}
Engine work_engine(int dtype) {
  switch (base_of(dtype)) {
    case NS_F64: return ENG_F64;
    case NS_F32: return ENG_F32;
    case NS_SPLIT_BF16: return ENG_BF16X3;
    case NS_F16_SCALED: return ENG_F16S;
    default: return ENG_F32;
  }
}

int radix_of(int method) {
  switch (method) {
    case NS_BINARY: return 2;
    case NS_TERNARY: return 3;
    case NS_QUINARY: return 5;
    case NS_RADIX9: case NS_RADIX9_RESID: return 9;
    case NS_RADIX15: case NS_RADIX15C: return 15;
    case NS_HENSEL: return 2;
    default: return 0;
  }
}
// products per level: mu_m + 2 (Sec. 2.2 cost model; Sec. 5.4 eq. (9))
int per_level(int method) {
  switch (method) {
    case NS_BINARY: return 2;
    case NS_TERNARY: return 3;
    case NS_QUINARY: return 4;
    case NS_RADIX9: case NS_RADIX9_RESID: return 5;
    case NS_RADIX15: case NS_RADIX15C: return 6;
    case NS_HENSEL: return 2;
    default: return 0;
  }
}

// ---------------------------------------------------------------------------
// exact plan for any k (NS_MIXED)
// ---------------------------------------------------------------------------
// Steps: m in {2, 3, 5, 9} is a radix-m update costing mu_m + 2 products; 1 is
// an additive step costing one product (free when it is the last step and a
// product came before it).  best(n) is the cheapest way from n = 1 to the pair
// (S_n, A^n): either n - 1 additive steps, or best(n / m) + cost(m) + n % m
// (an optimal plan never has m or more additive steps right after a radix-m
// update: one additive step before the update replaces m after it).
int mixed_cost(int m) { return m == 9 ? 5 : m == 5 ? 4 : m == 3 ? 3 : 2; }
constexpr int kMixedRadices[4] = {9, 5, 3, 2};

struct MixedBest {
  std::unordered_map<int64_t, std::pair<int64_t, int>> memo;   // n -> (cost, choice)
  std::pair<int64_t, int> best(int64_t n) {
    auto it = memo.find(n);
    if (it != memo.end()) return it->second;
    std::pair<int64_t, int> b{n - 1, 0};
    for (int m : kMixedRadices) {
      if (n < m) continue;
      const int64_t c = best(n / m).first + mixed_cost(m) + n % m;
      if (c < b.first) b = {c, m};
    }
    memo.emplace(n, b);
    return b;
  }
  void steps(int64_t n, std::vector<int>* out) {
    const int m = best(n).second;
    if (m == 0) {
      out->insert(out->end(), (size_t)(n - 1), 1);
      return;
    }
    steps(n / m, out);
    out->push_back(m);
    out->insert(out->end(), (size_t)(n % m), 1);
  }
};

// Cheapest exact plan for S_k; fills steps if non-null (k must then be small
// enough for an additive chain to be listed, which an optimal plan only picks
// for k <= 5).
int64_t mixed_plan(int64_t k, std::vector<int>* steps) {
  if (k <= 1) return 0;
  MixedBest mb;
  int64_t cost = (k == 2) ? 1 : k - 2;
  int choice = 0;
  for (int m : kMixedRadices) {
    if (k < m) continue;
    const int64_t r = k % m;
    const int64_t c = mb.best(k / m).first + mixed_cost(m) + (r > 0 ? r - 1 : 0);
    if (c < cost) {
      cost = c;
      choice = m;
    }
  }
  if (steps) {
    steps->clear();
    if (choice == 0) {
      steps->insert(steps->end(), (size_t)(k - 1), 1);
    } else {
      mb.steps(k / choice, steps);
      steps->push_back(choice);
      steps->insert(steps->end(), (size_t)(k % choice), 1);
    }
  }
  return cost;
}

int plan(int64_t k, int method, int64_t* k_eff, int32_t* levels, int32_t* gemms) {
  if (k < 1) return fail(NS_ERR_ARG, "k must be >= 1 (got %lld)", (long long)k);
  if (method == NS_MIXED) {
    std::vector<int> st;
    const int64_t cost = mixed_plan(k, &st);
    int32_t t = 0;
    for (int m : st) t += m > 1;
    if (cost > INT32_MAX || t > NS_MAX_LEVELS) return fail(NS_ERR_RANGE, "k too large");
    *k_eff = k;
    *levels = t;
    *gemms = (int32_t)cost;
    return NS_OK;
  }
  if (method == NS_NAIVE) {
    if (k - 1 > INT32_MAX) return fail(NS_ERR_RANGE, "naive k too large");
    *k_eff = k;
    *levels = (int32_t)(k - 1);
    *gemms = (int32_t)(k - 1);
    return NS_OK;
  }
  const int m = radix_of(method);
  if (m == 0) return fail(NS_ERR_ARG, "unknown method %d", method);
  int t = 0;
  __int128 p = 1;
  while (p < k) {
    p *= m;
    ++t;
  }
  if (p > INT64_MAX || t > NS_MAX_LEVELS)
    return fail(NS_ERR_RANGE, "k_eff = %d^%d overflows", m, t);
  *k_eff = (int64_t)p;
  *levels = t;
  *gemms = per_level(method) * t;
  return NS_OK;
}

int n_internal(int64_t n, int dtype) {
  const Engine e = work_engine(dtype);
  const int i8 = (resid_slices(dtype) || resid_crt(dtype)) ? i8_tile() : 1;
  int t = std::max(engine_tile(e, (int)n), i8);
  if (is_mixed(dtype)) t = std::max(t, engine_tile(ENG_F64, (int)n));
  int np = (int)((n + t - 1) / t * t);
  // the tile choice depends on the padded size; re-round if it changed
  int t2 = std::max(engine_tile(e, np), i8);
  if (is_mixed(dtype)) t2 = std::max(t2, engine_tile(ENG_F64, np));
  return (int)((np + t2 - 1) / t2 * t2);
}

// working-precision buffers and FP64 accumulators each schedule needs
void buffer_counts(int method, int dtype, int* nw, int* n64) {
  const bool mixed = is_mixed(dtype);
  switch (method) {
    case NS_NAIVE: *nw = 3; break;                       // A, S, S'
    case NS_BINARY: *nw = 4; break;                      // S, S', P, P'
    case NS_TERNARY: *nw = 6; break;                     // S, S', P, P2, P', T
    case NS_QUINARY: *nw = 7; break;                     // S, S', B, B', U, X1, T
    case NS_RADIX9: *nw = 9; break;                      // S, S', B, B', U, X1, P, Q, T
    case NS_HENSEL: *nw = 4; break;                      // A, R, Y, Y'
    case NS_MIXED: *nw = 10; break;                      // A, S, S', B, B', U, X1, P, Q, T
    case NS_RADIX9_RESID: *nw = 9; break;                // A, R, Y, Y', U, X1, P, Q, T
    case NS_RADIX15:
    case NS_RADIX15C: *nw = 12; break;                   // A, R, Y, Y', P1, L2, R2, L3, R3, L4, R4, F
    default: *nw = 0;
  }
  *n64 = mixed ? (is_residual(method) ? 2 : 1) : 0;    // Y64 + A64, or S64
  // the 16-bit panels of a product's two operands (each at most an FP32 matrix)
  if (base_of(dtype) == NS_SPLIT_BF16 || base_of(dtype) == NS_F16_SCALED) *nw += 2;
}

// bytes of the int8-emulated residual's buffers: digit planes of both
// operands, the FP64 partial sums, row and column max-abs.  The residue form:
// residue planes of both operands and the reduced products, max-abs.
size_t i8_bytes(int np, int slices, bool crt) {
  if (!slices) return 0;
  const size_t mat = (size_t)np * np;
  if (crt) return 3 * slices * mat + 2 * 8 * (size_t)np + 4 * 256;
  return 2 * slices * mat + 8 * mat + 2 * 8 * (size_t)np + 4 * 256;
}

// planes per operand of the emulated residual: slices, or moduli
int resid_planes(int dtype, int np) {
  return resid_crt(dtype) ? crt_moduli(np) : resid_slices(dtype);
}

size_t workspace_bytes(int64_t n, int method, int dtype) {
  const int np = n_internal(n, dtype);
  int nw, n64;
  buffer_counts(method, dtype, &nw, &n64);
  const size_t w = (base_of(dtype) == NS_F64) ? 8 : 4;
  const size_t mat = (size_t)np * np;
  return kScalarBytes + mat * (nw * w + n64 * 8) + 256 * (nw + n64 + 1) +
         i8_bytes(np, resid_planes(dtype, np), resid_crt(dtype));
}

// ---------------------------------------------------------------------------
// execution context
// ---------------------------------------------------------------------------
struct Buf {
  void* p = nullptr;
  int f64 = 0;
  unsigned* amax = nullptr;   // max-abs slot of the current contents (scaled FP16)
};

struct Out {
  Buf* b;
  double a;
  double z[kMaxZ];
  double id;
};

// A recorded device operation of a call.
struct Op {
  enum Kind { GEMM, IDENTITY, AMAX, PANELS, ZERO, PAD, UNPAD, MAXABS, SLICES } kind;
  Engine e;
  GemmParams p;      // GEMM
  bool panels;       // GEMM: X / Y are 16-bit panels
  bool pair_next;    // GEMM: independent of the next GEMM, which may share its launch
  void* ptr;         // IDENTITY / AMAX / ZERO target, PANELS / PAD / UNPAD source
  int f64;           // element type of the target (PAD / UNPAD: of the destination)
  unsigned* amax;
  void* dst;         // PANELS / PAD / UNPAD destination
  int transpose;     // PANELS: 1 for a Y operand
  int src_f64;       // PAD / UNPAD: element type of the source
  int64_t n, ld;     // PAD / UNPAD: the caller's n and leading dimension; ZERO: bytes in n
  // MAXABS: row max-abs into rmax, column max-abs into cmax (either may be
  // null) of ptr.  SLICES: the digit planes of ptr (by columns if transpose)
  // into dst, exponents from rmax.  GEMM on ENG_I8: X / Y are the digit
  // planes, acc the partial sums, rmax / cmax the max-abs of X rows / Y columns.
  unsigned long long* rmax;
  unsigned long long* cmax;
  double* acc;
  int slices;
  bool crt;          // SLICES / GEMM on ENG_I8: the residue form (planes are residues)
  void* tplanes;     // GEMM on ENG_I8, residue form: the reduced products
};

// Device memory of a call that allocates nothing (ns_eval_noalloc): the
// workspace and the parameter blocks' device copy live in a fixed region, the
// blocks are staged in a fixed host array.
struct FixedMem {
  char* ws;                 // scalar block + matrices
  size_t ws_bytes;
  GemmParams* params_host;  // host staging
  GemmParams* params_dev;   // device copy, inside the fixed region
  size_t params_cap;        // blocks
};

struct Ctx {
  ns_handle* h;             // null on the fixed-memory path
  const FixedMem* fixed;    // null on the handle path
  hipStream_t s;
  int n;              // caller's n
  int np;             // internal n
  Engine eng;         // working engine
  bool mixed;
  Scalars* scal;      // device
  int next_amax = 0;
  int gemms = 0;
  int64_t launches = 0;     // product launches of the call (a pair counts once)
  // int8-emulated residual products (NS_RESID_INT8): slice count, buffers, and
  // the X operand whose planes are current (A, sliced once per call)
  int slices = 0;
  bool crt = false;          // the residue form (NS_RESID_CRT): slices counts moduli
  void* i8_t = nullptr;      // its reduced products
  bool resid_last = false;
  void* i8_x = nullptr;
  void* i8_y = nullptr;
  double* i8_acc = nullptr;
  unsigned long long* i8_rmax = nullptr;
  unsigned long long* i8_cmax = nullptr;
  const void* i8_x_src = nullptr;
  int status = NS_OK;
  char* arena;
  size_t arena_off = 0;
  std::vector<Op> ops;
  Buf panel_x, panel_y;   // panels of the current product's operands (low precision, large n)

  Buf take(int f64) {
    Buf b;
    b.p = arena + arena_off;
    b.f64 = f64;
    arena_off += (size_t)np * np * (f64 ? 8 : 4);
    arena_off = (arena_off + 255) & ~(size_t)255;
    return b;
  }

  unsigned* new_amax_slot() {
    if (next_amax >= kAmaxSlots) {
      status = fail(NS_ERR_RANGE, "too many products for the max-abs slots");
      return nullptr;
    }
    return &scal->amax[next_amax++];
  }

  void identity(const Buf& b) {
    Op op{};
    op.kind = Op::IDENTITY;
    op.ptr = b.p;
    op.f64 = b.f64;
    ops.push_back(op);
  }

  void zero(void* p, size_t bytes) {
    Op op{};
    op.kind = Op::ZERO;
    op.ptr = p;
    op.n = (int64_t)bytes;
    ops.push_back(op);
  }

  // padded working copy dst <- the caller's n x n matrix src (leading dim ld)
  void pad(const void* src, int src_f64, int64_t ld, const Buf& dst) {
    Op op{};
    op.kind = Op::PAD;
    op.ptr = const_cast<void*>(src);
    op.src_f64 = src_f64;
    op.dst = dst.p;
    op.f64 = dst.f64;
    op.n = n;
    op.ld = ld;
    ops.push_back(op);
  }

  // the caller's n x n result dst (leading dim ld) <- top-left block of src
  void unpad(const Buf& src, void* dst, int dst_f64, int64_t ld) {
    Op op{};
    op.kind = Op::UNPAD;
    op.ptr = src.p;
    op.src_f64 = src.f64;
    op.dst = dst;
    op.f64 = dst_f64;
    op.n = n;
    op.ld = ld;
    ops.push_back(op);
  }

  void amax(Buf& b) {
    b.amax = new_amax_slot();
    if (!b.amax || b.f64) return;
    Op op{};
    op.kind = Op::AMAX;
    op.ptr = b.p;
    op.amax = b.amax;
    ops.push_back(op);
  }

  void panels(Engine e, const Buf& src, int transpose, Buf& dst) {
    if (!dst.p) dst = take(0);
    Op op{};
    op.kind = Op::PANELS;
    op.e = e;
    op.ptr = src.p;
    op.amax = src.amax;
    op.dst = dst.p;
    op.transpose = transpose;
    ops.push_back(op);
  }

  // Record C = X Y on engine e; Z inputs; outputs as affine combinations of
  // (C, Z..., I).  norm_level >= 0 accumulates ||output 0||_F^2 there.
  void gemm(Engine e, const Buf& X, const Buf& Y, std::initializer_list<Buf> Z,
            std::initializer_list<Out> outs, int norm_level = -1) {
    if (status != NS_OK) return;
    Op op{};
    op.kind = Op::GEMM;
    op.e = e;
    GemmParams& p = op.p;
    p.X = X.p;
    p.Y = Y.p;
    if (e == ENG_I8) {
      i8_operands(X, Y);
      p.X = i8_x;
      p.Y = i8_y;
      op.acc = i8_acc;
      op.rmax = i8_rmax;
      op.cmax = i8_cmax;
      op.slices = slices;
      op.crt = crt;
      op.tplanes = i8_t;
    } else if (panel_path(e, np)) {
      panels(e, X, 0, panel_x);
      panels(e, Y, 1, panel_y);
      p.X = panel_x.p;
      p.Y = panel_y.p;
      op.panels = true;
    }
    p.n = np;
    p.ld = np;
    p.nz = 0;
    for (const Buf& z : Z) {
      p.Z[p.nz] = z.p;
      p.zf64[p.nz] = z.f64;
      ++p.nz;
    }
    p.no = 0;
    for (const Out& o : outs) {
      EpiOut& e_ = p.out[p.no++];
      e_.ptr = o.b->p;
      e_.f64 = o.b->f64;
      e_.a = o.a;
      for (int i = 0; i < kMaxZ; ++i) e_.z[i] = o.z[i];
      e_.id = o.id;
    }
    p.sumsq = norm_level >= 0 ? &scal->level_sumsq[norm_level] : nullptr;
    p.nonfinite = &scal->nonfinite;
    if (eng == ENG_F16S) {
      // the scaled-FP16 engine needs each operand's max-abs.  Its own
      // products record it for every FP32 output in the epilogue; an FP64
      // product (the residual) for output 0, with a separate pass for others.
      p.xamax = X.amax;
      p.yamax = Y.amax;
      if (e == ENG_F16S) {
        int k = 0;
        for (const Out& o : outs) {
          if (!o.b->f64) {
            p.out[k].amax = new_amax_slot();
            o.b->amax = p.out[k].amax;
          }
          ++k;
        }
      } else {
        p.amax = new_amax_slot();
      }
    }
    ops.push_back(op);
    ++gemms;
    if (p.amax) {
      size_t i = 0;
      for (const Out& o : outs) {
        if (i++ == 0) o.b->amax = p.amax;
        else amax(*o.b);
      }
    }
  }

  // Digit planes of the FP64 operands of an int8-emulated product: X (the
  // copy of A, the same buffer at every level) once per call, Y every time.
  void i8_operands(const Buf& X, const Buf& Y) {
    if (i8_x_src != X.p) {
      zero(i8_rmax, 8 * (size_t)np);
      maxabs(X, i8_rmax, nullptr);
      slice(X, 0, i8_rmax, i8_x);
      i8_x_src = X.p;
    }
    zero(i8_cmax, 8 * (size_t)np);
    maxabs(Y, nullptr, i8_cmax);
    slice(Y, 1, i8_cmax, i8_y);
  }

  void maxabs(const Buf& b, unsigned long long* rmax, unsigned long long* cmax) {
    Op op{};
    op.kind = Op::MAXABS;
    op.ptr = b.p;
    op.rmax = rmax;
    op.cmax = cmax;
    ops.push_back(op);
  }

  void slice(const Buf& b, int transpose, unsigned long long* mx, void* dst) {
    Op op{};
    op.kind = Op::SLICES;
    op.ptr = b.p;
    op.transpose = transpose;
    op.rmax = mx;
    op.dst = dst;
    op.slices = slices;
    op.crt = crt;
    ops.push_back(op);
  }

  // The last two recorded operations are independent products (neither reads
  // what the other writes): let them share one launch when both are plain
  // products of the same engine (not from panels) and one product's grid
  // leaves the chip under-filled.
  void pair_last_two() {
    const size_t m = ops.size();
    if (status != NS_OK || m < 2) return;
    Op& a = ops[m - 2];
    const Op& b = ops[m - 1];
    if (a.kind == Op::GEMM && b.kind == Op::GEMM && !a.panels && !b.panels && a.e == b.e &&
        a.e != ENG_I8 && gemm_grid(a.e, np) <= kPairMaxGrid)
      a.pair_next = true;
  }

  // Upload every recorded parameter block with one copy, then launch the
  // recorded operations in order on the stream.
  int execute() {
    if (status != NS_OK) return status;
    size_t ng = 0;
    for (const Op& op : ops) ng += op.kind == Op::GEMM;
    GemmParams *ph, *pd;
    int slot = -1;
    if (fixed) {
      if (ng > fixed->params_cap)
        return fail(NS_ERR_RANGE, "%zu products exceed the %zu parameter blocks of the fixed region",
                    ng, fixed->params_cap);
      ph = fixed->params_host;
      pd = fixed->params_dev;
    } else {
      const int st = ring_slot(ng, &ph, &pd, &slot);
      if (st) return st;
    }
    size_t gi = 0;
    for (const Op& op : ops)
      if (op.kind == Op::GEMM) ph[gi++] = op.p;
    if (ng) {
      // from the fixed (pageable) staging array the copy is synchronous for
      // the host, so the array is free again when it returns
      NS_HIP(hipMemcpyAsync(pd, ph, ng * sizeof(GemmParams), hipMemcpyHostToDevice, s));
      if (slot >= 0) NS_HIP(hipEventRecord(h->params_free[slot], s));
    }
    return launch_all(pd);
  }

  // The handle's next parameter slot (grown when a call has more blocks).
  int ring_slot(size_t ng, GemmParams** ph, GemmParams** pd, int* slot_out) {
    constexpr int R = ns_handle::kParamSlots;
    if (ng > h->params_cap) {
      NS_HIP(hipDeviceSynchronize());   // earlier kernels may still read the old blocks
      if (h->params_host) NS_HIP(hipHostFree(h->params_host));
      if (h->params_dev) NS_HIP(hipFree(h->params_dev));
      h->params_host = nullptr;
      h->params_dev = nullptr;
      h->params_cap = 0;
      const size_t cap = std::max<size_t>(ng, 256);
      if (hipHostMalloc((void**)&h->params_host, R * cap * sizeof(GemmParams)) != hipSuccess ||
          hipMalloc((void**)&h->params_dev, R * cap * sizeof(GemmParams)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(NS_ERR_NOMEM, "parameter buffers (%zu blocks) could not be allocated", cap);
      }
      h->params_cap = cap;
    }
    // this call's slot.  Its device blocks were last read by the call a ring
    // earlier, which has finished: every call waits for the previous one on
    // the handle.  Its host blocks may still be in that call's upload.
    const int slot = (int)(h->params_next++ % R);
    if (!h->params_free[slot])
      NS_HIP(hipEventCreateWithFlags(&h->params_free[slot], hipEventDisableTiming));
    NS_HIP(hipEventSynchronize(h->params_free[slot]));
    *ph = h->params_host + (size_t)slot * h->params_cap;
    *pd = h->params_dev + (size_t)slot * h->params_cap;
    *slot_out = slot;
    return NS_OK;
  }

  // Launch the recorded operations in order; pd holds the GEMM blocks.
  int launch_all(const GemmParams* pd) {
    const bool timing = h && h->timing;
    launches = 0;
    size_t gi = 0;
    for (size_t oi = 0; oi < ops.size(); ++oi) {
      const Op& op = ops[oi];
      if (op.kind == Op::ZERO || op.kind == Op::PAD || op.kind == Op::IDENTITY) {
        // a run of consecutive fills (the call's prologue: scalar reset,
        // copies-in, identities) goes out as one launch; they write distinct
        // buffers and read only the caller's A
        Fill f[kMaxFills];
        int nf = 0;
        for (; oi < ops.size() && nf < kMaxFills; ++oi) {
          const Op& x = ops[oi];
          if (x.kind != Op::ZERO && x.kind != Op::PAD && x.kind != Op::IDENTITY) break;
          Fill& y = f[nf++];
          y = Fill{};
          y.kind = x.kind == Op::ZERO ? FILL_ZERO : x.kind == Op::PAD ? FILL_PAD : FILL_IDENTITY;
          y.src_f64 = x.src_f64;
          y.dst_f64 = x.f64;
          y.n_pad = np;
          y.n = x.n;
          y.lda = x.ld;
          y.src = x.ptr;
          y.dst = x.kind == Op::PAD ? x.dst : x.ptr;
          y.bytes = x.kind == Op::ZERO ? (size_t)x.n : 0;
        }
        --oi;   // the loop's own increment moves past the run
        NS_HIP(launch_fills(f, nf, s));
        continue;
      }
      if (op.kind == Op::UNPAD) {
        NS_HIP(launch_unpad_copy(op.ptr, op.src_f64, np, op.dst, op.f64, op.n, op.ld, s));
        continue;
      }
      if (op.kind == Op::AMAX) {
        NS_HIP(launch_amax(static_cast<const float*>(op.ptr), (size_t)np * np, op.amax, s));
        continue;
      }
      if (op.kind == Op::PANELS) {
        NS_HIP(launch_to_panels(op.e, static_cast<const float*>(op.ptr), np, np, op.transpose, op.dst,
                                op.amax, s));
        continue;
      }
      if (op.kind == Op::MAXABS) {
        NS_HIP(launch_maxabs_rc(static_cast<const double*>(op.ptr), np, op.rmax, op.cmax, s));
        continue;
      }
      if (op.kind == Op::SLICES) {
        if (op.crt)
          NS_HIP(launch_crt_slices(static_cast<const double*>(op.ptr), np, op.transpose, op.rmax,
                                   op.dst, s));
        else
          NS_HIP(launch_i8_slices(static_cast<const double*>(op.ptr), np, op.transpose, op.rmax,
                                  op.slices, op.dst, s));
        continue;
      }
      // an independent next product shares this launch
      const bool pair = op.pair_next && oi + 1 < ops.size() && ops[oi + 1].kind == Op::GEMM;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timing) {
        if (h->ev_used == h->ev.size()) {
          for (int i = 0; i < 32; ++i) {
            ns_handle::Timed t{};
            NS_HIP(hipEventCreate(&t.e0));
            NS_HIP(hipEventCreate(&t.e1));
            h->ev.push_back(t);
          }
        }
        ns_handle::Timed& t = h->ev[h->ev_used++];
        t.engine = op.e;
        t.flops = (pair ? 2 : 1) * 2.0 * (double)n * n * n;
        e0 = t.e0;
        e1 = t.e1;
        NS_HIP(hipEventRecord(e0, s));
      }
      hipError_t err;
      if (op.e == ENG_I8 && op.crt)
        err = launch_gemm_crt(op.p.X, op.p.Y, np, op.tplanes, op.rmax, op.cmax, pd + gi, s);
      else if (op.e == ENG_I8)
        err = launch_gemm_i8(op.p.X, op.p.Y, np, op.slices, op.acc, op.rmax, op.cmax, pd + gi, s);
      else if (op.panels) err = launch_gemm_panels(op.e, op.p, pd + gi, s);
      else if (pair) err = launch_gemm(op.e, op.p, pd + gi, s, &ops[oi + 1].p, pd + gi + 1);
      else err = launch_gemm(op.e, op.p, pd + gi, s);
      gi += pair ? 2 : 1;
      ++launches;
      if (err != hipSuccess) return fail(NS_ERR_HIP, "product launch failed: %s", hipGetErrorString(err));
      if (timing) NS_HIP(hipEventRecord(e1, s));
      if (pair) ++oi;
    }
    ops.clear();
    if (h) h->product_launches = launches;
    return NS_OK;
  }
};

Out o(Buf& b, double a, double z0 = 0, double z1 = 0, double z2 = 0, double id = 0) {
  return Out{&b, a, {z0, z1, z2}, id};
}

// ---------------------------------------------------------------------------
// schedules
// ---------------------------------------------------------------------------

// Running sum update S <- S + S (T - I)  (block concatenation, eq. (2)).
// Sw is the working-precision operand; S64 (mixed forms) the FP64 accumulator.
void sum_update(Ctx& c, Buf& Sw, Buf& Sw2, Buf* S64, Buf& Tm1) {
  if (S64) {
    c.gemm(c.eng, Sw, Tm1, {*S64}, {o(*S64, 1, 1), o(Sw2, 1, 1)});
  } else {
    c.gemm(c.eng, Sw, Tm1, {Sw}, {o(Sw2, 1, 1)});
  }
  std::swap(Sw, Sw2);
}

// Theorem 3.1 on B: after the three products T holds T9(B) - I.
//   U = B^2;  V = U (B + 2U);  P = 3/20 B + 2U + V;  Q = 11/40 B - 1/8 U + 1/4 V;
//   W = P Q;  T9 = W + I + B + 767/800 U + 15/32 V.
// The first product writes only U and the operand B + 2U; the second forms P,
// Q and T - W from V, B and U (8 matrix passes of epilogue traffic for the two
// products instead of 12 when the first one also wrote the partial sums).
void kernel_radix9(Ctx& c, Buf& B, Buf& U, Buf& X1, Buf& P, Buf& Q, Buf& T) {
  c.gemm(c.eng, B, B, {B}, {o(U, 1.0), o(X1, 2.0, 1.0)});
  c.gemm(c.eng, U, X1, {B, U},
         {o(P, 1.0, 3.0 / 20.0, 2.0), o(Q, 0.25, 11.0 / 40.0, -1.0 / 8.0),
          o(T, 15.0 / 32.0, 1.0, 767.0 / 800.0)});
  c.gemm(c.eng, P, Q, {T}, {o(T, 1.0, 1.0)});
}

// Gustafsson's quinary kernel (Sec. 2.3): U = B^2, V = U (B + U),
// T5 = I + B + U + V; T holds T5 - I.
void kernel_quinary(Ctx& c, Buf& B, Buf& U, Buf& X1, Buf& T) {
  c.gemm(c.eng, B, B, {B}, {o(U, 1.0), o(X1, 1.0, 1.0), o(T, 1.0, 1.0)});
  c.gemm(c.eng, U, X1, {T}, {o(T, 1.0, 1.0)});
}

// Sec. 4.1 eq. (4)-(5) on R with coefficients k[28]; F holds T15~(R) - I.
void kernel_radix15(Ctx& c, const double* k, Buf& R, Buf& P1, Buf& L2, Buf& R2, Buf& L3,
                    Buf& R3, Buf& L4, Buf& R4, Buf& F) {
  const double *l2 = k, *r2 = k + 3, *l3 = k + 6, *r3 = k + 10, *l4 = k + 14, *r4 = k + 19,
               *g = k + 24;
  // P1 = R R; the factors of P2 are combinations of {I, R, P1}
  c.gemm(c.eng, R, R, {R},
         {o(P1, 1.0), o(L2, l2[2], l2[1], 0, 0, l2[0]), o(R2, r2[2], r2[1], 0, 0, r2[0])});
  // P2 = L2 R2; factors of P3 complete, those of P4 and F partial
  c.gemm(c.eng, L2, R2, {R, P1},
         {o(L3, l3[3], l3[1], l3[2], 0, l3[0]), o(R3, r3[3], r3[1], r3[2], 0, r3[0]),
          o(L4, l4[3], l4[1], l4[2], 0, l4[0]), o(R4, r4[3], r4[1], r4[2], 0, r4[0]),
          o(F, g[2], g[0], g[1])});
  // P3 = L3 R3
  c.gemm(c.eng, L3, R3, {L4, R4, F}, {o(L4, l4[4], 1.0), o(R4, r4[4], 0, 1.0), o(F, g[3], 0, 0, 1.0)});
  // P4 = L4 R4
  c.gemm(c.eng, L4, R4, {F}, {o(F, 1.0, 1.0)});
}

struct Result {
  Buf S;          // what to copy out (FP64 accumulator for mixed forms)
};

// One step of the exact plan for any k (NS_MIXED).  m > 1: radix-m update of
// (S, B = A^n); m = 1: additive step S <- S + B, B <- A B.  With `fuse` the
// plan's final additive step S + A^(new n) is folded into the step's last
// product (its C is the new power).  Bn receives the new power.
void mixed_step(Ctx& c, int m, bool fuse, const Buf& A, Buf& S, Buf& S2, Buf* S64, Buf& B, Buf& Bn,
                Buf& U, Buf& X1, Buf& P, Buf& Q, Buf& T, int lv) {
  if (m == 1) {
    if (!S64) {
      c.gemm(c.eng, A, B, {S, B}, {o(Bn, 1.0), o(S2, fuse ? 1.0 : 0.0, 1.0, 1.0)});
      std::swap(S, S2);
    } else if (fuse) {
      c.gemm(c.eng, A, B, {*S64, B}, {o(Bn, 1.0), o(*S64, 1.0, 1.0, 1.0)});
    } else {
      c.gemm(c.eng, A, B, {*S64, B}, {o(Bn, 1.0), o(*S64, 0.0, 1.0, 1.0), o(S, 0.0, 1.0, 1.0)});
    }
    return;
  }
  // Without the fused final step, a step's last two products are independent
  // and share one launch; with it, the last product reads the sum the one
  // before it wrote.
  if (m == 2) {
    sum_update(c, S, S2, S64, B);                      // S_2n = S_n (I + A^n)
    // A^2n = A^n A^n (+ the final additive step S_2n + A^2n)
    if (!fuse) {
      c.gemm(c.eng, B, B, {}, {o(Bn, 1.0)}, lv);
      c.pair_last_two();
    } else if (S64) c.gemm(c.eng, B, B, {*S64}, {o(Bn, 1.0), o(*S64, 1.0, 1.0)}, lv);
    else {
      c.gemm(c.eng, B, B, {S}, {o(Bn, 1.0), o(S2, 1.0, 1.0)}, lv);
      std::swap(S, S2);
    }
    return;
  }
  if (m == 3) {
    // U = A^2n, T = A^n + A^2n = T3 - I; S_3n = S_n T3; A^3n = U A^n
    c.gemm(c.eng, B, B, {B}, {o(U, 1.0), o(T, 1.0, 1.0)});
    sum_update(c, S, S2, S64, T);
    if (!fuse) {
      c.gemm(c.eng, U, B, {}, {o(Bn, 1.0)}, lv);
      c.pair_last_two();
    } else if (S64) c.gemm(c.eng, U, B, {*S64}, {o(Bn, 1.0), o(*S64, 1.0, 1.0)}, lv);
    else {
      c.gemm(c.eng, U, B, {S}, {o(Bn, 1.0), o(S2, 1.0, 1.0)}, lv);
      std::swap(S, S2);
    }
    return;
  }
  if (m == 9) kernel_radix9(c, B, U, X1, P, Q, T);
  else kernel_quinary(c, B, U, X1, T);
  sum_update(c, S, S2, S64, T);
  // telescoping: A^mn = B - (T - I) + (T - I) B
  if (!fuse) {
    c.gemm(c.eng, T, B, {B, T}, {o(Bn, 1.0, 1.0, -1.0)}, lv);
    c.pair_last_two();
  } else if (S64) c.gemm(c.eng, T, B, {B, T, *S64}, {o(Bn, 1.0, 1.0, -1.0), o(*S64, 1.0, 1.0, -1.0, 1.0)}, lv);
  else {
    c.gemm(c.eng, T, B, {B, T, S}, {o(Bn, 1.0, 1.0, -1.0), o(S2, 1.0, 1.0, -1.0, 1.0)}, lv);
    std::swap(S, S2);
  }
}

int run_schedule(Ctx& c, int method, int64_t k, int levels, const Buf& Ain_w, const Buf* Ain64,
                 Result* res) {
  const int W64 = (c.eng == ENG_F64) ? 1 : 0;
  Buf A = Ain_w;
  switch (method) {
    case NS_NAIVE: {                                   // S <- I + A S
      Buf S = c.take(W64), S2 = c.take(W64);
      c.identity(S);
      for (int i = 0; i < levels; ++i) {
        c.gemm(c.eng, A, S, {}, {o(S2, 1.0, 0, 0, 0, 1.0)});
        std::swap(S, S2);
      }
      res->S = S;
      break;
    }
    case NS_BINARY:
    case NS_TERNARY:
    case NS_QUINARY:
    case NS_RADIX9: {
      Buf S = c.take(W64), S2 = c.take(W64), B = A, B2 = c.take(W64);
      Buf S64;
      if (c.mixed) {
        S64 = c.take(1);
        c.identity(S64);
      }
      c.identity(S);
      Buf U, X1, P, Q, T;
      if (method == NS_RADIX9) { U = c.take(W64); X1 = c.take(W64); P = c.take(W64); Q = c.take(W64); T = c.take(W64); }
      if (method == NS_QUINARY) { U = c.take(W64); X1 = c.take(W64); T = c.take(W64); }
      if (method == NS_TERNARY) { U = c.take(W64); T = c.take(W64); }
      for (int lv = 0; lv < levels && c.status == NS_OK; ++lv) {
        if (method == NS_BINARY) {
          // S_2n = S_n (I + A^n);  A^2n = A^n A^n (independent: one launch)
          sum_update(c, S, S2, c.mixed ? &S64 : nullptr, B);
          c.gemm(c.eng, B, B, {}, {o(B2, 1.0)}, lv);
          c.pair_last_two();
          std::swap(B, B2);
          continue;
        }
        if (method == NS_TERNARY) {
          // A^2n = A^n A^n;  A^3n = A^2n A^n;  S_3n = S_n (I + A^n + A^2n)
          c.gemm(c.eng, B, B, {B}, {o(U, 1.0), o(T, 1.0, 1.0)});
          c.gemm(c.eng, U, B, {}, {o(B2, 1.0)}, lv);
          sum_update(c, S, S2, c.mixed ? &S64 : nullptr, T);
          c.pair_last_two();
          std::swap(B, B2);
          continue;
        }
        if (method == NS_RADIX9) kernel_radix9(c, B, U, X1, P, Q, T);
        else kernel_quinary(c, B, U, X1, T);
        sum_update(c, S, S2, c.mixed ? &S64 : nullptr, T);
        // telescoping: A^{mn} = I - T + T A^n = B - (T - I) + (T - I) B,
        // independent of the sum update (one launch)
        c.gemm(c.eng, T, B, {B, T}, {o(B2, 1.0, 1.0, -1.0)}, lv);
        c.pair_last_two();
        std::swap(B, B2);   // after the first level the copy of A becomes the spare
      }
      res->S = c.mixed ? S64 : S;
      break;
    }
    case NS_MIXED: {
      std::vector<int> steps;
      mixed_plan(k, &steps);
      Buf S = c.take(W64), S2 = c.take(W64);
      Buf Bb[2] = {c.take(W64), c.take(W64)};
      Buf U = c.take(W64), X1 = c.take(W64), P = c.take(W64), Q = c.take(W64), T = c.take(W64);
      Buf S64;
      if (c.mixed) {
        S64 = c.take(1);
        c.identity(S64);
      }
      c.identity(S);
      Buf B = A;                  // A^n; the copy of A stays intact for the additive steps
      int bi = 0, lv = 0;
      for (size_t i = 0; i < steps.size() && c.status == NS_OK; ++i) {
        const bool fuse = i + 2 == steps.size() && steps[i + 1] == 1;
        mixed_step(c, steps[i], fuse, A, S, S2, c.mixed ? &S64 : nullptr, B, Bb[bi], U, X1, P, Q, T,
                   steps[i] > 1 ? lv : -1);
        if (steps[i] > 1) ++lv;
        B = Bb[bi];
        bi ^= 1;
        if (fuse) ++i;
      }
      res->S = c.mixed ? S64 : S;
      break;
    }
    case NS_HENSEL:
    case NS_RADIX9_RESID:
    case NS_RADIX15:
    case NS_RADIX15C: {
      // Y_0 = I, R_0 = A;  Y <- Y f(R);  R <- I - (I - A) Y   (eq. (8))
      Buf Y = c.take(W64), Y2 = c.take(W64), R = c.take(W64);
      Buf Y64, A64;
      c.identity(Y);
      if (c.mixed) {
        Y64 = c.take(1);
        c.identity(Y64);
        A64 = *Ain64;
      }
      // R_0 = A: the first level reads the copy of A directly
      Buf Rcur = A;
      double k15[28];
      Buf U, X1, P, Q, T, P1, L2, R2, L3, R3, L4, R4, F;
      if (method == NS_RADIX9_RESID) { U = c.take(W64); X1 = c.take(W64); P = c.take(W64); Q = c.take(W64); T = c.take(W64); }
      if (method == NS_RADIX15 || method == NS_RADIX15C) {
        const bool ok = method == NS_RADIX15 ? radix15_table(k15, nullptr, nullptr, nullptr)
                                             : radix15c_table(k15, nullptr, nullptr, nullptr);
        if (!ok) return fail(NS_ERR_RANGE, "radix-15 coefficient polish did not converge");
        P1 = c.take(W64); L2 = c.take(W64); R2 = c.take(W64); L3 = c.take(W64);
        R3 = c.take(W64); L4 = c.take(W64); R4 = c.take(W64); F = c.take(W64);
      }
      for (int lv = 0; lv < levels && c.status == NS_OK; ++lv) {
        Buf* Fm1;
        if (method == NS_HENSEL) Fm1 = &Rcur;                        // f(R) - I = R
        else if (method == NS_RADIX9_RESID) { kernel_radix9(c, Rcur, U, X1, P, Q, T); Fm1 = &T; }
        else { kernel_radix15(c, k15, Rcur, P1, L2, R2, L3, R3, L4, R4, F); Fm1 = &F; }
        sum_update(c, Y, Y2, c.mixed ? &Y64 : nullptr, *Fm1);
        // R = I - Y + A Y: the true residual of the new iterate.  The mixed
        // forms take A Y exactly (FP64 MFMA, or int8 slices) -- with
        // NS_RESID_LAST only at the last two levels, the earlier ones in
        // working precision against the FP64 Y
        if (!c.mixed) c.gemm(c.eng, A, Y, {Y}, {o(R, 1.0, -1.0, 0, 0, 1.0)}, lv);
        else if (c.resid_last && lv < levels - 2)
          c.gemm(c.eng, A, Y, {Y64}, {o(R, 1.0, -1.0, 0, 0, 1.0)}, lv);
        else c.gemm(c.slices ? ENG_I8 : ENG_F64, A64, Y64, {Y64}, {o(R, 1.0, -1.0, 0, 0, 1.0)}, lv);
        Rcur = R;
      }
      res->S = c.mixed ? Y64 : Y;
      break;
    }
    default:
      return fail(NS_ERR_ARG, "unknown method %d", method);
  }
  return c.status;
}

int check_args(const void* A, int64_t n, int64_t lda, int64_t k, int method, int dtype,
               const void* out, int64_t ldo) {
  if (!A || !out) return fail(NS_ERR_ARG, "null matrix pointer");
  if (n <= 0) return fail(NS_ERR_ARG, "n must be positive (got %lld)", (long long)n);
  if (n > 65536) return fail(NS_ERR_RANGE, "n = %lld above the supported 65536", (long long)n);
  if (lda < n || ldo < n) return fail(NS_ERR_ARG, "leading dimension below n");
  if (k < 1) return fail(NS_ERR_ARG, "k must be >= 1 (got %lld)", (long long)k);
  if (method < NS_NAIVE || method > NS_RADIX15C) return fail(NS_ERR_ARG, "unknown method %d", method);
  const int base = base_of(dtype);
  if (base < NS_F64 || base > NS_F32_ACC64 || (dtype & ~(kBaseMask | kModifierBits)))
    return fail(NS_ERR_ARG, "unknown dtype %d", dtype);
  if (dtype & ~kBaseMask) {
    if (!(dtype & kResidInt8) && (dtype >> kSliceShift))
      return fail(NS_ERR_ARG, "slice count without NS_RESID_INT8 (dtype 0x%x)", dtype);
    if (resid_slices(dtype) > kMaxI8Slices)
      return fail(NS_ERR_ARG, "NS_RESID_INT8 takes 1 to %d slices", kMaxI8Slices);
    if ((dtype & kResidInt8) && resid_crt(dtype))
      return fail(NS_ERR_ARG, "NS_RESID_INT8 and NS_RESID_CRT exclude each other");
    if (!is_mixed(dtype) || !is_residual(method))
      return fail(NS_ERR_UNSUPPORTED,
                  "residual modifiers need a residual method in an FP64-accumulating dtype");
    const int64_t np = n_internal(n, dtype);
    if (resid_crt(dtype) && (!crt_moduli((int)np) || np * 128 * 128 >= ((int64_t)1 << 31)))
      return fail(NS_ERR_RANGE, "NS_RESID_CRT at padded n = %lld: beyond its moduli or int32 sums",
                  (long long)np);
    if ((int64_t)resid_slices(dtype) * np * 127 * 127 >= ((int64_t)1 << 31))
      return fail(NS_ERR_RANGE, "%d int8 slices at padded n = %lld overflow int32 accumulation",
                  resid_slices(dtype), (long long)np);
  }
  if (method == NS_NAIVE && is_mixed(dtype))
    return fail(NS_ERR_UNSUPPORTED, "the naive Horner form has no FP64-accumulated variant");
  const size_t es = (base == NS_F32) ? 4 : 8;
  const char* a0 = static_cast<const char*>(A);
  const char* a1 = a0 + ((size_t)(n - 1) * lda + n) * es;
  const char* b0 = static_cast<const char*>(out);
  const char* b1 = b0 + ((size_t)(n - 1) * ldo + n) * es;
  if (a0 < b1 && b0 < a1) return fail(NS_ERR_ARG, "out overlaps A");
  return NS_OK;
}

int ensure_workspace(ns_handle* h, size_t bytes) {
  if (h->ws_bytes >= bytes) return NS_OK;
  if (h->ws) {
    NS_HIP(hipDeviceSynchronize());
    NS_HIP(hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  if (hipMalloc(&h->ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    h->ws = nullptr;
    return fail(NS_ERR_NOMEM, "workspace of %zu bytes could not be allocated", bytes);
  }
  h->ws_bytes = bytes;
  return NS_OK;
}

std::mutex g_default_mu;
ns_handle* g_default[64] = {};

}  // namespace

// One evaluation, either on a handle (h: its workspace, parameter ring,
// timing and call ordering) or on a fixed memory region (fx, h null: nothing
// is allocated and no event is used).  The caller has made the device current.
int eval_core(ns_handle* h, const FixedMem* fx, const void* A, int64_t n, int64_t lda, int64_t k,
              int method, int dtype, void* out, int64_t ldo, hipStream_t s, ns_report* rep) {
  int st = check_args(A, n, lda, k, method, dtype, out, ldo);
  if (st) return st;
  int64_t k_eff;
  int32_t levels, gemms_formula;
  if ((st = plan(k, method, &k_eff, &levels, &gemms_formula))) return st;
  const size_t need = workspace_bytes(n, method, dtype);
  char* ws;
  if (fx) {
    if (need > fx->ws_bytes)
      return fail(NS_ERR_RANGE,
                  "n = %lld needs %zu bytes of workspace for this method and dtype; the fixed "
                  "region holds %zu",
                  (long long)n, need, fx->ws_bytes);
    ws = fx->ws;
  } else {
    if ((st = ensure_workspace(h, need))) return st;
    if (!h->call_done) NS_HIP(hipEventCreateWithFlags(&h->call_done, hipEventDisableTiming));
    else NS_HIP(hipStreamWaitEvent(s, h->call_done, 0));
    ws = static_cast<char*>(h->ws);
  }

  Ctx c{};
  c.h = h;
  c.fixed = fx;
  c.s = s;
  c.n = (int)n;
  c.np = n_internal(n, dtype);
  c.eng = work_engine(dtype);
  c.mixed = is_mixed(dtype);
  c.resid_last = resid_last(dtype);
  c.crt = resid_crt(dtype);
  c.slices = resid_planes(dtype, c.np);
  c.scal = reinterpret_cast<Scalars*>(ws);
  c.arena = ws + kScalarBytes;
  c.zero(c.scal, sizeof(Scalars));
  if (c.slices) {
    // the int8-emulated residual's buffers sit at the end of the workspace
    const size_t mat = (size_t)c.np * c.np;
    char* q = ws + need - i8_bytes(c.np, c.slices, c.crt);
    q = reinterpret_cast<char*>(((uintptr_t)q + 255) & ~(uintptr_t)255);
    c.i8_x = q;
    c.i8_y = q + c.slices * mat;
    if (c.crt) {
      c.i8_t = q + 2 * c.slices * mat;
      c.i8_rmax = reinterpret_cast<unsigned long long*>(q + 3 * c.slices * mat);
    } else {
      c.i8_acc = reinterpret_cast<double*>(q + 2 * c.slices * mat);
      c.i8_rmax = reinterpret_cast<unsigned long long*>(q + 2 * c.slices * mat + 8 * mat);
    }
    c.i8_cmax = c.i8_rmax + c.np;
  }

  const int in64 = (base_of(dtype) != NS_F32);
  const int W64 = (c.eng == ENG_F64);
  Buf Aw = c.take(W64);
  c.pad(A, in64, lda, Aw);
  Buf A64;
  if (c.mixed && is_residual(method)) {
    A64 = c.take(1);
    c.pad(A, 1, lda, A64);
  }
  if (c.eng == ENG_F16S) c.amax(Aw);
  Result res;
  if ((st = run_schedule(c, method, k, levels, Aw, c.mixed ? &A64 : nullptr, &res))) return st;
  c.unpad(res.S, out, in64, ldo);
  if ((st = c.execute())) return st;
  if (h) NS_HIP(hipEventRecord(h->call_done, s));

  if (rep) {
    Scalars hs;
    NS_HIP(hipMemcpyAsync(&hs, c.scal, offsetof(Scalars, amax), hipMemcpyDeviceToHost, s));
    NS_HIP(hipStreamSynchronize(s));
    std::memset(rep, 0, sizeof(*rep));
    rep->k_eff = k_eff;
    rep->levels = levels;
    rep->gemms_performed = c.gemms;
    rep->gemms_formula = gemms_formula;
    rep->nonfinite = hs.nonfinite ? 1 : 0;
    rep->n_internal = c.np;
    rep->method = method;
    rep->dtype = dtype;
    rep->product_launches = (int32_t)c.launches;
    if (method != NS_NAIVE)
      for (int i = 0; i < levels && i < NS_MAX_LEVELS; ++i) rep->level_norm[i] = std::sqrt(hs.level_sumsq[i]);
    if (method == NS_RADIX15 || method == NS_RADIX15C) {
      double cc[28];
      if (method == NS_RADIX15) radix15_table(cc, &rep->kernel_prefix_err, &rep->spill15, &rep->spill16);
      else radix15c_table(cc, &rep->kernel_prefix_err, &rep->spill15, &rep->spill16);
    }
  }
  return NS_OK;
}

int eval_impl(ns_handle* h, const void* A, int64_t n, int64_t lda, int64_t k, int method,
              int dtype, void* out, int64_t ldo, hipStream_t s, ns_report* rep) {
  const DeviceGuard dg(h->device);
  NS_HIP(dg.err);
  return eval_core(h, nullptr, A, n, lda, k, method, dtype, out, ldo, s, rep);
}

// The fixed-region path of ns_eval_noalloc (noalloc.hip); the current device
// is the region's.
int eval_fixed(char* ws, size_t ws_bytes, GemmParams* params_host, GemmParams* params_dev,
               size_t params_cap, const void* A, int64_t n, int64_t lda, int64_t k, int method,
               int dtype, void* out, int64_t ldo, hipStream_t s, ns_report* rep) {
  const FixedMem fx{ws, ws_bytes, params_host, params_dev, params_cap};
  return eval_core(nullptr, &fx, A, n, lda, k, method, dtype, out, ldo, s, rep);
}

int fail_status(int status, const char* msg) { return fail(status, "%s", msg); }

Engine work_engine_of(int dtype) { return work_engine(dtype); }

// accessors for batched.hip
int batch_fail(int status, const char* msg) { return fail(status, "%s", msg); }
void* handle_batched_state(ns_handle* h) { return h->batched; }
void set_handle_batched_state(ns_handle* h, void* st) { h->batched = st; }
int handle_device(ns_handle* h) { return h->device; }

}  // namespace ns

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int ns_create(ns_handle** h, int device) {
  if (!h) return fail(NS_ERR_ARG, "null handle pointer");
  *h = nullptr;
  int count = 0;
  NS_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(NS_ERR_ARG, "device %d of %d", device, count);
  ns_handle* p = new (std::nothrow) ns_handle();
  if (!p) return fail(NS_ERR_NOMEM, "host allocation failed");
  p->device = device;
  *h = p;
  return NS_OK;
}

int ns_destroy(ns_handle* h) {
  if (!h) return NS_OK;
  {
    const ns::DeviceGuard dg(h->device);
    (void)hipDeviceSynchronize();
    ns::batched_release(h);
    for (const auto& t : h->ev) {
      (void)hipEventDestroy(t.e0);
      (void)hipEventDestroy(t.e1);
    }
    for (hipEvent_t e : h->params_free)
      if (e) (void)hipEventDestroy(e);
    if (h->call_done) (void)hipEventDestroy(h->call_done);
    if (h->params_host) (void)hipHostFree(h->params_host);
    if (h->params_dev) (void)hipFree(h->params_dev);
    if (h->ws) (void)hipFree(h->ws);
  }
  delete h;
  return NS_OK;
}

int ns_plan(int64_t k, int method, int64_t* k_eff, int32_t* levels, int32_t* gemms) {
  int64_t a;
  int32_t b, c;
  const int st = ns::plan(k, method, &a, &b, &c);
  if (st) return st;
  if (k_eff) *k_eff = a;
  if (levels) *levels = b;
  if (gemms) *gemms = c;
  return NS_OK;
}

int ns_workspace_bytes(int64_t n, int method, int dtype, size_t* bytes) {
  if (!bytes) return fail(NS_ERR_ARG, "null output pointer");
  if (n <= 0 || method < NS_NAIVE || method > NS_RADIX15C || ns::base_of(dtype) > NS_F32_ACC64 ||
      dtype < 0 || (dtype & ~(ns::kBaseMask | ns::kModifierBits)))
    return fail(NS_ERR_ARG, "bad arguments");
  *bytes = ns::workspace_bytes(n, method, dtype);
  return NS_OK;
}

int ns_eval_ex(ns_handle* h, const void* A, int64_t n, int64_t lda, int64_t k, int method,
               int dtype, void* out, int64_t ldo, hipStream_t stream, ns_report* rep) {
  if (!h) return fail(NS_ERR_ARG, "null handle");
  try {
    return ns::eval_impl(h, A, n, lda, k, method, dtype, out, ldo, stream, rep);
  } catch (...) {
    return fail(NS_ERR_HIP, "unexpected C++ exception");
  }
}

int ns_eval(const void* A, int64_t n, int64_t k, int method, int dtype, void* out) {
  int dev = 0;
  NS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(NS_ERR_ARG, "device index %d", dev);
  // every host thread shares the default handle, so the whole call (the
  // host-side recording and enqueueing) runs under the lock
  std::lock_guard<std::mutex> lk(ns::g_default_mu);
  if (!ns::g_default[dev]) {
    const int st = ns_create(&ns::g_default[dev], dev);
    if (st) return st;
  }
  return ns_eval_ex(ns::g_default[dev], A, n, n, k, method, dtype, out, n, nullptr, nullptr);
}

int ns_eval_batched(ns_handle* h, const void* A_packed, const int64_t* off_dev,
                    const int32_t* n_dev, const int32_t* n_host, int32_t batch, int64_t k,
                    int method, int dtype, void* out_packed, hipStream_t stream, ns_report* rep) {
  if (!h) return fail(NS_ERR_ARG, "null handle");
  try {
    return ns::batched_eval(h, A_packed, off_dev, n_dev, n_host, batch, k, method, dtype,
                            out_packed, stream, rep);
  } catch (...) {
    return fail(NS_ERR_HIP, "unexpected C++ exception");
  }
}

int ns_eval_batched_loop(ns_handle* h, const void* A_packed, const int64_t* off_host,
                         const int32_t* n_host, int32_t batch, int64_t k, int method, int dtype,
                         void* out_packed, hipStream_t stream) {
  if (!h || !A_packed || !off_host || !n_host || !out_packed || batch < 0)
    return fail(NS_ERR_ARG, "bad arguments");
  if (dtype != NS_F32) return fail(NS_ERR_UNSUPPORTED, "the batched forms are FP32");
  for (int32_t i = 0; i < batch; ++i) {
    const float* a = static_cast<const float*>(A_packed) + off_host[i];
    float* o = static_cast<float*>(out_packed) + off_host[i];
    const int st = ns_eval_ex(h, a, n_host[i], n_host[i], k, method, dtype, o, n_host[i], stream, nullptr);
    if (st) return st;
  }
  return NS_OK;
}

int ns_autotune_batched(ns_handle* h, const void* A_packed, const int64_t* off_dev,
                        const int32_t* n_dev, const int32_t* n_host, int32_t batch, int64_t k,
                        void* out_packed, hipStream_t stream, int32_t* n_timed) {
  if (!h) return fail(NS_ERR_ARG, "null handle");
  try {
    return ns::batched_autotune(h, A_packed, off_dev, n_dev, n_host, batch, k, out_packed, stream,
                                n_timed);
  } catch (...) {
    return fail(NS_ERR_HIP, "unexpected C++ exception");
  }
}

int ns_radix15_coeffs(double c28[28], double* prefix_err, double* spill15, double* spill16) {
  if (!c28) return fail(NS_ERR_ARG, "null output");
  if (!ns::radix15_table(c28, prefix_err, spill15, spill16))
    return fail(NS_ERR_RANGE, "radix-15 coefficient polish did not converge");
  return NS_OK;
}

int ns_radix15c_coeffs(double c28[28], double* prefix_err, double* spill15, double* spill16) {
  if (!c28) return fail(NS_ERR_ARG, "null output");
  if (!ns::radix15c_table(c28, prefix_err, spill15, spill16))
    return fail(NS_ERR_RANGE, "radix-15 coefficient polish did not converge");
  return NS_OK;
}

int ns_set_product_timing(ns_handle* h, int enable) {
  if (!h) return fail(NS_ERR_ARG, "null handle");
  h->timing = enable != 0;
  return NS_OK;
}

namespace {
// Sum the timed launches of one engine (-1: all), waiting for their events.
int sum_timing(ns_handle* h, int engine, int32_t* count, double* total_ms, double* total_flops) {
  double ms = 0.0, fl = 0.0;
  int32_t cnt = 0;
  for (size_t i = 0; i < h->ev_used; ++i) {
    const auto& t = h->ev[i];
    if (engine >= 0 && t.engine != engine) continue;
    NS_HIP(hipEventSynchronize(t.e1));
    float x = 0.f;
    NS_HIP(hipEventElapsedTime(&x, t.e0, t.e1));
    ms += x;
    fl += t.flops;
    ++cnt;
  }
  if (count) *count = cnt;
  if (total_ms) *total_ms = ms;
  if (total_flops) *total_flops = fl;
  return NS_OK;
}
}  // namespace

int ns_product_timing(ns_handle* h, int32_t* count, double* total_ms, double* total_flops,
                      int reset) {
  if (!h) return fail(NS_ERR_ARG, "null handle");
  const int st = sum_timing(h, -1, count, total_ms, total_flops);
  if (st) return st;
  if (reset) h->ev_used = 0;
  return NS_OK;
}

int ns_product_timing_dtype(ns_handle* h, int dtype, int32_t* count, double* total_ms,
                            double* total_flops) {
  if (!h) return fail(NS_ERR_ARG, "null handle");
  if (dtype == NS_RESID_INT8(0)) return sum_timing(h, ns::ENG_I8, count, total_ms, total_flops);
  if (dtype < NS_F64 || dtype > NS_F16_SCALED)
    return fail(NS_ERR_ARG, "dtype %d names no product engine", dtype);
  return sum_timing(h, ns::work_engine_of(dtype), count, total_ms, total_flops);
}

int ns_product_timing_launches(ns_handle* h, int32_t cap, float* ms, int32_t* engine,
                               int32_t* count) {
  if (!h || cap < 0) return fail(NS_ERR_ARG, "bad arguments");
  int32_t i = 0;
  for (size_t k = 0; k < h->ev_used; ++k, ++i) {
    if (i >= cap) continue;
    const auto& t = h->ev[k];
    if (ms) {
      NS_HIP(hipEventSynchronize(t.e1));
      NS_HIP(hipEventElapsedTime(&ms[i], t.e0, t.e1));
    }
    // engines are named by the dtype that uses them; the int8 residual engine
    // by its modifier
    if (engine) engine[i] = t.engine == ns::ENG_I8 ? NS_RESID_INT8(0) : t.engine;
  }
  if (count) *count = (int32_t)h->ev_used;
  return NS_OK;
}

const char* ns_status_string(int status) {
  switch (status) {
    case NS_OK: return "ok";
    case NS_ERR_ARG: return "invalid argument";
    case NS_ERR_UNSUPPORTED: return "unsupported combination";
    case NS_ERR_NOMEM: return "out of device memory";
    case NS_ERR_HIP: return "HIP runtime error";
    case NS_ERR_RANGE: return "size out of range";
    default: return "unknown status";
  }
}

const char* ns_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
