// Batched S_k over thousands of small matrices of uneven n in ONE persistent
// kernel launch (replayed from a cached HIP graph).
//
// Work distribution: a device queue of (matrix index, n) pairs in longest-first order
// (n descending, so the n = 256 matrices that carry most of the flops start
// first and the small ones fill the tail).  Each workgroup pops a ticket,
// evaluates that matrix's whole schedule itself, and pops again; when the
// queue is empty it counts itself out, and the last workgroup out resets the
// two counters, so every launch (and graph replay) starts from zero without a
// memset node.  Every workgroup exits once the ticket passes the batch size.
//
// Per matrix, the workgroup runs the same MFMA tile code and fused epilogue
// as the single-matrix products (gemm_device.h) on its private workspace
// slot: n is padded to the tile (64 for n <= 64, else a multiple of 128) and
// the padding is zero, which leaves the top-left n x n block of every
// polynomial in A exact.  Products are separated by workgroup barriers; the
// slot stays in L2/MALL while the workgroup works on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ns.h"
#include "gemm_device.h"

struct ns_handle;

namespace ns {

// defined in ns.cpp
int batch_fail(int status, const char* msg);
void* handle_batched_state(ns_handle* h);
void set_handle_batched_state(ns_handle* h, void* st);
int handle_device(ns_handle* h);

namespace {
using namespace dev;

constexpr int kMaxBatchN = 256;
constexpr int kSlotMats = 9;          // B, B', S, S', U, X1, P, Q, T
constexpr int kThreads = 256;

// One queue entry: matrix index and its n, taken from the caller's host array
// (validated to lie in [1, 256] before upload) -- the kernel never reads the
// caller's device copy of n.
struct Item {
  int32_t m;
  int32_t n;
};

struct BatchArgs {
  const float* A;
  float* out;
  const int64_t* off;
  const Item* items;          // longest first
  int batch;
  int levels;
  int method;
  float* work;                // grid slots of kSlotMats * 256^2 floats
  unsigned* counter;          // queue head
  unsigned* done;             // workgroups that found the queue empty
  double* sumsq;              // per level, summed over matrices
  int* nonfinite;
};

// One workgroup-wide product C = X Y on an np x np slot matrix (ld = np),
// tile by tile, with the fused epilogue `ep`.  Outputs never alias X or Y.
// The product's statistics (norm of output 0 if ep.sumsq is set, nonfinite
// flag) are published at the end; the trailing barrier keeps the next
// product's LDS stores behind the reduction's LDS reads.
template <class P>
__device__ __forceinline__ void wg_product(const float* X, const float* Y, int np,
                                           const GemmParams& ep, float* smem) {
  const int tn_count = np / P::BN, tiles = (np / P::BM) * tn_count;
  EpiState st{0.0, 0.f, 0};
  for (int t = 0; t < tiles; ++t) {
    const int row0 = (t / tn_count) * P::BM, col0 = (t % tn_count) * P::BN;
    typename P::Acc acc;
    P::zero(acc);
    if constexpr (DmaShape<P>::OK)        // 1 KB tile rows: np == BN, so rows stay in the slot
      tile_mainloop_dma<P>(X, Y, np, np, row0, col0, smem, acc);
    else
      tile_mainloop<P>(X, Y, np, np, row0, col0, smem, acc);
    tile_epilogue<P, true>(acc, ep, row0, col0, smem, st);   // all slot matrices are FP32
  }
  publish_stats<kThreads>(ep, st, reinterpret_cast<double*>(smem));
  __syncthreads();
}

__device__ __forceinline__ GemmParams ep0(int np, int* nonfinite) {
  GemmParams p{};
  p.n = np;
  p.ld = np;
  p.nonfinite = nonfinite;
  return p;
}
__device__ __forceinline__ void ep_z(GemmParams& p, const float* z) {
  p.Z[p.nz] = z;
  p.zf64[p.nz] = 0;
  ++p.nz;
}
__device__ __forceinline__ void ep_out(GemmParams& p, float* ptr, double a, double z0 = 0,
                                       double z1 = 0, double z2 = 0, double id = 0) {
  EpiOut& e = p.out[p.no++];
  e.ptr = ptr;
  e.f64 = 0;
  e.a = a;
  e.z[0] = z0;
  e.z[1] = z1;
  e.z[2] = z2;
  e.id = id;
}

// The schedule of one matrix on its slot (increment form of the updates, as
// in the single-matrix path):
//   radix-9 (Thm 3.1 in the telescoping update), binary splitting, naive Horner.
// Forced inline: each tile's instance is called from several kernels, and a
// call (measured) doubles the 128 x 128 kernel's private memory and its time.
template <class P>
__device__ __forceinline__ void one_matrix(const BatchArgs& a, int m, int n, float* slot, float* smem) {
  const int np = n <= 64 ? 64 : (n + 127) / 128 * 128;
  const size_t mat = (size_t)np * np;
  float* buf[kSlotMats];
#pragma unroll
  for (int i = 0; i < kSlotMats; ++i) buf[i] = slot + i * mat;
  float *B = buf[0], *B2 = buf[1], *S = buf[2], *S2 = buf[3], *U = buf[4], *X1 = buf[5],
        *Pm = buf[6], *Q = buf[7], *T = buf[8];
  // B <- A zero-padded to np, S <- I: four consecutive elements of a padded
  // row per thread step; np is 64, 128 or 256, so row and column are shifts
  // (a 64-bit division per element took 60 us of an n = 256 matrix's 1 ms)
  const int lg = np == 64 ? 6 : np == 128 ? 7 : 8;
  const float* Am = a.A + a.off[m];
  for (int i = threadIdx.x; i < (np * np) >> 2; i += kThreads) {
    const int r = i >> (lg - 2), c = (i & ((np >> 2) - 1)) << 2;
    float4 b = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < n) {
      const float* src = Am + (size_t)r * n + c;
      if (c < n) b.x = src[0];
      if (c + 1 < n) b.y = src[1];
      if (c + 2 < n) b.z = src[2];
      if (c + 3 < n) b.w = src[3];
    }
    *reinterpret_cast<float4*>(B + ((size_t)r << lg) + c) = b;
    *reinterpret_cast<float4*>(S + ((size_t)r << lg) + c) =
        make_float4(r == c ? 1.f : 0.f, r == c + 1 ? 1.f : 0.f, r == c + 2 ? 1.f : 0.f,
                    r == c + 3 ? 1.f : 0.f);
  }
  __syncthreads();
  for (int lv = 0; lv < a.levels; ++lv) {
    if (a.method == NS_NAIVE) {
      GemmParams e = ep0(np, a.nonfinite);                               // S <- I + A S
      ep_out(e, S2, 1.0, 0, 0, 0, 1.0);
      wg_product<P>(B, S, np, e, smem);
      __syncthreads();
      float* t = S; S = S2; S2 = t;
      continue;
    }
    if (a.method == NS_BINARY) {
      GemmParams e1 = ep0(np, a.nonfinite);                              // S <- S + S P
      ep_z(e1, S);
      ep_out(e1, S2, 1.0, 1.0);
      wg_product<P>(S, B, np, e1, smem);
      GemmParams e2 = ep0(np, a.nonfinite);                              // P <- P P
      ep_out(e2, B2, 1.0);
      e2.sumsq = a.sumsq + lv;
      wg_product<P>(B, B, np, e2, smem);
      __syncthreads();
      float* t = S; S = S2; S2 = t;
      t = B; B = B2; B2 = t;
      continue;
    }
    {   // radix-9: U = B^2, and the next product's operand B + 2U
      GemmParams e = ep0(np, a.nonfinite);
      ep_z(e, B);
      ep_out(e, U, 1.0);
      ep_out(e, X1, 2.0, 1.0);
      wg_product<P>(B, B, np, e, smem);
    }
    __syncthreads();
    {   // V = U (B + 2U); P, Q and T - W formed from V, B and U
      GemmParams e = ep0(np, a.nonfinite);
      ep_z(e, B);
      ep_z(e, U);
      ep_out(e, Pm, 1.0, 3.0 / 20.0, 2.0);
      ep_out(e, Q, 0.25, 11.0 / 40.0, -1.0 / 8.0);
      ep_out(e, T, 15.0 / 32.0, 1.0, 767.0 / 800.0);
      wg_product<P>(U, X1, np, e, smem);
    }
    __syncthreads();
    {   // W = P Q; T <- T9 - I
      GemmParams e = ep0(np, a.nonfinite);
      ep_z(e, T);
      ep_out(e, T, 1.0, 1.0);
      wg_product<P>(Pm, Q, np, e, smem);
    }
    __syncthreads();
    {   // S <- S + S (T - I)
      GemmParams e = ep0(np, a.nonfinite);
      ep_z(e, S);
      ep_out(e, S2, 1.0, 1.0);
      wg_product<P>(S, T, np, e, smem);
    }
    {   // B <- B - (T - I) + (T - I) B
      GemmParams e = ep0(np, a.nonfinite);
      ep_z(e, B);
      ep_z(e, T);
      ep_out(e, B2, 1.0, 1.0, -1.0);
      e.sumsq = a.sumsq + lv;
      wg_product<P>(T, B, np, e, smem);
    }
    __syncthreads();
    float* t = S; S = S2; S2 = t;
    t = B; B = B2; B2 = t;
  }
  // out <- the top-left n x n block of S, four elements of a row per step
  const int q = (n + 3) >> 2;
  float* Om = a.out + a.off[m];
  for (int i = threadIdx.x; i < n * q; i += kThreads) {
    const int r = i / q, c = (i - r * q) << 2;
    const float4 v = *reinterpret_cast<const float4*>(S + ((size_t)r << lg) + c);
    float* dst = Om + (size_t)r * n + c;
    dst[0] = v.x;
    if (c + 1 < n) dst[1] = v.y;
    if (c + 2 < n) dst[2] = v.z;
    if (c + 3 < n) dst[3] = v.w;
  }
  __syncthreads();
}

using Small = PolF32<2, 2, 2, 2>;     // 64 x 64 tiles for n <= 64
// 128 x 256 tiles with the direct-to-LDS k-loop for n in (128, 256]: the slot
// is padded to 256 there, so a tile row is one whole 1 KB slot row
struct Wide : PolF32<2, 2, 4, 8> {
  // three LDS stages: two k-chunks in flight behind the one the matrix cores
  // work on (74 KB of LDS, still two workgroups per CU)
  static constexpr int DMA_STAGES = 3;
};
static_assert(Wide::BN == kMaxBatchN && DmaShape<Wide>::OK, "wide tile spans a padded slot row");

template <class A, class B>
constexpr int max_smem() {
  return tile_smem_elems<A>() > tile_smem_elems<B>() ? tile_smem_elems<A>() : tile_smem_elems<B>();
}

// MINB: workgroups per CU the register allocation must allow (the compiler
// caps the registers accordingly; measured per tile, see kMinB0).  WIDE: the
// matrices with n > 128 use the Wide tile instead of Big.
template <class Big, int MINB, bool WIDE>
__global__ __launch_bounds__(kThreads, MINB) void batched_kernel(const BatchArgs a) {
  constexpr int E1 = max_smem<Big, Small>(), E2 = WIDE ? tile_smem_elems<Wide>() : 0;
  __shared__ __align__(16) float smem[E1 > E2 ? E1 : E2];
  __shared__ unsigned s_ticket;
  float* slot = a.work + (size_t)blockIdx.x * kSlotMats * kMaxBatchN * kMaxBatchN;
  for (;;) {
    if (threadIdx.x == 0) s_ticket = atomicAdd(a.counter, 1u);
    __syncthreads();
    const unsigned t = s_ticket;
    __syncthreads();
    if (t >= (unsigned)a.batch) break;
    const Item it = a.items[t];
    if (it.n <= 64) one_matrix<Small>(a, it.m, it.n, slot, smem);
    else if (WIDE && it.n > 128) one_matrix<Wide>(a, it.m, it.n, slot, smem);
    else one_matrix<Big>(a, it.m, it.n, slot, smem);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(a.done, 1u) == gridDim.x - 1) {   // last one out resets the queue
      atomicExch(a.counter, 0u);
      atomicExch(a.done, 0u);
    }
  }
}

__global__ void zero_doubles(double* p, int count, int* flag) {
  const int i = threadIdx.x;
  if (i < count) p[i] = 0.0;
  if (i == 0) *flag = 0;
}

// ---------------------------------------------------------------------------
// host side: configurations, graph cache, autotuner
// ---------------------------------------------------------------------------
struct Config {
  int big;          // index into kBigNames
  int per_cu;       // resident workgroups per CU to launch
};
const char* kBigNames[] = {"128x128", "64x128", "128x64", "128x128+128x256"};
constexpr int kNumBig = 4;

using Big0 = PolF32<2, 2, 4, 4>;
using Big1 = PolF32<2, 2, 2, 4>;
using Big2 = PolF32<2, 2, 4, 2>;
// Register caps (as resident workgroups per CU the allocation must allow),
// measured on the 2048-matrix workload launched two per CU: the 128 x 128 tile
// takes 2.50 ms compiled for three per CU (168 registers, 512 bytes of spill),
// 2.91 ms for four, 2.99 ms for two (no spill) and 3.81 ms uncapped (316
// registers: one per CU).  The 64 x 128 and 128 x 64 tiles are fastest uncapped
// (2.67 and 2.78 ms).
constexpr int kMinB0 = 3, kMinB1 = 1, kMinB2 = 1;
// with the Wide tile (128 accumulator registers per lane) the kernel is
// compiled for two workgroups per CU, which its 66.5 KB of LDS also sets
constexpr int kMinBW = 2;

void launch_batched(const Config& c, int grid, const BatchArgs& a, hipStream_t s) {
  switch (c.big) {
    case 0: hipLaunchKernelGGL((batched_kernel<Big0, kMinB0, false>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL((batched_kernel<Big1, kMinB1, false>), dim3(grid), dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((batched_kernel<Big2, kMinB2, false>), dim3(grid), dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((batched_kernel<Big0, kMinBW, true>), dim3(grid), dim3(kThreads), 0, s, a); break;
  }
}

int max_resident(const Config& c, int* out) {
  int per = 0;
  hipError_t e;
  switch (c.big) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_kernel<Big0, kMinB0, false>, kThreads, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_kernel<Big1, kMinB1, false>, kThreads, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_kernel<Big2, kMinB2, false>, kThreads, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_kernel<Big0, kMinBW, true>, kThreads, 0); break;
  }
  if (e != hipSuccess) return batch_fail(NS_ERR_HIP, "occupancy query failed");
  *out = per;
  return NS_OK;
}

struct GraphEntry {
  std::string key;
  std::vector<int32_t> n_host;    // the per-matrix n the items were built from
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  Item* items = nullptr;          // device, longest first
  Config cfg{};
  int grid = 0;
};

// Graphs cached per handle; beyond this many the oldest is dropped, so that
// calls on ever new buffers do not accumulate graphs and item arrays.
constexpr size_t kMaxGraphs = 16;

// Release one cached graph.  Its kernel arguments hold the workspace address
// and its item array, so the caller has synchronised the device first.
void drop_graph(GraphEntry& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  if (g.items) (void)hipFree(g.items);
  g = GraphEntry{};
}

struct State {
  int cus = 0;
  float* work = nullptr;
  size_t work_slots = 0;
  unsigned* counters = nullptr;   // [counter, done]
  double* sumsq = nullptr;        // NS_MAX_LEVELS
  int* nonfinite = nullptr;
  hipStream_t capture = nullptr;
  hipEvent_t done_ev = nullptr;      // after the last batched launch (cross-stream order)
  bool done_recorded = false;
  std::vector<GraphEntry> graphs;
  std::map<std::string, Config> tuned;    // n-histogram key -> config
  bool tune_loaded = false;
};

#define B_HIP(call)                                                                  \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return batch_fail(NS_ERR_HIP, #call " failed");            \
  } while (0)

int state_of(ns_handle* h, State** out) {
  State* st = static_cast<State*>(handle_batched_state(h));
  if (!st) {
    st = new State();
    B_HIP(hipDeviceGetAttribute(&st->cus, hipDeviceAttributeMultiprocessorCount, handle_device(h)));
    B_HIP(hipMalloc(&st->counters, 2 * sizeof(unsigned)));
    B_HIP(hipMemset(st->counters, 0, 2 * sizeof(unsigned)));
    B_HIP(hipMalloc(&st->sumsq, NS_MAX_LEVELS * sizeof(double)));
    B_HIP(hipMalloc(&st->nonfinite, sizeof(int)));
    B_HIP(hipStreamCreateWithFlags(&st->capture, hipStreamNonBlocking));
    B_HIP(hipEventCreateWithFlags(&st->done_ev, hipEventDisableTiming));
    set_handle_batched_state(h, st);
  }
  *out = st;
  return NS_OK;
}

int ensure_slots(State* st, size_t slots) {
  if (st->work_slots >= slots) return NS_OK;
  B_HIP(hipDeviceSynchronize());
  // every cached graph has the old workspace address in its kernel
  // arguments: drop them all, and the next call on each key captures again
  for (auto& g : st->graphs) drop_graph(g);
  st->graphs.clear();
  if (st->work) B_HIP(hipFree(st->work));
  st->work = nullptr;
  st->work_slots = 0;
  if (hipMalloc(&st->work, slots * kSlotMats * kMaxBatchN * kMaxBatchN * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return batch_fail(NS_ERR_NOMEM, "batched workspace allocation failed");
  }
  st->work_slots = slots;
  return NS_OK;
}

// key of the n histogram (tile choices depend only on it)
std::string hist_key(const int32_t* n_host, int batch) {
  int counts[kMaxBatchN + 1] = {0};
  for (int i = 0; i < batch; ++i) counts[n_host[i]]++;
  std::ostringstream os;
  for (int v = 1; v <= kMaxBatchN; ++v)
    if (counts[v]) os << v << ':' << counts[v] << ',';
  return os.str();
}

const char* tune_path() { return std::getenv("NS_TUNE_CACHE"); }

void load_tuned(State* st) {
  if (st->tune_loaded) return;
  st->tune_loaded = true;
  const char* path = tune_path();
  if (!path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    // one entry per line: {"hist": "...", "big": i, "per_cu": j}
    const auto h0 = line.find("\"hist\": \"");
    const auto b0 = line.find("\"big\": ");
    const auto p0 = line.find("\"per_cu\": ");
    if (h0 == std::string::npos || b0 == std::string::npos || p0 == std::string::npos) continue;
    const auto h1 = line.find('"', h0 + 9);
    Config c{std::atoi(line.c_str() + b0 + 7), std::atoi(line.c_str() + p0 + 10)};
    if (c.big < 0 || c.big >= kNumBig || c.per_cu < 1 || c.per_cu > 8) continue;
    st->tuned[line.substr(h0 + 9, h1 - h0 - 9)] = c;
  }
}

void save_tuned(State* st) {
  const char* path = tune_path();
  if (!path) return;
  std::ofstream f(path);
  for (const auto& kv : st->tuned)
    f << "{\"hist\": \"" << kv.first << "\", \"big\": " << kv.second.big
      << ", \"per_cu\": " << kv.second.per_cu << ", \"tile\": \"" << kBigNames[kv.second.big]
      << "\"}\n";
}

int check_batch_args(const void* A, const int64_t* off, const int32_t* nh, int32_t batch, int64_t k,
                     int method, int dtype, void* out) {
  if (batch < 0) return batch_fail(NS_ERR_ARG, "batch < 0");
  if (batch > 0 && (!A || !off || !nh || !out)) return batch_fail(NS_ERR_ARG, "null pointer");
  if (k < 1) return batch_fail(NS_ERR_ARG, "k must be >= 1");
  if (dtype != NS_F32) return batch_fail(NS_ERR_UNSUPPORTED, "the batched form computes in FP32");
  if (method != NS_RADIX9 && method != NS_BINARY && method != NS_NAIVE)
    return batch_fail(NS_ERR_UNSUPPORTED, "batched methods: radix-9, binary, naive");
  for (int i = 0; i < batch; ++i)
    if (nh[i] < 1 || nh[i] > kMaxBatchN)
      return batch_fail(NS_ERR_UNSUPPORTED, "batched n must be in [1, 256]");
  return NS_OK;
}

int levels_for(int64_t k, int method, int32_t* levels) {
  int64_t ke;
  int32_t g;
  return ns_plan(k, method, &ke, levels, &g);
}

BatchArgs make_args(State* st, const void* A, const int64_t* off, const Item* items, int batch,
                    int levels, int method, void* out) {
  BatchArgs a{};
  a.A = static_cast<const float*>(A);
  a.out = static_cast<float*>(out);
  a.off = off;
  a.items = items;
  a.batch = batch;
  a.levels = levels;
  a.method = method;
  a.work = st->work;
  a.counter = st->counters;
  a.done = st->counters + 1;
  a.sumsq = st->sumsq;
  a.nonfinite = st->nonfinite;
  return a;
}

// The queue: (matrix, n) pairs in longest-first order, n from the validated
// host array.
int upload_items(const int32_t* n_host, int batch, Item** items_dev) {
  std::vector<Item> items(batch);
  for (int i = 0; i < batch; ++i) items[i] = Item{i, n_host[i]};
  std::stable_sort(items.begin(), items.end(),
                   [](const Item& a, const Item& b) { return a.n > b.n; });   // longest first
  B_HIP(hipMalloc(items_dev, std::max(1, batch) * sizeof(Item)));
  if (batch) B_HIP(hipMemcpy(*items_dev, items.data(), batch * sizeof(Item), hipMemcpyHostToDevice));
  return NS_OK;
}

}  // namespace

int batched_eval(ns_handle* h, const void* A_packed, const int64_t* off_dev, const int32_t* n_dev,
                 const int32_t* n_host, int32_t batch, int64_t k, int method, int dtype,
                 void* out_packed, hipStream_t stream, ns_report* rep) {
  (void)n_dev;   // not read: the queue carries the library's copy of n_host
  int rc = check_batch_args(A_packed, off_dev, n_host, batch, k, method, dtype, out_packed);
  if (rc) return rc;
  int32_t levels;
  if ((rc = levels_for(k, method, &levels))) return rc;
  const DeviceGuard dg(handle_device(h));
  B_HIP(dg.err);
  State* st;
  if ((rc = state_of(h, &st))) return rc;
  load_tuned(st);
  if (batch == 0) return NS_OK;

  const std::string hk = hist_key(n_host, batch);
  std::ostringstream ks;
  ks << A_packed << '|' << out_packed << '|' << off_dev << '|' << batch << '|' << levels << '|'
     << method << '|' << hk;
  const std::string key = ks.str();
  Config cfg{0, 2};
  auto tt = st->tuned.find(hk);
  if (tt != st->tuned.end()) cfg = tt->second;

  GraphEntry* ge = nullptr;
  // a graph replays its item array, so the per-matrix n must match entry by
  // entry, not only in histogram
  for (auto& g : st->graphs)
    if (g.key == key && g.cfg.big == cfg.big && g.cfg.per_cu == cfg.per_cu &&
        std::equal(g.n_host.begin(), g.n_host.end(), n_host))
      ge = &g;
  if (!ge) {
    if (st->graphs.size() >= kMaxGraphs) {
      B_HIP(hipDeviceSynchronize());             // the oldest graph may still be in flight
      drop_graph(st->graphs.front());
      st->graphs.erase(st->graphs.begin());
    }
    GraphEntry g;
    g.key = key;
    g.n_host.assign(n_host, n_host + batch);
    g.cfg = cfg;
    int per = 0;
    if ((rc = max_resident(cfg, &per))) return rc;
    const int resident = std::max(1, std::min(per, cfg.per_cu)) * st->cus;
    g.grid = std::max(1, std::min(batch, resident));
    if ((rc = ensure_slots(st, g.grid))) return rc;
    if ((rc = upload_items(n_host, batch, &g.items))) return rc;
    const BatchArgs a = make_args(st, A_packed, off_dev, g.items, batch, levels, method, out_packed);
    // capture: zero the report accumulators (a kernel node), then the
    // persistent kernel; the queue counters are reset by the kernel itself
    B_HIP(hipStreamBeginCapture(st->capture, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(zero_doubles, dim3(1), dim3(64), 0, st->capture, st->sumsq, NS_MAX_LEVELS, st->nonfinite);
    launch_batched(cfg, g.grid, a, st->capture);
    B_HIP(hipStreamEndCapture(st->capture, &g.graph));
    B_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    st->graphs.push_back(g);
    ge = &st->graphs.back();
  }
  if (st->done_recorded) B_HIP(hipStreamWaitEvent(stream, st->done_ev, 0));
  B_HIP(hipGraphLaunch(ge->exec, stream));
  B_HIP(hipEventRecord(st->done_ev, stream));
  st->done_recorded = true;
  if (rep) {
    double ss[NS_MAX_LEVELS];
    int nf = 0;
    B_HIP(hipMemcpyAsync(ss, st->sumsq, sizeof(ss), hipMemcpyDeviceToHost, stream));
    B_HIP(hipMemcpyAsync(&nf, st->nonfinite, sizeof(int), hipMemcpyDeviceToHost, stream));
    B_HIP(hipStreamSynchronize(stream));
    std::memset(rep, 0, sizeof(*rep));
    int64_t ke;
    int32_t lv, g;
    ns_plan(k, method, &ke, &lv, &g);
    rep->k_eff = ke;
    rep->levels = lv;
    rep->gemms_formula = g;
    rep->gemms_performed = g;
    rep->nonfinite = nf ? 1 : 0;
    rep->method = method;
    rep->dtype = dtype;
    rep->product_launches = 1;           // every product of every matrix in one launch
    if (method != NS_NAIVE)
      for (int i = 0; i < lv && i < NS_MAX_LEVELS; ++i) rep->level_norm[i] = std::sqrt(ss[i]);
  }
  return NS_OK;
}

int batched_autotune(ns_handle* h, const void* A_packed, const int64_t* off_dev,
                     const int32_t* n_dev, const int32_t* n_host, int32_t batch, int64_t k,
                     void* out_packed, hipStream_t stream, int32_t* n_timed) {
  (void)n_dev;   // not read, as in batched_eval
  int rc = check_batch_args(A_packed, off_dev, n_host, batch, k, NS_RADIX9, NS_F32, out_packed);
  if (rc) return rc;
  int32_t levels;
  if ((rc = levels_for(k, NS_RADIX9, &levels))) return rc;
  const DeviceGuard dg(handle_device(h));
  B_HIP(dg.err);
  State* st;
  if ((rc = state_of(h, &st))) return rc;
  load_tuned(st);
  if (batch == 0) return NS_OK;
  Item* items = nullptr;
  if ((rc = upload_items(n_host, batch, &items))) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Config best_cfg{0, 2};
  int timed = 0;
  // the timing loop; every exit from it goes through the release below
  auto tune = [&]() -> int {
    if (st->done_recorded) B_HIP(hipStreamWaitEvent(stream, st->done_ev, 0));
    B_HIP(hipEventCreate(&e0));
    B_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    for (int big = 0; big < kNumBig; ++big) {
      for (int per_cu = 1; per_cu <= 4; ++per_cu) {
        Config c{big, per_cu};
        int per = 0;
        int r0;
        if ((r0 = max_resident(c, &per))) return r0;
        if (per_cu > per) continue;                    // not resident: skip
        const int grid = std::max(1, std::min(batch, per_cu * st->cus));
        if ((r0 = ensure_slots(st, grid))) return r0;
        const BatchArgs a = make_args(st, A_packed, off_dev, items, batch, levels, NS_RADIX9, out_packed);
        launch_batched(c, grid, a, stream);              // warm-up
        B_HIP(hipEventRecord(e0, stream));
        for (int r = 0; r < 3; ++r) launch_batched(c, grid, a, stream);
        B_HIP(hipEventRecord(e1, stream));
        B_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        B_HIP(hipEventElapsedTime(&ms, e0, e1));
        ++timed;
        if (ms < best) {
          best = ms;
          best_cfg = c;
        }
      }
    }
    B_HIP(hipEventRecord(st->done_ev, stream));
    st->done_recorded = true;
    return NS_OK;
  };
  rc = tune();
  // the launches may still read the item array: wait before releasing it
  const hipError_t se = hipStreamSynchronize(stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(items);
  if (rc) return rc;
  if (se != hipSuccess) return batch_fail(NS_ERR_HIP, "hipStreamSynchronize failed");
  st->tuned[hist_key(n_host, batch)] = best_cfg;
  save_tuned(st);
  if (n_timed) *n_timed = timed;
  return NS_OK;
}

void batched_release(ns_handle* h) {
  State* st = static_cast<State*>(handle_batched_state(h));
  if (!st) return;
  for (auto& g : st->graphs) drop_graph(g);
  if (st->work) (void)hipFree(st->work);
  if (st->counters) (void)hipFree(st->counters);
  if (st->sumsq) (void)hipFree(st->sumsq);
  if (st->nonfinite) (void)hipFree(st->nonfinite);
  if (st->capture) (void)hipStreamDestroy(st->capture);
  if (st->done_ev) (void)hipEventDestroy(st->done_ev);
  delete st;
  set_handle_batched_state(h, nullptr);
}

}  // namespace ns
