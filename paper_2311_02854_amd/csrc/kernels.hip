// HIP kernels for gfx950 (CDNA4) and the HIP runtime wrappers of device.h.
//
// The hot kernel is a grouped, batched GEMM driven by a task list: every
// workgroup owns one 64x64 output tile of one task (output-stationary), loops
// over the task's contributions (and, inside each, over a reduction index),
// stages 64x32 / 32x64 operand tiles in LDS and accumulates in registers with
// MFMA: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32) or
// split-BF16 (three v_mfma_f32_16x16x32_bf16 per step).  Accumulation order
// is fixed, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <atomic>
#include <map>
#include <mutex>

#include <chrono>
#include <cstdio>
#include <string>
#include <type_traits>

#include "../../include/dmrg.h"
#include "common.h"
#include "device.h"

namespace dmrg {

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      throw Error(DMRG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));         \
  } while (0)

static inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int MAX_DEVICES = 64;

// ---------------------------------------------------------------- runtime
void dev_set(int device) { HIPCHK(hipSetDevice(device)); }

// Static scratch of the allocation-free entry points (each device holds its
// own copy until the process ends).  In host code `scratch` is only a
// stand-in for the device symbol: its device address comes from
// hipGetSymbolAddress, per device, and is the only form passed to kernels or
// copies.
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::atomic<void*> g_scratch[MAX_DEVICES];

size_t scratch_bytes() { return SCRATCH_BYTES; }

void scratch_init(int device) {
  DMRG_CHECK(device >= 0 && device < MAX_DEVICES, DMRG_EINVAL, "device index beyond the scratch table");
  if (g_scratch[device].load(std::memory_order_acquire)) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  DMRG_CHECK(p != nullptr, DMRG_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
  g_scratch[device].store(p, std::memory_order_release);
}

void* scratch_get(int device) {
  DMRG_CHECK(device >= 0 && device < MAX_DEVICES, DMRG_EINVAL, "device index beyond the scratch table");
  void* p = g_scratch[device].load(std::memory_order_acquire);
  DMRG_CHECK(p != nullptr, DMRG_EINTERNAL, "static scratch not set up on this device (no context created on it)");
  return p;
}

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(DMRG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  // the fill runs on the null stream, which work on non-blocking streams does
  // not wait for: wait for it here
  HIPCHK(hipMemset(p, 0, bytes));
  HIPCHK(hipStreamSynchronize(nullptr));
  return p;
}

void* dev_alloc_nozero(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(DMRG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

void* host_alloc_pinned(size_t bytes) {
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, bytes ? bytes : 256, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(DMRG_ENOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void host_free_pinned(void* p) {
  if (p) (void)hipHostFree(p);
}

void dev_h2d_async(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, S(stream)));
}

void dev_h2d(void* dst, const void* src, size_t bytes) {
  if (!bytes) return;
  // a copy from pageable memory may return before its DMA has landed, and
  // kernels on non-blocking streams do not wait for the null stream
  HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  HIPCHK(hipStreamSynchronize(nullptr));
}

void dev_h2d_on(void* dst, const void* src, size_t bytes, void* stream) {
  if (!bytes) return;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, S(stream)));
  HIPCHK(hipStreamSynchronize(S(stream)));
}

void dev_d2h(void* dst, const void* src, size_t bytes, void* stream) {
  if (!bytes) return;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, S(stream)));
  HIPCHK(hipStreamSynchronize(S(stream)));
}

void dev_sync(void* stream) { HIPCHK(hipStreamSynchronize(S(stream))); }

void dev_check(const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(DMRG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

void* ev_create() {
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return (void*)e;
}
void ev_destroy(void* ev) {
  if (ev) (void)hipEventDestroy((hipEvent_t)ev);
}
void ev_record(void* ev, void* stream) { HIPCHK(hipEventRecord((hipEvent_t)ev, S(stream))); }
void stream_wait(void* stream, void* ev) { HIPCHK(hipStreamWaitEvent(S(stream), (hipEvent_t)ev, 0)); }
float ev_elapsed_ms(void* a, void* b) {
  float ms = 0;
  HIPCHK(hipEventSynchronize((hipEvent_t)b));
  HIPCHK(hipEventElapsedTime(&ms, (hipEvent_t)a, (hipEvent_t)b));
  return ms;
}

void* stream_create() {
  hipStream_t s;
  HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  return (void*)s;
}
void stream_destroy(void* s) {
  if (s) (void)hipStreamDestroy(S(s));
}
void graph_begin(void* s) { HIPCHK(hipStreamBeginCapture(S(s), hipStreamCaptureModeThreadLocal)); }
void* graph_end(void* s) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamEndCapture(S(s), &g));
  hipGraphExec_t e = nullptr;
  hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (r != hipSuccess) throw Error(DMRG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(r));
  return (void*)e;
}
void graph_launch(void* exec, void* stream) { HIPCHK(hipGraphLaunch((hipGraphExec_t)exec, S(stream))); }
void graph_destroy(void* exec) {
  if (exec) (void)hipGraphExecDestroy((hipGraphExec_t)exec);
}

double wall_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- GEMM
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int BK = 32, NT = 256, NT_BIG = 1024;

// Operand precision policies.  FP64 and FP32 stage op(A) and op(B) tiles in
// LDS k-major ([k][row], rows contiguous) and feed 16x16x4 MFMAs one element
// per lane.  BF16x3 reads FP32 operands, splits every value while staging into
// hi = bf16(x) and lo = bf16(x - hi) (round to nearest even, two values per
// conversion), stores them row-major ([row][k], k contiguous) and accumulates
// hi*hi + hi*lo + lo*hi in FP32 with 16x16x32 MFMAs.
struct PolF64 {
  using T = double;
  using Acc = d4_t;
  static constexpr bool split = false;
  static constexpr int depth = 1;  // k tiles in flight in registers
  static constexpr int PAD = 2;
  static constexpr int RL = 1, RV = 4;  // result row of element v in lane l: RL*(l/16) + RV*v
};
struct PolF32 {
  using T = float;
  using Acc = f4_t;
  static constexpr bool split = false;
  static constexpr int depth = 1;
  static constexpr int PAD = 4;
  static constexpr int RL = 4, RV = 1;
};
struct PolBF3 {
  using T = float;
  using Acc = f4_t;
  static constexpr bool split = true;
  static constexpr int depth = 2;
  static constexpr int PAD = 8;
  static constexpr int RL = 4, RV = 1;
};

// LDS staging of one k tile of op(A) (BM_ rows) and op(B) (BN_ columns).
template <class P, int BM_, int BN_, bool S = P::split>
struct alignas(16) Smem {
  typename P::T A[BK][BM_ + P::PAD];
  typename P::T B[BK][BN_ + P::PAD];
};
template <class P, int BM_, int BN_>
struct alignas(16) Smem<P, BM_, BN_, true> {
  uint16_t Ah[BM_][BK + P::PAD], Al[BM_][BK + P::PAD];
  uint16_t Bh[BN_][BK + P::PAD], Bl[BN_][BK + P::PAD];
};

__device__ __forceinline__ d4_t mfma4(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma4(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma32(bf8_t a, bf8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Every operand and output of the GEMM kernels lives in global memory: loads
// and stores go through address-space-1 pointers so that they compile to
// global (not flat) instructions, which do not count against the LDS wait
// counter the MFMA loop waits on.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(GLOBAL T*)p = v;
}

typedef float f2_t __attribute__((ext_vector_type(2)));
typedef __bf16 b2_t __attribute__((ext_vector_type(2)));

// Split x = hi + lo of two floats into packed bf16 pairs: hi = bf16(x),
// lo = bf16(x - hi), both rounded to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ void split_bf16x2(f2_t x, uint32_t& hi, uint32_t& lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, b2_t));
  const f2_t hf = {__uint_as_float(hi << 16), __uint_as_float(hi & 0xffff0000u)};
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(x - hf, b2_t));
}

// Task of a job: the bucket table narrows the search to the tasks that
// intersect the job's bucket of 2^shift consecutive jobs.
__device__ __forceinline__ int find_task(const GTask* __restrict__ tasks, const int* __restrict__ bucket,
                                         int shift, int64_t job) {
  // bucket points at this XCD's table; task indices are global
  const int64_t b = job >> shift;
  int lo = bucket[b], hi = bucket[b + 1];
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].job_begin <= job)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per-thread view of one ROWS x BK operand tile staged by NTH threads: element
// (r, k) of op(X) sits at X + r*sr + k*sk.  When k is contiguous (kc: sk == 1)
// threads walk k fastest (32 per row, NTH/32 rows per pass), otherwise r
// fastest (ROWS per row, NTH/ROWS k per pass); either way every thread owns
// E = ROWS*BK/NTH elements.
//
// Loads go through a buffer descriptor based at the k tile's first element
// whose range ends at the operand's last valid element among the tile's rows:
// elements outside it read as zero and nothing is ever read past that
// element.  Along the outer dimension of the storage (rows when kc, k
// otherwise) the range check therefore zeroes every element past the operand.
// Inside it, a kc tile's k tail (k >= K) holds neighbouring values of the
// same matrix: the LDS store zeroes it (one compare per thread: all of a
// thread's elements share one k); a row-contiguous tile's rows past the
// operand hold neighbouring values too, which only reach output rows or
// columns that are never stored.
template <typename T>
struct Opnd {
  const char* origin;  // element (0, 0) of the tile (first row, k = 0)
  int64_t range;       // bytes from origin to the end of the last element a load may read
  int64_t step_k;      // bytes of one BK tile
  int32_t lane_off;    // byte offset of the thread's first element within a k tile
  int32_t step_it;     // bytes between a thread's consecutive elements
  int32_t s2;          // split staging: bytes from a pair's first to its second element
  int r_inc, k_inc;    // increments per element (one of them is 0)
  T scale;
};

// Byte range of a tile: up to the operand's last valid element among the
// tile's rows (at most ROWS of them) -- row min(rows, ROWS) - 1, column K - 1.
template <int ROWS, typename T>
__device__ __forceinline__ int64_t tile_range(int64_t sr, int64_t sk, int rv, int K) {
  rv = rv < ROWS ? rv : ROWS;
  if (rv <= 0 || K <= 0) return 0;
  const int64_t last = sk == 1 ? (int64_t)(rv - 1) * sr + (K - 1) : (int64_t)(K - 1) * sk + (rv - 1);
  return (last + 1) * (int64_t)sizeof(T);
}

// Descriptor of k tile k0 / BK: based at its first element, so that the
// 32-bit offsets stay inside one tile whatever K and the strides are.  A range
// beyond 2^31 - 1 bytes is capped: the tile never reads that far (leading
// dimensions are below 2^20), and the zeroed elements past the operand all lie
// in the last k tile, whose remaining range is small.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const Opnd<T>& o, int k0) {
  const int64_t kb = (int64_t)(k0 / BK) * o.step_k;
  int64_t rem = o.range - kb;
  rem = rem < 0 ? 0 : (rem > 0x7fffffff ? 0x7fffffff : rem);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(o.origin + kb), (short)0, (int)rem, 0x00020000);
}

template <int ROWS, int NTH, typename T>
__device__ __forceinline__ void opnd_setup(Opnd<T>& o, const T* X, int64_t sr, int64_t sk, int r0, int rows,
                                           int K, T scale) {
  const int tid = threadIdx.x;
  int r_first, k_first;
  if (sk == 1) {
    r_first = tid >> 5;
    k_first = tid & 31;
    o.r_inc = NTH / 32;
    o.k_inc = 0;
    o.step_it = (int32_t)((NTH / 32) * sr * (int64_t)sizeof(T));
  } else {
    r_first = tid % ROWS;
    k_first = tid / ROWS;
    o.r_inc = 0;
    o.k_inc = NTH / ROWS;
    o.step_it = (int32_t)((NTH / ROWS) * sk * (int64_t)sizeof(T));
  }
  o.origin = reinterpret_cast<const char*>(X + (int64_t)r0 * sr);
  o.range = tile_range<ROWS, T>(sr, sk, rows - r0, K);
  o.lane_off = (int32_t)(((int64_t)r_first * sr + (int64_t)k_first * sk) * (int64_t)sizeof(T));
  o.step_k = (int64_t)BK * sk * (int64_t)sizeof(T);
  o.scale = scale;
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <int E, typename T>
__device__ __forceinline__ void opnd_load(const Opnd<T>& o, int k0, T (&v)[E]) {
  const __amdgpu_buffer_rsrc_t r = tile_rsrc(o, k0);
#pragma unroll
  for (int it = 0; it < E; ++it) v[it] = buf_load(r, o.lane_off + it * o.step_it, T(0));
}

// Element it of a thread's share of a ROWS x BK tile sits at (row, k) =
// (r_first + it*r_inc, k_first + it*k_inc), with the pattern opnd_setup
// picks for k-contiguous (kc) or row-contiguous operands.
template <int ROWS, int NTH>
__device__ __forceinline__ void tile_pattern(bool kc, int& r_first, int& k_first, int& r_inc, int& k_inc) {
  const int tid = threadIdx.x;
  r_first = kc ? tid >> 5 : tid % ROWS;
  k_first = kc ? tid & 31 : tid / ROWS;
  r_inc = kc ? NTH / 32 : 0;
  k_inc = kc ? 0 : NTH / ROWS;
}

// kvalid: valid k of this tile (the k tail of a kc tile is zeroed here)
template <int ROWS, int NTH, int E, typename T, int LD>
__device__ __forceinline__ void opnd_store(bool kc, int kvalid, T scale, const T (&v)[E], T (*L)[LD]) {
  int r_first, k_first, r_inc, k_inc;
  tile_pattern<ROWS, NTH>(kc, r_first, k_first, r_inc, k_inc);
  const bool keep = !kc || k_first < kvalid;
#pragma unroll
  for (int it = 0; it < E; ++it) L[k_first + it * k_inc][r_first + it * r_inc] = keep ? v[it] * scale : T(0);
}

// Split-BF16 staging: every thread owns E/2 pairs of k-consecutive elements
// (k contiguous in memory: 16 threads per row, NTH/16 rows per pass; else r
// fastest, 2*NTH/ROWS k per pass), so that each pair converts with one
// instruction and lands in LDS ([row][k]) as one 32-bit store per half.
template <int ROWS, int NTH>
__device__ __forceinline__ void opnd_setup_split(Opnd<float>& o, const float* X, int64_t sr, int64_t sk, int r0,
                                                 int rows, int K, float scale) {
  const int tid = threadIdx.x;
  int r_first, k_first;
  if (sk == 1) {
    r_first = tid >> 4;
    k_first = 2 * (tid & 15);
    o.r_inc = NTH / 16;
    o.k_inc = 0;
    o.step_it = (int32_t)((NTH / 16) * sr * 4);
  } else {
    r_first = tid % ROWS;
    k_first = 2 * (tid / ROWS);
    o.r_inc = 0;
    o.k_inc = 2 * NTH / ROWS;
    o.step_it = (int32_t)((2 * NTH / ROWS) * sk * 4);
  }
  o.s2 = (int32_t)(sk * 4);
  o.origin = reinterpret_cast<const char*>(X + (int64_t)r0 * sr);
  o.range = tile_range<ROWS, float>(sr, sk, rows - r0, K);
  o.lane_off = (int32_t)(((int64_t)r_first * sr + (int64_t)k_first * sk) * 4);
  o.step_k = (int64_t)BK * sk * 4;
  o.scale = scale;
}

template <int E>
__device__ __forceinline__ void opnd_load_split(const Opnd<float>& o, int k0, float (&v)[E]) {
  const __amdgpu_buffer_rsrc_t r = tile_rsrc(o, k0);
#pragma unroll
  for (int it = 0; it < E / 2; ++it) {
    v[2 * it] = buf_load(r, o.lane_off + it * o.step_it, 0.0f);
    v[2 * it + 1] = buf_load(r, o.lane_off + it * o.step_it + o.s2, 0.0f);
  }
}

template <int ROWS, int NTH>
__device__ __forceinline__ void tile_pattern_split(bool kc, int& r_first, int& k_first, int& r_inc, int& k_inc) {
  const int tid = threadIdx.x;
  r_first = kc ? tid >> 4 : tid % ROWS;
  k_first = kc ? 2 * (tid & 15) : 2 * (tid / ROWS);
  r_inc = kc ? NTH / 16 : 0;
  k_inc = kc ? 0 : 2 * NTH / ROWS;
}

template <int ROWS, int NTH, int E, int LD>
__device__ __forceinline__ void opnd_store_split(bool kc, int kvalid, float scale, const float (&v)[E],
                                                 uint16_t (*H)[LD], uint16_t (*Lo)[LD]) {
  int r_first, k_first, r_inc, k_inc;
  tile_pattern_split<ROWS, NTH>(kc, r_first, k_first, r_inc, k_inc);
  const bool keep0 = !kc || k_first < kvalid, keep1 = !kc || k_first + 1 < kvalid;
#pragma unroll
  for (int it = 0; it < E / 2; ++it) {
    const int r = r_first + it * r_inc, k = k_first + it * k_inc;
    const f2_t x = {keep0 ? v[2 * it] * scale : 0.0f, keep1 ? v[2 * it + 1] * scale : 0.0f};
    uint32_t hi, lo;
    split_bf16x2(x, hi, lo);
    *reinterpret_cast<uint32_t*>(&H[r][k]) = hi;
    *reinterpret_cast<uint32_t*>(&Lo[r][k]) = lo;
  }
}

// One step of the flattened (contribution, reduction index, k tile) sequence.
struct Step {
  int ci, t, k0;
  int K;
};

// One job of a grouped GEMM task: the tile `local` (batch-major) of task Tk.
// The NTH / 64 waves form a GW x GW grid and each wave owns WM x WN sub-tiles
// of 16 x 16, so the workgroup tile is (16 WM GW) x (16 WN GW): 256 threads
// in 2 x 2 waves, or 1024 threads in 4 x 4 waves (128 x 128 tiles).  smem
// holds at least sizeof(Smem<P, BM, BN>) bytes.
template <class P, int WM, int WN, int NTH = NT>
__device__ __forceinline__ void gemm_job(const GTask& Tk, int64_t local, void* smem,
                                         const GContrib* __restrict__ contribs,
                                         typename P::T* const* __restrict__ table, const typename P::T* p0,
                                         double* p1) {
  using T = typename P::T;
  using Acc = typename P::Acc;
  constexpr int GW = NTH == 1024 ? 4 : 2;
  static_assert(NTH == 64 * GW * GW, "workgroup of 2 x 2 or 4 x 4 waves");
  constexpr int BM = 16 * WM * GW, BN = 16 * WN * GW, EA = BM * BK / NTH, EB = BN * BK / NTH;
  Smem<P, BM, BN>& sm = *reinterpret_cast<Smem<P, BM, BN>*>(smem);
  // the wave index is uniform across its lanes: keep it (and the sub-tile
  // predicates derived from it) scalar, so that inactive sub-tiles branch
  // around their MFMAs instead of selecting whole accumulators
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave / GW) * 16 * WM, wn = (wave % GW) * 16 * WN;
  const int lr = lane & 15, lk = lane >> 4;
  auto opp = [&](int id) -> const T* { return id == 0 ? p0 : (id == 1 ? (const T*)p1 : table[id]); };
  {
    const int tiles = Tk.tiles_m * Tk.tiles_n;
    const int64_t batch = local / tiles;
    const int tile = (int)(local - batch * tiles);
    const int m0 = (tile / Tk.tiles_n) * BM, n0 = (tile % Tk.tiles_n) * BN;
    const int mrem = Tk.M - m0 - wm, nrem = Tk.N - n0 - wn;
    // sub-tile (i, j) of this wave holds valid rows and columns
    bool act[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) act[i][j] = mrem > 16 * i && nrem > 16 * j;
    const bool any = act[0][0];
    bool full = true;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) full = full && act[i][j];
    Acc acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    // identity contributions: acc += alpha op(B)  (M == K)
    for (int ci = Tk.contrib_begin; ci < Tk.contrib_end; ++ci) {
      const GContrib& Cb = contribs[ci];
      if (!(Cb.flags & GF_IDENT_A)) continue;
      const bool tb = Cb.flags & GF_TRANS_B;
      for (int t = 0; t < Cb.nred; ++t) {
        const T* B = opp(Cb.b_buf) + Cb.b_off + batch * Cb.b_bstride + (int64_t)t * Cb.b_rstride;
        T alpha = (T)Cb.alpha;
        if (Cb.s_buf >= 0) alpha *= gld(opp(Cb.s_buf) + Cb.s_off + batch * Cb.s_bstride + (int64_t)t * Cb.s_rstride);
#pragma unroll
        for (int mi = 0; mi < WM; ++mi)
#pragma unroll
          for (int ni = 0; ni < WN; ++ni) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              int r = m0 + wm + mi * 16 + lk * P::RL + v * P::RV, c = n0 + wn + ni * 16 + lr;
              if (r < Tk.M && c < Tk.N)
                acc[mi][ni][v] += alpha * gld(tb ? B + (int64_t)c * Cb.ldb + r : B + (int64_t)r * Cb.ldb + c);
            }
          }
      }
    }

    // MFMA contributions.  The flattened (contribution, member, k tile)
    // sequence streams through P::depth register sets: while step i is
    // multiplied out of LDS, the loads of steps i+1 .. i+depth are in flight.
    auto first_from = [&](int ci) {
      while (ci < Tk.contrib_end && (contribs[ci].flags & GF_IDENT_A)) ++ci;
      return ci;
    };
    auto setup = [&](const Step& s, Opnd<T>& oa, Opnd<T>& ob) {
      const GContrib& Cb = contribs[s.ci];
      const T* A = opp(Cb.a_buf) + Cb.a_off + batch * Cb.a_bstride + (int64_t)s.t * Cb.a_rstride;
      const T* B = opp(Cb.b_buf) + Cb.b_off + batch * Cb.b_bstride + (int64_t)s.t * Cb.b_rstride;
      T alpha = (T)Cb.alpha;
      if (Cb.s_buf >= 0) alpha *= gld(opp(Cb.s_buf) + Cb.s_off + batch * Cb.s_bstride + (int64_t)s.t * Cb.s_rstride);
      const bool ta = Cb.flags & GF_TRANS_A, tb = Cb.flags & GF_TRANS_B;
      // op(A)(m, k): stored M x K (lda) or K x M;  op(B)(k, n) seen as (n, k)
      if constexpr (P::split) {
        opnd_setup_split<BM, NTH>(oa, A, ta ? 1 : Cb.lda, ta ? Cb.lda : 1, m0, Tk.M, Cb.K, alpha);
        opnd_setup_split<BN, NTH>(ob, B, tb ? Cb.ldb : 1, tb ? 1 : Cb.ldb, n0, Tk.N, Cb.K, T(1));
      } else {
        opnd_setup<BM, NTH>(oa, A, ta ? 1 : Cb.lda, ta ? Cb.lda : 1, m0, Tk.M, Cb.K, alpha);
        opnd_setup<BN, NTH>(ob, B, tb ? Cb.ldb : 1, tb ? 1 : Cb.ldb, n0, Tk.N, Cb.K, T(1));
      }
    };
    // what staging a register set needs from the step it holds
    struct SetMeta {
      int kend;       // valid k in the tile
      bool akc, bkc;  // operand tile is k-contiguous in memory
      T scale;        // alpha of the contribution (applied to A)
    };
    Step lc{first_from(Tk.contrib_begin), 0, 0, 0};  // next step to load
    if (lc.ci < Tk.contrib_end) {
      Opnd<T> oa, ob;
      lc.K = contribs[lc.ci].K;
      setup(lc, oa, ob);
      bool lmore = true;
      T ra0[EA], rb0[EB], ra1[EA], rb1[EB];
      SetMeta m0, m1;
      // issue the loads of step lc into a register set, then advance lc
      auto load_step = [&](T (&ra)[EA], T (&rb)[EB], SetMeta& m) {
        m.kend = (lc.K - lc.k0 < BK) ? lc.K - lc.k0 : BK;
        m.akc = oa.r_inc != 0 || oa.k_inc == 0;
        m.bkc = ob.r_inc != 0 || ob.k_inc == 0;
        m.scale = oa.scale;
        if constexpr (P::split) {
          opnd_load_split(oa, lc.k0, ra);
          opnd_load_split(ob, lc.k0, rb);
        } else {
          opnd_load(oa, lc.k0, ra);
          opnd_load(ob, lc.k0, rb);
        }
        lc.k0 += BK;
        if (lc.k0 >= lc.K) {
          lc.k0 = 0;
          if (++lc.t >= contribs[lc.ci].nred) {
            lc.t = 0;
            lc.ci = first_from(lc.ci + 1);
            lmore = lc.ci < Tk.contrib_end;
          }
          if (lmore) {
            lc.K = contribs[lc.ci].K;
            setup(lc, oa, ob);
          }
        }
      };
      auto stage = [&](const T (&ra)[EA], const T (&rb)[EB], const SetMeta& m) {
        if constexpr (P::split) {
          opnd_store_split<BM, NTH>(m.akc, m.kend, m.scale, ra, sm.Ah, sm.Al);
          opnd_store_split<BN, NTH>(m.bkc, m.kend, T(1), rb, sm.Bh, sm.Bl);
        } else {
          opnd_store<BM, NTH>(m.akc, m.kend, m.scale, ra, sm.A);
          opnd_store<BN, NTH>(m.bkc, m.kend, T(1), rb, sm.B);
        }
      };
      auto multiply = [&](int kend) {
        if constexpr (P::split) {
          // one 16x16x32 step covers the whole k tile (entries past K are 0)
          if (any) {
            bf8_t ah[WM], al[WM], bh[WN], bl[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
              ah[i] = *reinterpret_cast<const bf8_t*>(&sm.Ah[wm + i * 16 + lr][8 * lk]);
              al[i] = *reinterpret_cast<const bf8_t*>(&sm.Al[wm + i * 16 + lr][8 * lk]);
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
              bh[j] = *reinterpret_cast<const bf8_t*>(&sm.Bh[wn + j * 16 + lr][8 * lk]);
              bl[j] = *reinterpret_cast<const bf8_t*>(&sm.Bl[wn + j * 16 + lr][8 * lk]);
            }
#pragma unroll
            for (int mi = 0; mi < WM; ++mi)
#pragma unroll
              for (int ni = 0; ni < WN; ++ni)
                if (act[mi][ni]) {
                  acc[mi][ni] = mfma32(al[mi], bh[ni], acc[mi][ni]);
                  acc[mi][ni] = mfma32(ah[mi], bl[ni], acc[mi][ni]);
                  acc[mi][ni] = mfma32(ah[mi], bh[ni], acc[mi][ni]);
                }
          }
        } else if (full && kend == BK) {
          // full tile: unrolled; the fragments of step kk+4 are read from
          // LDS while the MFMAs of step kk run
          T fa[2][WM], fb[2][WN];
#pragma unroll
          for (int i = 0; i < WM; ++i) fa[0][i] = sm.A[lk][wm + i * 16 + lr];
#pragma unroll
          for (int j = 0; j < WN; ++j) fb[0][j] = sm.B[lk][wn + j * 16 + lr];
#pragma unroll
          for (int s = 0; s < BK / 4; ++s) {
            const int cb = s & 1, nb = cb ^ 1;
            if (s + 1 < BK / 4) {
              const int kn = 4 * (s + 1) + lk;
#pragma unroll
              for (int i = 0; i < WM; ++i) fa[nb][i] = sm.A[kn][wm + i * 16 + lr];
#pragma unroll
              for (int j = 0; j < WN; ++j) fb[nb][j] = sm.B[kn][wn + j * 16 + lr];
            }
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
              for (int j = 0; j < WN; ++j) acc[i][j] = mfma4(fa[cb][i], fb[cb][j], acc[i][j]);
          }
        } else if (any) {
          for (int kk = 0; kk < kend; kk += 4) {
            T fa[WM], fb[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) fa[i] = sm.A[kk + lk][wm + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < WN; ++j) fb[j] = sm.B[kk + lk][wn + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
              for (int j = 0; j < WN; ++j)
                if (act[i][j]) acc[i][j] = mfma4(fa[i], fb[j], acc[i][j]);
          }
        }
      };
      load_step(ra0, rb0, m0);
      if constexpr (P::depth == 1) {
        for (;;) {
          stage(ra0, rb0, m0);
          __syncthreads();
          const int kend = m0.kend;
          const bool h0 = lmore;
          if (h0) load_step(ra0, rb0, m0);
          multiply(kend);
          __syncthreads();
          if (!h0) break;
        }
      } else {
        bool h1 = lmore;
        if (h1) load_step(ra1, rb1, m1);
        for (;;) {
          stage(ra0, rb0, m0);
          __syncthreads();
          int kend = m0.kend;
          const bool h0 = lmore;
          if (h0) load_step(ra0, rb0, m0);
          multiply(kend);
          __syncthreads();
          if (!h1) break;
          stage(ra1, rb1, m1);
          __syncthreads();
          kend = m1.kend;
          h1 = lmore;
          if (h1) load_step(ra1, rb1, m1);
          multiply(kend);
          __syncthreads();
          if (!h0) break;
        }
      }
    }
    // result element v of lane l in sub-tile (mi, ni): row RL*(l/16) + RV*v, column l%16
    auto store = [&](auto* Cp) {
#pragma unroll
      for (int mi = 0; mi < WM; ++mi)
#pragma unroll
        for (int ni = 0; ni < WN; ++ni) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              int r = m0 + wm + mi * 16 + lk * P::RL + v * P::RV, c = n0 + wn + ni * 16 + lr;
              if (r < Tk.M && c < Tk.N) {
                auto* dst = Cp + (int64_t)r * Tk.ldc + c;
                auto val = (decltype(*dst + 0))acc[mi][ni][v];
                if (Tk.accumulate & GT_ACCUM) val += gld(dst);
                gst(dst, val);
              }
            }
          }
    };
    if (Tk.accumulate & GT_C64)
      store((Tk.c_buf == 1 ? p1 : reinterpret_cast<double*>(table[Tk.c_buf])) + Tk.c_off + batch * Tk.c_bstride);
    else
      store(table[Tk.c_buf] + Tk.c_off + batch * Tk.c_bstride);
  }
}

// The jobs of this workgroup's XCD: units taken from the XCD's counter
// (dynamic launches), else every gridDim.x / NXCD-th job from blockIdx.x / NXCD.
template <class Run>
__device__ __forceinline__ void for_each_job(const XcdMap& map, int64_t* s_unit, Run&& run) {
  const int xcd = blockIdx.x % NXCD;
  if (map.dynamic) {
    const int64_t* __restrict__ U = map.units + map.unit_begin[xcd];
    const int64_t nu = map.nunits[xcd];
    for (;;) {
      if (threadIdx.x == 0) *s_unit = (int64_t)atomicAdd(map.counters + 64 * xcd, 1u);
      __syncthreads();
      const int64_t u = *s_unit;
      __syncthreads();
      if (u >= nu) break;
      const int64_t je = U[u + 1];
      for (int64_t job = U[u]; job < je; ++job) run(job);
    }
  } else {
    const int64_t njobs = map.njobs[xcd];
    for (int64_t job = blockIdx.x / NXCD; job < njobs; job += gridDim.x / NXCD) run(job);
  }
}

// Grouped GEMM over a task list (see device.h).  Operand buffers hold P::T;
// the output is P::T, or binary64 for tasks flagged GT_C64 (buffer 1 is p1).
// MIXED: every task carries its own tile shape (TILE_EDGE launches).
template <class P, int WM, int WN, bool MIXED>
__global__ __launch_bounds__(NT, 4) void gemm_kernel(const GTask* __restrict__ tasks, const XcdMap map,
                                                  const GContrib* __restrict__ contribs,
                                                  const int* __restrict__ bucket_all,
                                                  typename P::T* const* __restrict__ table,
                                                  const typename P::T* p0, double* p1) {
  using SmemT = std::conditional_t<MIXED, Smem<P, 64, 64>, Smem<P, 32 * WM, 32 * WN>>;
  __shared__ SmemT smem;
  __shared__ int64_t s_unit;
  const int* __restrict__ bucket = bucket_all + map.bucket_begin[blockIdx.x % NXCD];
  for_each_job(map, &s_unit, [&](int64_t job) {
    const GTask& Tk = tasks[find_task(tasks, bucket, map.shift, job)];
    const int64_t local = job - Tk.job_begin + Tk.job_off;
    if constexpr (!MIXED) {
      gemm_job<P, WM, WN>(Tk, local, &smem, contribs, table, p0, p1);
    } else {
      switch (Tk.shape) {
        case TILE_32x64:
          gemm_job<P, 1, 2>(Tk, local, &smem, contribs, table, p0, p1);
          break;
        case TILE_64x32:
          gemm_job<P, 2, 1>(Tk, local, &smem, contribs, table, p0, p1);
          break;
        case TILE_32x32:
          gemm_job<P, 1, 1>(Tk, local, &smem, contribs, table, p0, p1);
          break;
        default:
          gemm_job<P, 2, 2>(Tk, local, &smem, contribs, table, p0, p1);
          break;
      }
    }
  });
}

// 128 x 128 tiles on 1024-thread workgroups (TILE_128): sixteen waves, each
// with the 32 x 32 sub-tile of the 256-thread 64 x 64 path, share one operand
// tile in LDS, so that every operand byte fetched feeds twice the MFMA work.
// One workgroup fills a CU (four waves per SIMD).
template <class P>
__global__ __launch_bounds__(NT_BIG, 1) void gemm_kernel_big(const GTask* __restrict__ tasks, const XcdMap map,
                                                          const GContrib* __restrict__ contribs,
                                                          const int* __restrict__ bucket_all,
                                                          typename P::T* const* __restrict__ table,
                                                          const typename P::T* p0, double* p1) {
  __shared__ Smem<P, 128, 128> smem;
  __shared__ int64_t s_unit;
  const int* __restrict__ bucket = bucket_all + map.bucket_begin[blockIdx.x % NXCD];
  for_each_job(map, &s_unit, [&](int64_t job) {
    const GTask& Tk = tasks[find_task(tasks, bucket, map.shift, job)];
    gemm_job<P, 2, 2, NT_BIG>(Tk, job - Tk.job_begin + Tk.job_off, &smem, contribs, table, p0, p1);
  });
}

__global__ void zero_counters_kernel(unsigned* c) {
  if (threadIdx.x < NXCD) c[64 * threadIdx.x] = 0u;
}

template <class P>
static void launch_variant(int tile, dim3 grid, hipStream_t s, const GTask* t, const XcdMap& map,
                           const GContrib* c, const int* bk, typename P::T* const* tab, const typename P::T* p0,
                           double* p1) {
  switch (tile) {
    case TILE_64x64:
      hipLaunchKernelGGL((gemm_kernel<P, 2, 2, false>), grid, dim3(NT), 0, s, t, map, c, bk, tab, p0, p1);
      break;
    case TILE_32x32:
      hipLaunchKernelGGL((gemm_kernel<P, 1, 1, false>), grid, dim3(NT), 0, s, t, map, c, bk, tab, p0, p1);
      break;
    case TILE_64x32:
      hipLaunchKernelGGL((gemm_kernel<P, 2, 1, false>), grid, dim3(NT), 0, s, t, map, c, bk, tab, p0, p1);
      break;
    case TILE_32x64:
      hipLaunchKernelGGL((gemm_kernel<P, 1, 2, false>), grid, dim3(NT), 0, s, t, map, c, bk, tab, p0, p1);
      break;
    case TILE_EDGE:
      hipLaunchKernelGGL((gemm_kernel<P, 2, 2, true>), grid, dim3(NT), 0, s, t, map, c, bk, tab, p0, p1);
      break;
    case TILE_128:
      hipLaunchKernelGGL((gemm_kernel_big<P>), grid, dim3(NT_BIG), 0, s, t, map, c, bk, tab, p0, p1);
      break;
    default:
      throw Error(DMRG_EINVAL, "unknown GEMM tile shape");
  }
}

// Workgroups of one GEMM kernel variant resident per compute unit.
// Occupancy and CU counts are cached per device (devices may differ).
static int current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  DMRG_CHECK(dev >= 0 && dev < MAX_DEVICES, DMRG_EINVAL, "device index beyond the occupancy cache");
  return dev;
}

template <class P>
static int blocks_per_cu_of(int tile) {
  static std::atomic<int> cache[MAX_DEVICES][NTILE];
  const int dev = current_device();
  int v = cache[dev][tile].load(std::memory_order_relaxed);
  if (v == 0) {
    const void* f = nullptr;
    switch (tile) {
      case TILE_32x32:
        f = reinterpret_cast<const void*>(&gemm_kernel<P, 1, 1, false>);
        break;
      case TILE_64x32:
        f = reinterpret_cast<const void*>(&gemm_kernel<P, 2, 1, false>);
        break;
      case TILE_32x64:
        f = reinterpret_cast<const void*>(&gemm_kernel<P, 1, 2, false>);
        break;
      case TILE_EDGE:
        f = reinterpret_cast<const void*>(&gemm_kernel<P, 2, 2, true>);
        break;
      case TILE_128:
        f = reinterpret_cast<const void*>(&gemm_kernel_big<P>);
        break;
      default:
        f = reinterpret_cast<const void*>(&gemm_kernel<P, 2, 2, false>);
        break;
    }
    int nb = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, tile == TILE_128 ? NT_BIG : NT, 0));
    v = nb > 0 ? nb : 1;
    cache[dev][tile].store(v, std::memory_order_relaxed);
  }
  return v;
}
static int blocks_per_cu(int elem, int tile) {
  DMRG_CHECK(tile >= 0 && tile < NTILE, DMRG_EINVAL, "unknown GEMM tile shape");
  if (elem == P_F64) return blocks_per_cu_of<PolF64>(tile);
  if (elem == P_F32) return blocks_per_cu_of<PolF32>(tile);
  return blocks_per_cu_of<PolBF3>(tile);
}
static int cu_count() {
  static std::atomic<int> cache[MAX_DEVICES];
  const int dev = current_device();
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n == 0) {
    HIPCHK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    if (n < NXCD) n = NXCD;
    cache[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

void gemm_launch(const GTask* tasks_dev, int ntasks, const XcdMap& map, const GContrib* contribs_dev,
                 const int* bucket_dev, void* const* table_dev, const void* p0, void* p1, int elem, int tile,
                 int64_t grid_per_xcd, void* stream) {
  if (ntasks == 0 || map.max_jobs == 0) return;
  int64_t per = map.max_jobs < (1 << 19) ? map.max_jobs : (1 << 19);
  if (grid_per_xcd > 0 && grid_per_xcd < per) per = grid_per_xcd;
  XcdMap m = map;
  m.dynamic = grid_per_xcd < 0;
  if (m.dynamic) {
    DMRG_CHECK(map.units && map.counters, DMRG_EINVAL, "dynamic GEMM launch without units");
    per = (int64_t)(cu_count() / NXCD) * blocks_per_cu(elem, tile);
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, S(stream), map.counters);
  }
  const dim3 grid((unsigned)(per * NXCD));
  if (elem == P_F64) {
    launch_variant<PolF64>(tile, grid, S(stream), tasks_dev, m, contribs_dev, bucket_dev,
                           (double* const*)table_dev, (const double*)p0, (double*)p1);
  } else if (elem == P_F32) {
    launch_variant<PolF32>(tile, grid, S(stream), tasks_dev, m, contribs_dev, bucket_dev,
                           (float* const*)table_dev, (const float*)p0, (double*)p1);
  } else if (elem == P_BF16X3) {
    launch_variant<PolBF3>(tile, grid, S(stream), tasks_dev, m, contribs_dev, bucket_dev,
                           (float* const*)table_dev, (const float*)p0, (double*)p1);
  } else {
    throw Error(DMRG_EINVAL, "unknown GEMM precision");
  }
  dev_check("gemm_launch");
}

// One workgroup per (segment, slice): slice y of 8 takes every 8th run of
// 256 elements.  The partials of an element are added in order.
__global__ void reduce_kernel(const ReduceSeg* __restrict__ segs, void* const* __restrict__ table, double* p1) {
  const ReduceSeg sg = segs[blockIdx.x];
  double* dst = (sg.dst_buf == 1 ? p1 : reinterpret_cast<double*>(table[sg.dst_buf])) + sg.dst_off;
  const double* src = (sg.src_buf == 1 ? p1 : reinterpret_cast<const double*>(table[sg.src_buf])) + sg.src_off;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < sg.n; e += 256 * (int64_t)gridDim.y) {
    double v = dst[e];
    for (int s = 0; s < sg.nsrc; ++s) v += src[e + s * sg.src_stride];
    dst[e] = v;
  }
}

__global__ void copy_segments_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                     const int64_t* __restrict__ seg) {
  const int64_t s = seg[3 * blockIdx.x], d = seg[3 * blockIdx.x + 1], n = seg[3 * blockIdx.x + 2];
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < n; e += 256 * (int64_t)gridDim.y) dst[d + e] = src[s + e];
}

void k_copy_segments(const double* src, double* dst, const int64_t* seg_dev, int nseg, void* stream) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(copy_segments_kernel, dim3((unsigned)nseg, 8), dim3(256), 0, S(stream), src, dst, seg_dev);
  dev_check("k_copy_segments");
}

void reduce_launch(const ReduceSeg* segs_dev, int nseg, void* const* table_dev, void* p1, void* stream) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)nseg, 8), dim3(256), 0, S(stream), segs_dev, table_dev,
                     (double*)p1);
  dev_check("reduce_launch");
}

// ---------------------------------------------------------------- vector kernels
static inline unsigned nblocks(int64_t n, int per = 256) {
  int64_t b = (n + per - 1) / per;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

__global__ void fill_kernel(double* x, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}
__global__ void fill_f_kernel(float* x, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}
__global__ void d2f_kernel(const double* x, float* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = (float)x[i];
}
__global__ void f2d_kernel(const float* x, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = (double)x[i];
}
__global__ void axpby_kernel(double a, const double* x, double b, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}
__global__ void copy_kernel(const double* x, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = x[i];
}
__global__ void scale_kernel(double* y, double s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] *= s;
}

void k_fill(double* x, double v, int64_t n, void* s) {
  if (n > 0) hipLaunchKernelGGL(fill_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), x, v, n);
  dev_check("k_fill");
}
void k_zero_bytes(void* p, size_t bytes, void* s) {
  DMRG_CHECK(((uintptr_t)p & 7) == 0 && bytes % 8 == 0, DMRG_EINTERNAL,
             "k_zero_bytes needs 8-byte aligned whole words");
  const int64_t n = (int64_t)(bytes / 8);
  if (n > 0) hipLaunchKernelGGL(fill_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), (double*)p, 0.0, n);
  dev_check("k_zero_bytes");
}
void k_fill_f(float* x, float v, int64_t n, void* s) {
  if (n > 0) hipLaunchKernelGGL(fill_f_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), x, v, n);
  dev_check("k_fill_f");
}
void k_d2f(const double* x, float* y, int64_t n, void* s) {
  if (n > 0) hipLaunchKernelGGL(d2f_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), x, y, n);
  dev_check("k_d2f");
}
void k_f2d(const float* x, double* y, int64_t n, void* s) {
  if (n > 0) hipLaunchKernelGGL(f2d_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), x, y, n);
  dev_check("k_f2d");
}
void k_axpby(double a, const double* x, double b, double* y, int64_t n, void* s) {
  if (n > 0) hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), a, x, b, y, n);
  dev_check("k_axpby");
}
void k_copy(const double* x, double* y, int64_t n, void* s) {
  if (n > 0) hipLaunchKernelGGL(copy_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), x, y, n);
  dev_check("k_copy");
}
void k_scale(double* y, double sc, int64_t n, void* s) {
  if (n > 0) hipLaunchKernelGGL(scale_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), y, sc, n);
  dev_check("k_scale");
}

// Dots of m vectors with x: two passes (fixed-order partial sums) -> deterministic.
constexpr int MD_CHUNKS = MULTIDOT_PART;
__global__ void multidot_partial(const double* V, int64_t ld, const double* x, int64_t n, double* part) {
  const int j = blockIdx.y, c = blockIdx.x;
  const int64_t per = (n + MD_CHUNKS - 1) / MD_CHUNKS;
  const int64_t beg = c * per, end = (beg + per < n) ? beg + per : n;
  const double* v = V + j * ld;
  double s = 0;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) s += v[i] * x[i];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[j * MD_CHUNKS + c] = red[0];
}
__global__ void multidot_final(const double* part, int m, double* out) {
  const int j = blockIdx.x;
  __shared__ double red[256];
  double s = 0;
  for (int c = threadIdx.x; c < MD_CHUNKS; c += blockDim.x) s += part[j * MD_CHUNKS + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

void k_multidot(const double* V, int64_t ld, int m, const double* x, int64_t n, double* out, double* part,
                void* s) {
  if (m <= 0) return;
  DMRG_CHECK(part != nullptr, DMRG_EINVAL, "k_multidot without partial-sum scratch");
  hipLaunchKernelGGL(multidot_partial, dim3(MD_CHUNKS, m), dim3(256), 0, S(s), V, ld, x, n, part);
  hipLaunchKernelGGL(multidot_final, dim3(m), dim3(256), 0, S(s), part, m, out);
  dev_check("k_multidot");
}

__global__ void lincomb_kernel(const double* V, int64_t ld, int m, const double* c, int64_t n, double* y,
                               int mode) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0;
    for (int j = 0; j < m; ++j) s += c[j] * V[j * ld + i];
    if (mode == 0)
      y[i] = s;
    else
      y[i] -= s;
  }
}
void k_lincomb(const double* V, int64_t ld, int m, const double* c, int64_t n, double* y, void* s) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), V, ld, m, c, n, y, 0);
  dev_check("k_lincomb");
}
void k_sub_lincomb(const double* V, int64_t ld, int m, const double* c, int64_t n, double* y, void* s) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), V, ld, m, c, n, y, 1);
  dev_check("k_sub_lincomb");
}

// rocSOLVER handles, one per (device, stream), kept for the process lifetime.
static rocblas_handle solver_handle(void* stream) {
  static std::mutex mu;
  static std::map<std::pair<int, void*>, rocblas_handle> handles;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = handles.find({dev, stream});
  if (it != handles.end()) return it->second;
  rocblas_handle h = nullptr;
  DMRG_CHECK(rocblas_create_handle(&h) == rocblas_status_success, DMRG_EHIP, "rocblas_create_handle failed");
  DMRG_CHECK(rocblas_set_stream(h, S(stream)) == rocblas_status_success, DMRG_EHIP, "rocblas_set_stream failed");
  handles[{dev, stream}] = h;
  return h;
}

void dev_syevd(double* A, int n, int lda, double* w, double* work_e, int* info, void* stream) {
  if (n <= 0) return;
  const rocblas_status st = rocsolver_dsyevd(solver_handle(stream), rocblas_evect_original, rocblas_fill_upper, n,
                                             A, lda, w, work_e, info);
  DMRG_CHECK(st == rocblas_status_success, DMRG_EHIP, "rocsolver_dsyevd failed to launch");
  dev_check("dev_syevd");
}

// Cyclic Jacobi on one wave; matrix in LDS.  m <= 32.
__global__ void small_eigh_kernel(const double* G, int ld, int m, double* w, double* Z) {
  __shared__ double a[32][33];
  __shared__ double z[32][33];
  __shared__ double cs[2];
  const int t = threadIdx.x;
  for (int i = t; i < m * m; i += blockDim.x) {
    int r = i / m, c = i % m;
    a[r][c] = 0.5 * (G[r * ld + c] + G[c * ld + r]);
    z[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    // convergence: off-diagonal norm relative to the matrix norm
    __shared__ double offn, totn;
    if (t == 0) {
      double o = 0, d = 0;
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
          if (r != c) o += a[r][c] * a[r][c];
          d += a[r][c] * a[r][c];
        }
      offn = o;
      totn = d;
    }
    __syncthreads();
    if (offn <= 1e-30 * (totn > 0 ? totn : 1.0)) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        if (t == 0) {
          double apq = a[p][q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
            double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            s = tt * c;
          }
          cs[0] = c;
          cs[1] = s;
        }
        __syncthreads();
        const double c = cs[0], s = cs[1];
        if (s != 0.0) {
          // A <- J^T A J on rows/cols p,q; Z <- Z J
          if (t < m) {
            double akp = a[t][p], akq = a[t][q];
            a[t][p] = c * akp - s * akq;
            a[t][q] = s * akp + c * akq;
          }
          __syncthreads();
          if (t < m) {
            double apk = a[p][t], aqk = a[q][t];
            a[p][t] = c * apk - s * aqk;
            a[q][t] = s * apk + c * aqk;
            double zkp = z[t][p], zkq = z[t][q];
            z[t][p] = c * zkp - s * zkq;
            z[t][q] = s * zkp + c * zkq;
          }
        }
        __syncthreads();
      }
  }
  __syncthreads();
  if (t == 0) {
    // selection sort ascending
    int idx[32];
    for (int i = 0; i < m; ++i) idx[i] = i;
    for (int i = 0; i < m; ++i) {
      int b = i;
      for (int j = i + 1; j < m; ++j)
        if (a[idx[j]][idx[j]] < a[idx[b]][idx[b]]) b = j;
      int tmp = idx[i];
      idx[i] = idx[b];
      idx[b] = tmp;
    }
    for (int i = 0; i < m; ++i) {
      w[i] = a[idx[i]][idx[i]];
      for (int r = 0; r < m; ++r) Z[r * m + i] = z[r][idx[i]];
    }
  }
}
void k_small_eigh(const double* G, int ld, int m, double* w, double* Z, void* s) {
  hipLaunchKernelGGL(small_eigh_kernel, dim3(1), dim3(64), 0, S(s), G, ld, m, w, Z);
  dev_check("k_small_eigh");
}

__global__ void precond_diag_kernel(const double* r, const double* d, const double* theta, double fl,
                                    double* t, int64_t n) {
  const double th = *theta;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double den = th - d[i];
    if (fabs(den) < fl) den = (den < 0 ? -fl : fl);
    t[i] = r[i] / den;
  }
}
void k_precond_diag(const double* r, const double* d, const double* theta, double fl, double* t, int64_t n,
                    void* s) {
  hipLaunchKernelGGL(precond_diag_kernel, dim3(nblocks(n)), dim3(256), 0, S(s), r, d, theta, fl, t, n);
  dev_check("k_precond_diag");
}

// meta: per block (src_off, dim, dst_off)
__global__ void gather_diag_kernel(const double* src, const int64_t* meta, int nblk, int64_t sstride,
                                   int64_t dstride, double* dst) {
  const int mem = blockIdx.y;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t so = meta[3 * b], dim = meta[3 * b + 1], dO = meta[3 * b + 2];
    for (int64_t l = threadIdx.x; l < dim; l += blockDim.x)
      dst[mem * dstride + dO + l] = src[mem * sstride + so + l * dim + l];
  }
}
void k_gather_diag(const double* src, const int64_t* meta, int nblk, int64_t sstride, int64_t dstride,
                   int nmem, double* dst, void* s) {
  if (nblk <= 0 || nmem <= 0) return;
  unsigned gx = nblk < 1024 ? nblk : 1024;
  hipLaunchKernelGGL(gather_diag_kernel, dim3(gx, nmem), dim3(64), 0, S(s), src, meta, nblk, sstride, dstride, dst);
  dev_check("k_gather_diag");
}

}  // namespace dmrg
