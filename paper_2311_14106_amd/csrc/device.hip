// Device layer of libmdmrg for gfx950 (CDNA4): memory, the grouped
// sector-block GEMM (FP64 MFMA) that carries the effective-Hamiltonian
// product, renormalisation, density matrices and operator combinations, the
// diagonal of H_eff, deterministic FP64 vector reductions, a counter-based
// Gaussian generator and the symmetric eigensolver (rocSOLVER).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <numeric>
#include <type_traits>

#include "internal.h"

namespace mdmrg {

#define HIP_CHECK(x)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw Error(-3, std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x);  \
  } while (0)

struct Device {
  int id = 0;
  hipStream_t stream = nullptr;
  bool own_stream = true;  // false: the caller's stream, not destroyed here
  rocblas_handle blas = nullptr;
  double *red = nullptr;       // reduction partials
  double *red_out = nullptr;   // reduction results (device)
  double *host_red = nullptr;  // pinned host mirror
  int *info = nullptr;
  double *syevd_work = nullptr;
  size_t syevd_work_n = 0;
  // allocation budget of the context (dev_alloc / dev_free)
  std::unordered_map<void *, size_t> live;
  size_t live_bytes = 0, budget_bytes = 0, budget_default = 0;
  // launch timing
  bool timing = false;
  bool capturing = false;  // stream capture in progress: no events, no host syncs
  int force_variant = -1;  // >= 0: tile variant of every grouped launch
  unsigned char *staging = nullptr;  // device address of this GPU's copy of `scratch` (set at creation)
  std::vector<hipEvent_t> ev_pool;
  struct Pending {
    int tag, prec, variant;  // variant < 0: a graph replay (whole product), not one kernel
    hipEvent_t a, b;
    double flop;
  };
  std::vector<Pending> pending;
  double ms[kTags] = {}, launches[kTags] = {}, flop[kTags] = {};
};

static hipEvent_t ev_get(Device *d) {
  if (!d->ev_pool.empty()) {
    hipEvent_t e = d->ev_pool.back();
    d->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}

// Process-wide totals of the grouped kernel per precision form (0 FP64,
// 1 FP32, 2 3xBF16, 3 6xBF16) and tile variant, summed over every device
// context of the process, including destroyed ones.
static std::mutex g_timing_mu;
static double g_ms[kPrecs][kGemmVariants], g_launches[kPrecs][kGemmVariants], g_flop[kPrecs][kGemmVariants];

static void timing_drain(Device *d) {
  if (d->pending.empty()) return;
  HIP_CHECK(hipEventSynchronize(d->pending.back().b));
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (auto &p : d->pending) {
    float t = 0.f;
    HIP_CHECK(hipEventElapsedTime(&t, p.a, p.b));
    d->ms[p.tag] += t;
    d->launches[p.tag] += 1;
    d->flop[p.tag] += p.flop;
    if (p.variant >= 0) {
      g_ms[p.prec][p.variant] += t;
      g_launches[p.prec][p.variant] += 1;
      g_flop[p.prec][p.variant] += p.flop;
    }
    d->ev_pool.push_back(p.a);
    d->ev_pool.push_back(p.b);
  }
  d->pending.clear();
}

void dev_timing_process(Device *d, double ms[kPrecs][kGemmVariants], double launches[kPrecs][kGemmVariants],
                        double flop[kPrecs][kGemmVariants]) {
  timing_drain(d);
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (int p = 0; p < kPrecs; ++p)
    for (int v = 0; v < kGemmVariants; ++v) {
      ms[p][v] = g_ms[p][v];
      launches[p][v] = g_launches[p][v];
      flop[p][v] = g_flop[p][v];
    }
}

void dev_timing_enable(Device *d, bool on) { d->timing = on; }
void dev_timing_collect(Device *d, double ms[kTags], double launches[kTags], double flop[kTags]) {
  timing_drain(d);
  for (int i = 0; i < kTags; ++i) {
    ms[i] = d->ms[i];
    launches[i] = d->launches[i];
    flop[i] = d->flop[i];
  }
}

double wall_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr int kRedBlocks = 256;
constexpr int kMaxDot = 64;

// Staging area of the allocation-free grouped GEMM (dev_gemm_run_noalloc):
// the plan's segment, output and tile descriptors.  Every GPU the library
// runs on holds its own copy of the array until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: kernels and
// copies take the address hipGetSymbolAddress gives for the device, looked
// up once per device when the first context on it is created.
static __device__ __align__(256) unsigned char scratch[kNoAllocStagingBytes];
static std::mutex g_scratch_mu;
static std::unordered_map<int, unsigned char *> g_scratch_addr;  // device id -> its copy of `scratch`

static unsigned char *scratch_address(int device) {  // the device must be current
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void *ptr = nullptr;
  HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  MDMRG_REQUIRE(ptr != nullptr, -3, "hipGetSymbolAddress returned no address for the staging array");
  g_scratch_addr[device] = static_cast<unsigned char *>(ptr);
  return static_cast<unsigned char *>(ptr);
}

Device *dev_create(int device, void *stream) {
  std::unique_ptr<Device> owner(new Device());  // deleted if a set-up call below fails
  Device *d = owner.get();
  d->id = device;
  HIP_CHECK(hipSetDevice(device));
  if (stream) {
    // the caller's stream (it keeps ownership); its device must be ours
    d->stream = static_cast<hipStream_t>(stream);
    d->own_stream = false;
    int sdev = -1;
    HIP_CHECK(hipStreamGetDevice(d->stream, &sdev));
    MDMRG_REQUIRE(sdev == device, -1, "mdmrg_create: the stream belongs to another device");
  } else {
    // blocking stream: ordered with work that callers queue on the legacy default stream
    HIP_CHECK(hipStreamCreate(&d->stream));
    d->own_stream = true;
  }
  if (rocblas_create_handle(&d->blas) != rocblas_status_success) throw Error(-3, "rocblas_create_handle failed");
  rocblas_set_stream(d->blas, d->stream);
  HIP_CHECK(hipMalloc(&d->red, sizeof(double) * kRedBlocks * kMaxDot));
  HIP_CHECK(hipMalloc(&d->red_out, sizeof(double) * kMaxDot));
  HIP_CHECK(hipHostMalloc(&d->host_red, sizeof(double) * kMaxDot));
  HIP_CHECK(hipMalloc(&d->info, sizeof(int)));
  d->staging = scratch_address(device);
  size_t free_b = 0, total_b = 0;
  HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
  d->budget_bytes = d->budget_default = size_t(0.95 * double(free_b));
  return owner.release();
}

void dev_destroy(Device *d) {
  if (!d) return;
  (void)hipSetDevice(d->id);
  (void)hipStreamSynchronize(d->stream);
  try {
    timing_drain(d);  // keep the process-wide totals complete
  } catch (...) {
  }
  for (auto &p : d->pending) {
    d->ev_pool.push_back(p.a);
    d->ev_pool.push_back(p.b);
  }
  for (auto e : d->ev_pool) (void)hipEventDestroy(e);
  (void)hipFree(d->red);
  (void)hipFree(d->red_out);
  (void)hipHostFree(d->host_red);
  (void)hipFree(d->info);
  if (d->syevd_work) (void)hipFree(d->syevd_work);
  if (d->blas) rocblas_destroy_handle(d->blas);
  if (d->own_stream) (void)hipStreamDestroy(d->stream);
  delete d;
}

// Every allocation of the context is counted against a budget fixed at
// creation (95% of the device memory free then), so that a workload larger
// than the card fails here, with ENOMEM and the sizes, instead of in the
// stream-ordered allocator.
void *dev_alloc(Device *d, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (d->live_bytes + bytes > d->budget_bytes)
    throw Error(-2, "device memory budget exceeded: " + std::to_string(bytes) + " bytes requested, " +
                        std::to_string(d->live_bytes) + " in use of " + std::to_string(d->budget_bytes));
  void *p = nullptr;
  hipError_t e = hipMallocAsync(&p, bytes, d->stream);
  if (e != hipSuccess || !p) {
    // the stream-ordered pool keeps freed blocks reserved: once the stream
    // has drained, return them to the device and try once more (a large
    // workload frees and allocates blocks of ~100 GB in turn)
    (void)hipGetLastError();
    HIP_CHECK(hipStreamSynchronize(d->stream));
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, d->id) == hipSuccess && pool) (void)hipMemPoolTrimTo(pool, 0);
    (void)hipGetLastError();
    p = nullptr;
    e = hipMallocAsync(&p, bytes, d->stream);
  }
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(-2, "device allocation of " + std::to_string(bytes) + " bytes failed (" +
                        std::to_string(d->live_bytes) + " bytes in use by the context)");
  }
  d->live[p] = bytes;
  d->live_bytes += bytes;
  return p;
}
void dev_set_budget(Device *d, size_t bytes) {
  d->budget_bytes = bytes ? std::min(bytes, d->budget_default) : d->budget_default;
}
size_t dev_live_bytes(Device *d) { return d->live_bytes; }
void dev_free(Device *d, void *p) {
  if (!p) return;
  auto it = d->live.find(p);
  if (it != d->live.end()) {
    d->live_bytes -= it->second;
    d->live.erase(it);
  }
  HIP_CHECK(hipFreeAsync(p, d->stream));
}
void dev_h2d(Device *d, void *dst, const void *src, size_t b) {
  if (b) HIP_CHECK(hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, d->stream));
  HIP_CHECK(hipStreamSynchronize(d->stream));
}
void dev_d2h(Device *d, void *dst, const void *src, size_t b) {
  if (b) HIP_CHECK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, d->stream));
  HIP_CHECK(hipStreamSynchronize(d->stream));
}
void dev_d2d(Device *d, void *dst, const void *src, size_t b) {
  if (b) HIP_CHECK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, d->stream));
}
void dev_sync(Device *d) { HIP_CHECK(hipStreamSynchronize(d->stream)); }
size_t dev_free_bytes(Device *d) {
  size_t f = 0, t = 0;
  HIP_CHECK(hipMemGetInfo(&f, &t));
  return f;
}

// ------------------------------------------------------------------ zero
// Zero fill of n8 doubles followed by `tail` (< 8) single bytes.
__global__ void k_zero(double *x, int64_t n8, int tail) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < n8; i += (int64_t)gridDim.x * blockDim.x) x[i] = 0.0;
  if (i0 < tail) reinterpret_cast<unsigned char *>(x + n8)[i0] = 0;
}
void dev_zero(Device *d, void *dst, size_t bytes) {
  // every byte by a fill kernel, never a memset node, so that the call may
  // sit inside a captured graph (an FP32 vector of odd length ends in a
  // 4-byte tail)
  const int64_t n = int64_t(bytes / 8);
  const int tail = int(bytes % 8);
  if (n == 0 && tail == 0) return;
  const int grid = int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)));
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, d->stream, (double *)dst, n, tail);
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------- grouped GEMM (FP64 and FP32)
// Workgroup = 8 waves (2 x 4) = 64x64 output tile; each wave owns a 32x16
// block as 2x1 MFMA 16x16x4 accumulators.  K is staged through LDS in steps
// of 8 or 16.  Operand layout of v_mfma_f64_16x16x4f64: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator element r of lane l is
// C[l/16 + 4r][l%16] for FP64 and C[4(l/16) + r][l%16] for FP32.
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kTKmax = 16;  // largest K step of the grouped kernel (checked against every TileCfg)
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

// one MFMA 16x16x4 step in the element type of the kernel: FP64
// (v_mfma_f64_16x16x4f64) or FP32 (v_mfma_f32_16x16x4f32), same operand
// layout
template <class T>
struct Mfma;
// accumulator element r of lane l holds C[row(l/16, r)][l%16]; the FP64 and
// FP32 instructions differ (both checked on gfx950 against host references)
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
  static __device__ inline acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
  static __device__ inline acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Workgroup tile of the grouped kernel: BM x BN outputs per workgroup of
// WY x WX waves, each wave a (BM/WY) x (BN/WX) block of 16x16 MFMA tiles;
// K staged through LDS in steps of TK with one step of register prefetch.
template <int BM_, int BN_, int WY_, int WX_, int TK_>
struct TileCfg {
  static constexpr int BM = BM_, BN = BN_, WY = WY_, WX = WX_, TK = TK_;
  static constexpr int NT = 64 * WY * WX;                      // threads per workgroup
  static constexpr int MI = BM / WY / 16, NI = BN / WX / 16;  // MFMA tiles per wave
};
// Tile variants (all 64x64 outputs per workgroup, so one tile list serves
// them all; they differ in how the tile is split over waves).  Every output
// element is accumulated over K in the same order in all of them, so their
// results are bitwise identical; the autotuner picks one per plan.
// K step: FP64 stages 8 columns per step in the 8- and 4-wave splits (half
// the LDS of a 16-column step, so twice the workgroups per CU; measured
// faster on split-K H_eff products) and 16 in the 16-wave split, which keeps
// the unsplit long-K case; FP32 stages 16 everywhere (32, the same LDS bytes
// per stage as FP64 at 16, measured slower).
// The BF16 forms stage 16 columns per step (a 32-column step holds twice
// the LDS and measured 25% slower); their products go in pairs into
// v_mfma_f32_16x16x32_bf16 (tile_mfma_bfs).
struct Bf16x3 {};  // element-type tag: FP32 data, two BF16 parts, 3 products
struct Bf16x6 {};  // element-type tag: FP32 data, three BF16 parts, 6 products
template <class T>
struct KStep {  // FP32
  static constexpr int small = 16, wide = 16;
};
template <>
struct KStep<double> {
  static constexpr int small = 8, wide = 16;
};
template <>
struct KStep<Bf16x3> {
  static constexpr int small = 16, wide = 16;
};
template <>
struct KStep<Bf16x6> {
  static constexpr int small = 16, wide = 16;
};
template <class T>
using Cfg64 = TileCfg<64, 64, 2, 4, KStep<T>::small>;  // variant 0, k_gemm: 8 waves of 32x16
template <class T>
using Cfg64w = TileCfg<64, 64, 4, 4, KStep<T>::wide>;  // variant 1, k_gemm_w16: 16 waves of 16x16
template <class T>
using Cfg64q = TileCfg<64, 64, 2, 2, KStep<T>::small>;  // variant 2, k_gemm_w4: 4 waves of 32x32
// variant 3, k_gemm_t128: 128x128 outputs per workgroup, 8 waves (2 x 4) of
// 64x32 (twice the operand reuse per fetched byte of the 64x64 tiles; its
// own tile list).  Eight waves keep 4 (FP64, 3xBF16) or 5 (FP32) waves per
// SIMD; four waves of 64x64 held two and measured 9-55% slower per product
// (6x6 Hubbard, D=2048: FP64 62.9 -> 57.8 ms, FP32 53.2 -> 34.4 ms, 3xBF16
// 32.7 -> 23.3 ms).
template <class T>
using Cfg128 = TileCfg<128, 128, 2, 4, KStep<T>::small>;
static_assert(KStep<double>::small <= kTKmax && KStep<double>::wide <= kTKmax && KStep<float>::small <= kTKmax &&
                  KStep<float>::wide <= kTKmax && KStep<Bf16x3>::small <= kTKmax && KStep<Bf16x3>::wide <= kTKmax &&
                  KStep<Bf16x6>::small <= kTKmax && KStep<Bf16x6>::wide <= kTKmax,
              "a K step exceeds kTKmax, which bounds the offsets the host checks");
constexpr int kTileM = 64, kTileN = 64;  // output tile of variants 0-2 (variant 3: 128 x 128)
constexpr int kPad = 2;  // LDS row padding (doubles) of the staged A / B tiles

// Operand loads of the grouped kernel are buffer loads: a workgroup-uniform
// base (the tile's first row / column of the operand at the step's first K
// position, advanced by scalar arithmetic per K step) and per-thread byte
// offsets fixed for a whole segment.  An element outside the output, or
// past K in a segment's last step, gets an offset beyond the buffer's range,
// for which the hardware returns 0 without a memory access, so a K step
// needs no address or mask arithmetic.  The host keeps every valid offset
// below 2^30 (plan_check).
constexpr int32_t kOffOut = int32_t(0x80000000u);  // beyond the buffer range: the load returns 0
constexpr int32_t kBufRange = 0x7fffffff;          // buffer size in bytes

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const char *base) {
  // raw buffer (stride 0), range kBufRange bytes; dword 3 as the gfx9 family needs
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(base), short(0), kBufRange, 0x00020000);
}
template <class T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, int32_t off);
template <>
__device__ inline float buf_load<float>(__amdgpu_buffer_rsrc_t r, int32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ inline double buf_load<double>(__amdgpu_buffer_rsrc_t r, int32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Per-thread load state of one segment (FP64 and FP32 forms): each thread
// stages EA elements of op(A) and EB of op(B) per K step.  Element `it` of
// a thread sits at row i0 + di*it and K offset ka0 + dka*it of the staged A
// tile (K offset kb0 + dkb*it and column j0 + dj*it of the B tile); (di, dka)
// and (dkb, dj) follow from the operand's transposition, chosen so that
// consecutive threads read consecutive addresses.
template <class T, class C>
struct SegLoad {
  static constexpr int BM = C::BM, BN = C::BN, NT = C::NT, TK = C::TK;
  static constexpr int EA = BM * TK / NT, EB = BN * TK / NT;
  static_assert(EA >= 1 && EB >= 1 && NT % BM == 0 && NT % BN == 0 && NT % TK == 0, "tile / thread mismatch");
  const char *A, *B;       // step-0 bases of the tile's operand panels (uniform)
  int64_t da, db;          // bytes per K step (uniform)
  int32_t oa[EA], ob[EB];  // byte offsets of the thread's elements from the step base, or kOffOut
  int i0, di, ka0, dka;    // A tile: row and K offset of element 0, increments
  int j0, dj, kb0, dkb;    // B tile: column and K offset, increments
  int ga, ma;              // A: output row of element 0, rows of the output (identity operands)
  int k;
  T alpha;
  bool idA;
};

template <class T, class C>
__device__ inline void seg_setup(SegLoad<T, C> &L, const GSeg &sg, const Bases &bases, const GOut &o, int row0,
                                 int col0, int tid) {
  constexpr int BM = C::BM, BN = C::BN, NT = C::NT, TK = C::TK, EA = SegLoad<T, C>::EA, EB = SegLoad<T, C>::EB;
  constexpr int ES = int(sizeof(T));
  const T *A = reinterpret_cast<const T *>(bases.p[sg.a_slot]) + sg.a_off;
  const T *B = reinterpret_cast<const T *>(bases.p[sg.b_slot]) + sg.b_off;
  const bool tA = sg.flags & SEG_TA, tB = sg.flags & SEG_TB;
  L.idA = sg.flags & SEG_AID;
  L.alpha = T(sg.alpha);
  L.k = sg.k;
  L.ma = o.m;
  // A tile BM x TK: row-major source -> (i, kk) = (e / TK, e % TK);
  // transposed source -> (e % BM, e / BM); e = tid + NT it
  L.i0 = tA ? tid % BM : tid / TK;
  L.di = tA ? 0 : NT / TK;
  L.ka0 = tA ? tid / BM : tid % TK;
  L.dka = tA ? NT / BM : 0;
  L.ga = row0 + L.i0;
  L.A = reinterpret_cast<const char *>(tA ? A + row0 : A + int64_t(row0) * sg.lda);
  L.da = ES * (tA ? int64_t(TK) * sg.lda : int64_t(TK));
#pragma unroll
  for (int it = 0; it < EA; ++it) {
    const int i = L.i0 + L.di * it, kk = L.ka0 + L.dka * it;
    L.oa[it] = row0 + i < o.m ? ES * (tA ? kk * sg.lda + i : i * sg.lda + kk) : kOffOut;
  }
  // B tile TK x BN: row-major source -> (kb, j) = (e / BN, e % BN);
  // transposed source -> (e % TK, e / TK)
  L.j0 = tB ? tid / TK : tid % BN;
  L.dj = tB ? NT / TK : 0;
  L.kb0 = tB ? tid % TK : tid / BN;
  L.dkb = tB ? 0 : NT / BN;
  L.B = reinterpret_cast<const char *>(tB ? B + int64_t(col0) * sg.ldb : B + col0);
  L.db = ES * (tB ? int64_t(TK) : int64_t(TK) * sg.ldb);
#pragma unroll
  for (int it = 0; it < EB; ++it) {
    const int j = L.j0 + L.dj * it, kb = L.kb0 + L.dkb * it;
    L.ob[it] = col0 + j < o.n ? ES * (tB ? j * sg.ldb + kb : kb * sg.ldb + j) : kOffOut;
  }
}

// Loads of one K step.  EDGE: the step may reach past K (only a segment's
// last step can); the offsets of positions past K are replaced by kOffOut.
// Nothing is computed from the loaded values here, so no wait on them is
// needed before the MFMAs of the current step.
template <bool EDGE, class T, class C>
__device__ inline void seg_fetch(const SegLoad<T, C> &L, int step, T (&ra)[SegLoad<T, C>::EA],
                                 T (&rb)[SegLoad<T, C>::EB]) {
  const int k0 = step * C::TK;
  const __amdgpu_buffer_rsrc_t rA = buf_rsrc(L.A + step * L.da), rB = buf_rsrc(L.B + step * L.db);
  if (!L.idA) {
#pragma unroll
    for (int it = 0; it < SegLoad<T, C>::EA; ++it)
      ra[it] = buf_load<T>(rA, !EDGE || k0 + L.ka0 + L.dka * it < L.k ? L.oa[it] : kOffOut);
  }
#pragma unroll
  for (int it = 0; it < SegLoad<T, C>::EB; ++it)
    rb[it] = buf_load<T>(rB, !EDGE || k0 + L.kb0 + L.dkb * it < L.k ? L.ob[it] : kOffOut);
}

// Write one fetched K step to an LDS stage: A stage [kk][BM + kPad], B stage
// [kb][BN + kPad].  alpha is folded into A; identity factors are generated.
template <class T, class C>
__device__ inline void seg_store(const SegLoad<T, C> &L, int step, const T (&ra)[SegLoad<T, C>::EA],
                                 const T (&rb)[SegLoad<T, C>::EB], T *As, T *Bs) {
  constexpr int BM = C::BM, BN = C::BN;
  const int k0 = step * C::TK;
#pragma unroll
  for (int it = 0; it < SegLoad<T, C>::EA; ++it) {
    const int kk = L.ka0 + L.dka * it;
    T v;
    if (L.idA) {
      const int g = L.ga + L.di * it;
      v = (g < L.ma && k0 + kk < L.k && g == k0 + kk) ? L.alpha : T(0);
    } else {
      v = L.alpha * ra[it];
    }
    As[kk * (BM + kPad) + L.i0 + L.di * it] = v;
  }
#pragma unroll
  for (int it = 0; it < SegLoad<T, C>::EB; ++it) Bs[(L.kb0 + L.dkb * it) * (BN + kPad) + L.j0 + L.dj * it] = rb[it];
}

// MFMAs of one K step on the LDS stage (Ab, Bb) for this wave's block.  A
// wave whose block lies wholly outside the output skips the step; a partly
// covered block runs every MFMA (rows and columns outside the output are
// staged as zeros and their accumulators are never stored), which keeps the
// step free of per-tile branches.
template <class T, class C>
__device__ inline void tile_mfma(const T *Ab, const T *Bb, int wm, int wn, int lr, int lk, int qm, int qn,
                                 typename Mfma<T>::acc_t (&acc)[C::MI][C::NI]) {
  constexpr int BM = C::BM, BN = C::BN, MI = C::MI, NI = C::NI, TK = C::TK;
  if (qm <= 0 || qn <= 0) return;
#pragma unroll
  for (int kk = 0; kk < TK; kk += 4) {
    T a[MI], b[NI];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi) a[mi] = Ab[(kk + lk) * (BM + kPad) + wm + 16 * mi + lr];
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) b[ni] = Bb[(kk + lk) * (BN + kPad) + wn + 16 * ni + lr];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = Mfma<T>::step(a[mi], b[ni], acc[mi][ni]);
  }
}

template <class T, class C>
__device__ inline void gemm_tile(const GTile *__restrict__ tiles, const GOut *__restrict__ outs,
                                 const GSeg *__restrict__ segs, const Bases &bases) {
  constexpr int BM = C::BM, BN = C::BN, MI = C::MI, NI = C::NI, TK = C::TK;
  typedef typename Mfma<T>::acc_t acc_t;
  typedef SegLoad<T, C> SL;
  __shared__ T As[2][TK * (BM + kPad)];
  __shared__ T Bs[2][TK * (BN + kPad)];
  const GTile tl = tiles[blockIdx.x];
  if (tl.out < 0) return;  // queue padding; uniform over the workgroup, before any barrier
  const GOut o = outs[tl.out];
  const int row0 = int(tl.ti) * BM, col0 = int(tl.tj) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / C::WX) * (BM / C::WY), wn = (wave % C::WX) * (BN / C::WX);
  const int lr = lane & 15, lk = lane >> 4;
  // rows / columns of this wave's quadrant inside the output (wave-uniform)
  const int qm = o.m - (row0 + wm), qn = o.n - (col0 + wn);
  acc_t acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  SL L;
  T ra[SL::EA], rb[SL::EB];
  for (int si = 0; si < o.seg_count; ++si) {
    seg_setup(L, segs[o.seg_begin + si], bases, o, row0, col0, tid);
    const int nsteps = (L.k + TK - 1) / TK;
    if (nsteps == 0) continue;
    // double-buffered LDS: while the MFMAs consume stage `buf`, the next K
    // step is fetched into registers and then written to the other stage;
    // steps 0 .. nsteps-2 are whole, the last one may end past K
    int buf = 0;
    seg_fetch<true>(L, 0, ra, rb);
    seg_store(L, 0, ra, rb, As[buf], Bs[buf]);
    __syncthreads();
    for (int step = 1; step + 1 < nsteps; ++step) {
      seg_fetch<false>(L, step, ra, rb);
      tile_mfma<T, C>(As[buf], Bs[buf], wm, wn, lr, lk, qm, qn, acc);
      buf ^= 1;
      seg_store(L, step, ra, rb, As[buf], Bs[buf]);
      __syncthreads();
    }
    if (nsteps > 1) {
      seg_fetch<true>(L, nsteps - 1, ra, rb);
      tile_mfma<T, C>(As[buf], Bs[buf], wm, wn, lr, lk, qm, qn, acc);
      buf ^= 1;
      seg_store(L, nsteps - 1, ra, rb, As[buf], Bs[buf]);
      __syncthreads();
    }
    tile_mfma<T, C>(As[buf], Bs[buf], wm, wn, lr, lk, qm, qn, acc);
    __syncthreads();  // the next segment's first store reuses the stages
  }
  T *Cp = reinterpret_cast<T *>(bases.p[o.c_slot]) + o.c_off;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = row0 + wm + mi * 16 + Mfma<T>::row(lk, r);
        const int gj = col0 + wn + ni * 16 + lr;
        if (gi < o.m && gj < o.n) {
          T *p = Cp + (int64_t)gi * o.ldc + gj;
          const T v = acc[mi][ni][r];
          *p = o.accumulate ? (*p + v) : v;
        }
      }
}

// ---------------------------------------------- BF16 split products
// Every FP32 operand element x is split when it is staged to LDS.  3xBF16:
// hi = RNE_bf16(x), lo = RNE_bf16(x - hi) (x - hi is exact in FP32); a
// product is hi*lo + lo*hi + hi*hi with FP32 accumulation (lo*lo dropped):
// about 16 significant bits per operand instead of FP32's 24, at BF16 MFMA
// rate.  6xBF16 adds a middle part (hi, mid, lo) and the terms mid*mid,
// hi*mid, mid*hi: about 24 bits per operand.  The staged tiles are
// K-contiguous ([row][k] for A, [column][k] for B, rows of TK + 8 BF16), so
// a lane's 4 values of one part are one 8-byte LDS read; the MFMA takes
// from lane l the values of row / column l % 16 at K positions fixed by
// l / 16, the same for both operands, so any staged K order is a valid
// product order.
typedef short v4s __attribute__((ext_vector_type(4)));  // 4 BF16 bit patterns


// LDS stage of one operand: NP part arrays, rows of TK + 8 BF16 (K-contiguous)
template <class C, int NP>
using StageA = __bf16[NP][C::BM * (C::TK + 8)];
template <class C, int NP>
using StageB = __bf16[NP][C::BN * (C::TK + 8)];

// Staging of the split forms.  Each thread stages R = BM*TK/NT (1, 2 or
// 4) elements of op(A) and as many of op(B) per K step, mapped so that
// every load instruction is coalesced:
// * an operand stored M- (N-)contiguous: consecutive threads take
//   consecutive rows (columns) and a thread holds R consecutive K positions
//   of its row, so each BF16 part goes to LDS as one packed write of R values;
// * an operand stored K-contiguous: consecutive threads take consecutive K
//   positions of a row and a thread holds R consecutive rows; neighbouring
//   lanes exchange values (pair_store) so that each BF16 part again goes to
//   LDS as packed K pairs.
// Element `it` of a thread is at row r0 + dr*it and K position k0 + dk*it of
// the staged tile.  Loads are buffer loads from a workgroup-uniform base
// (the tile's first row / column at the step's first K position, advanced
// by scalar arithmetic per step) at per-thread byte offsets fixed for the
// whole segment; an element outside the output, or past K in the last
// step, gets an offset beyond the buffer's range, for which the hardware
// returns 0 -- so no per-step address or mask arithmetic is needed.

template <class C>
struct SegLoadK {
  static constexpr int BM = C::BM, BN = C::BN, NT = C::NT, TK = C::TK;
  static constexpr int RA = BM * TK / NT, RB = BN * TK / NT;
  static_assert((RA == 1 || RA == 2 || RA == 4) && (RB == 1 || RB == 2 || RB == 4), "R must be 1, 2 or 4");
  const char *A, *B;          // step-0 bases of the tile's operand panels (uniform)
  int64_t da, db;             // bytes per K step (uniform)
  int32_t oa[RA], ob[RB];     // byte offsets of the thread's elements from the step base, or kOffOut
  int ia, dia, ka, dka;       // A: row and K position of element 0 and their per-element increments
  int jb, djb, kb, dkb;       // B: column and K position, the same
  int k;
  float alpha;
  bool idA, pa, pb;  // identity A; packed staging of A, of B
  int ga;            // A: output row of element 0 (identity operands)
  int ma;            // A: rows of the output (identity operands)
};

template <class C>
__device__ inline void segk_setup(SegLoadK<C> &L, const GSeg &sg, const Bases &bases, const GOut &o, int row0,
                                  int col0, int tid) {
  constexpr int BM = C::BM, BN = C::BN, TK = C::TK, RA = SegLoadK<C>::RA, RB = SegLoadK<C>::RB;
  const bool tA = sg.flags & SEG_TA, tB = sg.flags & SEG_TB;
  const float *A = reinterpret_cast<const float *>(bases.p[sg.a_slot]) + sg.a_off;
  const float *B = reinterpret_cast<const float *>(bases.p[sg.b_slot]) + sg.b_off;
  L.idA = sg.flags & SEG_AID;
  L.alpha = float(sg.alpha);
  L.k = sg.k;
  L.ma = o.m;
  // op(A) element (i, kk) of step s sits at A[(row0+i)*lda + s*TK+kk] (row-major, K-contiguous)
  // or A[(s*TK+kk)*lda + row0+i] (transposed, M-contiguous)
  L.pa = tA;
  L.ia = tA ? tid % BM : RA * (tid / TK);
  L.dia = tA ? 0 : 1;
  L.ka = tA ? (tid / BM) * RA : tid % TK;
  L.dka = tA ? 1 : 0;
  L.ga = row0 + L.ia;
  L.A = reinterpret_cast<const char *>(tA ? A + row0 : A + int64_t(row0) * sg.lda);
  L.da = 4 * (tA ? int64_t(TK) * sg.lda : int64_t(TK));
#pragma unroll
  for (int it = 0; it < RA; ++it) {
    const int i = L.ia + L.dia * it, kk = L.ka + L.dka * it;
    L.oa[it] = row0 + i < o.m ? 4 * (tA ? kk * sg.lda + i : i * sg.lda + kk) : kOffOut;
  }
  // op(B) element (kk, j) sits at B[(s*TK+kk)*ldb + col0+j] (row-major, N-contiguous)
  // or B[(col0+j)*ldb + s*TK+kk] (transposed, K-contiguous)
  L.pb = !tB;
  L.jb = tB ? RB * (tid / TK) : tid % BN;
  L.djb = tB ? 1 : 0;
  L.kb = tB ? tid % TK : (tid / BN) * RB;
  L.dkb = tB ? 0 : 1;
  L.B = reinterpret_cast<const char *>(tB ? B + int64_t(col0) * sg.ldb : B + col0);
  L.db = 4 * (tB ? int64_t(TK) : int64_t(TK) * sg.ldb);
#pragma unroll
  for (int it = 0; it < RB; ++it) {
    const int j = L.jb + L.djb * it, kk = L.kb + L.dkb * it;
    L.ob[it] = col0 + j < o.n ? 4 * (tB ? j * sg.ldb + kk : kk * sg.ldb + j) : kOffOut;
  }
}

// Loads of one K step.  EDGE: the step may reach past K (only a segment's
// last step can), and the offsets of positions past K are replaced by
// kOffOut; other steps load at the segment's fixed offsets.
template <bool EDGE, class C>
__device__ inline void segk_fetch(const SegLoadK<C> &L, int step, float (&ra)[SegLoadK<C>::RA],
                                  float (&rb)[SegLoadK<C>::RB]) {
  constexpr int RA = SegLoadK<C>::RA, RB = SegLoadK<C>::RB;
  const int k0 = step * C::TK;
  const __amdgpu_buffer_rsrc_t rA = buf_rsrc(L.A + step * L.da), rB = buf_rsrc(L.B + step * L.db);
  if (!L.idA) {
#pragma unroll
    for (int it = 0; it < RA; ++it)
      ra[it] = buf_load<float>(rA, !EDGE || k0 + L.ka + L.dka * it < L.k ? L.oa[it] : kOffOut);
  }
#pragma unroll
  for (int it = 0; it < RB; ++it) rb[it] = buf_load<float>(rB, !EDGE || k0 + L.kb + L.dkb * it < L.k ? L.ob[it] : kOffOut);
}

// R consecutive BF16 values of one part, written as one LDS access
template <int R>
struct Packed;
template <>
struct Packed<1> {
  typedef __bf16 bf_t;
  typedef float f_t;
};
template <>
struct Packed<2> {
  typedef __bf16 bf_t __attribute__((ext_vector_type(2)));
  typedef float f_t __attribute__((ext_vector_type(2)));
};
template <>
struct Packed<4> {
  typedef __bf16 bf_t __attribute__((ext_vector_type(4)));
  typedef float f_t __attribute__((ext_vector_type(4)));
};

// Split R values into NP parts (NP = 2: hi = RNE(v), lo = RNE(v - hi);
// NP = 3: hi, mid = RNE(v - hi), lo = RNE(v - hi - mid); every difference is
// exact in FP32) and write part q to P[q][e .. e+R).
template <int NP, int R, int LEN>
__device__ inline void split_store(const float (&v)[R], __bf16 (&P)[NP][LEN], int e) {
  typedef typename Packed<R>::bf_t bf_t;
  typedef typename Packed<R>::f_t f_t;
  f_t x;
  if constexpr (R == 1) {
    x = v[0];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[r];
  }
  bf_t part[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    if constexpr (R == 1)
      part[q] = __bf16(x);
    else
      part[q] = __builtin_convertvector(x, bf_t);
    if (q + 1 < NP) {
      if constexpr (R == 1)
        x = x - float(part[q]);
      else
        x = x - __builtin_convertvector(part[q], f_t);
    }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) *reinterpret_cast<bf_t *>(&P[q][e]) = part[q];
}

// Staging of a K-contiguous operand: the thread holds R values of R
// consecutive rows at K position kk, and so does its neighbour lane at
// kk ^ 1.  The two exchange half of their values (one DPP lane swap per
// pair) so that the even lane holds the first R/2 rows and the odd lane the
// last R/2 at K positions (kk & ~1, kk | 1); each part is then written as
// one packed pair per row.  With rows of TK + 8 BF16 the 64 lanes of such a
// write cover the 64 LDS banks once.
template <int NP, int R, int LEN>
__device__ inline void pair_store(const float (&v)[R], __bf16 (&P)[NP][LEN], int row, int kk, int ld) {
  if constexpr (R == 1) {
    split_store<NP>(v, P, row * ld + kk);
  } else {
    constexpr int H = R / 2;
    const bool odd = kk & 1;
#pragma unroll
    for (int p = 0; p < H; ++p) {
      const float send = odd ? v[p] : v[H + p];
      // quad_perm [1, 0, 3, 2]: every lane receives the value of lane ^ 1
      const float recv =
          __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, send), 0xB1, 0xF, 0xF, false));
      const float pr[2] = {odd ? recv : v[p], odd ? v[H + p] : recv};
      split_store<NP>(pr, P, (row + (odd ? H : 0) + p) * ld + (kk & ~1));
    }
  }
}

// Write one fetched K step to an LDS stage of NP part arrays ([row][k] for
// A, [column][k] for B, rows of TK + 8): alpha folded into A, identity
// factors generated, then the split.
template <class C, int NP>
__device__ inline void segk_store(const SegLoadK<C> &L, int step, const float (&ra)[SegLoadK<C>::RA],
                                  const float (&rb)[SegLoadK<C>::RB], StageA<C, NP> &Ap, StageB<C, NP> &Bp) {
  constexpr int RA = SegLoadK<C>::RA, LD = C::TK + 8;
  const int k0 = step * C::TK;
  float va[RA];
  if (L.idA) {
#pragma unroll
    for (int it = 0; it < RA; ++it) {
      const int g = L.ga + L.dia * it, kk = k0 + L.ka + L.dka * it;
      va[it] = (g < L.ma && kk < L.k && g == kk) ? L.alpha : 0.f;
    }
  } else {
#pragma unroll
    for (int it = 0; it < RA; ++it) va[it] = L.alpha * ra[it];
  }
  if (L.pa)
    split_store<NP>(va, Ap, L.ia * LD + L.ka);
  else
    pair_store<NP>(va, Ap, L.ia, L.ka, LD);
  if (L.pb)
    split_store<NP>(rb, Bp, L.jb * LD + L.kb);
  else
    pair_store<NP>(rb, Bp, L.jb, L.kb, LD);
}

// One 16-deep K step of BF16 products.  Pairs of products go into one
// v_mfma_f32_16x16x32_bf16 (the full-rate gfx950 instruction): a lane's 8
// operand values are the 4 of part X followed by the 4 of part Y at the same
// K positions, for A and B alike, so the 32-deep product is X_A.X_B +
// Y_A.Y_B over the step's 16 K positions.  NP = 2: (hi*lo + lo*hi), then
// (hi*hi + 0); NP = 3: (hi*lo + mid*mid), (lo*hi + hi*mid), (mid*hi + hi*hi)
// -- smallest terms first, so that the FP32 accumulator rounds them before
// the large ones.  Every product of a chain on one accumulator is the same
// instruction: a 16-deep v_mfma_f32_16x16x16_bf16 issued straight after a
// 32-deep one on the same accumulator (the 16x16-per-wave split, where no
// other MFMA sits between them) gave results without the cross terms in the
// kernel test against the product model, as if it had read the
// accumulator before the 32-deep product was written.  The 16-deep
// instruction runs at half the rate of the 32-deep one on gfx950, so the
// zero half costs nothing.
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
__device__ inline v4f mfma32(v4s ax, v4s ay, v4s bx, v4s by, v4f c) {
  const v8s a = __builtin_shufflevector(ax, ay, 0, 1, 2, 3, 4, 5, 6, 7);
  const v8s b = __builtin_shufflevector(bx, by, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
template <class C, int NP>
__device__ inline void tile_mfma_bfs(const StageA<C, NP> &Ap, const StageB<C, NP> &Bp, int wm, int wn, int lr,
                                     int lk, int qm, int qn, v4f (&acc)[C::MI][C::NI]) {
  constexpr int MI = C::MI, NI = C::NI;
  static_assert(C::TK == 16, "one MFMA K step per staged step");
  // a wave whose block lies wholly outside the output skips the step; a
  // partly covered block runs every MFMA (rows and columns outside the
  // output are staged as zeros and their accumulators are never stored),
  // which keeps the step free of per-tile branches
  if (qm <= 0 || qn <= 0) return;
  v4s a[NP][MI], b[NP][NI];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
      a[q][mi] = *reinterpret_cast<const v4s *>(Ap[q] + (wm + 16 * mi + lr) * (C::TK + 8) + 4 * lk);
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
      b[q][ni] = *reinterpret_cast<const v4s *>(Bp[q] + (wn + 16 * ni + lr) * (C::TK + 8) + 4 * lk);
  }
  constexpr int H = 0, M = 1, Lo = NP - 1;  // part indices (M unused for NP = 2)
  const v4s z = {0, 0, 0, 0};
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      v4f c = acc[mi][ni];
      if constexpr (NP == 2) {
        c = mfma32(a[H][mi], a[Lo][mi], b[Lo][ni], b[H][ni], c);
        acc[mi][ni] = mfma32(a[H][mi], z, b[H][ni], z, c);
      } else {
        c = mfma32(a[H][mi], a[M][mi], b[Lo][ni], b[M][ni], c);
        c = mfma32(a[Lo][mi], a[H][mi], b[H][ni], b[M][ni], c);
        acc[mi][ni] = mfma32(a[M][mi], a[H][mi], b[H][ni], b[H][ni], c);
      }
    }
}

// Same tile walk as gemm_tile (FP32 data in HBM, FP32 accumulators and
// results); only the staging and the MFMA step differ.  NP BF16 parts per
// operand element, each in its own K-contiguous LDS array.
template <class C, int NP>
__device__ inline void gemm_tile_bfs(const GTile *__restrict__ tiles, const GOut *__restrict__ outs,
                                     const GSeg *__restrict__ segs, const Bases &bases) {
  constexpr int BM = C::BM, BN = C::BN, MI = C::MI, NI = C::NI, TK = C::TK;
  typedef SegLoadK<C> SL;
  __shared__ __attribute__((aligned(16))) StageA<C, NP> As[2];
  __shared__ __attribute__((aligned(16))) StageB<C, NP> Bs[2];
  const GTile tl = tiles[blockIdx.x];
  if (tl.out < 0) return;
  const GOut o = outs[tl.out];
  const int row0 = int(tl.ti) * BM, col0 = int(tl.tj) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / C::WX) * (BM / C::WY), wn = (wave % C::WX) * (BN / C::WX);
  const int lr = lane & 15, lk = lane >> 4;
  const int qm = o.m - (row0 + wm), qn = o.n - (col0 + wn);
  v4f acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = v4f{0, 0, 0, 0};
  SL L;
  float ra[SL::RA], rb[SL::RB];
  for (int si = 0; si < o.seg_count; ++si) {
    segk_setup(L, segs[o.seg_begin + si], bases, o, row0, col0, tid);
    const int nsteps = (L.k + TK - 1) / TK;
    if (nsteps == 0) continue;
    // double-buffered LDS, one step of register prefetch; steps 0 .. nsteps-2
    // are whole, the last one may end past K
    int buf = 0;
    segk_fetch<true>(L, 0, ra, rb);
    segk_store<C, NP>(L, 0, ra, rb, As[buf], Bs[buf]);
    __syncthreads();
    for (int step = 1; step + 1 < nsteps; ++step) {
      segk_fetch<false>(L, step, ra, rb);
      tile_mfma_bfs<C, NP>(As[buf], Bs[buf], wm, wn, lr, lk, qm, qn, acc);
      buf ^= 1;
      segk_store<C, NP>(L, step, ra, rb, As[buf], Bs[buf]);
      __syncthreads();
    }
    if (nsteps > 1) {
      segk_fetch<true>(L, nsteps - 1, ra, rb);
      tile_mfma_bfs<C, NP>(As[buf], Bs[buf], wm, wn, lr, lk, qm, qn, acc);
      buf ^= 1;
      segk_store<C, NP>(L, nsteps - 1, ra, rb, As[buf], Bs[buf]);
      __syncthreads();
    }
    tile_mfma_bfs<C, NP>(As[buf], Bs[buf], wm, wn, lr, lk, qm, qn, acc);
    __syncthreads();  // the next segment's first store reuses the stages
  }
  float *Cp = reinterpret_cast<float *>(bases.p[o.c_slot]) + o.c_off;
#pragma unroll
  for (int mi = 0; mi < MI; ++mi)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = row0 + wm + mi * 16 + Mfma<float>::row(lk, r);
        const int gj = col0 + wn + ni * 16 + lr;
        if (gi < o.m && gj < o.n) {
          float *p = Cp + (int64_t)gi * o.ldc + gj;
          const float v = acc[mi][ni][r];
          *p = o.accumulate ? (*p + v) : v;
        }
      }
}

template <class T, class C>
__device__ inline void gemm_any(const GTile *__restrict__ tiles, const GOut *__restrict__ outs,
                                const GSeg *__restrict__ segs, const Bases &bases) {
  if constexpr (std::is_same<T, Bf16x3>::value)
    gemm_tile_bfs<C, 2>(tiles, outs, segs, bases);
  else if constexpr (std::is_same<T, Bf16x6>::value)
    gemm_tile_bfs<C, 3>(tiles, outs, segs, bases);
  else
    gemm_tile<T, C>(tiles, outs, segs, bases);
}

template <class T>
__global__ __launch_bounds__(Cfg64<T>::NT) void k_gemm(const GTile *__restrict__ tiles, const GOut *__restrict__ outs,
                                                    const GSeg *__restrict__ segs, Bases bases) {
  gemm_any<T, Cfg64<T>>(tiles, outs, segs, bases);
}
template <class T>
__global__ __launch_bounds__(Cfg64w<T>::NT) void k_gemm_w16(const GTile *__restrict__ tiles,
                                                         const GOut *__restrict__ outs,
                                                         const GSeg *__restrict__ segs, Bases bases) {
  gemm_any<T, Cfg64w<T>>(tiles, outs, segs, bases);
}
template <class T>
__global__ __launch_bounds__(Cfg64q<T>::NT) void k_gemm_w4(const GTile *__restrict__ tiles, const GOut *__restrict__ outs,
                                                        const GSeg *__restrict__ segs, Bases bases) {
  gemm_any<T, Cfg64q<T>>(tiles, outs, segs, bases);
}

// 128x128 tiles: 116 (FP64), 90 (FP32), 114 (3xBF16) and 128 (6xBF16)
// registers per lane, 33 KB (FP64, FP32), 48 KB (3xBF16) and 72 KB (6xBF16)
// of LDS stages per workgroup; held at 4 waves per SIMD (two workgroups of
// 8 waves per CU).
template <class T>
__global__ __launch_bounds__(Cfg128<T>::NT) __attribute__((amdgpu_waves_per_eu(4))) void k_gemm_t128(const GTile *__restrict__ tiles,
                                                          const GOut *__restrict__ outs,
                                                          const GSeg *__restrict__ segs, Bases bases) {
  gemm_any<T, Cfg128<T>>(tiles, outs, segs, bases);
}

template <class T>
static void launch_variant(int v, hipStream_t st, const DevPlan *p, const Bases &b) {
  const dim3 g(unsigned(p->n_tiles));
  if (v == 3)
    hipLaunchKernelGGL(k_gemm_t128<T>, dim3(unsigned(p->n_tiles128)), dim3(Cfg128<T>::NT), 0, st, p->tiles128,
                       p->outs, p->segs, b);
  else if (v == 1)
    hipLaunchKernelGGL(k_gemm_w16<T>, g, dim3(Cfg64w<T>::NT), 0, st, p->tiles, p->outs, p->segs, b);
  else if (v == 2)
    hipLaunchKernelGGL(k_gemm_w4<T>, g, dim3(Cfg64q<T>::NT), 0, st, p->tiles, p->outs, p->segs, b);
  else
    hipLaunchKernelGGL(k_gemm<T>, g, dim3(Cfg64<T>::NT), 0, st, p->tiles, p->outs, p->segs, b);
}

// Range limits of the kernels' 32-bit element and tile arithmetic, checked
// on the host for every output and segment of a plan.
static void plan_check(const GemmPlan &plan) {
  // the kernels keep 32-bit offsets: element offsets inside an operand
  // block below 2^31, byte offsets inside one tile's K step below 2^30
  for (const GOut &o : plan.outs) {
    // tile origins and row / column indices inside the kernel are 32-bit
    MDMRG_REQUIRE(o.m >= 1 && o.n >= 1 && o.m < (1 << 30) && o.n < (1 << 30), -6,
                  "grouped GEMM: output block dimensions out of range");
    for (int q = 0; q < o.seg_count; ++q) {
      const GSeg &g = plan.segs[o.seg_begin + q];
      const int64_t ext_a = (g.flags & SEG_TA) ? int64_t(kTKmax) * g.lda + o.m : int64_t(o.m) * g.lda + kTKmax;
      const int64_t ext_b = (g.flags & SEG_TB) ? int64_t(o.n) * g.ldb + kTKmax : int64_t(kTKmax) * g.ldb + o.n;
      MDMRG_REQUIRE(ext_a < (int64_t(1) << 31) && ext_b < (int64_t(1) << 31), -6,
                    "grouped GEMM: operand block too large for 32-bit element offsets");
      // buffer-load byte offsets inside one tile's K step (128 x 128 tiles at
      // most, K steps of at most kTKmax, 8-byte elements) stay below 2^30,
      // under the buffer range
      const int64_t tile_a = (g.flags & SEG_TA) ? int64_t(kTKmax) * g.lda + 128 : int64_t(128) * g.lda + kTKmax;
      const int64_t tile_b = (g.flags & SEG_TB) ? int64_t(128) * g.ldb + kTKmax : int64_t(kTKmax) * g.ldb + 128;
      MDMRG_REQUIRE(8 * tile_a < (int64_t(1) << 30) && 8 * tile_b < (int64_t(1) << 30), -6,
                    "grouped GEMM: leading dimension too large for 32-bit tile offsets");
    }
  }
}

static double plan_flop(const GemmPlan &plan) {
  double f = 0.0;  // identity segments excluded
  for (const GOut &o : plan.outs)
    for (int q = 0; q < o.seg_count; ++q) {
      const GSeg &g = plan.segs[o.seg_begin + q];
      if (!(g.flags & SEG_AID)) f += 2.0 * o.m * o.n * g.k;
    }
  return f;
}

// Launch order of the tm x tn output tiles of a plan.  One launch covers
// every output, largest first (longest-processing-time order; small outputs
// fill the tail).  Workgroups of a launch go to the 8 XCDs round-robin
// (workgroup b to XCD b mod 8) and every XCD has its own L2, so outputs are
// cut into chunks of whole tile rows (at most chunk_tiles tiles: a few A
// panels against all B panels of the output), chunks are dealt to per-XCD
// queues (largest first, to the queue with the least work) and the queues
// interleaved: the tiles of a chunk run on one XCD and share its L2.  Queues
// are padded with empty tiles (out = -1).
static std::vector<GTile> plan_tiles(const GemmPlan &plan, int tm, int tn, int chunk_tiles) {
  std::vector<std::pair<double, int32_t>> work(plan.outs.size());
  for (size_t i = 0; i < plan.outs.size(); ++i) {
    const GOut &o = plan.outs[i];
    double kk = 0;
    for (int s = 0; s < o.seg_count; ++s) kk += plan.segs[o.seg_begin + s].k;
    work[i] = {-(kk + 16.0) * o.m * o.n, int32_t(i)};
  }
  std::stable_sort(work.begin(), work.end());
  std::vector<std::vector<GTile>> q(kXcds);
  double load[kXcds] = {};
  for (auto &w : work) {
    const GOut &o = plan.outs[w.second];
    const int nti = (o.m + tm - 1) / tm, ntj = (o.n + tn - 1) / tn;
    const int rows = std::max(1, chunk_tiles / ntj);
    for (int i0 = 0; i0 < nti; i0 += rows) {
      const int i1 = std::min(nti, i0 + rows);
      const int x = int(std::min_element(load, load + kXcds) - load);
      load[x] += -w.first * double(i1 - i0) / nti;
      for (int i = i0; i < i1; ++i)
        for (int j = 0; j < ntj; ++j) q[x].push_back(GTile{w.second, int32_t(i), int32_t(j)});
    }
  }
  size_t maxq = 0;
  for (auto &qq : q) maxq = std::max(maxq, qq.size());
  std::vector<GTile> tiles;
  for (size_t u = 0; u < maxq; ++u)
    for (auto &qq : q) tiles.push_back(u < qq.size() ? qq[u] : GTile{-1, 0, 0});
  while (!tiles.empty() && tiles.back().out < 0) tiles.pop_back();  // trailing empty workgroups are not launched
  MDMRG_REQUIRE(tiles.size() < (size_t(1) << 31), -6, "grouped GEMM plan has too many tiles");
  return tiles;
}

DevPlan *dev_plan_upload(Device *d, const GemmPlan &plan) {
  plan_check(plan);
  auto *dp = new DevPlan();
  dp->n_outs = int64_t(plan.outs.size());
  dp->n_segs = int64_t(plan.segs.size());
  dp->flop = plan_flop(plan);  // algorithmic FLOP of the launch
  const std::vector<GTile> tiles = plan_tiles(plan, kTileM, kTileN, 64), tiles128 = plan_tiles(plan, 128, 128, 16);
  dp->n_tiles = int64_t(tiles.size());
  dp->n_tiles128 = int64_t(tiles128.size());
  if (dp->n_tiles) {
    dp->segs = (GSeg *)dev_alloc(d, sizeof(GSeg) * std::max<size_t>(1, plan.segs.size()));
    dp->outs = (GOut *)dev_alloc(d, sizeof(GOut) * plan.outs.size());
    dp->tiles = (GTile *)dev_alloc(d, sizeof(GTile) * tiles.size());
    dp->tiles128 = (GTile *)dev_alloc(d, sizeof(GTile) * tiles128.size());
    if (!plan.segs.empty()) dev_h2d(d, dp->segs, plan.segs.data(), sizeof(GSeg) * plan.segs.size());
    dev_h2d(d, dp->outs, plan.outs.data(), sizeof(GOut) * plan.outs.size());
    dev_h2d(d, dp->tiles, tiles.data(), sizeof(GTile) * tiles.size());
    dev_h2d(d, dp->tiles128, tiles128.data(), sizeof(GTile) * tiles128.size());
  }
  return dp;
}

void dev_plan_free(Device *d, DevPlan *p) {
  if (!p) return;
  for (auto &evs : p->trial_ev)
    for (void *e : evs)
      if (e) d->ev_pool.push_back(static_cast<hipEvent_t>(e));
  dev_free(d, p->segs);
  dev_free(d, p->outs);
  dev_free(d, p->tiles);
  dev_free(d, p->tiles128);
  delete p;
}

void dev_force_variant(Device *d, int v) { d->force_variant = v; }

void dev_gemm_run(Device *d, DevPlan *p, const Bases &b, int tag, int prec) {
  if (!p || p->n_tiles == 0) return;
  if (tag <= 0 || tag >= kTags) tag = 6;  // untagged launches are timed as "other"
  // autotuner: the first kGemmVariants launches of a plan (per element type)
  // run one variant each (they are the plan's real work) and are timed with
  // their own events; the next launch reads the times and keeps the fastest
  MDMRG_REQUIRE(prec >= 0 && prec < kPrecs, -6, "grouped GEMM: unknown precision form");
  const int pr = prec;
  int v = d->force_variant >= 0 ? d->force_variant : p->variant[pr];
  if (!d->capturing && v < 0) {
    if (p->trials[pr] < kGemmVariants) {
      v = p->trials[pr];
    } else {
      void **ev = p->trial_ev[pr];
      HIP_CHECK(hipEventSynchronize(static_cast<hipEvent_t>(ev[2 * kGemmVariants - 1])));
      float best = 0.f;
      for (int q = 0; q < kGemmVariants; ++q) {
        float t = 0.f;
        HIP_CHECK(hipEventElapsedTime(&t, static_cast<hipEvent_t>(ev[2 * q]), static_cast<hipEvent_t>(ev[2 * q + 1])));
        p->trial_ms[pr][q] = t;
        if (q == 0 || t < best) {
          best = t;
          v = q;
        }
      }
      for (int q = 0; q < 2 * kGemmVariants; ++q) {
        d->ev_pool.push_back(static_cast<hipEvent_t>(ev[q]));
        ev[q] = nullptr;
      }
      p->variant[pr] = v;
    }
  }
  if (v < 0) v = 0;  // captured before the plan was tuned
  const bool trial = !d->capturing && d->force_variant < 0 && p->variant[pr] < 0;
  const bool timed = d->timing && !d->capturing;
  hipEvent_t e0 = nullptr, e1 = nullptr, t0 = nullptr, t1 = nullptr;
  if (timed) {
    if (d->pending.size() > 512) timing_drain(d);
    e0 = ev_get(d);
    e1 = ev_get(d);
    HIP_CHECK(hipEventRecord(e0, d->stream));
  }
  if (trial) {
    t0 = ev_get(d);
    t1 = ev_get(d);
    HIP_CHECK(hipEventRecord(t0, d->stream));
  }
  if (prec == 0)
    launch_variant<double>(v, d->stream, p, b);
  else if (prec == 1)
    launch_variant<float>(v, d->stream, p, b);
  else if (prec == 2)
    launch_variant<Bf16x3>(v, d->stream, p, b);
  else
    launch_variant<Bf16x6>(v, d->stream, p, b);
  HIP_CHECK(hipGetLastError());
  if (trial) {
    HIP_CHECK(hipEventRecord(t1, d->stream));
    p->trial_ev[pr][2 * p->trials[pr]] = t0;
    p->trial_ev[pr][2 * p->trials[pr] + 1] = t1;
    p->trials[pr] += 1;
  }
  if (timed) {
    HIP_CHECK(hipEventRecord(e1, d->stream));
    d->pending.push_back(Device::Pending{tag, prec, v, e0, e1, p->flop});
  }
}

// Allocation-free form of dev_plan_upload + dev_gemm_run: the descriptors
// and the tile list are copied into this device's static staging array
// (kNoAllocStagingBytes) instead of allocations; the launch uses the forced
// tile variant, else k_gemm_w4 (no autotuning trials, no timing events).
// Waits for the launch, so the staging array is free again on return.  Calls
// that overlap on one device (two host threads, or contexts on different
// streams) race on the array.
void dev_gemm_run_noalloc(Device *d, const GemmPlan &plan, const Bases &b) {
  plan_check(plan);
  const int v = d->force_variant >= 0 ? d->force_variant : 2;
  const std::vector<GTile> tiles = plan_tiles(plan, v == 3 ? 128 : kTileM, v == 3 ? 128 : kTileN, v == 3 ? 16 : 64);
  if (tiles.empty()) return;
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t b_segs = sizeof(GSeg) * std::max<size_t>(1, plan.segs.size());
  const size_t b_outs = sizeof(GOut) * plan.outs.size(), b_tiles = sizeof(GTile) * tiles.size();
  const size_t need = up(b_segs) + up(b_outs) + up(b_tiles);
  if (need > kNoAllocStagingBytes)
    throw Error(-1, "gemm_grouped_noalloc: the plan needs " + std::to_string(need) +
                        " bytes of descriptors and tiles, above the static staging limit of " +
                        std::to_string(kNoAllocStagingBytes) + " bytes");
  MDMRG_REQUIRE(d->staging != nullptr, -4, "gemm_grouped_noalloc: no staging address for this device");
  DevPlan p;
  p.segs = reinterpret_cast<GSeg *>(d->staging);
  p.outs = reinterpret_cast<GOut *>(d->staging + up(b_segs));
  GTile *t = reinterpret_cast<GTile *>(d->staging + up(b_segs) + up(b_outs));
  (v == 3 ? p.tiles128 : p.tiles) = t;
  p.n_outs = int64_t(plan.outs.size());
  p.n_segs = int64_t(plan.segs.size());
  (v == 3 ? p.n_tiles128 : p.n_tiles) = int64_t(tiles.size());
  if (!plan.segs.empty()) dev_h2d(d, p.segs, plan.segs.data(), sizeof(GSeg) * plan.segs.size());
  dev_h2d(d, p.outs, plan.outs.data(), b_outs);
  dev_h2d(d, t, tiles.data(), b_tiles);
  launch_variant<double>(v, d->stream, &p, b);
  HIP_CHECK(hipGetLastError());
  // the host descriptor vectors and the staging array stay in use until here
  dev_sync(d);
}

// ------------------------------------------------------------ graph capture
struct DevGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
void dev_capture_begin(Device *d) {
  MDMRG_REQUIRE(!d->capturing, -4, "stream capture already in progress");
  HIP_CHECK(hipStreamBeginCapture(d->stream, hipStreamCaptureModeThreadLocal));
  d->capturing = true;
}
DevGraph *dev_capture_end(Device *d) {
  MDMRG_REQUIRE(d->capturing, -4, "no stream capture in progress");
  auto *g = new DevGraph();
  d->capturing = false;
  HIP_CHECK(hipStreamEndCapture(d->stream, &g->graph));
  HIP_CHECK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  return g;
}
void dev_capture_abort(Device *d) {
  if (!d->capturing) return;
  d->capturing = false;
  hipGraph_t g = nullptr;
  (void)hipStreamEndCapture(d->stream, &g);
  if (g) (void)hipGraphDestroy(g);
}
void dev_graph_launch(Device *d, DevGraph *g, int tag, double flop) {
  const bool timed = d->timing;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    if (d->pending.size() > 512) timing_drain(d);
    e0 = ev_get(d);
    e1 = ev_get(d);
    HIP_CHECK(hipEventRecord(e0, d->stream));
  }
  HIP_CHECK(hipGraphLaunch(g->exec, d->stream));
  if (timed) {
    HIP_CHECK(hipEventRecord(e1, d->stream));
    d->pending.push_back(Device::Pending{tag, 0, -1, e0, e1, flop});
  }
}
void dev_graph_free(Device *d, DevGraph *g) {
  if (!g) return;
  (void)d;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

// ------------------------------------------------------ split-K reduction
template <class T>
__global__ void k_reduce(const int64_t *__restrict__ off, const int32_t *__restrict__ len, int n_split,
                         int64_t stride, const T *__restrict__ P, T *__restrict__ y) {
  const int64_t o = off[blockIdx.y];
  const int n = len[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    T s = y[o + i];
    for (int q = 0; q < n_split; ++q) s += P[q * stride + o + i];
    y[o + i] = s;
  }
}
DevReduce *dev_reduce_upload(Device *d, const std::vector<int64_t> &off, const std::vector<int32_t> &len,
                             int n_split, int64_t stride) {
  auto *r = new DevReduce();
  r->n_blk = int64_t(off.size());
  r->n_split = n_split;
  r->stride = stride;
  for (int32_t l : len) r->max_len = std::max<int64_t>(r->max_len, l);
  if (r->n_blk) {
    r->off = (int64_t *)dev_alloc(d, sizeof(int64_t) * off.size());
    r->len = (int32_t *)dev_alloc(d, sizeof(int32_t) * len.size());
    dev_h2d(d, r->off, off.data(), sizeof(int64_t) * off.size());
    dev_h2d(d, r->len, len.data(), sizeof(int32_t) * len.size());
  }
  return r;
}
void dev_reduce_free(Device *d, DevReduce *r) {
  if (!r) return;
  dev_free(d, r->off);
  dev_free(d, r->len);
  delete r;
}
void dev_reduce_run(Device *d, const DevReduce *r, const double *P, double *y, int prec) {
  if (!r || r->n_blk == 0) return;
  MDMRG_REQUIRE(r->n_blk < 65536, -6, "split-K reduction: too many blocks for one launch");
  const unsigned gx = unsigned(std::min<int64_t>((r->max_len + 255) / 256, 64));
  if (prec == 0)
    hipLaunchKernelGGL(k_reduce<double>, dim3(gx, unsigned(r->n_blk)), dim3(256), 0, d->stream, r->off, r->len,
                       r->n_split, r->stride, P, y);
  else
    hipLaunchKernelGGL(k_reduce<float>, dim3(gx, unsigned(r->n_blk)), dim3(256), 0, d->stream, r->off, r->len,
                       r->n_split, r->stride, reinterpret_cast<const float *>(P), reinterpret_cast<float *>(y));
  HIP_CHECK(hipGetLastError());
}

// --------------------------------------------------------- precision casts
__global__ void k_d2f(const double *__restrict__ x, float *__restrict__ y, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] = float(x[k]);
}
__global__ void k_f2d(const float *__restrict__ x, double *__restrict__ y, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] = double(x[k]);
}
void dev_d2f(Device *d, const double *x, float *y, int64_t n) {
  int grid = int(std::min<int64_t>((n + 255) / 256, 8192));
  if (grid < 1) return;
  hipLaunchKernelGGL(k_d2f, dim3(grid), dim3(256), 0, d->stream, x, y, n);
  HIP_CHECK(hipGetLastError());
}
void dev_f2d(Device *d, const float *x, double *y, int64_t n) {
  int grid = int(std::min<int64_t>((n + 255) / 256, 8192));
  if (grid < 1) return;
  hipLaunchKernelGGL(k_f2d, dim3(grid), dim3(256), 0, d->stream, x, y, n);
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------- diagonal of H_eff
__global__ void k_diag(const DiagTask *__restrict__ tasks, const int32_t *__restrict__ beg,
                       const int64_t *__restrict__ off, const int32_t *__restrict__ bm,
                       const int32_t *__restrict__ bn, Bases bases, double *__restrict__ d) {
  const int b = blockIdx.x;
  const int m = bm[b], n = bn[b];
  double *D = d + off[b];
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int t = beg[b]; t < beg[b + 1]; ++t) {
      const DiagTask tk = tasks[t];
      const double l = tk.l_id ? 1.0 : bases.p[tk.l_slot][tk.l_off + (int64_t)i * tk.ls];
      const double r = tk.r_id ? 1.0 : bases.p[tk.r_slot][tk.r_off + (int64_t)j * tk.rs];
      s += tk.alpha * l * r;
    }
    D[e] = s;
  }
}

DevDiag *dev_diag_upload(Device *d, const std::vector<DiagTask> &tasks, const std::vector<int64_t> &blk_off,
                         const std::vector<int32_t> &blk_m, const std::vector<int32_t> &blk_n) {
  // tasks must be grouped by output block (d_off order matches blk_off)
  auto *dd = new DevDiag();
  const int64_t nb = int64_t(blk_off.size());
  std::vector<int32_t> beg(nb + 1, 0);
  std::unordered_map<int64_t, int> bidx;
  for (int64_t i = 0; i < nb; ++i) bidx[blk_off[i]] = int(i);
  std::vector<std::vector<DiagTask>> per(nb);
  for (auto &t : tasks) per[bidx.at(t.d_off)].push_back(t);
  std::vector<DiagTask> flat;
  for (int64_t i = 0; i < nb; ++i) {
    beg[i] = int32_t(flat.size());
    flat.insert(flat.end(), per[i].begin(), per[i].end());
  }
  beg[nb] = int32_t(flat.size());
  dd->n_tasks = int64_t(flat.size());
  dd->n_blk = nb;
  dd->tasks = (DiagTask *)dev_alloc(d, sizeof(DiagTask) * std::max<size_t>(1, flat.size()));
  dd->blk_begin = (int32_t *)dev_alloc(d, sizeof(int32_t) * (nb + 1));
  dd->blk_off = (int64_t *)dev_alloc(d, sizeof(int64_t) * std::max<int64_t>(1, nb));
  dd->blk_m = (int32_t *)dev_alloc(d, sizeof(int32_t) * std::max<int64_t>(1, nb));
  dd->blk_n = (int32_t *)dev_alloc(d, sizeof(int32_t) * std::max<int64_t>(1, nb));
  if (!flat.empty()) dev_h2d(d, dd->tasks, flat.data(), sizeof(DiagTask) * flat.size());
  dev_h2d(d, dd->blk_begin, beg.data(), sizeof(int32_t) * (nb + 1));
  if (nb) {
    dev_h2d(d, dd->blk_off, blk_off.data(), sizeof(int64_t) * nb);
    dev_h2d(d, dd->blk_m, blk_m.data(), sizeof(int32_t) * nb);
    dev_h2d(d, dd->blk_n, blk_n.data(), sizeof(int32_t) * nb);
  }
  return dd;
}

void dev_diag_free(Device *d, DevDiag *p) {
  if (!p) return;
  dev_free(d, p->tasks);
  dev_free(d, p->blk_begin);
  dev_free(d, p->blk_off);
  dev_free(d, p->blk_m);
  dev_free(d, p->blk_n);
  delete p;
}

void dev_diag_run(Device *d, const DevDiag *p, const Bases &b, double *out) {
  if (!p || p->n_blk == 0) return;
  hipLaunchKernelGGL(k_diag, dim3(unsigned(p->n_blk)), dim3(256), 0, d->stream, p->tasks, p->blk_begin, p->blk_off,
                     p->blk_m, p->blk_n, b, out);
  HIP_CHECK(hipGetLastError());
}

// -------------------------------------------------- FP64 vector primitives
__device__ inline double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(256) void k_multidot_partial(const double *__restrict__ V, int64_t ldv,
                                                          const double *__restrict__ x, int64_t n,
                                                          double *__restrict__ part) {
  __shared__ double sh[256];
  const int y = blockIdx.y;
  const double *v = V + (int64_t)y * ldv;
  double s = 0.0;
  for (int64_t k = blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) s += v[k] * x[k];
  const double r = block_sum(s, sh);
  if (threadIdx.x == 0) part[y * gridDim.x + blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_multidot_final(const double *__restrict__ part, int nb,
                                                        double *__restrict__ out) {
  __shared__ double sh[256];
  const int y = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[y * nb + i];
  const double r = block_sum(s, sh);
  if (threadIdx.x == 0) out[y] = r;
}

void dev_multidot(Device *d, const double *V, int64_t ldv, int m, const double *x, int64_t n, double *out_host) {
  MDMRG_REQUIRE(m >= 0 && m <= kMaxDot, -1, "multidot: too many vectors");
  if (m == 0) return;
  hipLaunchKernelGGL(k_multidot_partial, dim3(kRedBlocks, m), dim3(256), 0, d->stream, V, ldv, x, n, d->red);
  hipLaunchKernelGGL(k_multidot_final, dim3(m), dim3(256), 0, d->stream, d->red, kRedBlocks, d->red_out);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipMemcpyAsync(d->host_red, d->red_out, sizeof(double) * m, hipMemcpyDeviceToHost, d->stream));
  HIP_CHECK(hipStreamSynchronize(d->stream));
  std::memcpy(out_host, d->host_red, sizeof(double) * m);
}

struct Coefs {
  double c[kMaxDot];
};
__global__ void k_lincomb(const double *__restrict__ V, int64_t ldv, int m, Coefs c, double beta,
                          double *__restrict__ y, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double s = (beta == 0.0) ? 0.0 : beta * y[k];
    for (int i = 0; i < m; ++i) s += c.c[i] * V[(int64_t)i * ldv + k];
    y[k] = s;
  }
}
void dev_lincomb(Device *d, const double *V, int64_t ldv, int m, const double *c_host, double beta, double *y,
                 int64_t n) {
  MDMRG_REQUIRE(m >= 0 && m <= kMaxDot, -1, "lincomb: too many vectors");
  Coefs c{};
  for (int i = 0; i < m; ++i) c.c[i] = c_host[i];
  int grid = int(std::min<int64_t>((n + 255) / 256, 8192));
  if (grid < 1) return;
  hipLaunchKernelGGL(k_lincomb, dim3(grid), dim3(256), 0, d->stream, V, ldv, m, c, beta, y, n);
  HIP_CHECK(hipGetLastError());
}

__global__ void k_axpy(double a, const double *__restrict__ x, double *__restrict__ y, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    y[k] += a * x[k];
}
void dev_axpy(Device *d, double a, const double *x, double *y, int64_t n) {
  int grid = int(std::min<int64_t>((n + 255) / 256, 8192));
  if (grid < 1) return;
  hipLaunchKernelGGL(k_axpy, dim3(grid), dim3(256), 0, d->stream, a, x, y, n);
  HIP_CHECK(hipGetLastError());
}
__global__ void k_scale(double a, double *__restrict__ x, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    x[k] *= a;
}
void dev_scale(Device *d, double a, double *x, int64_t n) {
  int grid = int(std::min<int64_t>((n + 255) / 256, 8192));
  if (grid < 1) return;
  hipLaunchKernelGGL(k_scale, dim3(grid), dim3(256), 0, d->stream, a, x, n);
  HIP_CHECK(hipGetLastError());
}
__global__ void k_precond(const double *__restrict__ r, const double *__restrict__ dg, double theta, double eps,
                          double *__restrict__ t, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    double den = theta - dg[k];
    if (fabs(den) < eps) den = (den < 0.0) ? -eps : eps;
    t[k] = r[k] / den;
  }
}
void dev_precond(Device *d, const double *r, const double *dg, double theta, double eps, double *t, int64_t n) {
  int grid = int(std::min<int64_t>((n + 255) / 256, 8192));
  if (grid < 1) return;
  hipLaunchKernelGGL(k_precond, dim3(grid), dim3(256), 0, d->stream, r, dg, theta, eps, t, n);
  HIP_CHECK(hipGetLastError());
}

// splitmix64 (Steele, Lea, Flood 2014) as a counter-based generator,
// Box-Muller to N(0,1).
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_randn(double *x, int64_t n, uint64_t seed) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t base = seed * 0x2545F4914F6CDD1Dull + 2 * (uint64_t)k;
    const double u1 = ((splitmix64(base) >> 11) + 1) * (1.0 / 9007199254740993.0);
    const double u2 = (splitmix64(base + 1) >> 11) * (1.0 / 9007199254740992.0);
    x[k] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}
void dev_randn(Device *d, double *x, int64_t n, uint64_t seed) {
  int grid = int(std::min<int64_t>((n + 255) / 256, 8192));
  if (grid < 1) return;
  hipLaunchKernelGGL(k_randn, dim3(grid), dim3(256), 0, d->stream, x, n, seed);
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------- eigensolver
void dev_syevd(Device *d, double *A, int n, double *w) {
  if (n <= 0) return;
  if (d->syevd_work_n < size_t(n)) {
    if (d->syevd_work) HIP_CHECK(hipFree(d->syevd_work));
    HIP_CHECK(hipMalloc(&d->syevd_work, sizeof(double) * n));
    d->syevd_work_n = size_t(n);
  }
  rocblas_status st = rocsolver_dsyevd(d->blas, rocblas_evect_original, rocblas_fill_upper, n, A, n, w,
                                       d->syevd_work, d->info);
  MDMRG_REQUIRE(st == rocblas_status_success, -3, "rocsolver_dsyevd failed");
  int info = 0;
  HIP_CHECK(hipMemcpyAsync(&info, d->info, sizeof(int), hipMemcpyDeviceToHost, d->stream));
  HIP_CHECK(hipStreamSynchronize(d->stream));
  MDMRG_REQUIRE(info == 0, -3, "rocsolver_dsyevd did not converge (info " + std::to_string(info) + ")");
}

// ------------------------------------------------------------------ gather
__global__ void k_gather(const GatherBlk *__restrict__ blks, const int32_t *__restrict__ cols,
                         const double *__restrict__ E, double *__restrict__ out, int transpose_out) {
  const GatherBlk g = blks[blockIdx.x];
  const int total = g.rows * g.ncol;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = e / g.ncol, j = e % g.ncol;
    const double v = E[g.e_off + (int64_t)cols[g.col_begin + j] * g.ldE + g.row0 + i];
    if (transpose_out)
      out[g.out_off + (int64_t)j * g.rows + i] = v;
    else
      out[g.out_off + (int64_t)i * g.ncol + j] = v;
  }
}
void dev_gather(Device *d, const std::vector<GatherBlk> &blks, const std::vector<int32_t> &cols, const double *E,
                double *out, bool transpose_out) {
  if (blks.empty()) return;
  auto *db = (GatherBlk *)dev_alloc(d, sizeof(GatherBlk) * blks.size());
  auto *dc = (int32_t *)dev_alloc(d, sizeof(int32_t) * std::max<size_t>(1, cols.size()));
  dev_h2d(d, db, blks.data(), sizeof(GatherBlk) * blks.size());
  if (!cols.empty()) dev_h2d(d, dc, cols.data(), sizeof(int32_t) * cols.size());
  hipLaunchKernelGGL(k_gather, dim3(unsigned(blks.size())), dim3(256), 0, d->stream, db, dc, E, out,
                     transpose_out ? 1 : 0);
  HIP_CHECK(hipGetLastError());
  dev_free(d, db);
  dev_free(d, dc);
}

}  // namespace mdmrg
