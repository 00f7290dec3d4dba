// HIP kernels of libbbp for gfx950 (MI355X): the split-layer fit visit of
// block BP (App. A of Guo, Poletti, Arad), Householder QR/LQ, and the small
// gather / extract / normalise / overlap steps around it.
//
// Every MPS site lives in a zero-padded slot of S = K*P*K doubles (K the
// bond cap, P = D^2 the fused double-layer leg), so all contractions of a
// batch have the same shape; zero padding stays exactly zero through every
// contraction, and the QR works on the true panel only.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "bbp_internal.h"

namespace bbp {

// ---------------------------------------------------------------------------
// Launch timing
// ---------------------------------------------------------------------------
namespace {
struct TimedLaunch {
  int cls;
  hipEvent_t a, b;
  double flops, bytes, pflops, pbytes;
};
// Launch timing is process-wide; its lists are guarded so contexts used from
// several host threads (the request server) can time concurrently.
struct TimingState {
  std::atomic<bool> on{false};
  std::recursive_mutex mu;
  std::vector<TimedLaunch> done;
  std::vector<hipEvent_t> pool;
  long long launches[KC_COUNT] = {};
  double ms[KC_COUNT] = {}, flops[KC_COUNT] = {}, bytes[KC_COUNT] = {};
  double pflops[KC_COUNT] = {}, pbytes[KC_COUNT] = {};
};
TimingState &timing() {
  static TimingState t;
  return t;
}
hipEvent_t take_event() {
  TimingState &t = timing();
  std::lock_guard<std::recursive_mutex> lk(t.mu);
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
// Folds completed event pairs into the per-class totals.
hipError_t drain() {
  TimingState &t = timing();
  std::lock_guard<std::recursive_mutex> lk(t.mu);
  for (TimedLaunch &l : t.done) {
    hipError_t e = hipEventSynchronize(l.b);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, l.a, l.b);
    if (e != hipSuccess) return e;
    t.launches[l.cls] += 1;
    t.ms[l.cls] += ms;
    t.flops[l.cls] += l.flops;
    t.bytes[l.cls] += l.bytes;
    t.pflops[l.cls] += l.pflops;
    t.pbytes[l.cls] += l.pbytes;
    t.pool.push_back(l.a);
    t.pool.push_back(l.b);
  }
  t.done.clear();
  return hipSuccess;
}
// Brackets one launch with events when timing is on.  f, b: algorithmic
// counts on the true extents; pf, pb: padded counts and the kernel's own
// byte traffic (the same as f, b where a launch has no padding).
struct Span {
  int cls;
  hipStream_t st;
  double flops, bytes, pflops, pbytes;
  hipEvent_t a = nullptr;
  Span(int c, hipStream_t s, double f, double b, double pf = -1.0, double pb = -1.0)
      : cls(c), st(s), flops(f), bytes(b), pflops(pf < 0 ? f : pf), pbytes(pb < 0 ? b : pb) {
    if (!timing().on) return;
    std::lock_guard<std::recursive_mutex> lk(timing().mu);
    if (timing().done.size() > 4096) (void)drain();
    a = take_event();
    if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;
  }
  ~Span() {
    if (!a) return;
    std::lock_guard<std::recursive_mutex> lk(timing().mu);
    hipEvent_t b = take_event();
    if (b && hipEventRecord(b, st) == hipSuccess)
      timing().done.push_back(TimedLaunch{cls, a, b, flops, bytes, pflops, pbytes});
  }
};
const char *kClassNames[KC_COUNT] = {"fit_visit", "fit_T1",  "fit_ket",
                                     "fit_bra",   "fit_local", "fit_env",
                                     "fit_end",   "qr",       "other"};
}  // namespace

void timing_enable(bool on) { timing().on = on; }
bool timing_enabled() { return timing().on; }
void timing_reset() {
  TimingState &t = timing();
  std::lock_guard<std::recursive_mutex> lk(t.mu);
  (void)drain();
  for (int i = 0; i < KC_COUNT; ++i) {
    t.launches[i] = 0;
    t.ms[i] = t.flops[i] = t.bytes[i] = t.pflops[i] = t.pbytes[i] = 0.0;
  }
}
hipError_t timing_query(int cls, const char **name, long long *launches,
                        double *ms, double *flops, double *bytes, double *pflops,
                        double *pbytes) {
  TimingState &t = timing();
  std::lock_guard<std::recursive_mutex> lk(t.mu);
  hipError_t e = drain();
  if (e != hipSuccess) return e;
  if (name) *name = kClassNames[cls];
  if (launches) *launches = t.launches[cls];
  if (ms) *ms = t.ms[cls];
  if (flops) *flops = t.flops[cls];
  if (bytes) *bytes = t.bytes[cls];
  if (pflops) *pflops = t.pflops[cls];
  if (pbytes) *pbytes = t.pbytes[cls];
  return hipSuccess;
}

namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// Batched FP64 GEMM engine.  C(it, m, n) = sum_k A(it, m, k) B(it, k, n) for
// the items of a batch (blockIdx.z).  The operand and result index maps are
// supplied by an op struct (a(), b(), st()); each workgroup stages BK-deep
// slices of A and B in LDS and 16 x 16 threads accumulate TM x TN tiles.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));

// LDS row strides that keep the MFMA operand reads free of bank conflicts
// (64-bit words, 32 word pairs per bank row; a read serves 16 lanes along the
// tile and 2 lane groups along k together): a row that the 16 lanes walk as
// the A operand gets a stride of 2 (mod 32), a row that 2 lane groups walk as
// the B operand a stride of 16 (mod 32).
__host__ __device__ constexpr int pad_a(int x) { return x + (34 - x % 32) % 32; }
__host__ __device__ constexpr int pad_b(int x) { return x + (48 - x % 32) % 32; }

__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Device global memory seen through a pointer whose origin the compiler
// cannot trace (taken from a pointer table or a struct member): accesses
// through the returned pointer are global loads and stores, not flat ones,
// which would also count against the LDS wait counter.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}

// Loads and stores through a buffer descriptor: the base lives in SGPRs and
// each lane supplies a 32-bit byte offset, so a loop keeps one 32-bit offset
// per element instead of a 64-bit address.  Descriptor word 3 selects the
// 32-bit data format, which untyped buffer accesses on this GPU family
// require.  The hardware checks every offset against the `bytes` declared: a
// load at or beyond it returns zero and a store there is dropped; the visit
// and the environment update load the elements outside their operands that
// way (offset `bytes`).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const double *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const float *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}
template <class T>
__device__ __forceinline__ void buf_st_t(__amdgpu_buffer_rsrc_t r, unsigned byte_off, T v);
template <>
__device__ __forceinline__ void buf_st_t<double>(__amdgpu_buffer_rsrc_t r, unsigned o, double v) {
  typedef unsigned int v2u __attribute__((__vector_size__(8)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, o, 0, 0);
}
template <>
__device__ __forceinline__ void buf_st_t<float>(__amdgpu_buffer_rsrc_t r, unsigned o, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, o, 0, 0);
}
template <class T> __device__ __forceinline__ T buf_ld_t(__amdgpu_buffer_rsrc_t r, unsigned byte_off);
template <> __device__ __forceinline__ double buf_ld_t<double>(__amdgpu_buffer_rsrc_t r, unsigned o) {
  return buf_ld(r, o);
}
template <> __device__ __forceinline__ float buf_ld_t<float>(__amdgpu_buffer_rsrc_t r, unsigned o) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
}

// Workgroups are dealt to the 8 XCDs round-robin by linear id, and each XCD
// has its own L2.  For a (tile, item) grid this returns the tile and item of
// the calling workgroup such that every tile of item i < 8 floor(items / 8)
// runs on XCD i % 8 (an item's shared operands stay in one L2); the items
// beyond follow in plain order.
__device__ __forceinline__ void xcd_tile_item(int *tile, int *item) {
  constexpr int kXcds = 8;
  const int nx = gridDim.x, ny = gridDim.y, ny8 = ny - ny % kXcds;
  const int w = blockIdx.x + nx * blockIdx.y;
  if (w >= nx * ny8) {
    *item = ny8 + (w - nx * ny8) / nx;
    *tile = (w - nx * ny8) % nx;
    return;
  }
  const int xcd = w % kXcds, slot = w / kXcds;
  *item = (slot / nx) * kXcds + xcd;
  *tile = slot % nx;
}

// Orders one wave's LDS writes before its later LDS reads (other lanes).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Contraction type of the specialised kernels: FP64, or FP32 on FP32 MFMA
// with FP32 accumulation (the precision option).  LDS stride residues for
// 4-byte words: A-operand rows 4 (mod 64), B-operand rows 16 (mod 64).
typedef float v4f __attribute__((ext_vector_type(4)));
template <class T> struct Mma;
// crow(r, lq): tile row held by accumulator register r of a lane in row
// group lq (FP64 MFMA: 4r + lq; FP32 16x16x4 MFMA: 4lq + r, as probed).
template <> struct Mma<double> {
  typedef v4d acc;
  static __device__ __forceinline__ int crow(int r, int lq) { return 4 * r + lq; }
  static __device__ __forceinline__ v4d run(double a, double b, v4d c) { return mfma16(a, b, c); }
  static __host__ __device__ constexpr int pad_a(int x) { return bbp::pad_a(x); }
  static __host__ __device__ constexpr int pad_b(int x) { return bbp::pad_b(x); }
  // smallest A-operand row stride >= x whose 16 rows x 2 lane groups of a
  // half wave fall in distinct banks: any stride = 2 (mod 4)
  static __host__ __device__ constexpr int pad_a_min(int x) { return x + (6 - x % 4) % 4; }
};
template <> struct Mma<float> {
  typedef v4f acc;
  static __device__ __forceinline__ int crow(int r, int lq) { return 4 * lq + r; }
  static __device__ __forceinline__ v4f run(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __host__ __device__ constexpr int pad_a(int x) { return x + (68 - x % 64) % 64; }
  static __host__ __device__ constexpr int pad_b(int x) { return x + (80 - x % 64) % 64; }
  static __host__ __device__ constexpr int pad_a_min(int x) { return x + (12 - x % 8) % 8; }
};

// BF16 contraction step (the precision option's lowest stage): FP32 operands
// rounded to BF16 (nearest even), BF16 MFMA 16x16x16 with FP32 accumulation.
// Each lane supplies four k values of its A row and B column; the product
// sums over the 16 (lane group, slot) pairs, so any assignment of k values
// to slots is valid as long as A and B use the same one.  The accumulator
// layout is that of the FP32 MFMA (Mma<float>::crow).
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4f mfma_bf16(const float *a, const float *b, v4f c) {
  v4bf x, y;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x[j] = (__bf16)a[j];
    y[j] = (__bf16)b[j];
  }
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, x),
                                                   __builtin_bit_cast(v4s, y), c, 0, 0, 0);
}

template <int BM, int BN, int BK, class Op>
__global__ __launch_bounds__(kThreads) void k_gemm(Op op) {
  const int it = blockIdx.z;
  if (op.flag && !op.flag[it]) return;
  // 16 x 16 MFMA tiles of the BM x BN block, spread over the four waves
  constexpr int TMX = BM / 16, TNX = BN / 16, NT = TMX * TNX;
  constexpr int TPW = (NT + 3) / 4;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  v4d acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < op.Kd; k0 += BK) {
    for (int i = tid; i < BM * BK; i += kThreads) {
      const int kk = i % BK, mm = i / BK;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < op.M && k < op.Kd) ? op.a(it, m, k) : 0.0;
    }
    for (int i = tid; i < BK * BN; i += kThreads) {
      const int nn = i % BN, kk = i / BN;
      const int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < op.N && k < op.Kd) ? op.b(it, k, n) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wave + 4 * q;
      if (t < NT) {
        const int tm = (t / TNX) * 16, tn = (t % TNX) * 16;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4)
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              As[kk + lq][tm + lr], Bs[kk + lq][tn + lr], acc[q], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wave + 4 * q;
    if (t < NT) {
      const int tm = (t / TNX) * 16, tn = (t % TNX) * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + tm + 4 * r + lq, n = n0 + tn + lr;
        if (m < op.M && n < op.N) op.st(it, m, n, acc[q][r]);
      }
    }
  }
}

template <int BM, int BN, int BK, class Op>
hipError_t run_gemm(const Op &op, int items, hipStream_t st) {
  if (items <= 0 || op.M <= 0 || op.N <= 0) return hipSuccess;
  dim3 grid((op.N + BN - 1) / BN, (op.M + BM - 1) / BM, items);
  hipLaunchKernelGGL((k_gemm<BM, BN, BK, Op>), grid, dim3(kThreads), 0, st,
                     op);
  return hipGetLastError();
}

// Split-K form for a few output tiles per item and a long reduction (the
// end-site local update: one 32 x 32 tile from K P = 512 terms at chi = 32,
// which one workgroup per item walks in eight dependent chunks): NS
// workgroups per tile each reduce one contiguous k range into a partial
// tile of `part` ([item][NS][M][N]), and k_splitk_sum adds the NS partials
// of every element in a fixed order (k range 0 first) and stores the sum
// through the op.
template <int BM, int BN, int BK, int NS, class Op>
__global__ __launch_bounds__(kThreads) void k_gemm_part(Op op, double *part,
                                                        size_t part_stride) {
  const int it = blockIdx.z;
  if (op.flag && !op.flag[it]) return;
  constexpr int TMX = BM / 16, TNX = BN / 16, NT = TMX * TNX;
  constexpr int TPW = (NT + 3) / 4;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int ks = blockIdx.x % NS;
  const int m0 = blockIdx.y * BM, n0 = (blockIdx.x / NS) * BN;
  const int span = ((op.Kd + NS - 1) / NS + BK - 1) / BK * BK;
  const int kb = ks * span, ke = min(op.Kd, kb + span);
  v4d acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += BK) {
    for (int i = tid; i < BM * BK; i += kThreads) {
      const int kk = i % BK, mm = i / BK;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < op.M && k < ke) ? op.a(it, m, k) : 0.0;
    }
    for (int i = tid; i < BK * BN; i += kThreads) {
      const int nn = i % BN, kk = i / BN;
      const int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < op.N && k < ke) ? op.b(it, k, n) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wave + 4 * q;
      if (t < NT) {
        const int tm = (t / TNX) * 16, tn = (t % TNX) * 16;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4)
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              As[kk + lq][tm + lr], Bs[kk + lq][tn + lr], acc[q], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  double *pp = part + (size_t)it * part_stride + (size_t)ks * op.M * op.N;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wave + 4 * q;
    if (t < NT) {
      const int tm = (t / TNX) * 16, tn = (t % TNX) * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + tm + 4 * r + lq, n = n0 + tn + lr;
        if (m < op.M && n < op.N) pp[(size_t)m * op.N + n] = acc[q][r];
      }
    }
  }
}

template <int NS, class Op>
__global__ __launch_bounds__(kThreads) void k_splitk_sum(Op op, const double *part,
                                                         size_t part_stride) {
  const int it = blockIdx.y;
  if (op.flag && !op.flag[it]) return;
  const size_t mn = (size_t)op.M * op.N;
  const double *pp = part + (size_t)it * part_stride;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < mn;
       i += (size_t)gridDim.x * kThreads) {
    double v = pp[i];
#pragma unroll
    for (int ks = 1; ks < NS; ++ks) v += pp[(size_t)ks * mn + i];
    op.st(it, (int)(i / op.N), (int)(i % op.N), v);
  }
}

// Split-K GEMM of `items` items: part holds NS M N doubles per item (stride
// part_stride).
template <int BM, int BN, int BK, int NS, class Op>
hipError_t run_gemm_splitk(const Op &op, int items, double *part, size_t part_stride,
                           hipStream_t st) {
  if (items <= 0 || op.M <= 0 || op.N <= 0) return hipSuccess;
  if (part_stride < (size_t)NS * op.M * op.N) return hipErrorInvalidValue;
  dim3 grid(NS * ((op.N + BN - 1) / BN), (op.M + BM - 1) / BM, items);
  hipLaunchKernelGGL((k_gemm_part<BM, BN, BK, NS, Op>), grid, dim3(kThreads), 0, st, op,
                     part, part_stride);
  const int blocks = (int)std::min<size_t>(8, ((size_t)op.M * op.N + kThreads - 1) / kThreads);
  hipLaunchKernelGGL((k_splitk_sum<NS, Op>), dim3(blocks, items), dim3(kThreads), 0, st, op,
                     (const double *)part, part_stride);
  return hipGetLastError();
}

// Site tensor A'[s][u][l][d][r] of the rotated block, flat index.
__device__ __forceinline__ size_t aidx(int D, int s, int u, int l, int dd,
                                       int r) {
  return ((((size_t)s * D + u) * D + l) * D + dd) * D + r;
}

struct Shape {
  int K, P, D, d;
};

// ---- inner-site visit ---------------------------------------------------
// Front view: "front" is the side the sweep comes from (left for LR, right
// for RL).  X_f[xf][a][xb], A_f[s][wf][l][wb][a] with wf the MPO leg on the
// front side, F the front environment, G the back environment.

// T1[yf][wfb][ab][xb][wfk][ak] = sum_xf F[yf][wf][xf] X_f[xf][a][xb]
struct OpK1 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  Ptr X, F;
  double *t1;
  size_t t1s;
  __device__ double a(int it, int m, int k) const {
    return F.at(it)[(size_t)m * s.K + k];
  }
  __device__ double b(int it, int k, int n) const {
    const int a = n / s.K, xb = n - a * s.K;
    const double *x = X.at(it);
    return rl ? x[((size_t)xb * s.P + a) * s.K + k]
              : x[((size_t)k * s.P + a) * s.K + xb];
  }
  __device__ void st(int it, int m, int n, double v) const {
    const int D = s.D, K = s.K, P = s.P;
    const int yf = m / P, wf = m - yf * P, wfk = wf / D, wfb = wf - wfk * D;
    const int a = n / K, xb = n - a * K, ak = a / D, ab = a - ak * D;
    const size_t idx =
        (((((size_t)yf * D + wfb) * D + ab) * K + xb) * D + wfk) * D + ak;
    t1[(size_t)it * t1s + idx] = v;
  }
};

// T2[yf][xb][lk][wbk][s][wfb][ab] = sum_{wfk,ak} T1[...][wfk][ak] Aket_f[s][wfk][lk][wbk][ak]
struct OpK2 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  const double *t1;
  size_t t1s;
  const double *A;  // item 0, site (j-1, c)
  size_t as;
  double *t2;
  size_t t2s;
  __device__ double a(int it, int m, int k) const {
    return t1[(size_t)it * t1s + (size_t)m * s.P + k];
  }
  __device__ double b(int it, int k, int n) const {
    const int D = s.D;
    const int wfk = k / D, ak = k - wfk * D;
    const int sp = n / s.P, r = n - sp * s.P, lk = r / D, wbk = r - lk * D;
    const double *A0 = A + (size_t)it * as;
    return rl ? A0[aidx(D, sp, wbk, lk, wfk, ak)]
              : A0[aidx(D, sp, wfk, lk, wbk, ak)];
  }
  __device__ void st(int it, int m, int n, double v) const {
    const int D = s.D, K = s.K;
    int t = m;
    const int xb = t % K;
    t /= K;
    const int ab = t % D;
    t /= D;
    const int wfb = t % D;
    const int yf = t / D;
    const int sp = n / s.P, r = n - sp * s.P, lk = r / D, wbk = r - lk * D;
    const size_t idx =
        (((((((size_t)yf * K + xb) * D + lk) * D + wbk) * s.d + sp) * D + wfb) *
             D +
         ab);
    t2[(size_t)it * t2s + idx] = v;
  }
};

// T3[yf][lk][lb][xb][wbk][wbb] = sum_{s,wfb,ab} T2[...] Abra_f[s][wfb][lb][wbb][ab]
struct OpK3 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  const double *t2;
  size_t t2s;
  const double *A;
  size_t as;
  double *t3;
  size_t t3s;
  __device__ double a(int it, int m, int k) const {
    return t2[(size_t)it * t2s + (size_t)m * Kd + k];
  }
  __device__ double b(int it, int k, int n) const {
    const int D = s.D;
    const int sp = k / s.P, r = k - sp * s.P, wfb = r / D, ab = r - wfb * D;
    const int lb = n / D, wbb = n - lb * D;
    const double *A0 = A + (size_t)it * as;
    return rl ? A0[aidx(D, sp, wbb, lb, wfb, ab)]
              : A0[aidx(D, sp, wfb, lb, wbb, ab)];
  }
  __device__ void st(int it, int m, int n, double v) const {
    const int D = s.D, K = s.K, P = s.P;
    int t = m;
    const int wbk = t % D;
    t /= D;
    const int lk = t % D;
    t /= D;
    const int xb = t % K;
    const int yf = t / K;
    const int lb = n / D, wbb = n - lb * D;
    const size_t idx =
        (((size_t)yf * P + lk * D + lb) * K + xb) * P + wbk * D + wbb;
    t3[(size_t)it * t3s + idx] = v;
  }
};

// Yt[yf][l][yb] = sum_{xb,wb} T3[yf][l][xb][wb] G[yb][wb][xb]
struct OpK4 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  const double *t3;
  size_t t3s;
  Ptr G, Y;
  __device__ double a(int it, int m, int k) const {
    return t3[(size_t)it * t3s + (size_t)m * Kd + k];
  }
  __device__ double b(int it, int k, int n) const {
    const int xb = k / s.P, wb = k - xb * s.P;
    return G.at(it)[((size_t)n * s.P + wb) * s.K + xb];
  }
  __device__ void st(int it, int m, int n, double v) const {
    const int yf = m / s.P, l = m - yf * s.P;
    const size_t idx = rl ? ((size_t)n * s.P + l) * s.K + yf
                          : ((size_t)yf * s.P + l) * s.K + n;
    Y.at(it)[idx] = v;
  }
};

// env'[yb][wb][xb] = sum_{yf,l} Y[yf][l][yb] T3[yf][l][xb][wb]
struct OpK5 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  const double *t3;
  size_t t3s;
  Ptr Y, E;
  __device__ double a(int it, int m, int k) const {
    const int yf = k / s.P, l = k - yf * s.P;
    const size_t idx = rl ? ((size_t)m * s.P + l) * s.K + yf
                          : ((size_t)yf * s.P + l) * s.K + m;
    return Y.at(it)[idx];
  }
  __device__ double b(int it, int k, int n) const {
    return t3[(size_t)it * t3s + (size_t)k * N + n];
  }
  __device__ void st(int it, int m, int n, double v) const {
    const int xb = n / s.P, wb = n - xb * s.P;
    E.at(it)[((size_t)m * s.P + wb) * s.K + xb] = v;
  }
};

// ---- environment update after the QR, Lenv' = T3 . Y ----------------------
// E[y'][wb][xb] = sum_{yf, l} Y[yf][l][y'] T3[yf][l][xb][wb]  (RL: Y[y'][l][yf]).
// One workgroup per (item, 64 columns n = (xb, wb)) of 4 KS waves: wave w owns
// the 16 columns w % 4 and all MT row tiles of y', over the k part w / 4 of
// every chunk.  The T3 operand is read straight from global memory (16 lanes,
// 128 contiguous bytes); Y is staged in LDS in chunks of 32 KS k = (yf, l).
// The next chunk of both is fetched into registers while the current one is
// multiplied; one barrier per chunk.  The KS partial sums of a column tile are
// added at the end in a fixed order (k part 0, 1, ...).
struct EnvArgs {
  int K, P, rl;
  const double *t3;
  size_t t3s;
  Ptr Y, E;
  // true extents of site j of column c (null: the full bond cap K): the k
  // range stops at the true front bond of Y and the T3 columns past the
  // true X bond are not read (the pair-per-wave visit does not write them)
  const FitDims *dims;
  int W, c, j, N;
};

// k parts per workgroup: two up to 32 rows (MT <= 2); from MT = 3 one, which
// leaves the registers for T3 two chunks ahead at MT = 3
template <int MT> struct EnvShape {
  static constexpr int KS = MT <= 2 ? 2 : 1;
  static constexpr int kThreads = 256 * KS;
  static constexpr int kWaves = KS == 2 ? 4 : 2;  // waves per SIMD the registers allow
};

// B16 (T = float): BF16 MFMA, the eight T3 rows a lane holds per chunk
// feeding two 16-deep steps (rows 4i + lq, i = 0-3 and 4-7).
template <int MT, class T, bool B16 = false>
__global__ __launch_bounds__(EnvShape<MT>::kThreads)
__attribute__((amdgpu_waves_per_eu(EnvShape<MT>::kWaves))) void k_env(EnvArgs e) {
  typedef Mma<T> M;
  typedef typename M::acc Acc;
  constexpr int KS = EnvShape<MT>::KS, NT = EnvShape<MT>::kThreads;
  constexpr int MW = MT * 16, AS = M::pad_b(MW), CH = 32 * KS;
  constexpr int NA = CH * MW / NT;  // A elements staged per thread
  __shared__ T As[2][CH][AS];
  const int K = e.K, P = e.P, N = K * P;
  int tile, it;
  xcd_tile_item(&tile, &it);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4, cg = wave & 3, h = wave >> 2;
  const int n = tile * 64 + cg * 16 + lr;
  // k = (yf, l) runs to the true front bond of Y, columns n = (xb, wb) to the
  // true X bond; past them every product is zero (Y padding) or T3 was not
  // written, so they are skipped (or masked) without changing any sum.  E is
  // still written in full (zeros in the padding).
  int Kd = K * P, Nt = N;
  if (e.dims) {
    const SiteExt ex = site_ext(e.dims[(size_t)it * e.W + e.c], e.j, e.N, e.rl != 0);
    Kd = ex.yf * P;
    Nt = ex.xb * P;
  }
  if (tile * 64 >= Nt) {  // every column of the tile is padding
    if (tid < 64 * 4) {
      auto *Ez = gmem(e.E.at(it));
      const int nz = tile * 64 + tid % 64;
      if (nz < N) {
        const int xb = nz / P, wb = nz - xb * P;
        for (int m = tid / 64; m < K; m += 4) Ez[((size_t)m * P + wb) * K + xb] = 0.0;
      }
    }
    return;
  }
  // Y (K P K doubles) and this item's T3 (K P x K P) through buffer
  // descriptors; an element outside the operand (or past the true extents)
  // loads at the descriptor's end, where the range check returns zero
  const T *T3 = reinterpret_cast<const T *>(e.t3) + (size_t)it * e.t3s;
  const unsigned ybytes = (unsigned)(K * P * K) * 8u;
  const unsigned tbytes = (unsigned)(Kd * N) * (unsigned)sizeof(T);
  const __amdgpu_buffer_rsrc_t yrs = buf_rsrc(e.Y.at(it), ybytes);
  const __amdgpu_buffer_rsrc_t trs = buf_rsrc(T3, tbytes);
  const bool rl = e.rl != 0;
  // Y elements of the next chunk (raw loads, staged in LDS by put)
  double an[NA];
  // RL layout: (yf, l) of k = k0 + kk for each staged element, packed as
  // yf * 256 + l and carried from chunk to chunk (no division in the loop)
  int yfl[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int kk = (tid + u * NT) / MW;
    yfl[u] = (kk / P) * 256 + kk % P;
  }
  const int dyfl = (CH / P) * 256 + CH % P;
  auto fetch_a = [&](int k0) {  // chunks in order 0, CH, 2 CH, ...
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int i = tid + u * NT, kk = i / MW, m = i % MW, k = k0 + kk;
      const bool ok = m < K && k < Kd;
      const unsigned off = rl ? (m * P + (yfl[u] & 255)) * K + (yfl[u] >> 8) : k * K + m;
      an[u] = buf_ld(yrs, ok ? off * 8u : ybytes);
      yfl[u] += dyfl;
      if ((yfl[u] & 255) >= P) yfl[u] += 256 - P;
    }
  };
  // T3 rows of chunk k0 for this wave's k part (two chunks are in flight)
  auto fetch_b = [&](int k0, T (&b)[8]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + h * 32 + 4 * i + lq;
      const bool ok = n < Nt && k < Kd;
      b[i] = buf_ld_t<T>(trs, ok ? (unsigned)(k * N + n) * (unsigned)sizeof(T) : tbytes);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int i = tid + u * NT;
      As[buf][i / MW][i % MW] = (T)an[u];
    }
  };
  // two accumulation chains per row tile, one where MT tiles already give
  // three or more independent chains
  constexpr int NC = MT >= 3 ? 1 : 2;
  Acc acc[MT][NC];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[mt][q] = Acc{0, 0, 0, 0};
  // T3 rows are fetched DB chunks ahead (two while the registers allow)
  constexpr int DB = MT <= 3 ? 2 : 1;
  T b0[8], b1[8];
  fetch_a(0);
  fetch_b(0, b0);
  if (DB == 2 && CH < Kd) fetch_b(CH, b1);
  put(0);
  __syncthreads();
  int buf = 0;
  // one chunk: multiply with the staged Y and the given T3 rows, then
  // refill those rows DB chunks ahead and stage the next Y chunk
  auto step = [&](int k0, T (&b)[8]) {
    if (k0 + CH < Kd) fetch_a(k0 + CH);
    if constexpr (B16) {  // copy out, refill, then two BF16 steps per row tile
      float bc[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) bc[i] = (float)b[i];
      if (k0 + DB * CH < Kd) fetch_b(k0 + DB * CH, b);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        float a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = As[buf][h * 32 + 4 * i + lq][mt * 16 + lr];
        acc[mt][0] = mfma_bf16(a, bc, acc[mt][0]);
        acc[mt][NC - 1] = mfma_bf16(a + 4, bc + 4, acc[mt][NC - 1]);
      }
    } else if constexpr (DB == 1) {  // copy out, then refill the same registers
      T bc[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) bc[i] = b[i];
      if (k0 + CH < Kd) fetch_b(k0 + CH, b);
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][i % NC] =
              M::run(As[buf][h * 32 + 4 * i + lq][mt * 16 + lr], bc[i], acc[mt][i % NC]);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const T bc = b[i];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][i % NC] =
              M::run(As[buf][h * 32 + 4 * i + lq][mt * 16 + lr], bc, acc[mt][i % NC]);
      }
      if (k0 + 2 * CH < Kd) fetch_b(k0 + 2 * CH, b);
    }
    if (k0 + CH < Kd) put(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  };
  for (int k0 = 0; k0 < Kd; k0 += DB * CH) {
    step(k0, b0);
    if (DB == 2 && k0 + CH < Kd) step(k0 + CH, b1);
  }
  Acc c[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) c[mt] = NC == 1 ? acc[mt][0] : acc[mt][0] + acc[mt][NC - 1];
  if (KS > 1) {  // k parts 1.. hand their sums to part 0 through LDS
    T *red = &As[0][0][0];
    static_assert((KS - 1) * 4 * MT * 4 * 64 <= 2 * CH * AS, "reduction fits");
    if (h > 0) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          red[((((h - 1) * 4 + cg) * MT + mt) * 4 + r) * 64 + lane] = c[mt][r];
    }
    __syncthreads();
    if (h > 0) return;
#pragma unroll
    for (int hh = 1; hh < KS; ++hh)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          c[mt][r] += red[((((hh - 1) * 4 + cg) * MT + mt) * 4 + r) * 64 + lane];
  }
  if (n >= N) return;
  const int xb = n / P, wb = n - xb * P;
  auto *E = gmem(e.E.at(it));
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = mt * 16 + M::crow(r, lq);
      if (m < K) E[((size_t)m * P + wb) * K + xb] = (double)c[mt][r];
    }
  }
}

// ---- end-site visit (message site as MPO: Mend[a][q][a']) ----------------
// T[a][q][xb] = sum_{a'} Mend[a][q][a'] X_e[a'][xb]
struct OpE1 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  Ptr Mend, Xe;
  double *t3;
  size_t t3s;
  __device__ double a(int it, int m, int k) const {
    return Mend.at(it)[(size_t)m * s.K + k];
  }
  __device__ double b(int it, int k, int n) const {
    return rl ? Xe.at(it)[(size_t)n * s.K + k] : Xe.at(it)[(size_t)k * s.K + n];
  }
  __device__ void st(int it, int m, int n, double v) const {
    t3[(size_t)it * t3s + (size_t)m * s.K + n] = v;
  }
};

// Yt_e[a][yb] = sum_{q,xb} T[a][q][xb] G[yb][q][xb]
struct OpE2 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  const double *t3;
  size_t t3s;
  Ptr G, Ye;
  __device__ double a(int it, int m, int k) const {
    return t3[(size_t)it * t3s + (size_t)m * Kd + k];
  }
  __device__ double b(int it, int k, int n) const {
    return gmem((const double *)G.at(it))[(size_t)n * Kd + k];
  }
  __device__ void st(int it, int m, int n, double v) const {
    gmem(Ye.at(it))[rl ? (size_t)n * s.K + m : (size_t)m * s.K + n] = v;
  }
};

// env'[yb][q][xb] = sum_a Y_e[a][yb] T[a][q][xb]
struct OpE3 {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  bool rl;
  const double *t3;
  size_t t3s;
  Ptr Ye, E;
  __device__ double a(int it, int m, int k) const {
    return rl ? Ye.at(it)[(size_t)m * s.K + k] : Ye.at(it)[(size_t)k * s.K + m];
  }
  __device__ double b(int it, int k, int n) const {
    return t3[(size_t)it * t3s + (size_t)k * N + n];
  }
  __device__ void st(int it, int m, int n, double v) const {
    E.at(it)[(size_t)m * N + n] = v;
  }
};

// Y <- Y . L with L[k][n] = R[n][k]: rows of the slot times the bond.
struct OpApplyL {
  int M, N, Kd;
  const int32_t *flag;
  Shape s;
  Ptr Y;
  const double *rbuf;
  double *tmp;
  size_t S;
  __device__ double a(int it, int m, int k) const {
    return Y.at(it)[(size_t)m * s.K + k];
  }
  __device__ double b(int it, int k, int n) const {
    return rbuf[(size_t)it * s.K * s.K + (size_t)n * s.K + k];
  }
  __device__ void st(int it, int m, int n, double v) const {
    tmp[(size_t)it * S + (size_t)m * s.K + n] = v;
  }
};

// Transfer-matrix steps of <a|b>.
struct OpOv1 {  // U[b'][q][a] = sum_{a'} E[a'][b'] a_i[a'][q][a]
  int M, N, Kd;
  const int32_t *flag;
  int K;
  const double *E;
  const double *const *ap;
  size_t off;
  double *U;
  size_t S;
  __device__ double a(int it, int m, int k) const {
    return E[(size_t)it * K * K + (size_t)k * K + m];
  }
  __device__ double b(int it, int k, int n) const {
    return ap[it][off + (size_t)k * N + n];
  }
  __device__ void st(int it, int m, int n, double v) const {
    U[(size_t)it * S + (size_t)m * N + n] = v;
  }
};
struct OpOv2 {  // E'[a][b] = sum_{b',q} U[b'][q][a] b_i[b'][q][b]
  int M, N, Kd;
  const int32_t *flag;
  int K, P;
  const double *U;
  size_t S;
  const double *const *bp;
  size_t off;
  double *E;
  __device__ double a(int it, int m, int k) const {
    return U[(size_t)it * S + (size_t)k * K + m];
  }
  __device__ double b(int it, int k, int n) const {
    return bp[it][off + (size_t)k * K + n];
  }
  __device__ void st(int it, int m, int n, double v) const {
    E[(size_t)it * K * K + (size_t)m * K + n] = v;
  }
};

// ---------------------------------------------------------------------------
// Fused fit visit on FP64 MFMA (v_mfma_f64_16x16x4f64).  One workgroup per
// (item, tile of TY front bonds yf); it walks all tiles of TX back bonds xb
// and, per tile, runs four LDS-resident contractions:
//   (a) T1[yf,wf][a,xb]      = sum_xf F[yf][wf][xf] X_f[xf][a][xb]
//   (b) T2[wfb,ab][s,lk,wbk] = sum_{wfk,ak} T1 Aket_f[s][wfk][lk][wbk][ak]  (per pair)
//   (c) T3[lk,wbk][lb,wbb]   = sum_{s,wfb,ab} T2 Abra_f[s][wfb][lb][wbb][ab] (per pair)
//   (e) Yt[yf,l][yb]        += sum_{xb,wb} T3 G[yb][wb][xb]
// T3 goes to HBM once (the environment update reads it); T1 and T2 never do.
// MFMA operand layout: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator register r holds D[4r + l/16][l%16].
// ---------------------------------------------------------------------------
struct VisitArgs {
  int K, P, D, d, TY, TX;
  int rl, do_local;
  // true extents of site j of column c (null: the full bond cap K); only
  // the pair-per-wave D = 4 kernel uses them to skip zero padding
  const FitDims *dims;
  int W, c, j, N;
  Ptr F, X, G, Y;
  const double *aket;
  size_t aket_stride;
  const double *abra;
  size_t abra_stride;
  double *t3;
  size_t t3_stride;
};

constexpr int kVisitThreads = 512;
constexpr int kVisitWaves = kVisitThreads / 64;

// One batched LDS GEMM: for batch p < nb, C_p[M][N] = A_p[M][Kd] B_p[Kd][N];
// 16 x 16 output tiles spread over the waves, two per wave at a time when
// there are enough; each tile keeps two accumulators (even and odd k-steps)
// and its operands are read two k-steps ahead of the MFMAs.  afn/bfn read
// operands (zero outside), sfn stores the result tile element.  T: FP64, or
// FP32 on FP32 MFMA with FP32 accumulation; B16 (T = float): BF16 MFMA, 32
// k per step, lane slot s holding k = k0 + 4s + lq (slots 0-3 and 4-7 feed
// the two accumulators).
template <class T, bool B16 = false, class AF, class BF, class SF>
__device__ __forceinline__ void lds_gemm(int nb, int M, int N, int Kd, AF afn,
                                         BF bfn, SF sfn) {
  typedef Mma<T> MM;
  typedef typename MM::acc Acc;
  const Acc zero = Acc{0, 0, 0, 0};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  const int ntiles = nb * tm * tn;
  for (int t0 = wave; t0 < ntiles; t0 += 2 * kVisitWaves) {
    int p[2], m0[2], n0[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = min(t0 + h * kVisitWaves, ntiles - 1);
      p[h] = t / (tm * tn);
      const int r2 = t - p[h] * tm * tn;
      m0[h] = (r2 / tn) << 4;
      n0[h] = (r2 % tn) << 4;
    }
    const bool two = t0 + kVisitWaves < ntiles;
    Acc acc[2][2] = {{zero, zero}, {zero, zero}};
    if constexpr (B16) {
      static_assert(sizeof(T) == 4, "BF16 steps stage FP32 operands");
      for (int k0 = 0; k0 < Kd; k0 += 32) {
        float av[2][8], bv[2][8];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int k = k0 + 4 * s + lq, am = m0[h] + lr, bn = n0[h] + lr;
            const bool on = h == 0 || two;
            av[h][s] = (on && am < M && k < Kd) ? (float)afn(p[h], am, k) : 0.f;
            bv[h][s] = (on && bn < N && k < Kd) ? (float)bfn(p[h], k, bn) : 0.f;
          }
        const bool hi = k0 + 16 < Kd;  // slots 4-7 hold k0 + 16 .. k0 + 31
        acc[0][0] = mfma_bf16(av[0], bv[0], acc[0][0]);
        if (hi) acc[0][1] = mfma_bf16(av[0] + 4, bv[0] + 4, acc[0][1]);
        if (two) {
          acc[1][0] = mfma_bf16(av[1], bv[1], acc[1][0]);
          if (hi) acc[1][1] = mfma_bf16(av[1] + 4, bv[1] + 4, acc[1][1]);
        }
      }
    } else {
      for (int k0 = 0; k0 < Kd; k0 += 8) {
        T av[2][2], bv[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int k = k0 + 4 * u + lq, am = m0[h] + lr, bn = n0[h] + lr;
            const bool on = h == 0 || two;
            av[h][u] = (on && am < M && k < Kd) ? afn(p[h], am, k) : (T)0;
            bv[h][u] = (on && bn < N && k < Kd) ? bfn(p[h], k, bn) : (T)0;
          }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          acc[0][u] = MM::run(av[0][u], bv[0][u], acc[0][u]);
          if (two) acc[1][u] = MM::run(av[1][u], bv[1][u], acc[1][u]);
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !two) break;
      const Acc c = acc[h][0] + acc[h][1];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0[h] + MM::crow(r, lq), n = n0[h] + lr;
        if (m < M && n < N) sfn(p[h], m, n, c[r]);
      }
    }
  }
}

// Doubles of dynamic LDS for one fused-visit workgroup with tiles TY x TX.
__host__ __device__ inline size_t visit_lds(int K, int P, int d, int TY, int TX) {
  const size_t P2 = (size_t)P * P;
  return (size_t)TY * P * pad_a(K) + (size_t)K * pad_b(P * TX) + (size_t)TY * TX * P2 +
         (size_t)TY * TX * P * pad_b(d * P) + (size_t)TY * TX * P2 +
         (size_t)TX * P * pad_b(K) + 2 * (size_t)d * P2;
}

// DT > 0 fixes D (and P = D^2) at compile time; DT = 0 reads them at run time.
// B16 (T = float): every contraction on BF16 MFMA with FP32 accumulation.
// LDS layouts (index order, fastest last):
//   Fs [ty, wf][xf]          stride pad_a(K)
//   Xs [xf][a, tx]           stride pad_b(P TX)
//   T1s[pair][wfk, akx][wfb, abx]
//   T2s[pair][wfb, abx][s, lk, wbk]   stride pad_b(d P)
//   T3s[pair][wbk, wbb][lk, lb]
//   Gs [tx, wb][yb]          stride pad_b(K)
//   Ak, Ab [s][wf][a][l][wb] of the front view (ket and bra roles alike)
template <int DT, class T, bool B16 = false>
__global__ __launch_bounds__(kVisitThreads) void k_visit(VisitArgs v) {
  extern __shared__ double sm_raw[];
  T *sm = reinterpret_cast<T *>(sm_raw);
  typedef Mma<T> MM;
  typedef typename MM::acc Acc;
  constexpr bool kFixed = DT > 0;
  const int D = kFixed ? DT : v.D;
  const int P = kFixed ? DT * DT : v.P;
  const int K = v.K, d = v.d, TY = v.TY, TX = v.TX;
  const int dP = d * P, P2 = P * P;
  const int FS = pad_a(K), XS = pad_b(P * TX), T2S = pad_b(dP), GS = pad_b(K);
  const int it = blockIdx.y, y0 = blockIdx.x * TY;
  const int tid = threadIdx.x;
  T *Fs = sm;
  T *Xs = Fs + (size_t)TY * P * FS;
  T *T1s = Xs + (size_t)K * XS;
  T *T2s = T1s + (size_t)TY * TX * P2;
  T *T3s = T2s + (size_t)TY * TX * P * T2S;
  T *Gs = T3s + (size_t)TY * TX * P2;
  T *Ak = Gs + (size_t)TX * P * GS;
  T *Ab = Ak + (size_t)d * P2;
  const auto *F = gmem((const double *)v.F.at(it));
  const auto *X = gmem((const double *)v.X.at(it));
  const auto *G = gmem((const double *)v.G.at(it));
  const double *ak = v.aket + (size_t)it * v.aket_stride;
  const double *ab = v.abra + (size_t)it * v.abra_stride;
  T *T3g = reinterpret_cast<T *>(v.t3) + (size_t)it * v.t3_stride;
  const bool rl = v.rl != 0;

  // front-view site tensors A_f[s][wf][l][wb][a] (RL swaps the u/d legs),
  // stored as [s][wf][a][l][wb]
  for (int i = tid; i < d * P2; i += kVisitThreads) {
    int t = i;
    const int wb = t % D; t /= D;
    const int l = t % D; t /= D;
    const int a = t % D; t /= D;
    const int wf = t % D;
    const int s = t / D;
    const int u = rl ? wb : wf, dd = rl ? wf : wb;
    const size_t src = ((((size_t)s * D + u) * D + l) * D + dd) * D + a;
    Ak[i] = (T)ak[src];
    Ab[i] = (T)ab[src];
  }
  // F rows of this y tile: F[yf][wf][xf]
  for (int i = tid; i < TY * P * K; i += kVisitThreads) {
    const int row = i / K, xf = i - row * K;
    const int yf = y0 + row / P;
    Fs[row * FS + xf] = (T)(yf < K ? F[(size_t)(y0 * P + row) * K + xf] : 0.0);
  }
  // Yt accumulators: tiles of [(ty,l)][yb], kept in registers.  With at
  // most half as many tiles as waves, each tile's k range is split over two
  // waves (kh = 0, 1) and the halves are summed at the end.
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int Me = TY * P, tme = (Me + 15) >> 4, tne = (K + 15) >> 4;
  const int ntile_e = tme * tne;
  const bool split_e = 2 * ntile_e <= kVisitWaves;
  constexpr int kMaxE = 4;  // tiles per wave (host keeps ntile_e <= 4 * waves)
  Acc accE[kMaxE];
#pragma unroll
  for (int q = 0; q < kMaxE; ++q) accE[q] = Acc{0, 0, 0, 0};

  for (int x0 = 0; x0 < K; x0 += TX) {
    __syncthreads();  // previous tile's Xs/Gs/T3s consumers are done
    // X_f[xf][a][xb] for the tile, as Xs[xf][a*TX + tx]; the loop runs along
    // the contiguous global index (xb for LR, xf for RL)
    for (int i = tid; i < K * P * TX; i += kVisitThreads) {
      int xf, a, tx;
      if (rl) {
        xf = i % K;
        const int r = i / K;
        a = r % P;
        tx = r / P;
      } else {
        tx = i % TX;
        const int r = i / TX;
        a = r % P;
        xf = r / P;
      }
      const int xb = x0 + tx;
      double val = 0.0;
      if (xb < K)
        val = rl ? X[((size_t)xb * P + a) * K + xf] : X[((size_t)xf * P + a) * K + xb];
      Xs[xf * XS + a * TX + tx] = (T)val;
    }
    if (v.do_local)
      // G[yb][wb][xb] as Gs[(tx*P + wb)][yb], read along xb
      for (int i = tid; i < TX * P * K; i += kVisitThreads) {
        const int tx = i % TX, r = i / TX;
        const int wb = r % P, yb = r / P, xb = x0 + tx;
        Gs[(tx * P + wb) * GS + yb] = (T)(xb < K ? G[((size_t)yb * P + wb) * K + xb] : 0.0);
      }
    __syncthreads();
    // (a) T1: rows (ty, wf), cols (a, tx), stored [pair][wfk, akx][wfb, abx]
    lds_gemm<T, B16>(
        1, TY * P, P * TX, K,
        [&](int, int m, int k) { return Fs[m * FS + k]; },
        [&](int, int k, int n) { return Xs[k * XS + n]; },
        [&](int, int m, int n, T val) {
          const int ty = m / P, wf = m - ty * P, a = n / TX, tx = n - a * TX;
          const int wfk = wf / D, wfb = wf - wfk * D, akx = a / D, abx = a - akx * D;
          T1s[(ty * TX + tx) * P2 + (wfk * D + akx) * P + wfb * D + abx] = val;
        });
    __syncthreads();
    // (b) ket: per pair, rows m = (wfb, abx), k = (wfk, akx), cols n = (s, lk, wbk)
    lds_gemm<T, B16>(
        TY * TX, P, dP, P,
        [&](int p, int m, int k) { return T1s[p * P2 + k * P + m]; },
        [&](int, int k, int n) {
          const int s = n / P;
          return Ak[(s * P + k) * P + (n - s * P)];
        },
        [&](int p, int m, int n, T val) { T2s[(p * P + m) * T2S + n] = val; });
    __syncthreads();
    // (c) bra: per pair, rows m = (lk, wbk), k = (s, wfb, abx), cols n = (lb, wbb);
    // stored as T3s[pair][wb][l]
    lds_gemm<T, B16>(
        TY * TX, P, P, dP,
        [&](int p, int m, int k) {
          const int s = k / P;
          return T2s[(p * P + (k - s * P)) * T2S + s * P + m];
        },
        [&](int, int k, int n) { return Ab[k * P + n]; },
        [&](int p, int m, int n, T val) {
          const int lk = m / D, wbk = m - lk * D, lb = n / D, wbb = n - lb * D;
          T3s[p * P2 + (wbk * D + wbb) * P + lk * D + lb] = val;
        });
    __syncthreads();
    // T3 tile to HBM as T3[yf][l][xb][wb]
    for (int i = tid; i < TY * TX * P2; i += kVisitThreads) {
      int t = i;
      const int wb = t % P; t /= P;
      const int tx = t % TX; t /= TX;
      const int l = t % P;
      const int ty = t / P;
      const int yf = y0 + ty, xb = x0 + tx;
      if (yf < K && xb < K)
        T3g[(((size_t)yf * P + l) * K + xb) * P + wb] = T3s[(ty * TX + tx) * P2 + wb * P + l];
    }
    // (e) local update, accumulated over the xb tiles
    if (v.do_local) {
      const int Ke = TX * P;
      const int kh = split_e ? wave / (kVisitWaves / 2) : 0;
      const int wt = split_e ? wave % (kVisitWaves / 2) : wave;
      const int wstep = split_e ? kVisitWaves / 2 : kVisitWaves;
      const int kb = split_e ? kh * (Ke / 2) : 0, ke = split_e ? kb + Ke / 2 : Ke;
#pragma unroll
      for (int q = 0; q < kMaxE; ++q) {
        const int t = wt + q * wstep;
        if (t >= ntile_e) break;
        const int m0 = (t / tne) << 4, n0 = (t % tne) << 4;
        const int am = m0 + lr, bn = n0 + lr;
        const int ty = am / P, l = am - ty * P;
        Acc acc[2] = {accE[q], Acc{0, 0, 0, 0}};
        if constexpr (B16) {  // 32 k per step, slot s holding k0 + 4s + lq
          for (int k0 = kb; k0 < ke; k0 += 32) {
            float av[8], bv[8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
              const int k = k0 + 4 * s + lq;
              const int tx = k / P, wb = k - tx * P;
              av[s] = (am < Me && k < ke) ? T3s[(ty * TX + tx) * P2 + wb * P + l] : 0.f;
              bv[s] = (bn < K && k < ke) ? Gs[k * GS + bn] : 0.f;
            }
            acc[0] = mfma_bf16(av, bv, acc[0]);
            if (k0 + 16 < ke) acc[1] = mfma_bf16(av + 4, bv + 4, acc[1]);
          }
        } else {
          for (int k0 = kb; k0 < ke; k0 += 8) {
            T av[2], bv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int k = k0 + 4 * u + lq;
              const int tx = k / P, wb = k - tx * P;
              av[u] = (am < Me && k < ke) ? T3s[(ty * TX + tx) * P2 + wb * P + l] : (T)0;
              bv[u] = (bn < K && k < ke) ? Gs[k * GS + bn] : (T)0;
            }
            acc[0] = MM::run(av[0], bv[0], acc[0]);
            acc[1] = MM::run(av[1], bv[1], acc[1]);
          }
        }
        accE[q] = acc[0] + acc[1];
      }
    }
  }
  if (v.do_local && split_e) {  // add the second k half into the first
    __syncthreads();
    T *red = sm;  // every LDS buffer is free after the last tile
    if (wave >= kVisitWaves / 2) {
      const int wt = wave - kVisitWaves / 2;
#pragma unroll
      for (int q = 0; q < kMaxE; ++q) {
        const int t = wt + q * (kVisitWaves / 2);
        if (t >= ntile_e) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(t * 4 + r) * 64 + lane] = accE[q][r];
      }
    }
    __syncthreads();
    if (wave < kVisitWaves / 2) {
#pragma unroll
      for (int q = 0; q < kMaxE; ++q) {
        const int t = wave + q * (kVisitWaves / 2);
        if (t >= ntile_e) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) accE[q][r] += red[(t * 4 + r) * 64 + lane];
      }
    }
  }
  if (v.do_local && (!split_e || wave < kVisitWaves / 2)) {
    auto *Y = gmem(v.Y.at(it));
    const int wstep = split_e ? kVisitWaves / 2 : kVisitWaves;
#pragma unroll
    for (int q = 0; q < kMaxE; ++q) {
      const int t = wave + q * wstep;
      if (t >= ntile_e) break;
      const int m0 = (t / tne) << 4, n0 = (t % tne) << 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + MM::crow(r, lq), yb = n0 + lr;
        const int ty = m / P, l = m - ty * P, yf = y0 + ty;
        if (m < Me && yb < K && yf < K) {
          const size_t idx = rl ? ((size_t)yb * P + l) * K + yf
                                : ((size_t)yf * P + l) * K + yb;
          Y[idx] = (double)accE[q][r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fused fit visit specialised for D = 4 (P = 16) and d = 2, tiles TY x TX
// fixed at compile time.  Same four contractions and layouts as k_visit; every
// MFMA operand is read through a per-lane pointer with a compile-time step, the
// k loops are unrolled, and the operand tiles are zero-padded in LDS (rows and
// columns up to a multiple of 4 in k, of 16 in yb) so that no bounds test sits
// in an MFMA loop.
// ---------------------------------------------------------------------------
__host__ __device__ inline int ceil4(int x) { return (x + 3) & ~3; }
__host__ __device__ inline int ceil16(int x) { return (x + 15) & ~15; }

// LDS elements (of T) of one k_visit4 workgroup.
template <class T>
__host__ __device__ inline size_t visit4_lds(int K, int TY, int TX) {
  typedef Mma<T> M;
  const int K4 = ceil4(K);
  return (size_t)TY * 16 * M::pad_a(K4) + (size_t)K4 * M::pad_b(16 * TX) + (size_t)TY * TX * 256 +
         (size_t)TY * TX * 16 * M::pad_b(32) + (size_t)TY * TX * 256 +
         (size_t)TX * 16 * M::pad_b(K) + 2 * 2 * 256;
}

// acc[0] / acc[1] += sum over N k-steps (even / odd) of A(pa + i*da) B(pb + i*db)
template <int N, class T>
__device__ __forceinline__ void mma_steps(typename Mma<T>::acc (&acc)[2], const T *pa, int da,
                                          const T *pb, int db) {
  T av[N], bv[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    av[i] = pa[i * da];
    bv[i] = pb[i * db];
  }
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i & 1] = Mma<T>::run(av[i], bv[i], acc[i & 1]);
}

template <int TY, int TX, class T>
__global__ __launch_bounds__(kVisitThreads) void k_visit4(VisitArgs v) {
  extern __shared__ double sm_raw[];
  T *sm = reinterpret_cast<T *>(sm_raw);
  typedef Mma<T> M;
  typedef typename M::acc Acc;
  const Acc zero = Acc{0, 0, 0, 0};
  constexpr int D = 4, P = 16, P2 = 256, NP = TY * TX;
  constexpr int XS = M::pad_b(16 * TX), T2S = M::pad_b(32);
  const int K = v.K, K4 = ceil4(K), FS = M::pad_a(K4), GS = M::pad_b(K), KY = ceil16(K);
  const int it = blockIdx.y, y0 = blockIdx.x * TY;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  T *Fs = sm;
  T *Xs = Fs + TY * 16 * FS;
  T *T1s = Xs + K4 * XS;
  T *T2s = T1s + NP * P2;
  T *T3s = T2s + NP * 16 * T2S;
  T *Gs = T3s + NP * P2;
  T *Ak = Gs + TX * 16 * GS;
  T *Ab = Ak + 2 * P2;
  const auto *F = gmem((const double *)v.F.at(it));
  const auto *X = gmem((const double *)v.X.at(it));
  const auto *G = gmem((const double *)v.G.at(it));
  const double *ak = v.aket + (size_t)it * v.aket_stride;
  const double *ab = v.abra + (size_t)it * v.abra_stride;
  T *T3g = reinterpret_cast<T *>(v.t3) + (size_t)it * v.t3_stride;
  const bool rl = v.rl != 0;

  // site tensors as [s][wf][a][l][wb] of the front view (RL swaps u and d)
  for (int i = tid; i < 2 * P2; i += kVisitThreads) {
    const int wb = i & 3, l = (i >> 2) & 3, a = (i >> 4) & 3, wf = (i >> 6) & 3, s = i >> 8;
    const int u = rl ? wb : wf, dd = rl ? wf : wb;
    const int src = ((((s * D + u) * D + l) * D + dd) * D + a);
    Ak[i] = (T)ak[src];
    Ab[i] = (T)ab[src];
  }
  // F rows of the y tile, zero beyond K (and beyond the lattice edge in yf)
  for (int row = wave; row < TY * 16; row += kVisitWaves) {
    const bool ok = y0 + (row >> 4) < K;
    for (int xf = lane; xf < K4; xf += 64)
      Fs[row * FS + xf] = (T)((ok && xf < K) ? F[(size_t)(y0 * P + row) * K + xf] : 0.0);
  }
  // local-update accumulators: TY x (KY/16) tiles of [(ty, l)][yb]; each
  // tile's k range (tx, wb) is split over two waves when tiles are few
  const int tne = KY >> 4, ntile_e = TY * tne;
  const bool split_e = 2 * ntile_e <= kVisitWaves;
  constexpr int kMaxE = 4;
  Acc accE[kMaxE];
#pragma unroll
  for (int q = 0; q < kMaxE; ++q) accE[q] = zero;

  // The X and G tiles of the next xb step are fetched into registers while
  // the current step computes.  Each thread moves up to kLd elements of each;
  // their offsets (global relative to the tile, LDS) are decoded once.
  constexpr int kLd = 8;  // host keeps K4*16*TX and KY*16*TX within 8*512
  int xg[kLd], xl[kLd], gg[kLd], gl[kLd];
  T xr[kLd], gr[kLd];
#pragma unroll
  for (int u = 0; u < kLd; ++u) {
    const int i = tid + u * kVisitThreads;
    int xf, a, tx;
    if (rl) {
      xf = i % K4;
      const int r = i / K4;
      a = r & 15;
      tx = r >> 4;
    } else {
      tx = i % TX;
      const int r = i / TX;
      a = r & 15;
      xf = r >> 4;
    }
    const bool ok = i < K4 * 16 * TX && xf < K;
    xg[u] = !ok ? -1 : (rl ? (tx * P + a) * K + xf : (xf * P + a) * K + tx);
    xl[u] = i < K4 * 16 * TX ? xf * XS + a * TX + tx : -1;
    xl[u] |= (tx << 24);  // keep tx to test xb < K per step
    const int gtx = i % TX, gr2 = i / TX, wb = gr2 & 15, yb = gr2 >> 4;
    const bool gok = i < KY * 16 * TX && yb < K;
    gg[u] = gok ? (yb * P + wb) * K + gtx : -1;
    gl[u] = i < KY * 16 * TX ? ((gtx * 16 + wb) * GS + yb) | (gtx << 24) : -1;
  }
  auto fetch = [&](int x0) {
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      const int xtx = (xl[u] >> 24) & 0x7f, gtx = (gl[u] >> 24) & 0x7f;
      const size_t xo = rl ? (size_t)x0 * P * K : (size_t)x0;
      xr[u] = (T)((xg[u] >= 0 && x0 + xtx < K) ? X[xo + xg[u]] : 0.0);
      gr[u] = (T)((v.do_local && gg[u] >= 0 && x0 + gtx < K) ? G[(size_t)x0 + gg[u]] : 0.0);
    }
  };
  fetch(0);

  for (int x0 = 0; x0 < K; x0 += TX) {
    __syncthreads();  // the previous step's readers of Xs, Gs, T3s are done
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      if (xl[u] >= 0) Xs[xl[u] & 0xffffff] = xr[u];
      if (gl[u] >= 0) Gs[gl[u] & 0xffffff] = gr[u];
    }
    __syncthreads();
    if (x0 + TX < K) fetch(x0 + TX);
    // (a) T1: tiles (ty, tn): rows (ty, wf), cols n = (a, tx) in [16 tn, 16 tn + 16)
    for (int t = wave; t < TY * TX; t += kVisitWaves) {
      const int ty = t / TX, tn = t % TX;
      Acc acc[2] = {zero, zero};
      const T *pa = Fs + (ty * 16 + lr) * FS + lq;
      const T *pb = Xs + lq * XS + tn * 16 + lr;
      int k0 = 0;
      for (; k0 + 16 <= K4; k0 += 16) mma_steps<4>(acc, pa + k0, 4, pb + k0 * XS, 4 * XS);
      for (; k0 < K4; k0 += 4) mma_steps<1>(acc, pa + k0, 4, pb + k0 * XS, 4 * XS);
      const Acc c = acc[0] + acc[1];
      const int n = tn * 16 + lr, a = n / TX, tx = n % TX;
      T *dst = T1s + (ty * TX + tx) * P2 + (a >> 2) * 16 + (a & 3);
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // wf = (wfk, wfb)
        const int wf = M::crow(r, lq);
        dst[(wf >> 2) * 64 + (wf & 3) * 4] = c[r];
      }
    }
    __syncthreads();
    // (b) ket: per pair, rows m = (wfb, abx), k = (wfk, akx), cols n = (s, lk, wbk)
    for (int t = wave; t < 2 * NP; t += kVisitWaves) {
      const int pp = t >> 1, sn = t & 1;
      Acc acc[2] = {zero, zero};
      mma_steps<4>(acc, T1s + pp * P2 + lq * 16 + lr, 64, Ak + sn * P2 + lq * 16 + lr, 64);
      const Acc c = acc[0] + acc[1];
      T *dst = T2s + pp * 16 * T2S + sn * 16 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[M::crow(r, lq) * T2S] = c[r];
    }
    __syncthreads();
    // (c) bra: per pair, rows m = (lk, wbk), k = (s, wfb, abx), cols n = (lb, wbb)
    for (int t = wave; t < NP; t += kVisitWaves) {
      Acc acc[2] = {zero, zero};
#pragma unroll
      for (int sn = 0; sn < 2; ++sn)
        mma_steps<4>(acc, T2s + (t * 16 + lq) * T2S + sn * 16 + lr, 4 * T2S,
                     Ab + (sn * 16 + lq) * 16 + lr, 64);
      const Acc c = acc[0] + acc[1];
      // m = (lk, wbk), n = lr: lb = lr/4, wbb = lr%4
      T *dst = T3s + t * P2 + (lr & 3) * 16 + (lr >> 2);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = M::crow(r, lq);
        dst[(m & 3) * 64 + (m >> 2) * 4] = c[r];
      }
    }
    __syncthreads();
    // T3 tile to HBM as T3[yf][l][xb][wb]
    for (int i = tid; i < NP * P2; i += kVisitThreads) {
      const int wb = i & 15, r = i >> 4, tx = r % TX, r2 = r / TX, l = r2 & 15, ty = r2 >> 4;
      const int yf = y0 + ty, xb = x0 + tx;
      if (yf < K && xb < K)
        T3g[(((size_t)yf * P + l) * K + xb) * P + wb] = T3s[(ty * TX + tx) * P2 + wb * 16 + l];
    }
    // (e) local update: Yt[(ty, l)][yb] += sum_{tx, wb} T3[(ty, l)][(tx, wb)] G[(tx, wb)][yb]
    if (v.do_local) {
      const int half = split_e ? wave / (kVisitWaves / 2) : 0;
      const int wt = split_e ? wave % (kVisitWaves / 2) : wave;
      const int wstep = split_e ? kVisitWaves / 2 : kVisitWaves;
#pragma unroll
      for (int q = 0; q < kMaxE; ++q) {
        const int t = wt + q * wstep;
        if (t >= ntile_e) break;
        const int ty = t / tne, n0 = (t % tne) << 4;
        Acc acc[2] = {accE[q], zero};
#pragma unroll
        for (int tx = 0; tx < TX; ++tx)
#pragma unroll
          for (int wh = 0; wh < 2; ++wh) {  // wb in [8 wh, 8 wh + 8)
            if (split_e && ((tx * 2 + wh) & 1) != half) continue;
            mma_steps<2>(acc, T3s + (ty * TX + tx) * P2 + (wh * 8 + lq) * 16 + lr, 64,
                         Gs + (tx * 16 + wh * 8 + lq) * GS + n0 + lr, 4 * GS);
          }
        accE[q] = acc[0] + acc[1];
      }
    }
  }
  if (v.do_local && split_e) {  // add the second k half into the first
    __syncthreads();
    T *red = sm;
    if (wave >= kVisitWaves / 2) {
      const int wt = wave - kVisitWaves / 2;
#pragma unroll
      for (int q = 0; q < kMaxE; ++q) {
        const int t = wt + q * (kVisitWaves / 2);
        if (t >= ntile_e) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(t * 4 + r) * 64 + lane] = accE[q][r];
      }
    }
    __syncthreads();
    if (wave < kVisitWaves / 2) {
#pragma unroll
      for (int q = 0; q < kMaxE; ++q) {
        const int t = wave + q * (kVisitWaves / 2);
        if (t >= ntile_e) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) accE[q][r] += red[(t * 4 + r) * 64 + lane];
      }
    }
  }
  if (v.do_local && (!split_e || wave < kVisitWaves / 2)) {
    auto *Y = gmem(v.Y.at(it));
    const int wstep = split_e ? kVisitWaves / 2 : kVisitWaves;
#pragma unroll
    for (int q = 0; q < kMaxE; ++q) {
      const int t = wave + q * wstep;
      if (t >= ntile_e) break;
      const int ty = t / tne, n0 = (t % tne) << 4, yf = y0 + ty, yb = n0 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int l = M::crow(r, lq);
        if (yb < K && yf < K) {
          const size_t idx = rl ? ((size_t)yb * P + l) * K + yf : ((size_t)yf * P + l) * K + yb;
          Y[idx] = (double)accE[q][r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same visit with one (yf, xb) pair per wave (TY * TX waves): each wave
// runs T1 -> ket -> bra -> T3 store -> its local-update contribution for its
// own pair with wave-level LDS ordering only, so an xb step needs just the
// two barriers around the X/G refill.  The local-update partials of the TX
// waves that share yf are summed at the end in a fixed order.
//
// The ket's output tile for one s, C[(wfb, abx)][(lk, wbk)], sits in the MFMA
// accumulator with register i of lane (lr, lq) holding row 4i + lq (FP64) or
// 4lq + i (FP32) of column lr: that is the bra's A operand (rows (lk, wbk),
// k = (s, wfb, abx)) for k step i, with the bra's B rows read in the matching
// k order.  T2 therefore never leaves registers.  T1 and T3 share one LDS
// region per pair (T1 is consumed by the ket before the bra writes T3).
//
// NE = ceil(K / 16) bounds the local-update tiles; each thread moves LD
// elements of the X and G tiles per step.
// LDS: Fs [(ty, wf)][xf] (row stride pad_a_min(K4)); Xs [tx][xf][a] (rows
// of 16, tile stride 16 K4 + 32 / TX); per pair T1 [wfk,akx][wfb,abx] and
// T3 [wbk,wbb][lk,lb] (rows of 16); Gs [(tx, wb)][yb] (stride pad_b(K));
// Ak, Ab [s][wf][a][l][wb].  Rows of Fs, Xs, T1, T3 and Gs are stored with
// their column index XOR-ed by a function of the row (v4p_*_sw below), which
// leaves every MFMA operand read conflict-free and also makes the accesses
// that walk a column (the refill stores, the MFMA result stores, the T3 read
// for the HBM store) hit distinct LDS banks, for both a half wave over 32
// 8-byte banks and a quarter wave over 16 (the F, T1 and T3 swizzles were
// chosen to satisfy both).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int v4p_x_sw(int xf) { return (xf >> 1) & 15; }
__host__ __device__ constexpr int v4p_t1_sw(int k) { return (k & 3) << 2; }
__host__ __device__ constexpr int v4p_t3_sw(int wb) {
  return ((wb & 3) << 2) ^ (((wb >> 2) & 1) * 5) ^ (((wb >> 3) & 1) << 1);
}
__host__ __device__ constexpr int v4p_f_sw(int row) { return (row >> 3) & 1; }
__host__ __device__ constexpr int v4p_g_sw(int row) { return ((row >> 1) ^ ((row >> 4) << 2)) & 15; }
__host__ __device__ constexpr int v4p_xt(int K4, int TX) { return 16 * K4 + 32 / TX; }
template <class T>
__host__ __device__ inline size_t visit4p_lds(int K, int TY, int TX) {
  typedef Mma<T> M;
  const int K4 = ceil4(K), tne = ceil16(K) / 16;
  const size_t body = (size_t)TY * 16 * M::pad_a_min(K4) + (size_t)TX * v4p_xt(K4, TX) +
                      (size_t)TY * TX * 256 + (size_t)TX * 16 * M::pad_b(K) + 2 * 2 * 256;
  return std::max(body, (size_t)TY * TX * tne * 256);
}

// One wave per (yf, xb) pair of a TY x TX tile: NT threads.  LD elements of
// each of the X and G tiles (16 NE x 16 x TX) per thread and step.  Up to
// NE = 3 (K <= 48) three workgroups share a CU (2 x 2 pairs at NE = 2, LDS
// <= 47 KB; 4 x 1 at NE = 3, LDS <= 52 KB), so the registers are held to 3
// waves per SIMD; at NE = 4 to 2, and for the 1 x 4 tiles of small batches
// (which leave most of the CUs free anyway) to 2.
template <int TY, int TX, int NE>
struct Visit4pShape {
  static constexpr int NWV = TY * TX, NT = 64 * NWV;
  static constexpr int LD = (NE * 16 * 16 * TX + NT - 1) / NT;
};

template <int TY, int TX, class T, int NE>
__global__ __launch_bounds__(64 * TY * TX)
__attribute__((amdgpu_waves_per_eu(NE <= 3 && TY > 1 ? 3 : 2)))
void k_visit4p(VisitArgs v) {
  constexpr int NT = Visit4pShape<TY, TX, NE>::NT, NWV = Visit4pShape<TY, TX, NE>::NWV;
  extern __shared__ double sm_raw[];
  T *sm = reinterpret_cast<T *>(sm_raw);
  typedef Mma<T> M;
  typedef typename M::acc Acc;
  const Acc zero = Acc{0, 0, 0, 0};
  constexpr int D = 4, P = 16, P2 = 256, NP = TY * TX;
  constexpr int LD = Visit4pShape<TY, TX, NE>::LD;
  constexpr bool f64 = sizeof(T) == 8;
  const int K = v.K, K4 = ceil4(K), FS = M::pad_a_min(K4), GS = M::pad_b(K), KY = ceil16(K);
  const int XT = v4p_xt(K4, TX);
  int tile, it;
  xcd_tile_item(&tile, &it);
  const int y0 = tile * TY;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  // True extents of this item's operands; every slot entry beyond them is
  // zero, so tiles, xb steps, k blocks and local-update tiles past them
  // would only add zeros: they are skipped, which leaves every sum's order
  // over its nonzero terms, and so its bits, unchanged.  Y is still written
  // in full (zeros in the padding).
  int nyf = K, nyb = K, nxf = K, nxb = K;
  if (v.dims) {
    const SiteExt ex = site_ext(v.dims[(size_t)it * v.W + v.c], v.j, v.N, v.rl != 0);
    nyf = ex.yf;
    nyb = ex.yb;
    nxf = ex.xf;
    nxb = ex.xb;
  }
  if (y0 >= nyf) {  // every front bond of the tile is padding: Y rows are zero
    if (v.do_local) {
      auto *Yz = gmem(v.Y.at(it));
      const int rows = min(TY, K - y0);
      for (int i = tid; i < rows * P * K; i += NT) {
        const int yb = i % K, l = (i / K) % P, yf = y0 + i / (K * P);
        Yz[v.rl ? ((size_t)yb * P + l) * K + yf : ((size_t)yf * P + l) * K + yb] = 0.0;
      }
    }
    return;
  }
  const int K4x = ceil4(nxf), tnb = ceil16(nyb) >> 4;
  T *Fs = sm;
  T *Xs = Fs + TY * 16 * FS;
  T *T13s = Xs + TX * XT;
  T *Gs = T13s + NP * P2;
  T *Ak = Gs + TX * 16 * GS;
  T *Ab = Ak + 2 * P2;
  const auto *F = gmem((const double *)v.F.at(it));
    const double *ak = v.aket + (size_t)it * v.aket_stride;
  const double *ab = v.abra + (size_t)it * v.abra_stride;
  T *T3g = reinterpret_cast<T *>(v.t3) + (size_t)it * v.t3_stride;
  const __amdgpu_buffer_rsrc_t t3rs =
      __builtin_amdgcn_make_buffer_rsrc(T3g, 0, (int)((unsigned)K * P * K * P * sizeof(T)), 0x00020000);
  const bool rl = v.rl != 0;
  const int ty = wave / TX, tx = wave % TX, pp = wave;  // this wave's pair
  T *Tp = T13s + pp * P2;

  for (int i = tid; i < 2 * P2; i += NT) {
    const int wb = i & 3, l = (i >> 2) & 3, a = (i >> 4) & 3, wf = (i >> 6) & 3, s = i >> 8;
    const int u = rl ? wb : wf, dd = rl ? wf : wb;
    const int src = ((((s * D + u) * D + l) * D + dd) * D + a);
    Ak[i] = (T)ak[src];
    Ab[i] = (T)ab[src];
  }
  for (int row = wave; row < TY * 16; row += NWV) {
    const bool ok = y0 + (row >> 4) < nyf;
    for (int xf = lane; xf < K4; xf += 64)
      Fs[row * FS + (xf ^ v4p_f_sw(row))] = (T)((ok && xf < nxf) ? F[(size_t)(y0 * P + row) * K + xf] : 0.0);
  }
  const int tne = KY >> 4;  // <= NE
  Acc accE[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) accE[q] = zero;

  // X and G of the next xb step are fetched into registers while the
  // current step computes.  Thread element u is i = tid + NT u of the tile
  // [xf][a][tx] (rl: [tx][a][xf]) and [yb][wb][tx], each index taken over
  // the compile-time extent XF = 16 NE >= K4; the decode is recomputed where
  // needed rather than held in registers.
  constexpr int XF = 16 * NE, NX = XF * 16 * TX;
  auto xdec = [&](int u, int &txx, int &a, int &xf) {
    const int i = tid + u * NT;
    if (rl) {
      xf = i % XF;
      a = (i / XF) & 15;
      txx = i / (XF * 16);
    } else {
      txx = i % TX;
      a = (i / TX) & 15;
      xf = i / (TX * 16);
    }
  };
  auto gdec = [&](int u, int &gtx, int &wb, int &yb) {
    const int i = tid + u * NT;
    gtx = i % TX;
    wb = (i / TX) & 15;
    yb = i / (TX * 16);
  };
  // raw loads of the pending step: nothing waits on them before the refill at
  // the next step.  X and G of one item are K P K doubles each; an element
  // outside the tile loads at offset K P K doubles, past the descriptor's
  // range, and reads zero.  Without the local update there is no G (null):
  // nothing is loaded from it.
  double xr[LD], gr[LD];
  const unsigned xgbytes = (unsigned)K * P * K * sizeof(double);
  const __amdgpu_buffer_rsrc_t xrs = buf_rsrc(v.X.at(it), xgbytes);
  const __amdgpu_buffer_rsrc_t grs = buf_rsrc(v.do_local ? v.G.at(it) : v.X.at(it), xgbytes);
  auto fetch = [&](int x0) {
#pragma unroll
    for (int u = 0; u < LD; ++u) {
      int txx, a, xf;
      xdec(u, txx, a, xf);
      const bool xv = tid + u * NT < NX && xf < nxf && x0 + txx < nxb;
      const unsigned off = rl ? ((x0 + txx) * P + a) * K + xf : (xf * P + a) * K + x0 + txx;
      xr[u] = buf_ld(xrs, xv ? off * 8u : xgbytes);
    }
    if (v.do_local) {
#pragma unroll
      for (int u = 0; u < LD; ++u) {
        int gtx, wb, yb;
        gdec(u, gtx, wb, yb);
        const bool gv = tid + u * NT < NX && yb < nyb && x0 + gtx < nxb;
        gr[u] = buf_ld(grs, gv ? ((yb * P + wb) * K + x0 + gtx) * 8u : xgbytes);
      }
    }
  };
  fetch(0);

  for (int x0 = 0; x0 < nxb; x0 += TX) {
    __syncthreads();  // the previous step's readers of Xs, Gs and T3 are done
#pragma unroll
    for (int u = 0; u < LD; ++u) {  // rows up to K4 and K rows of G (zero where not real)
      if (tid + u * NT >= NX) continue;
      int txx, a, xf, gtx, wb, yb;
      xdec(u, txx, a, xf);
      gdec(u, gtx, wb, yb);
      if (xf < K4) Xs[txx * XT + xf * 16 + (a ^ v4p_x_sw(xf))] = (T)xr[u];
      const int grow = gtx * 16 + wb;
      if (yb < KY) Gs[grow * GS + (yb ^ v4p_g_sw(grow))] = (T)(v.do_local ? gr[u] : 0.0);
    }
    __syncthreads();
    if (x0 + TX < nxb) fetch(x0 + TX);
    // (a) T1 of the pair: rows wf, cols a, k = xf
    {
      Acc acc[2] = {zero, zero};
      const T *pa = Fs + (ty * 16 + lr) * FS + (lq ^ v4p_f_sw(lr));
      const T *px = Xs + tx * XT;
      // Xs row xf = k0 + lq (k0 = 0 mod 4): swizzle ((k0 >> 1) & 15) ^ (lq >> 1)
      const int xb0 = lq * 16 + (lr ^ (lq >> 1));
      int k0 = 0;
      for (; k0 + 16 <= K4x; k0 += 16) {
        const T *pk = px + k0 * 16;
        const int sw = (k0 >> 1) & 8;
        T av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          av[i] = pa[k0 + 4 * i];
          bv[i] = pk[(xb0 ^ (sw | 2 * i)) + 64 * i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i & 1] = M::run(av[i], bv[i], acc[i & 1]);
      }
      for (; k0 < K4x; k0 += 4)
        acc[0] = M::run(pa[k0], px[k0 * 16 + (xb0 ^ ((k0 >> 1) & 15))], acc[0]);
      const Acc c = acc[0] + acc[1];
      // a = lr (akx = lr/4, abx = lr%4), wf = (wfk, wfb): row (wfk, akx),
      // column (wfb, abx)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int wf = M::crow(r, lq), row = (wf >> 2) * 4 + (lr >> 2);
        Tp[row * 16 + (((wf & 3) * 4 + (lr & 3)) ^ v4p_t1_sw(row))] = c[r];
      }
    }
    wave_lds_order();
    // (b) ket, one tile per s: rows m = (wfb, abx), k = (wfk, akx), cols n = (lk, wbk)
    Acc t2[2];
#pragma unroll
    for (int sn = 0; sn < 2; ++sn) {
      Acc acc[2] = {zero, zero};
      // T1 row 4i + lq: its swizzle depends on lq only
      mma_steps<4>(acc, Tp + lq * 16 + (lr ^ v4p_t1_sw(lq)), 64, Ak + sn * P2 + lq * 16 + lr, 64);
      t2[sn] = acc[0] + acc[1];
    }
    wave_lds_order();  // every lane's T1 reads precede the T3 writes below
    // (c) bra: rows m = (lk, wbk), k = (s, wfb, abx), cols n = (lb, wbb); the
    // A operand of k step i is register i of t2[s]
    {
      Acc acc[2] = {zero, zero};
#pragma unroll
      for (int sn = 0; sn < 2; ++sn) {
        // B rows in the order the accumulator holds k: 4i + lq (FP64), 4lq + i (FP32)
        const T *pb = f64 ? Ab + (sn * 16 + lq) * 16 + lr : Ab + (sn * 16 + 4 * lq) * 16 + lr;
        constexpr int db = f64 ? 64 : 16;
        T bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = pb[i * db];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i & 1] = M::run(t2[sn][i], bv[i], acc[i & 1]);
      }
      const Acc c = acc[0] + acc[1];
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // m = (lk, wbk), n = lr = (lb, wbb)
        const int m = M::crow(r, lq), wb = (m & 3) * 4 + (lr & 3), l = (m >> 2) * 4 + (lr >> 2);
        Tp[wb * 16 + (l ^ v4p_t3_sw(wb))] = c[r];
      }
    }
    wave_lds_order();
    // T3 of the pair to HBM as T3[yf][l][xb][wb] (16 lanes per 128-byte row),
    // through the item's descriptor (32-bit offsets)
    {
      const int yf = y0 + ty, xb = x0 + tx;
      if (yf < nyf && xb < nxb) {
        const unsigned o0 = (unsigned)(yf * P * K + xb) * P;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int idx = u * 64 + lane, wb = idx & 15, l = idx >> 4;
          buf_st_t<T>(t3rs, (o0 + (unsigned)(l * K * P + wb)) * (unsigned)sizeof(T),
                      Tp[wb * 16 + (l ^ v4p_t3_sw(wb))]);
        }
      }
    }
    // (e) this pair's contribution to Yt[(ty, l)][yb]: k = wb of column tx
    if (v.do_local) {
      // A: T3 row wb = 4i + lq, column lr: swizzle t3_sw(lq) ^ t3_sw(4i) (linear);
      // B: Gs row tx 16 + 4i + lq: swizzle w ^ (lq >> 1) ^ 2i, w from tx
      const int ta = lq * 16 + (lr ^ v4p_t3_sw(lq));
      const int w = ((tx & 1) << 3) ^ ((tx << 2) & 15);
      const int gb = (tx * 16 + lq) * GS + (lr ^ w ^ (lq >> 1));
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        if (q >= tnb) break;
        T av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          av[i] = Tp[(ta ^ v4p_t3_sw(4 * i)) + 64 * i];
          bv[i] = Gs[(gb ^ (2 * i)) + 4 * i * GS + q * 16];
        }
        Acc acc[2] = {accE[q], zero};
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i & 1] = M::run(av[i], bv[i], acc[i & 1]);
        accE[q] = acc[0] + acc[1];
      }
    }
  }
  if (!v.do_local) return;
  // sum the TX partials of each yf tile in a fixed order (tx = 0, 1, ...)
  __syncthreads();
  T *red = sm;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    if (q >= tne) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) red[((pp * tne + q) * 4 + r) * 64 + lane] = accE[q][r];
  }
  __syncthreads();
  if (tx != 0) return;
  auto *Y = gmem(v.Y.at(it));
  const int yf = y0 + ty;
#pragma unroll
  for (int q = 0; q < NE; ++q) {
    if (q >= tne) break;
    const int yb = q * 16 + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      T acc = red[((pp * tne + q) * 4 + r) * 64 + lane];
      for (int t2i = 1; t2i < TX; ++t2i) acc += red[(((pp + t2i) * tne + q) * 4 + r) * 64 + lane];
      const int l = M::crow(r, lq);
      if (yb < K && yf < K) {
        const size_t idx = rl ? ((size_t)yb * P + l) * K + yf : ((size_t)yf * P + l) * K + yb;
        Y[idx] = (double)acc;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Householder QR (LAPACK conventions: dlarfg reflectors, dorg2r formation).
// One workgroup per item; the true panel (rows r = r1*n2 + r2, columns c at
// base[r1*s1 + r2*s2 + c*sc]) is copied column-major into LDS, factorised,
// and Q written back in place (panels too large for LDS: k_qrg below).
// ---------------------------------------------------------------------------
// x / n and x % n for 0 <= x < 2^22 and 1 <= n < 2^22 through one FP32
// multiply: x and 1/n are within one rounding of exact, so the truncated
// product is the quotient or one off, and the remainder's sign and size
// correct it.  Replaces an integer division (a few dozen VALU operations)
// in the panel copies.
struct DivN {
  int n;
  float inv;
  __device__ explicit DivN(int n_) : n(n_), inv(1.0f / (float)n_) {}
  __device__ __forceinline__ int quot(int x) const {
    int q = (int)((float)x * inv);
    const int r = x - q * n;
    if (r < 0) --q;
    else if (r >= n) ++q;
    return q;
  }
};

struct QrArgs {
  FitDims *dims;
  int W, c, j, mode, K, P;
  Ptr Y;
  double *rbuf;
  double *scratch;
  size_t scratch_stride;
  const int32_t *flag;
  int want_r;
};

constexpr int kQrLds = 19968;  // doubles (156 KB of the 160 KB LDS)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kThreads) void k_qr(QrArgs q) {
  const int it = blockIdx.x;
  if (q.flag && !q.flag[it]) return;
  const FitDims &dm = q.dims[(size_t)it * q.W + q.c];
  const int K = q.K, P = q.P, j = q.j;
  int n1, n2, ncol;
  size_t s1, s2, sc;
  switch (q.mode) {
    case LR_INNER:
      n1 = dm.bl[j]; s1 = (size_t)P * K; n2 = P; s2 = K; ncol = dm.br[j]; sc = 1;
      break;
    case RL_INNER:  // rows (l, yb), l-major, as in the QR of the transpose
      n1 = P; s1 = K; n2 = dm.br[j]; s2 = 1; ncol = dm.bl[j]; sc = (size_t)P * K;
      break;
    case LR_TOP:
      n1 = dm.p[j]; s1 = K; n2 = 1; s2 = 0; ncol = dm.br[j]; sc = 1;
      break;
    default:  // RL_BOT
      n1 = dm.p[j]; s1 = 1; n2 = 1; s2 = 0; ncol = dm.bl[j]; sc = K;
      break;
  }
  const int m = n1 * n2, n = ncol;
  double *base = q.Y.at(it);
  __shared__ double lds[kQrLds];
  __shared__ double red[8];
  __shared__ double tau_s[128];
  double *A = lds;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  const DivN divm(m), dn2(n2);
  for (int idx = tid; idx < m * n; idx += kThreads) {
    const int col = divm.quot(idx), r = idx - col * m;
    const int r1 = dn2.quot(r), r2 = r - r1 * n2;
    A[idx] = base[r1 * s1 + r2 * s2 + col * sc];
  }
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    double *v = A + (size_t)k * m;
    double part = 0.0;
    for (int i = k + 1 + tid; i < m; i += kThreads) part += v[i] * v[i];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) {
      const double sigma2 = red[0] + red[1] + red[2] + red[3];
      const double alpha = v[k];
      double tau = 0.0, scal = 0.0, beta = alpha;
      if (sigma2 > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      tau_s[k] = tau;
      red[4] = scal;
      v[k] = beta;
    }
    __syncthreads();
    const double scal = red[4], tau = tau_s[k];
    if (tau != 0.0)
      for (int i = k + 1 + tid; i < m; i += kThreads) v[i] *= scal;
    __syncthreads();
    if (tau != 0.0) {
      for (int jj = k + 1 + wave; jj < n; jj += kThreads / 64) {
        double *a = A + (size_t)jj * m;
        double w = 0.0;
        for (int i = k + 1 + lane; i < m; i += 64) w += v[i] * a[i];
        w = wave_sum(w) + a[k];
        w *= tau;
        if (lane == 0) a[k] -= w;
        for (int i = k + 1 + lane; i < m; i += 64) a[i] -= v[i] * w;
      }
    }
    __syncthreads();
  }

  if (q.want_r) {
    double *R = q.rbuf + (size_t)it * K * K;
    for (int idx = tid; idx < K * K; idx += kThreads) {
      const int r = idx / K, cc = idx - r * K;
      R[idx] = (r < n && cc < n && r <= cc) ? A[(size_t)cc * m + r] : 0.0;
    }
  }
  __syncthreads();

  // Q = H_0 ... H_{n-1} [I; 0], formed in place from the last reflector.
  for (int k = n - 1; k >= 0; --k) {
    double *v = A + (size_t)k * m;
    const double tau = tau_s[k];
    if (k < n - 1 && tau != 0.0) {
      for (int jj = k + 1 + wave; jj < n; jj += kThreads / 64) {
        double *a = A + (size_t)jj * m;
        double w = 0.0;
        for (int i = k + 1 + lane; i < m; i += 64) w += v[i] * a[i];
        w = wave_sum(w) + a[k];
        w *= tau;
        if (lane == 0) a[k] -= w;
        for (int i = k + 1 + lane; i < m; i += 64) a[i] -= v[i] * w;
      }
    }
    __syncthreads();
    for (int i = tid; i < m; i += kThreads) {
      if (i > k) v[i] *= -tau;
      else if (i == k) v[i] = 1.0 - tau;
      else v[i] = 0.0;
    }
    __syncthreads();
  }

  for (int idx = tid; idx < m * n; idx += kThreads) {
    const int col = divm.quot(idx), r = idx - col * m;
    const int r1 = dn2.quot(r), r2 = r - r1 * n2;
    base[r1 * s1 + r2 * s2 + col * sc] = A[idx];
  }
}

// ---------------------------------------------------------------------------
// The same Householder QR for tall panels kept in a global scratch (D = 6
// and larger bonds): one workgroup of 16 waves per item.  Each reflector is
// staged in LDS once (read in place where a panel has more than kQrgRows
// rows), and a wave updates up to kQrgCols trailing columns in
// one pass over the rows (one dot product and one axpy per column, the
// columns' loads interleaved), so the trailing matrix is read twice and
// written once per reflector.  Reflectors, their order and the formation of
// Q are those of the kernel above.
// ---------------------------------------------------------------------------
constexpr int kQrgThreads = 1024;
constexpr int kQrgWaves = kQrgThreads / 64;
constexpr int kQrgRows = 8192;  // rows of the staged reflector (64 KB of LDS)
constexpr int kQrgCols = 8;     // trailing columns per wave and pass (n <= 128)

// a_c -= tau v (a_kc + v^T a_c) for the columns c = c0, c0 + kQrgWaves, ...
// (< n) of this wave; v = (1, vs[k+1..m-1]).  Rows go kQrgUnroll at a time
// per lane, their loads issued together (the panel streams from L2).
constexpr int kQrgUnroll = 2;
__device__ __forceinline__ void qrg_apply(double *A, const double *vs, int m, int n, int k,
                                          double tau, int c0, int lane) {
  double *a[kQrgCols];
  double w[kQrgCols];
  int nc = 0;
#pragma unroll
  for (int u = 0; u < kQrgCols; ++u) {
    const int c = c0 + u * kQrgWaves;
    a[u] = A + (size_t)(c < n ? c : k) * m;
    w[u] = 0.0;
    if (c < n) nc = u + 1;
  }
  if (nc == 0) return;
  for (int i0 = k + 1 + lane; i0 < m; i0 += 64 * kQrgUnroll) {
    double v[kQrgUnroll], x[kQrgUnroll][kQrgCols];
#pragma unroll
    for (int r = 0; r < kQrgUnroll; ++r) {
      const int i = i0 + 64 * r;
      v[r] = i < m ? vs[i] : 0.0;
#pragma unroll
      for (int u = 0; u < kQrgCols; ++u) x[r][u] = (u < nc && i < m) ? a[u][i] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kQrgUnroll; ++r)
#pragma unroll
      for (int u = 0; u < kQrgCols; ++u) w[u] = fma(v[r], x[r][u], w[u]);
  }
#pragma unroll
  for (int u = 0; u < kQrgCols; ++u) {
    if (u >= nc) break;
    w[u] = tau * (wave_sum(w[u]) + a[u][k]);
  }
  if (lane == 0) {
#pragma unroll
    for (int u = 0; u < kQrgCols; ++u)
      if (u < nc) a[u][k] -= w[u];
  }
  for (int i0 = k + 1 + lane; i0 < m; i0 += 64 * kQrgUnroll) {
    double v[kQrgUnroll], x[kQrgUnroll][kQrgCols];
#pragma unroll
    for (int r = 0; r < kQrgUnroll; ++r) {
      const int i = i0 + 64 * r;
      v[r] = i < m ? vs[i] : 0.0;
#pragma unroll
      for (int u = 0; u < kQrgCols; ++u) x[r][u] = (u < nc && i < m) ? a[u][i] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kQrgUnroll; ++r) {
      const int i = i0 + 64 * r;
      if (i >= m) break;
#pragma unroll
      for (int u = 0; u < kQrgCols; ++u)
        if (u < nc) a[u][i] = x[r][u] - v[r] * w[u];
    }
  }
}

// Copies between the strided panel and the column-major scratch, eight
// elements in flight per thread.
template <bool kIn>
__device__ __forceinline__ void qrg_copy(double *A, double *base, int m, int n, int n2,
                                         size_t s1, size_t s2, size_t sc, int tid) {
  constexpr int U = 8;
  const int total = m * n;
  const DivN divm(m), dn2(n2);
  for (int i0 = tid; i0 < total; i0 += kQrgThreads * U) {
    double x[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int idx = i0 + r * kQrgThreads;
      const int col = divm.quot(idx), row = idx - col * m;
      const int r1 = dn2.quot(row), r2 = row - r1 * n2;
      const size_t g = r1 * s1 + r2 * s2 + col * sc;
      x[r] = idx < total ? (kIn ? base[g] : A[idx]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int idx = i0 + r * kQrgThreads;
      if (idx >= total) break;
      const int col = divm.quot(idx), row = idx - col * m;
      const int r1 = dn2.quot(row), r2 = row - r1 * n2;
      const size_t g = r1 * s1 + r2 * s2 + col * sc;
      if (kIn) A[idx] = x[r];
      else base[g] = x[r];
    }
  }
}

__global__ __launch_bounds__(kQrgThreads) void k_qrg(QrArgs q) {
  const int it = blockIdx.x;
  if (q.flag && !q.flag[it]) return;
  const FitDims &dm = q.dims[(size_t)it * q.W + q.c];
  const int K = q.K, P = q.P, j = q.j;
  int n1, n2, ncol;
  size_t s1, s2, sc;
  switch (q.mode) {
    case LR_INNER:
      n1 = dm.bl[j]; s1 = (size_t)P * K; n2 = P; s2 = K; ncol = dm.br[j]; sc = 1;
      break;
    case RL_INNER:  // rows (l, yb), l-major, as in the QR of the transpose
      n1 = P; s1 = K; n2 = dm.br[j]; s2 = 1; ncol = dm.bl[j]; sc = (size_t)P * K;
      break;
    case LR_TOP:
      n1 = dm.p[j]; s1 = K; n2 = 1; s2 = 0; ncol = dm.br[j]; sc = 1;
      break;
    default:  // RL_BOT
      n1 = dm.p[j]; s1 = 1; n2 = 1; s2 = 0; ncol = dm.bl[j]; sc = K;
      break;
  }
  const int m = n1 * n2, n = ncol;
  double *base = q.Y.at(it);
  __shared__ double vs[kQrgRows];
  __shared__ double red[kQrgWaves];
  __shared__ double tau_s[128];
  __shared__ double scal_s;
  double *A = q.scratch + (size_t)it * q.scratch_stride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool stage = m <= kQrgRows;

  qrg_copy<true>(A, base, m, n, n2, s1, s2, sc, tid);
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    double *v = A + (size_t)k * m;
    double part = 0.0;
    for (int i = k + 1 + tid; i < m; i += kQrgThreads) part = fma(v[i], v[i], part);
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (tid == 0) {  // dlarfg
      double sigma2 = 0.0;
      for (int w = 0; w < kQrgWaves; ++w) sigma2 += red[w];
      const double alpha = v[k];
      double tau = 0.0, scal = 0.0, beta = alpha;
      if (sigma2 > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      tau_s[k] = tau;
      scal_s = scal;
      v[k] = beta;
    }
    __syncthreads();
    const double tau = tau_s[k];
    if (tau != 0.0) {
      const double scal = scal_s;
      for (int i = k + 1 + tid; i < m; i += kQrgThreads) {
        const double x = v[i] * scal;
        v[i] = x;
        if (stage) vs[i] = x;
      }
      __syncthreads();
      qrg_apply(A, stage ? vs : v, m, n, k, tau, k + 1 + wave, lane);
    }
    __syncthreads();
  }

  if (q.want_r) {
    double *R = q.rbuf + (size_t)it * K * K;
    for (int idx = tid; idx < K * K; idx += kQrgThreads) {
      const int r = idx / K, cc = idx - r * K;
      R[idx] = (r < n && cc < n && r <= cc) ? A[(size_t)cc * m + r] : 0.0;
    }
  }
  __syncthreads();

  // Q = H_0 ... H_{n-1} [I; 0], formed in place from the last reflector.
  for (int k = n - 1; k >= 0; --k) {
    double *v = A + (size_t)k * m;
    const double tau = tau_s[k];
    if (stage)
      for (int i = k + 1 + tid; i < m; i += kQrgThreads) vs[i] = v[i];
    __syncthreads();
    if (k < n - 1 && tau != 0.0) qrg_apply(A, stage ? vs : v, m, n, k, tau, k + 1 + wave, lane);
    if (!stage) __syncthreads();  // column k is read in place by the update
    for (int i = tid; i < m; i += kQrgThreads) {
      if (i > k) v[i] = -tau * (stage ? vs[i] : v[i]);
      else if (i == k) v[i] = 1.0 - tau;
      else v[i] = 0.0;
    }
    __syncthreads();
  }

  qrg_copy<false>(A, base, m, n, n2, s1, s2, sc, tid);
}

// ---------------------------------------------------------------------------
// Blocked Householder QR on FP64 MFMA tiles, one workgroup of NW waves per
// item.  The panel stays in registers as 16x16 tiles in the MFMA accumulator
// layout (register s of lane l holds row 4s + l/16, column l%16 of its tile);
// wave w owns row tiles w, w + NW, ... of every column tile.  Columns are
// factorised in blocks of 16 as in dgeqrf.  Inside a block, step k
// broadcasts column k along each 16-lane row (DPP row_newbcast) and forms,
// in one pass and one cross-wave sum, x^T a_c for every column c (x = column
// k below the diagonal) and the row-k entries a_kc; column k's own entries
// give sigma^2 and alpha for dlarfg, and w_c = a_kc + scal x^T a_c gives the
// dlarf update of the block's later columns.  The block reflector
// I - V T V^T (T from dlarft) is then applied to the columns on the right on
// MFMA (W = V^T A, A -= V T^T W).  Q is formed backwards over the blocks as
// in dorgqr: the block reflector updates the columns on the right, and the
// block's own columns are E - V (T V_top^T), E the unit columns, both on
// MFMA.  The reflectors are those of the unblocked algorithm (dgeqr2); only
// the rounding order of sums and updates differs.  Cross-wave sums are taken
// in a fixed order that every wave repeats, so all waves hold the same bits.
// ---------------------------------------------------------------------------

constexpr int kQmRowCap = 768;        // rows held by one workgroup, at most
// V column c of the block starts at c * kQmVs + (c & 14) doubles: with the
// column stride 16 (mod 32) and that shift, both the per-lane column walk
// (lane (lr, lc) reads column lc, rows 4s + lr) and the MFMA operand read
// (column 4kk + lr, row lc) touch 32 distinct banks per half-wave, and the
// per-lane part of every address stays a base plus compile-time offsets.
constexpr int kQmVs = kQmRowCap + 16;
__device__ __forceinline__ int qm_col(int c) { return c * kQmVs + (c & 14); }

__device__ __forceinline__ double join_f64(int lo, int hi) {
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the four 16-lane rows: row pairs (0,1), (2,3) through
// permlane16_swap, then the two pair sums through permlane32_swap; the same
// bits land in every row.
__device__ __forceinline__ double sum_rows4(double x) {
  long long b = __double_as_longlong(x);
  auto lo = __builtin_amdgcn_permlane16_swap((int)b, (int)b, false, false);
  auto hi = __builtin_amdgcn_permlane16_swap((int)(b >> 32), (int)(b >> 32), false, false);
  x = join_f64(lo[0], hi[0]) + join_f64(lo[1], hi[1]);
  b = __double_as_longlong(x);
  lo = __builtin_amdgcn_permlane32_swap((int)b, (int)b, false, false);
  hi = __builtin_amdgcn_permlane32_swap((int)(b >> 32), (int)(b >> 32), false, false);
  return join_f64(lo[0], hi[0]) + join_f64(lo[1], hi[1]);
}

__device__ __forceinline__ int cl_index(int i, int j) {  // accumulator slot of (i, j)
  return (i >> 2) * 64 + (i & 3) * 16 + j;
}

template <int CTRL, int N>
__device__ __forceinline__ void newbcast_all(double *d, const double *x) {
#pragma unroll
  for (int i = 0; i < N; ++i)
    d[i] = __longlong_as_double(
        __builtin_amdgcn_mov_dpp(__double_as_longlong(x[i]), CTRL, 0xf, 0xf, true));
}

// d[i] = x[i] of lane `src` of the same 16-lane row (64-bit row_newbcast)
template <int N>
__device__ __forceinline__ void row_bcast(double *d, const double *x, int src) {
  switch (src) {
    case 0: newbcast_all<0x150, N>(d, x); break;
    case 1: newbcast_all<0x151, N>(d, x); break;
    case 2: newbcast_all<0x152, N>(d, x); break;
    case 3: newbcast_all<0x153, N>(d, x); break;
    case 4: newbcast_all<0x154, N>(d, x); break;
    case 5: newbcast_all<0x155, N>(d, x); break;
    case 6: newbcast_all<0x156, N>(d, x); break;
    case 7: newbcast_all<0x157, N>(d, x); break;
    case 8: newbcast_all<0x158, N>(d, x); break;
    case 9: newbcast_all<0x159, N>(d, x); break;
    case 10: newbcast_all<0x15A, N>(d, x); break;
    case 11: newbcast_all<0x15B, N>(d, x); break;
    case 12: newbcast_all<0x15C, N>(d, x); break;
    case 13: newbcast_all<0x15D, N>(d, x); break;
    case 14: newbcast_all<0x15E, N>(d, x); break;
    default: newbcast_all<0x15F, N>(d, x); break;
  }
}

// f(integral_constant<int, I>) for I = I0 .. N-1, unrolled at compile time.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int NW, int RT, int CT>
__global__ __launch_bounds__(NW * 64) void k_qrm(QrArgs q) {
  static_assert(NW % 4 == 0 && NW >= CT && 16 * NW * RT <= kQmRowCap, "panel shape");
  const int it = blockIdx.x;
  if (q.flag && !q.flag[it]) return;
  const FitDims &dm = q.dims[(size_t)it * q.W + q.c];
  const int K = q.K, P = q.P, j = q.j;
  int n1, n2, ncol;
  size_t s1, s2, sc;
  switch (q.mode) {
    case LR_INNER:
      n1 = dm.bl[j]; s1 = (size_t)P * K; n2 = P; s2 = K; ncol = dm.br[j]; sc = 1;
      break;
    case RL_INNER:  // rows (l, yb), l-major, as in the QR of the transpose
      n1 = P; s1 = K; n2 = dm.br[j]; s2 = 1; ncol = dm.bl[j]; sc = (size_t)P * K;
      break;
    case LR_TOP:
      n1 = dm.p[j]; s1 = K; n2 = 1; s2 = 0; ncol = dm.br[j]; sc = 1;
      break;
    default:  // RL_BOT
      n1 = dm.p[j]; s1 = 1; n2 = 1; s2 = 0; ncol = dm.bl[j]; sc = K;
      break;
  }
  const int m = n1 * n2, n = min(ncol, m);
  double *base = q.Y.at(it);
  __shared__ double VT[16 * kQmVs];  // V of the current block, column c at qm_col(c)
  __shared__ double wred[NW][256];
  __shared__ double Ws[256], Zs[256];
  __shared__ double Tm[CT][16][16];
  __shared__ double wp[2][NW][16], wq[2][16];
  __shared__ double tau_s[16 * CT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane >> 4, lc = lane & 15;
  // Row tiles t > 0 start at row 16 * NW >= n, below every diagonal entry.
  auto rowof = [&](int t, int s) { return 16 * (wave + NW * t) + 4 * s + lr; };
  const DivN dn2(n2);
  auto gaddr = [&](int row, int col) {
    const int r1 = dn2.quot(row), r2 = row - r1 * n2;
    return r1 * s1 + r2 * s2 + col * sc;
  };

  v4d a[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = rowof(t, s), col = 16 * ct + lc;
        a[t][ct][s] = (row < m && col < n) ? base[gaddr(row, col)] : 0.0;
      }

  // Column tile b's reflectors to LDS: 0 above the diagonal, 1 on it.
  auto store_v = [&](int b, int nbb) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = rowof(t, s), pr = 16 * b + lc;
        VT[qm_col(lc) + row] = lc < nbb ? ((t > 0 || row > pr) ? a[t][b][s] : (row == pr ? 1.0 : 0.0))
                               : 0.0;
      }
    wave_lds_order();
  };

  // Sum of the per-wave 16x16 accumulators into Ws (accumulator slots).
  auto reduce_tiles = [&](const v4d &acc) {
#pragma unroll
    for (int r = 0; r < 4; ++r) wred[wave][r * 64 + lane] = acc[r];
    __syncthreads();
    if (tid < 256) {
      double x = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) x += wred[w][tid];
      Ws[tid] = x;
    }
    __syncthreads();
  };

  // C += V Zs for column tile ct, Zs = -(16x16 coefficients), K = 16 (MFMA)
  auto update_tile = [&](v4d (&c)[RT]) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        c[t] = mfma16(VT[qm_col(4 * kk + lr) + 16 * (wave + NW * t) + lc],
                      Zs[(4 * kk + lr) * 16 + lc], c[t]);
  };

  // C -= V op(T) (V^T C) for the column tiles right of block b.
  auto apply_block = [&](int b, bool trans) {
    double xo[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) xo[t][s] = VT[qm_col(lc) + 16 * (wave + NW * t) + 4 * s + lr];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      if (ct <= b || 16 * ct >= n) continue;
      v4d acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s & 1] = mfma16(xo[t][s], a[t][ct][s], acc[s & 1]);
      reduce_tiles(acc[0] + acc[1]);  // W = V^T C
      if (tid < 256) {
        const int p = tid >> 4, jj = tid & 15;
        double z = 0.0;
#pragma unroll 4
        for (int qq = 0; qq < 16; ++qq)
          z += (trans ? Tm[b][qq][p] : Tm[b][p][qq]) * Ws[cl_index(qq, jj)];
        Zs[tid] = -z;
      }
      __syncthreads();
      v4d c[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) c[t] = a[t][ct];
      update_tile(c);
#pragma unroll
      for (int t = 0; t < RT; ++t) a[t][ct] = c[t];
    }
  };

  // ---- factorisation (dgeqrf order) ----
  int pb = 0;
#pragma unroll
  for (int b = 0; b < CT; ++b) {
    const int b0 = 16 * b;
    if (b0 >= n) break;
    const int nbb = min(16, n - b0);
    double my_scal = 0.0, my_beta = 0.0, my_tau = 0.0;  // of column b0 + lc
    // step kc of the block (KC: an int, or a compile-time constant whose
    // broadcast takes the source lane as an immediate)
    auto column = [&](auto KC) {
      const int kc = KC;
      if (kc >= nbb) return;
      const int k = b0 + kc;
      // x = column k below row k, broadcast along the rows from lane kc
      double cv[RT * 4], xb[RT * 4];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) cv[t * 4 + s] = a[t][b][s];
      if constexpr (std::is_integral_v<decltype(KC)>)
        row_bcast<RT * 4>(xb, cv, kc);  // source lane chosen at run time
      else
        newbcast_all<0x150 + decltype(KC)::value, RT * 4>(xb, cv);
      // x^T a_c over this wave's rows, and the row-k entries a_kc, which the
      // lanes holding row k store on their own
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = rowof(0, s);
        if (row <= k) xb[s] = 0.0;
        if (row == k) wq[pb][lc] = a[0][b][s];
      }
      double pp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) pp[s] = fma(xb[t * 4 + s], a[t][b][s], pp[s]);
      const double pdot = sum_rows4((pp[0] + pp[1]) + (pp[2] + pp[3]));
      if (lr == 0) wp[pb][wave][lc] = pdot;
      __syncthreads();
      // x^T a_c over all rows (the waves' partials summed pairwise in a
      // fixed order), for this lane's column and for column k; every lane
      // reads the same words per column, so all hold the same bits.  All
      // reads are issued before the first sum.
      double vp[NW], vs[NW];
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        vp[ww] = wp[pb][ww][lc];
        vs[ww] = wp[pb][ww][kc];
      }
      const double qc = wq[pb][lc];
      // dlarfg on column k: sigma^2 = x^T x, alpha = a_kk
      const double alpha = wq[pb][kc];
#pragma unroll
      for (int h = 1; h < NW; h *= 2)
#pragma unroll
        for (int ww = 0; ww + h < NW; ww += 2 * h) {
          vp[ww] += vp[ww + h];
          vs[ww] += vs[ww + h];
        }
      const double pc = vp[0], sigma2 = vs[0];
      pb ^= 1;
      double tau = 0.0, scal = 0.0, beta = alpha;
      if (sigma2 > 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      if (tid == 0) tau_s[k] = tau;
      if (lc == kc) {
        my_scal = scal;
        my_beta = beta;
        my_tau = tau;
      }
      // dlarf on the block's columns c > k: w_c = a_kc + scal x^T a_c,
      // a_c -= tau v w_c with v = (1, scal x)
      const double wt = (lc > kc && lc < nbb) ? -(tau * (qc + scal * pc)) : 0.0;
      const double cs = scal * wt;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a[t][b][s] = fma(xb[t * 4 + s], cs, a[t][b][s]);
          if (t == 0 && rowof(0, s) == k) a[0][b][s] += wt;
        }
        };
    // up to two column tiles the block's steps are unrolled (a lane switch
    // less per step: 512x32 panels 62.4 -> 54.2 us); at three the unrolled
    // code outgrows the instruction cache
    if constexpr (CT <= 2)
      static_for<0, 16>(column);
    else
      for (int kc = 0; kc < nbb; ++kc) column(kc);
    // reflectors scaled in place, beta on the diagonal
    if (lc < nbb) {
      const int pr = b0 + lc;
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int row = rowof(t, s);
          if (t > 0 || row > pr) {
            if (my_tau != 0.0) a[t][b][s] *= my_scal;
          } else if (row == pr) {
            a[t][b][s] = my_beta;
          }
        }
    }
    store_v(b, nbb);

    // Gram matrix V^T V of the block, then T as in dlarft (forward, columnwise)
    v4d g[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double x = VT[qm_col(lc) + 16 * (wave + NW * t) + 4 * s + lr];
        g[s & 1] = mfma16(x, x, g[s & 1]);
      }
    reduce_tiles(g[0] + g[1]);
    if (wave == 0) {
      // lane (lr, lc) keeps T[lc][lr + 4u]; column i of T needs columns < i
      double tr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double ti = i < nbb ? tau_s[b0 + i] : 0.0;
        double x = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (4 * u < i && lr + 4 * u < i) x += tr[u] * Ws[cl_index(lr + 4 * u, i)];
        x = sum_rows4(x);
        const double t = lc < i ? -ti * x : (lc == i ? ti : 0.0);
        if (lr == (i & 3)) tr[i >> 2] = t;
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) Tm[b][lc][lr + 4 * u] = tr[u];
    }
    __syncthreads();
    apply_block(b, true);
  }

  if (q.want_r) {
    double *Rm = q.rbuf + (size_t)it * K * K;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = rowof(0, s), col = 16 * ct + lc;
        if (row < K && col < K)
          Rm[(size_t)row * K + col] =
              (row < n && col < n && col >= row) ? a[0][ct][s] : 0.0;
      }
#pragma unroll
    for (int t = 1; t < RT; ++t)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int row = rowof(t, s), col = 16 * ct + lc;
          if (row < K && col < K) Rm[(size_t)row * K + col] = 0.0;
        }
  }

  // ---- Q = H_0 ... H_{n-1} [I; 0], backwards over the blocks (dorgqr) ----
#pragma unroll
  for (int b = CT - 1; b >= 0; --b) {
    const int b0 = 16 * b;
    if (b0 >= n) continue;
    const int nbb = min(16, n - b0);
    store_v(b, nbb);
    apply_block(b, false);
    __syncthreads();  // V of every wave visible
    // the block's own columns: E - V (T V_top^T), E the unit columns at rows b0..
    if (tid < 256) {
      const int p = tid >> 4, jj = tid & 15;
      double z = 0.0;
#pragma unroll 4
      for (int qq = 0; qq < 16; ++qq) z += Tm[b][p][qq] * VT[qm_col(qq) + b0 + jj];
      Zs[tid] = -z;
    }
    __syncthreads();
    v4d c[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        c[t][s] = (t == 0 && rowof(0, s) == b0 + lc && lc < nbb) ? 1.0 : 0.0;
    update_tile(c);
#pragma unroll
    for (int t = 0; t < RT; ++t) a[t][b] = c[t];
  }

  // Recompute the store addresses instead of keeping the load's alive.
  size_t os1 = s1, os2 = s2, osc = sc;
  int on2 = n2;
  asm volatile("" : "+s"(os1), "+s"(os2), "+s"(osc), "+s"(on2));
  const DivN don2(on2);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = rowof(t, s), col = 16 * ct + lc;
        const int r1 = don2.quot(row), r2 = row - r1 * on2;
        if (row < m && col < n) base[r1 * os1 + r2 * os2 + col * osc] = a[t][ct][s];
      }
}


// ---------------------------------------------------------------------------
// Counter-based uniform numbers: SplitMix64 (Steele, Lea, Flood 2014).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One workgroup per (site, item): zero the slot, then fill the true
// (bl, p, br) tensor with 2*(h >> 11)*2^-52... values indexed by the compact
// C-order position, exactly as the oracle does.
__global__ __launch_bounds__(kThreads) void k_rand_init(
    FitDims *dims, int W, int c, int N, int K, int P, size_t S, Ptr Y,
    const uint64_t *slot, uint64_t seed, const int32_t *flag) {
  const int j = blockIdx.x, it = blockIdx.y;
  if (!flag[it]) return;
  const FitDims &dm = dims[(size_t)it * W + c];
  double *y = Y.at(it) + (size_t)j * S;
  for (size_t i = threadIdx.x; i < S; i += kThreads) y[i] = 0.0;
  __syncthreads();
  const int bl = dm.bl[j], p = dm.p[j], br = dm.br[j];
  const uint64_t h = splitmix(splitmix(splitmix(seed) ^ (slot[it] + c)) ^
                              (uint64_t)j);
  const int total = bl * p * br;
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const uint64_t v = splitmix(h ^ (uint64_t)idx);
    const double u = (double)(v >> 11) * 0x1p-52 - 1.0;
    const int y0 = idx / (p * br), rem = idx - y0 * p * br;
    const int a = rem / br, y1 = rem - a * br;
    size_t addr;
    if (j == 0) addr = (size_t)a * K + y1;               // [p][br]
    else if (j == N - 1) addr = (size_t)y0 * K + a;      // [bl][p]
    else addr = ((size_t)y0 * P + a) * K + y1;           // [bl][p][br]
    y[addr] = u;
  }
}

__global__ void k_set_unit(Ptr slot, size_t S) {
  double *s = slot.at(blockIdx.y);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < S;
       i += (size_t)gridDim.x * blockDim.x)
    s[i] = (i == 0) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(kThreads) void k_copy_flagged(
    const double *src, size_t sstride, Ptr dst, size_t n, const int32_t *flag) {
  const int it = blockIdx.y;
  if (flag && !flag[it]) return;
  double *d = dst.at(it);
  const double *s = src + (size_t)it * sstride;
  for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n;
       i += (size_t)gridDim.x * kThreads)
    d[i] = s[i];
}

// Norm of the end slot (K*K doubles) per item; scale to unit norm.
// nu[it*W] receives the norm (nu already offset to the column).
__global__ __launch_bounds__(kThreads) void k_normalize(Ptr Y0, int K,
                                                        double *nu, int W,
                                                        int32_t *err) {
  const int it = blockIdx.x;
  double *y = Y0.at(it);
  const int n = K * K;
  double part = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) part += y[i] * y[i];
  part = wave_sum(part);
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = part;
  __syncthreads();
  const double nrm = sqrt(red[0] + red[1] + red[2] + red[3]);
  const bool ok = nrm > 0.0 && isfinite(nrm);
  if (threadIdx.x == 0) {
    nu[(size_t)it * W] = nrm;
    if (!ok) atomicOr(err, 1);
  }
  if (ok) {
    const double inv = 1.0 / nrm;
    for (int i = threadIdx.x; i < n; i += kThreads) y[i] *= inv;
  }
}

// Copy one message site [a][q][b] from a slot with bond cap ks to a slot
// with bond cap kd (kd >= ks), optionally transposed to [b][q][a].  The
// destination slot is fully written (zero padding included).
__device__ __forceinline__ void copy_site(const double *src, double *dst,
                                          int ks, int kd, int P, bool tr,
                                          double scale, int tid, int nt) {
  const size_t S = (size_t)kd * P * kd;
  for (size_t i = tid; i < S; i += nt) {
    const int a = (int)(i / ((size_t)P * kd));
    const int rem = (int)(i - (size_t)a * P * kd);
    const int qq = rem / kd, b = rem - qq * kd;
    double v = 0.0;
    if (a < ks && b < ks)
      v = tr ? src[((size_t)b * P + qq) * ks + a] : src[((size_t)a * P + qq) * ks + b];
    dst[i] = scale * v;
  }
}

// blockIdx.x: site, blockIdx.y: which (0 top, 1 boundary, 2 bottom),
// blockIdx.z: item.
__global__ __launch_bounds__(kThreads) void k_gather(FitBatch f,
                                                     const GatherSrc *srcs) {
  const int site = blockIdx.x, which = blockIdx.y, it = blockIdx.z;
  const GatherSrc &g = srcs[it];
  const int K = f.K, P = f.P;
  const size_t S = f.S;
  int k, i;
  double *dst;
  if (which == 1) {
    if (site >= f.N) return;
    dst = f.xin + ((size_t)it * f.N + site) * S;
    if (site == 0 || site == f.N - 1) {
      for (size_t t = threadIdx.x; t < S; t += kThreads)
        dst[t] = (t == 0) ? 1.0 : 0.0;
      return;
    }
    k = 1;
    i = site - 1;
  } else {
    if (site >= f.W) return;
    k = which == 0 ? 0 : 2;
    i = site;
    dst = (which == 0 ? f.mt : f.mb) + ((size_t)it * f.W + site) * S;
  }
  const int seg = i < g.n[k][0] ? 0 : 1;
  const int loc = seg ? i - g.n[k][0] : i;
  const int n = g.n[k][seg];
  const bool rev = g.rev[k][seg] != 0;
  const int src_site = rev ? n - 1 - loc : loc;
  const size_t Ss = (size_t)g.ksrc * P * g.ksrc;
  copy_site(g.src[k][seg] + (size_t)src_site * Ss, dst, g.ksrc, K, P, rev, 1.0,
            threadIdx.x, kThreads);
}

// Final boundary (column 0) of each item -> message of H sites.
__global__ __launch_bounds__(kThreads) void k_extract(FitBatch f,
                                                      double *const *dst,
                                                      const int32_t *rev) {
  const int i = blockIdx.x, it = blockIdx.y;
  const int L = f.H;
  const double *Y = f.store + ((size_t)it * f.W * f.N) * f.S;  // column 0
  double scale = 1.0;
  if (i == 0) scale *= Y[0];                              // site 0 scalar
  if (i == L - 1) scale *= Y[(size_t)(f.N - 1) * f.S];    // site N-1 scalar
  const int out = rev[it] ? L - 1 - i : i;
  copy_site(Y + (size_t)(i + 1) * f.S, dst[it] + (size_t)out * f.S, f.K, f.K,
            f.P, rev[it] != 0, scale, threadIdx.x, kThreads);
}

__global__ __launch_bounds__(kThreads) void k_copy_jobs(const CopyJob *jobs,
                                                        int K, int P) {
  const CopyJob j = jobs[blockIdx.y];
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < j.n;
       i += (int64_t)gridDim.x * kThreads) {
    int64_t from = i;
    if (j.mode == 1) {
      const int64_t a = i / ((int64_t)P * K), rem = i - a * P * K;
      const int64_t qq = rem / K, b = rem - qq * K;
      from = (b * P + qq) * K + a;
    } else if (j.mode == 2) {
      if (i >= (int64_t)K * K) {
        j.dst[i] = 0.0;
        continue;
      }
      const int64_t a = i / K, b = i - a * K;
      from = b * K + a;
    }
    j.dst[i] = j.src[from];
  }
}

__global__ __launch_bounds__(kThreads) void k_dots(const double *const *a,
                                                   const double *const *b,
                                                   size_t n, double *out) {
  const int it = blockIdx.x;
  const double *x = a[it], *y = b[it];
  double part = 0.0;
  for (size_t i = threadIdx.x; i < n; i += kThreads) part += x[i] * y[i];
  part = wave_sum(part);
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = part;
  __syncthreads();
  if (threadIdx.x == 0) out[it] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_ov_init(double *E, int K) {
  const int it = blockIdx.x;
  for (int i = threadIdx.x; i < K * K; i += blockDim.x)
    E[(size_t)it * K * K + i] = (i == 0) ? 1.0 : 0.0;
}
__global__ void k_ov_out(const double *E, int K, int items, double *out) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it < items) out[it] = E[(size_t)it * K * K];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static Shape shape_of(const FitBatch &f) { return Shape{f.K, f.P, f.D, f.d}; }
static size_t t1_stride(const FitBatch &f) { return (size_t)f.K * f.P * f.P * f.K; }
static size_t t2_stride(const FitBatch &f) {
  return (size_t)f.d * f.K * f.K * f.P * f.P;
}
static size_t a_site(const FitBatch &f) { return (size_t)f.d * f.P * f.P; }
static size_t a_stride(const FitBatch &f) { return (size_t)f.H * f.W * a_site(f); }

// Tile shape of the fused visit: the largest TY x TX pair set whose LDS
// footprint fits, or TY = 0 when none does (generic chain then).
static void visit_tiles(const FitBatch &f, int *TY, int *TX, size_t *bytes) {
  const size_t K = f.K, P = f.P;
  const int cand[][2] = {{2, 8}, {2, 4}, {4, 2}, {2, 2}, {1, 4}, {1, 2}, {1, 1}};
  for (auto &c : cand) {
    const size_t ty = c[0], tx = c[1];
    if ((int)ty > f.K) continue;
    size_t n = visit_lds(f.K, f.P, f.d, (int)ty, (int)tx);
    const size_t tiles = ((ty * P + 15) / 16) * ((K + 15) / 16);
    if (2 * tiles <= (size_t)kVisitWaves) n = std::max(n, tiles * 256);  // k-half sums
    if (n * 8 <= 150 * 1024 && tiles <= 4 * (size_t)kVisitWaves) {
      *TY = (int)ty;
      *TX = (int)tx;
      *bytes = n * 8;
      return;
    }
  }
  *TY = 0;
}

using VisitKernel = void (*)(VisitArgs);

template <class T, bool B16 = false>
static VisitKernel visit_kernel(int D) {
  switch (D) {
    case 2: return k_visit<2, T, B16>;
    case 3: return k_visit<3, T, B16>;
    case 4: return k_visit<4, T, B16>;
    case 5: return k_visit<5, T, B16>;
    case 6: return k_visit<6, T, B16>;
    default: return k_visit<0, T, B16>;
  }
}

// Tiles of the D = 4, d = 2 kernel: the first candidate whose LDS fits.
template <class T>
static bool visit4_tiles(const FitBatch &f, int *TY, int *TX, size_t *bytes) {
  if (f.D != 4 || f.d != 2 || f.K > 128) return false;
  const int cand[][2] = {{2, 4}, {4, 2}, {2, 2}, {1, 2}, {1, 1}};
  for (auto &c : cand) {
    if (c[0] > f.K) continue;
    const size_t n = visit4_lds<T>(f.K, c[0], c[1]) * sizeof(T);
    const size_t moved = (size_t)std::max(ceil4(f.K), ceil16(f.K)) * 16 * c[1];
    if (n <= 150 * 1024 && moved <= 8 * (size_t)kVisitThreads) {
      *TY = c[0];
      *TX = c[1];
      *bytes = n;
      return true;
    }
  }
  return false;
}

template <class T>
static VisitKernel visit4_kernel(int TY, int TX) {
  if (TY == 2 && TX == 4) return k_visit4<2, 4, T>;
  if (TY == 4 && TX == 2) return k_visit4<4, 2, T>;
  if (TY == 2 && TX == 2) return k_visit4<2, 2, T>;
  if (TY == 1 && TX == 2) return k_visit4<1, 2, T>;
  return k_visit4<1, 1, T>;
}

// NE = number of 16-wide local-update tiles the kernel is built for (>= 2).
static int visit4p_ne(int K) { return std::max(2, ceil16(K) / 16); }

// Pair-per-wave visit (K <= 64): 2 x 2 pairs, 4 x 1 at NE = 3.  A small
// batch at NE <= 2, whose 2 x 2 grid would not give every CU a workgroup,
// takes 1 x 4 pairs: twice the workgroups, each walking a quarter of the
// columns xb.
template <class T>
static bool visit4p_tiles(const FitBatch &f, int *TY, int *TX, size_t *bytes) {
  if (f.D != 4 || f.d != 2 || f.K > 64) return false;
  const int ne = visit4p_ne(f.K);
  const long sel = f.tile_items > 0 ? f.tile_items : f.items;
  const bool small = ne <= 2 && sel * ((f.K + 1) / 2) < 256;
  const int ty = ne == 3 ? 4 : small ? 1 : 2, tx = ne == 3 ? 1 : small ? 4 : 2;
  const size_t n = visit4p_lds<T>(f.K, ty, tx) * sizeof(T);
  if (n > 150 * 1024) return false;
  *TY = ty;
  *TX = tx;
  *bytes = n;
  return true;
}


template <class T>
static VisitKernel visit4p_kernel(int NE, int TY) {
  if (NE <= 2) return TY == 1 ? k_visit4p<1, 4, T, 2> : k_visit4p<2, 2, T, 2>;
  if (NE == 3) return k_visit4p<4, 1, T, 3>;
  return k_visit4p<2, 2, T, 4>;
}

// BF16 contractions (precision 16) run in the generic fused visit and the
// environment update at bond caps <= 64, any D; T3 passes between them in
// FP32.  Elsewhere precision 16 leaves FP64 in place.
static bool visit_bf16(const FitBatch &f) {
  int TY, TX;
  size_t lds;
  if (f.prec != 16 || f.K > 64) return false;
  visit_tiles(f, &TY, &TX, &lds);
  return TY > 0;
}

// FP32 T3 and environment update: the FP32 contractions (precision 32) run
// where both the visit and the environment update have an FP32 form (every
// fused visit at K <= 64), and the BF16 ones (above) keep T3 in FP32 too.
// Elsewhere the precision option leaves FP64 in place.
static bool visit_f32(const FitBatch &f) {
  int TY, TX;
  size_t lds;
  if (f.prec == 16) return visit_bf16(f);
  if (f.prec != 32 || f.K > 64) return false;
  if (visit4_tiles<float>(f, &TY, &TX, &lds)) return true;
  visit_tiles(f, &TY, &TX, &lds);  // the generic fused visit
  return f.D != 4 && TY > 0;
}

// ---- algorithmic counts on the true extents (timing only) -----------------
// Floating-point operations and operand bytes of the split-layer
// contractions of one launch, summed over its items with each item's true
// bonds (f.hdims, present for the column absorptions).  Launches without
// them (the observables' line sandwiches) count at the bond cap.
enum : int { TC_T1 = 1, TC_KET = 2, TC_BRA = 4, TC_LOCAL = 8, TC_ENV = 16 };
struct Count {
  double flops = 0.0, bytes = 0.0;
};
static Count count_inner(const FitBatch &f, int c, int j, bool rl, int parts) {
  Count t;
  if (!timing_enabled()) return t;
  const double P = f.P, d = f.d;
  for (int i = 0; i < f.items; ++i) {
    double yf = f.K, yb = f.K, xf = f.K, xb = f.K;
    if (f.hdims) {
      const SiteExt e = site_ext(f.hdims[(size_t)i * f.W + c], j, f.N, rl);
      yf = e.yf, yb = e.yb, xf = e.xf, xb = e.xb;
    }
    double m = 0.0, b = 0.0;  // multiply-adds, doubles moved
    if (parts & TC_T1) m += yf * P * xf * P * xb, b += yf * P * xf + xf * P * xb;
    if (parts & TC_KET) m += yf * xb * d * P * P * P, b += d * P * P;
    if (parts & TC_BRA) m += yf * xb * d * P * P * P;
    if (parts & TC_LOCAL) m += yf * P * xb * P * yb, b += yb * P * xb + yf * P * yb;
    if (parts & TC_ENV) m += yb * P * xb * yf * P, b += yf * P * yb + yb * P * xb;
    t.flops += 2.0 * m;
    t.bytes += 8.0 * b;
  }
  return t;
}
// End site (0 in LR, N-1 in RL): the message site of the column as an MPO
// Mend[a][q][a'] against the X corner [a'][xe]; parts 1 chain, 2 local, 4 env.
static Count count_end(const FitBatch &f, int c, bool rl, int parts) {
  Count t;
  if (!timing_enabled()) return t;
  const double P = f.P;
  for (int i = 0; i < f.items; ++i) {
    double a = f.K, ap = f.K, xe = f.K, ye = f.K;
    if (f.hdims) {
      const FitDims &d = f.hdims[(size_t)i * f.W + c];
      const int j = rl ? f.N - 1 : 0;
      a = d.p[j];
      ap = c == f.W - 1 ? 1 : f.hdims[(size_t)i * f.W + c + 1].p[j];
      xe = rl ? d.xb[f.N - 2] : d.xb[0];
      ye = rl ? d.bl[f.N - 1] : d.br[0];
    }
    double m = 0.0, b = 0.0;
    if (parts & 1) m += a * P * ap * xe, b += a * P * ap + ap * xe;
    if (parts & 2) m += a * P * xe * ye, b += ye * P * xe + a * ye;
    if (parts & 4) m += ye * a * P * xe, b += a * ye + ye * P * xe;
    t.flops += 2.0 * m;
    t.bytes += 8.0 * b;
  }
  return t;
}
// Householder QR/LQ of the true panels: 4 m n^2 - 4 n^3 / 3 (R and Q).
static Count count_qr(const FitBatch &f, int c, int j, int mode) {
  Count t;
  if (!timing_enabled()) return t;
  for (int i = 0; i < f.items; ++i) {
    double m = (double)f.K * f.P, n = f.K;
    if (f.hdims) {
      const FitDims &d = f.hdims[(size_t)i * f.W + c];
      const bool lr = mode == LR_INNER || mode == LR_TOP;
      m = (double)(lr ? d.bl[j] : d.br[j]) * d.p[j];
      n = lr ? d.br[j] : d.bl[j];
    }
    t.flops += 4.0 * m * n * n - 4.0 * n * n * n / 3.0;
    t.bytes += 16.0 * m * n;
  }
  return t;
}

static hipError_t launch_fused(const FitBatch &f, int c, int j, bool rl, Ptr X,
                               Ptr F, Ptr G, Ptr Y, bool do_local, int TY,
                               int TX, size_t lds, hipStream_t st) {
  static std::once_flag attr_once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(attr_once, [] {
    for (int D : {0, 2, 3, 4, 5, 6})
      for (VisitKernel kf : {visit_kernel<double>(D), visit_kernel<float>(D),
                             visit_kernel<float, true>(D)}) {
        hipError_t e = hipFuncSetAttribute((const void *)kf,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) attr_err = e;
      }
    for (auto t : {std::make_pair(2, 4), std::make_pair(4, 2), std::make_pair(2, 2),
                   std::make_pair(1, 2), std::make_pair(1, 1)})
      for (VisitKernel kf : {visit4_kernel<double>(t.first, t.second),
                             visit4_kernel<float>(t.first, t.second)}) {
        hipError_t e = hipFuncSetAttribute((const void *)kf,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) attr_err = e;
      }
    for (int ne = 2; ne <= 4; ++ne)
      for (VisitKernel kf : {visit4p_kernel<double>(ne, 2), visit4p_kernel<float>(ne, 2),
                             visit4p_kernel<double>(ne, 1), visit4p_kernel<float>(ne, 1)}) {
        hipError_t e = hipFuncSetAttribute(
            (const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) attr_err = e;
      }
  });
  if (attr_err != hipSuccess) return attr_err;
  int TY4, TX4;
  size_t lds4;
  const bool b16 = visit_bf16(f), f32 = visit_f32(f);
  const bool spec = !b16 && (f32 ? visit4_tiles<float>(f, &TY4, &TX4, &lds4)
                                 : visit4_tiles<double>(f, &TY4, &TX4, &lds4));
  const size_t site_off = ((size_t)(j - 1) * f.W + c) * a_site(f);
  VisitArgs v;
  v.K = f.K; v.P = f.P; v.D = f.D; v.d = f.d; v.TY = TY; v.TX = TX;
  v.rl = rl ? 1 : 0;
  v.do_local = do_local ? 1 : 0;
  v.F = F; v.X = X; v.G = G; v.Y = Y;
  v.aket = f.acan + site_off;
  v.aket_stride = a_stride(f);
  v.abra = f.bra_one ? f.bra_one : (f.abra ? f.abra : f.acan) + site_off;
  v.abra_stride = f.bra_one ? 0 : a_stride(f);
  v.t3 = f.t3;
  v.t3_stride = t1_stride(f);
  v.dims = nullptr;
  v.W = f.W; v.c = c; v.j = j; v.N = f.N;
  const double it = f.items, K = f.K, P = f.P, d = f.d;
  double flops = it * (2 * K * K * K * P * P + 4 * d * K * K * P * P * P);
  double bytes = it * 8 * (2 * K * P * K + K * K * P * P + 2 * d * P * P);
  if (do_local) {
    flops += it * 2 * K * K * K * P * P;
    bytes += it * 8 * 2 * K * P * K;
  }
  const Count tc = count_inner(f, c, j, rl, TC_T1 | TC_KET | TC_BRA | (do_local ? TC_LOCAL : 0));
  Span sp(KC_VISIT, st, tc.flops, tc.bytes, flops, bytes);
  int TYp, TXp;
  size_t ldsp;
  const bool pairw = !b16 && (f32 ? visit4p_tiles<float>(f, &TYp, &TXp, &ldsp)
                                  : visit4p_tiles<double>(f, &TYp, &TXp, &ldsp));
  if (pairw) {  // one (yf, xb) pair per wave; skips the zero padding
    v.TY = TYp;
    v.TX = TXp;
    v.dims = f.bounded && f.hdims ? f.dims : nullptr;
    const int ne = visit4p_ne(f.K);
    hipLaunchKernelGGL(f32 ? visit4p_kernel<float>(ne, TYp) : visit4p_kernel<double>(ne, TYp),
                       dim3((f.K + TYp - 1) / TYp, f.items), dim3(64 * TYp * TXp), ldsp, st, v);
  } else if (spec) {
    v.TY = TY4;
    v.TX = TX4;
    hipLaunchKernelGGL(f32 ? visit4_kernel<float>(TY4, TX4) : visit4_kernel<double>(TY4, TX4),
                       dim3((f.K + TY4 - 1) / TY4, f.items), dim3(kVisitThreads), lds4, st, v);
  } else {
    const VisitKernel kf = b16   ? visit_kernel<float, true>(f.D)
                           : f32 ? visit_kernel<float>(f.D)
                                 : visit_kernel<double>(f.D);
    hipLaunchKernelGGL(kf, dim3((f.K + TY - 1) / TY, f.items), dim3(kVisitThreads), lds, st, v);
  }
  return hipGetLastError();
}

bool visit_fused_fits(const FitBatch &f) {
  int TY, TX;
  size_t lds;
  visit_tiles(f, &TY, &TX, &lds);
  return TY > 0;
}

// Blocked MFMA QR (8 waves) for panels up to 768 x 48: row tiles per wave and
// column tiles from the bond cap K and the physical dimension P.
constexpr int kQmWavesUsed = 8;

bool qrm_fits(const FitBatch &f) {
  return f.K <= 48 && f.K * f.P <= 16 * kQmWavesUsed * 6;
}

bool qr_needs_scratch(const FitBatch &f) {
  if (qrm_fits(f)) return false;
  return (size_t)f.K * f.P * f.K > (size_t)kQrLds;
}

template <int RT>
void launch_qrm_rt(int CT, int items, hipStream_t st, const QrArgs &q) {
  constexpr int NW = kQmWavesUsed;
  if (CT == 1) hipLaunchKernelGGL((k_qrm<NW, RT, 1>), dim3(items), dim3(NW * 64), 0, st, q);
  else if (CT == 2) hipLaunchKernelGGL((k_qrm<NW, RT, 2>), dim3(items), dim3(NW * 64), 0, st, q);
  else hipLaunchKernelGGL((k_qrm<NW, RT, 3>), dim3(items), dim3(NW * 64), 0, st, q);
}

void launch_qrm(const FitBatch &f, hipStream_t st, const QrArgs &q) {
  const int rt = (f.K * f.P + 16 * kQmWavesUsed - 1) / (16 * kQmWavesUsed);
  const int CT = (f.K + 15) / 16;
  if (rt <= 1) launch_qrm_rt<1>(CT, f.items, st, q);
  else if (rt <= 2) launch_qrm_rt<2>(CT, f.items, st, q);
  else if (rt <= 4) launch_qrm_rt<4>(CT, f.items, st, q);
  else launch_qrm_rt<6>(CT, f.items, st, q);
}

hipError_t launch_inner_visit(const FitBatch &f, int c, int j, bool rl, Ptr X,
                              Ptr F, Ptr G, Ptr Y, hipStream_t st) {
  int TY, TX;
  size_t lds;
  visit_tiles(f, &TY, &TX, &lds);
  if (TY > 0) return launch_fused(f, c, j, rl, X, F, G, Y, true, TY, TX, lds, st);
  hipError_t e = launch_inner_chain_generic(f, c, j, rl, X, F, st);
  if (e != hipSuccess) return e;
  return launch_inner_local(f, c, j, rl, G, Y, st);
}

hipError_t launch_inner_chain(const FitBatch &f, int c, int j, bool rl, Ptr X,
                              Ptr F, hipStream_t st) {
  int TY, TX;
  size_t lds;
  visit_tiles(f, &TY, &TX, &lds);
  if (TY > 0)
    return launch_fused(f, c, j, rl, X, F, Ptr{}, Ptr{}, false, TY, TX, lds, st);
  return launch_inner_chain_generic(f, c, j, rl, X, F, st);
}

hipError_t launch_inner_chain_generic(const FitBatch &f, int c, int j, bool rl,
                                      Ptr X, Ptr F, hipStream_t st) {
  const Shape s = shape_of(f);
  const size_t t1s = t1_stride(f), t2s = t2_stride(f), t3s = t1s;
  const size_t site_off = ((size_t)(j - 1) * f.W + c) * a_site(f);
  const double *Ak = f.acan + site_off;
  const double *Ab = f.bra_one ? f.bra_one : (f.abra ? f.abra : f.acan) + site_off;
  const double it = f.items, K = f.K, P = f.P, d = f.d;
  OpK1 k1{f.K * f.P, f.P * f.K, f.K, nullptr, s, rl, X, F, f.t1, t1s};
  hipError_t e;
  {
    const Count tc = count_inner(f, c, j, rl, TC_T1);
    Span sp(KC_T1, st, tc.flops, tc.bytes, it * 2 * K * P * P * K * K,
            it * 8 * (2 * K * P * K + K * K * P * P));
    e = run_gemm<64, 64, 16>(k1, f.items, st);
  }
  if (e != hipSuccess) return e;
  OpK2 k2{f.K * f.P * f.K, f.d * f.P, f.P, nullptr, s, rl, f.t1, t1s, Ak,
          a_stride(f), f.t2, t2s};
  {
    const Count tc = count_inner(f, c, j, rl, TC_KET);
    Span sp(KC_KET, st, tc.flops, tc.bytes, it * 2 * K * P * K * d * P * P,
            it * 8 * (K * K * P * P + d * P * P + d * K * K * P * P));
    e = run_gemm<128, 32, 16>(k2, f.items, st);
  }
  if (e != hipSuccess) return e;
  OpK3 k3{f.K * f.K * f.P, f.P, f.d * f.P, nullptr, s, rl, f.t2, t2s, Ab,
          f.bra_one ? 0 : a_stride(f), f.t3, t3s};
  const Count tc = count_inner(f, c, j, rl, TC_BRA);
  Span sp(KC_BRA, st, tc.flops, tc.bytes, it * 2 * K * K * P * P * d * P,
          it * 8 * (d * K * K * P * P + d * P * P + K * K * P * P));
  return run_gemm<256, 16, 16>(k3, f.items, st);
}

hipError_t launch_inner_local(const FitBatch &f, int c, int j, bool rl, Ptr G, Ptr Y,
                              hipStream_t st) {
  OpK4 k4{f.K * f.P, f.K, f.K * f.P, nullptr, shape_of(f), rl, f.t3,
          t1_stride(f), G, Y};
  const double it = f.items, K = f.K, P = f.P;
  const Count tc = count_inner(f, c, j, rl, TC_LOCAL);
  Span sp(KC_LOCAL, st, tc.flops, tc.bytes, it * 2 * K * P * K * K * P,
          it * 8 * (K * K * P * P + 2 * K * P * K));
  return run_gemm<64, 32, 16>(k4, f.items, st);
}

hipError_t launch_inner_env(const FitBatch &f, int c, int j, bool rl, Ptr Y,
                            Ptr envOut, hipStream_t st) {
  const double it = f.items, K = f.K, P = f.P;
  const Count tc = count_inner(f, c, j, rl, TC_ENV);
  Span sp(KC_ENV, st, tc.flops, tc.bytes, it * 2 * K * K * P * K * P,
          it * 8 * (K * K * P * P + 2 * K * P * K));
  if (f.K <= 64) {
    EnvArgs e{f.K, f.P, rl ? 1 : 0, f.t3, t1_stride(f), Y, envOut,
              f.bounded && f.hdims ? f.dims : nullptr, f.W, c, j, f.N};
    const dim3 grid((f.K * f.P + 63) / 64, f.items);
    const int mt = (f.K + 15) / 16;
    // BF16 or FP32 only where the visit wrote FP32 T3
    if (visit_bf16(f)) {
      if (mt <= 1) hipLaunchKernelGGL((k_env<1, float, true>), grid, dim3(EnvShape<1>::kThreads), 0, st, e);
      else if (mt <= 2) hipLaunchKernelGGL((k_env<2, float, true>), grid, dim3(EnvShape<2>::kThreads), 0, st, e);
      else if (mt <= 3) hipLaunchKernelGGL((k_env<3, float, true>), grid, dim3(EnvShape<3>::kThreads), 0, st, e);
      else hipLaunchKernelGGL((k_env<4, float, true>), grid, dim3(EnvShape<4>::kThreads), 0, st, e);
      return hipGetLastError();
    }
    if (visit_f32(f)) {
      if (mt <= 1) hipLaunchKernelGGL((k_env<1, float>), grid, dim3(EnvShape<1>::kThreads), 0, st, e);
      else if (mt <= 2) hipLaunchKernelGGL((k_env<2, float>), grid, dim3(EnvShape<2>::kThreads), 0, st, e);
      else if (mt <= 3) hipLaunchKernelGGL((k_env<3, float>), grid, dim3(EnvShape<3>::kThreads), 0, st, e);
      else hipLaunchKernelGGL((k_env<4, float>), grid, dim3(EnvShape<4>::kThreads), 0, st, e);
      return hipGetLastError();
    }
    if (mt <= 1) hipLaunchKernelGGL((k_env<1, double>), grid, dim3(EnvShape<1>::kThreads), 0, st, e);
    else if (mt <= 2) hipLaunchKernelGGL((k_env<2, double>), grid, dim3(EnvShape<2>::kThreads), 0, st, e);
    else if (mt <= 3) hipLaunchKernelGGL((k_env<3, double>), grid, dim3(EnvShape<3>::kThreads), 0, st, e);
    else hipLaunchKernelGGL((k_env<4, double>), grid, dim3(EnvShape<4>::kThreads), 0, st, e);
    return hipGetLastError();
  }
  OpK5 k5{f.K, f.K * f.P, f.K * f.P, nullptr, shape_of(f), rl, f.t3,
          t1_stride(f), Y, envOut};
  return run_gemm<32, 64, 16>(k5, f.items, st);
}

hipError_t launch_end_chain(const FitBatch &f, int c, bool rl, Ptr Mend, Ptr Xe,
                            hipStream_t st) {
  OpE1 e1{f.K * f.P, f.K, f.K, nullptr, shape_of(f), rl, Mend, Xe, f.t3,
          t1_stride(f)};
  const double it = f.items, K = f.K, P = f.P;
  const Count tc = count_end(f, c, rl, 1);
  Span sp(KC_END, st, tc.flops, tc.bytes, it * 2 * K * P * K * K,
          it * 8 * (2 * K * P * K + K * K));
  return run_gemm<64, 32, 16>(e1, f.items, st);
}

hipError_t launch_end_local(const FitBatch &f, int c, bool rl, Ptr G, Ptr Ye,
                            hipStream_t st) {
  OpE2 e2{f.K, f.K, f.P * f.K, nullptr, shape_of(f), rl, f.t3, t1_stride(f),
          G, Ye};
  const double it = f.items, K = f.K, P = f.P;
  const Count tc = count_end(f, c, rl, 2);
  Span sp(KC_END, st, tc.flops, tc.bytes, it * 2 * K * K * P * K,
          it * 8 * (2 * K * P * K + K * K));
  // one 32x32 tile, K P long: split over eight (P >= 8) workgroups per tile
  // through the item's tmp slot (K P K doubles >= 8 K^2), which nothing
  // else holds at this point of a column
  if (f.P >= 8 && f.tmp) return run_gemm_splitk<32, 32, 64, 8>(e2, f.items, f.tmp, f.S, st);
  return run_gemm<32, 32, 64>(e2, f.items, st);
}

hipError_t launch_end_env(const FitBatch &f, int c, bool rl, Ptr Ye, Ptr envOut,
                          hipStream_t st) {
  OpE3 e3{f.K, f.P * f.K, f.K, nullptr, shape_of(f), rl, f.t3, t1_stride(f),
          Ye, envOut};
  const double it = f.items, K = f.K, P = f.P;
  const Count tc = count_end(f, c, rl, 4);
  Span sp(KC_END, st, tc.flops, tc.bytes, it * 2 * K * P * K * K,
          it * 8 * (2 * K * P * K + K * K));
  return run_gemm<32, 64, 16>(e3, f.items, st);
}

hipError_t launch_qr(const FitBatch &f, int c, int j, int mode, Ptr Y,
                     bool want_r, bool only_flagged, hipStream_t st) {
  QrArgs q{f.dims, f.W, c, j, mode, f.K, f.P, Y, f.rbuf, f.t1, t1_stride(f),
           only_flagged ? f.flag : nullptr, want_r ? 1 : 0};
  const size_t panel = (size_t)f.K * f.P * f.K;  // upper bound of m*n
  const double m = (double)f.K * f.P, n = f.K;
  const Count tc = count_qr(f, c, j, mode);
  Span sp(KC_QR, st, tc.flops, tc.bytes, f.items * (4.0 * m * n * n - 4.0 * n * n * n / 3.0),
          f.items * 16.0 * m * n);
  // The blocked MFMA kernel for panels up to 768 x 48 (every shape of the
  // D <= 4 workloads); otherwise the LDS kernel, or the 16-wave global-memory
  // one (up to 128 columns: every bond cap the context accepts).
  if (qrm_fits(f)) {
    launch_qrm(f, st, q);
  } else if (panel <= (size_t)kQrLds) {
    hipLaunchKernelGGL(k_qr, dim3(f.items), dim3(kThreads), 0, st, q);
  } else {
    if (!f.t1 || t1_stride(f) < panel)
      return hipErrorInvalidValue;  // global panel scratch missing or too small
    if (f.K > kQrgWaves * kQrgCols) return hipErrorInvalidValue;  // bond caps are <= 128
    hipLaunchKernelGGL(k_qrg, dim3(f.items), dim3(kQrgThreads), 0, st, q);
  }
  (void)panel;
  return hipGetLastError();
}

hipError_t launch_apply_l(const FitBatch &f, bool end_site, Ptr Y,
                          hipStream_t st) {
  const int rows = end_site ? f.K : f.K * f.P;
  OpApplyL op{rows, f.K, f.K, f.flag, shape_of(f), Y, f.rbuf, f.tmp, f.S};
  hipError_t e = run_gemm<64, 32, 16>(op, f.items, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_flagged, dim3(64, f.items), dim3(kThreads), 0, st,
                     (const double *)f.tmp, f.S, Y, f.S, (const int32_t *)f.flag);
  return hipGetLastError();
}

hipError_t launch_rand_init(const FitBatch &f, int c, Ptr Ybase,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_rand_init, dim3(f.N, f.items), dim3(kThreads), 0, st,
                     f.dims, f.W, c, f.N, f.K, f.P, f.S, Ybase,
                     (const uint64_t *)f.slot, f.seed, (const int32_t *)f.flag);
  return hipGetLastError();
}

__global__ void k_zero_words(uint32_t *p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>(1024, (n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(kThreads), 0, st, (uint32_t *)p, n);
  return hipGetLastError();
}

hipError_t launch_set_unit(const FitBatch &f, Ptr slot, hipStream_t st) {
  hipLaunchKernelGGL(k_set_unit, dim3(16, f.items), dim3(kThreads), 0, st,
                     slot, f.S);
  return hipGetLastError();
}

hipError_t launch_normalize(const FitBatch &f, int c, Ptr Y0, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize, dim3(f.items), dim3(kThreads), 0, st, Y0,
                     f.K, f.nu + c, f.W, f.err);
  return hipGetLastError();
}

hipError_t launch_gather(const FitBatch &f, const GatherSrc *srcs,
                         hipStream_t st) {
  const int nx = f.N > f.W ? f.N : f.W;
  hipLaunchKernelGGL(k_gather, dim3(nx, 3, f.items), dim3(kThreads), 0, st, f,
                     srcs);
  return hipGetLastError();
}

hipError_t launch_extract(const FitBatch &f, double *const *dst,
                          const int32_t *rev, hipStream_t st) {
  hipLaunchKernelGGL(k_extract, dim3(f.H, f.items), dim3(kThreads), 0, st, f,
                     dst, rev);
  return hipGetLastError();
}

hipError_t launch_copy_jobs(const CopyJob *jobs, int njobs, int K, int P,
                            hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_jobs, dim3(8, njobs), dim3(kThreads), 0, st, jobs,
                     K, P);
  return hipGetLastError();
}

hipError_t launch_dots(int items, const double *const *a,
                       const double *const *b, size_t n, double *out,
                       hipStream_t st) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dots, dim3(items), dim3(kThreads), 0, st, a, b, n, out);
  return hipGetLastError();
}

hipError_t launch_overlap(int items, int K, int P, int L,
                          const double *const *a, const double *const *b,
                          double *E, double *U, double *out, hipStream_t st) {
  if (items <= 0) return hipSuccess;
  const size_t S = (size_t)K * P * K;
  hipLaunchKernelGGL(k_ov_init, dim3(items), dim3(64), 0, st, E, K);
  for (int i = 0; i < L; ++i) {
    OpOv1 o1{K, P * K, K, nullptr, K, E, a, (size_t)i * S, U, S};
    hipError_t e = run_gemm<32, 64, 16>(o1, items, st);
    if (e != hipSuccess) return e;
    OpOv2 o2{K, K, K * P, nullptr, K, P, U, S, b, (size_t)i * S, E};
    e = run_gemm<32, 32, 64>(o2, items, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ov_out, dim3((items + 63) / 64), dim3(64), 0, st, E, K,
                     items, out);
  return hipGetLastError();
}

}  // namespace bbp
