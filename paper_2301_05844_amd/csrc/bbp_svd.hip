// libbbp: batched truncated singular value decomposition by one-sided
// (Hestenes) Jacobi rotations, FP64.
//
// The compression step of the standard alternative to the zip-up fit (App.
// A: multiply the MPO into the MPS, then compress the result) truncates
// each bond by an SVD; the same primitive gives the singular values of the
// trace distance (App. C).  For a tall matrix A (m >= n) the columns are
// rotated pairwise until every pair is orthogonal: A V = U diag(S) with V
// the product of the rotations, S the column norms and U the normalised
// columns.
//
// One workgroup per matrix.  The matrix is held column-major in LDS (column
// j contiguous, so a pair's dot products are lane-strided reads), V beside
// it.  A sweep is n' - 1 rounds of the round-robin (circle) pairing of the
// n' = n rounded up to even columns: the n'/2 pairs of a round share no
// column, so the 16 waves rotate them side by side, a wave per pair, with
// one barrier per round.  Each pair's three sums (|a_p|^2, |a_q|^2,
// a_p . a_q) are accumulated per lane in row order and reduced across the
// wave in a fixed order (DPP moves within rows of 16 lanes, then the four row
// sums), so every result is reproducible bit for bit and independent of the
// other items of the batch.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <mutex>

#include "../../include/bbp.h"

namespace bbp {
namespace {

constexpr int kSvdWaves = 16, kSvdThreads = 64 * kSvdWaves;
constexpr int kSvdMaxN = 64;

struct SvdArgs {
  const double *A;
  double *U, *S, *V, *err2;
  int32_t *sweeps;
  int m, n, k, max_sweeps;
  double tol;
};

// v of lane (lane within its row of 16, permuted by the DPP control CTRL).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over the 64 lanes, the same bits in every lane: within each row of 16
// lanes by DPP moves (partner 1 apart, 2 apart, the other half of 8, the
// other half of 16; each step adds a lane's value to its partner's, so the
// partners hold equal sums), then the four row sums in a fixed order.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Columns of round r (0 <= r < np - 1) of the circle pairing of np (even)
// players: pair 0 is (r, np - 1), pair i > 0 is (r + i, r - i) mod np - 1.
__device__ __forceinline__ void round_pair(int r, int i, int np, int *p, int *q) {
  const int h = np - 1;
  int a, b;
  if (i == 0) {
    a = r;
    b = h;
  } else {
    a = (r + i) % h;
    b = (r - i + h) % h;
  }
  *p = min(a, b);
  *q = max(a, b);
}

__global__ __launch_bounds__(kSvdThreads) void k_svd_jacobi(SvdArgs g) {
  extern __shared__ double sm[];
  __shared__ double sig[kSvdMaxN];
  __shared__ int perm[kSvdMaxN], sgn[kSvdMaxN];
  __shared__ int rot[2];
  const int m = g.m, n = g.n, k = g.k, item = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *a = sm;              // a[j m + i] = A[i][j]
  double *v = sm + (size_t)m * n;  // v[j n + i] = V[i][j]
  const double *Ag = g.A + (size_t)item * m * n;
  for (int t = tid; t < m * n; t += kSvdThreads) {
    const int i = t / n, j = t % n;
    a[(size_t)j * m + i] = Ag[t];
  }
  for (int t = tid; t < n * n; t += kSvdThreads) v[t] = (t / n == t % n) ? 1.0 : 0.0;
  const int np = n + (n & 1);
  int sweep = 0;
  bool clean = false;
  while (sweep < g.max_sweeps) {
    if (tid == 0) rot[sweep & 1] = 0;
    __syncthreads();
    for (int r = 0; r + 1 < np; ++r) {
      for (int pi = wave; pi < np / 2; pi += kSvdWaves) {
        int p, q;
        round_pair(r, pi, np, &p, &q);
        if (q >= n) continue;  // the padding column of an odd n
        double *ap = a + (size_t)p * m, *aq = a + (size_t)q * m;
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll 8
        for (int i = lane; i < m; i += 64) {
          const double x = ap[i], y = aq[i];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        al = wave_total(al);
        be = wave_total(be);
        ga = wave_total(ga);
        // rotate unless the pair is already orthogonal to the tolerance
        if (!(fabs(ga) > g.tol * (sqrt(al) * sqrt(be)))) continue;
        const double ze = (be - al) / (2.0 * ga);
        const double t = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll 8
        for (int i = lane; i < m; i += 64) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double *vp = v + (size_t)p * n, *vq = v + (size_t)q * n;
        for (int i = lane; i < n; i += 64) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
        if (lane == 0) atomicOr(&rot[sweep & 1], 1);
      }
      __syncthreads();  // the next round pairs these columns with others
    }
    ++sweep;
    if (rot[(sweep - 1) & 1] == 0) {
      clean = true;
      break;
    }
  }
  // singular values (column norms) and the sign of each column: the
  // largest-magnitude entry (the first of equal ones) made positive
  for (int j = wave; j < n; j += kSvdWaves) {
    const double *aj = a + (size_t)j * m;
    double ss = 0.0, big = -1.0;
    int at = m;
    for (int i = lane; i < m; i += 64) {
      const double x = aj[i];
      ss = fma(x, x, ss);
      if (fabs(x) > big) big = fabs(x), at = i;
    }
    ss = wave_total(ss);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(big, o, 64);
      const int oa = __shfl_xor(at, o, 64);
      if (ob > big || (ob == big && oa < at)) big = ob, at = oa;
    }
    if (lane == 0) {
      sig[j] = sqrt(ss);
      sgn[j] = (at < m && aj[at] < 0.0) ? -1 : 1;
    }
  }
  __syncthreads();
  // descending order, ties by column index; a NaN norm (non-finite input)
  // sorts last, so the ranks stay a permutation
  if (tid < n) {
    auto key = [](double x) { return x == x ? x : -1.0; };
    const double sj = key(sig[tid]);
    int rk = 0;
    for (int i = 0; i < n; ++i) {
      const double si = key(sig[i]);
      rk += (si > sj) || (si == sj && i < tid);
    }
    perm[rk] = tid;
  }
  __syncthreads();
  double *U = g.U + (size_t)item * m * k, *V = g.V + (size_t)item * n * k;
  for (int t = tid; t < m * k; t += kSvdThreads) {
    const int i = t / k, r = t % k, j = perm[r];
    const double sj = sig[j];
    U[t] = sj > 0.0 ? sgn[j] * (a[(size_t)j * m + i] / sj) : 0.0;
  }
  for (int t = tid; t < n * k; t += kSvdThreads) {
    const int i = t / k, r = t % k, j = perm[r];
    V[t] = sgn[j] * v[(size_t)j * n + i];
  }
  if (tid < k) g.S[(size_t)item * k + tid] = sig[perm[tid]];
  if (tid == 0) {
    if (g.err2) {
      double e = 0.0;
      for (int r = k; r < n; ++r) e = fma(sig[perm[r]], sig[perm[r]], e);
      g.err2[item] = e;
    }
    if (g.sweeps) g.sweeps[item] = clean ? sweep : -sweep;
  }
}

}  // namespace
}  // namespace bbp

extern "C" bbp_status bbp_svd_jacobi(int32_t batch, int32_t m, int32_t n, int32_t k,
                                     const double *A, double *U, double *S, double *V,
                                     double *err2, int32_t *sweeps, int32_t max_sweeps,
                                     double tol, void *hip_stream) {
  using namespace bbp;
  if (batch < 0 || n < 1 || n > kSvdMaxN || m < n || k < 1 || k > n || max_sweeps < 1 ||
      max_sweeps > 100 || !(tol >= 0.0 && tol < 1.0) ||
      (size_t)m * n + (size_t)n * n > BBP_SVD_MAX_WORDS)
    return BBP_EINVAL;
  if (batch == 0) return BBP_OK;
  if (!A || !U || !S || !V) return BBP_EINVAL;
  static std::once_flag once;
  static hipError_t attr = hipSuccess;
  std::call_once(once, [] {
    attr = hipFuncSetAttribute((const void *)k_svd_jacobi,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(BBP_SVD_MAX_WORDS * sizeof(double)));
  });
  if (attr != hipSuccess) return BBP_EDEVICE;
  SvdArgs g;
  g.A = A;
  g.U = U;
  g.S = S;
  g.V = V;
  g.err2 = err2;
  g.sweeps = sweeps;
  g.m = m;
  g.n = n;
  g.k = k;
  g.max_sweeps = max_sweeps;
  g.tol = tol > 0.0 ? tol : std::sqrt((double)m) * DBL_EPSILON;
  const size_t lds = ((size_t)m * n + (size_t)n * n) * sizeof(double);
  hipLaunchKernelGGL(k_svd_jacobi, dim3(batch), dim3(kSvdThreads), lds,
                     (hipStream_t)hip_stream, g);
  return hipGetLastError() == hipSuccess ? BBP_OK : BBP_EDEVICE;
}
