// Internal declarations shared by the host orchestration and the kernels of
// libbbp.  Not part of the public ABI (include/bbp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/bbp.h"

namespace bbp {

// Largest number of sites of a boundary MPS (column height + 2 corners).
constexpr int NMAX = 68;

// Shapes of the fit result Y for one work item and one absorbed column:
// site j of Y is (bl[j], p[j], br[j]) with bl[0] = br[N-1] = 1.  xb[j]
// (j = 0..N-2) is the bond j|j+1 of the boundary X the column is absorbed
// into, so X site j is (j ? xb[j-1] : 1, ., j < N-1 ? xb[j] : 1).  Every
// slot entry outside these true extents is zero.
struct FitDims {
  int32_t bl[NMAX];
  int32_t br[NMAX];
  int32_t p[NMAX];
  int32_t xb[NMAX];
  int32_t rnd;      // 1: start from the counter-based random state
  int32_t pad_[3];
};

// True extents of inner site j of one item in one visit direction: the
// front/back bonds of Y (yf, yb) and of X (xf, xb), "front" being the side
// the sweep comes from (left for LR, right for RL).
struct SiteExt {
  int yf, yb, xf, xb;
};
__host__ __device__ inline SiteExt site_ext(const FitDims &d, int j, int N, bool rl) {
  const int xl = j ? d.xb[j - 1] : 1, xr = j < N - 1 ? d.xb[j] : 1;
  SiteExt e;
  e.yf = rl ? d.br[j] : d.bl[j];
  e.yb = rl ? d.bl[j] : d.br[j];
  e.xf = rl ? xr : xl;
  e.xb = rl ? xl : xr;
  return e;
}

// Device buffers of one batch of independent column absorptions ("items"),
// all with the same boundary length N, width W and bond cap K.  Every MPS
// site lives in a zero-padded slot of S = K*P*K doubles; end sites use the
// first K*K doubles of their slot as a [phys][bond] or [bond][phys] matrix.
struct FitBatch {
  int items = 0;
  // items the visit's tiling is chosen for: the whole batch's count where a
  // batch is split over streams, so that every part runs the same kernels
  int tile_items = 0;
  int K = 0, P = 0, D = 0, d = 0;  // bond cap, D^2, D, physical dim
  int H = 0, W = 0, N = 0;          // column height, width, N = H + 2
  size_t S = 0;                     // slot size (doubles)
  double *store = nullptr;  // [items][W][N][S]  fit result per column
  double *xin = nullptr;    // [items][N][S]     boundary before column W-1
  double *mt = nullptr;     // [items][W][S]     top message sites (rotated)
  double *mb = nullptr;     // [items][W][S]     bottom message sites
  double *lenv = nullptr;   // [items][N][S]
  double *renv = nullptr;   // [items][N][S]
  double *t1 = nullptr;     // [items][K*P*P*K]
  double *t2 = nullptr;     // [items][d*K*K*P*P]
  double *t3 = nullptr;     // [items][K*P*K*P]
  double *tmp = nullptr;    // [items][S]
  double *acan = nullptr;   // [items][H][W][d*D^4]  rotated site tensors (ket)
  double *abra = nullptr;   // bra tensors if different from acan (or null)
  // single-layer networks: one bra tensor (every virtual leg at index 0) for
  // every site and item, in place of abra/acan
  const double *bra_one = nullptr;
  double *rbuf = nullptr;   // [items][K*K]
  double *nu = nullptr;     // [items][W] norm of each column's fit
  int32_t *flag = nullptr;  // [items] per-item active flags
  int32_t *err = nullptr;   // [1] numeric error flag
  FitDims *dims = nullptr;  // [items][W]
  // host copy of dims (same layout), read by the launchers only to count
  // the floating-point operations and bytes of the true shapes
  const FitDims *hdims = nullptr;
  // 1: kernels that can read dims stop at the true extents (the padding
  // they skip only ever adds zeros)
  int bounded = 0;
  uint64_t *slot = nullptr; // [items] random-state slot base
  uint64_t seed = 0;
  int prec = 64;  // 64: FP64 contractions; 32 (16): visit and environment update on FP32 (BF16) MFMA
};

// Visit kinds of the fit engine.
enum VisitMode : int {
  LR_INNER = 0,  // left-to-right visit of an inner site (QR)
  RL_INNER = 1,  // right-to-left visit of an inner site (LQ)
  LR_TOP = 2,    // left-to-right visit of site 0 (top corner/message site)
  RL_BOT = 3     // right-to-left visit of site N-1 (bottom corner)
};

// A per-item device pointer: item i uses p + i*stride, or, with a pointer
// table, tab[i] + stride.
struct Ptr {
  double *p = nullptr;
  size_t stride = 0;
  double *const *tab = nullptr;
  __host__ __device__ double *at(int i) const {
    return tab ? tab[i] + stride : p + (size_t)i * stride;
  }
};

// Offset of site j of column c inside one item's fit-result store.
inline size_t slot_store(const FitBatch &f, int c, int j) {
  return ((size_t)c * f.N + j) * f.S;
}

// Launchers (bbp_kernels.hip).  All enqueue on `st`.
// Inner-site chain T1 -> T2 -> T3 (split layers) for site j of column c
// (fused MFMA kernel when its tiles fit in LDS, else the generic chain).
hipError_t launch_inner_chain(const FitBatch &f, int c, int j, bool rl,
                              Ptr X, Ptr F, hipStream_t st);
hipError_t launch_inner_chain_generic(const FitBatch &f, int c, int j, bool rl,
                                      Ptr X, Ptr F, hipStream_t st);
// Whether the fused visit kernel's tiles fit in LDS for this batch shape
// (otherwise the generic chain with its T1/T2 scratch runs), and whether the
// QR panel needs the global scratch (t1).
bool visit_fused_fits(const FitBatch &f);
bool qr_needs_scratch(const FitBatch &f);
// Chain plus the local update Yt = T3 . G written into Y.
hipError_t launch_inner_visit(const FitBatch &f, int c, int j, bool rl, Ptr X,
                              Ptr F, Ptr G, Ptr Y, hipStream_t st);
// Yt = T3 . G  (local update), written into Y.
hipError_t launch_inner_local(const FitBatch &f, int c, int j, bool rl, Ptr G,
                              Ptr Y, hipStream_t st);
// env' = Y . T3 after the visit of site j of column c
hipError_t launch_inner_env(const FitBatch &f, int c, int j, bool rl, Ptr Y,
                            Ptr envOut, hipStream_t st);
// End-site chain T = Mend . Xe (top corner in LR, bottom corner in RL).
hipError_t launch_end_chain(const FitBatch &f, int c, bool rl, Ptr Mend, Ptr Xe,
                            hipStream_t st);
hipError_t launch_end_local(const FitBatch &f, int c, bool rl, Ptr G, Ptr Ye,
                            hipStream_t st);
hipError_t launch_end_env(const FitBatch &f, int c, bool rl, Ptr Ye, Ptr envOut,
                          hipStream_t st);
// Householder QR of the site panel (mode: VisitMode); Q replaces the panel.
hipError_t launch_qr(const FitBatch &f, int c, int j, int mode, Ptr Y,
                     bool want_r, bool only_flagged, hipStream_t st);
// Y_{j-1} <- Y_{j-1} . L with L = R^T from rbuf (flagged items only).
hipError_t launch_apply_l(const FitBatch &f, bool end_site, Ptr Y,
                          hipStream_t st);
// Counter-based random start for all N sites of column c (flagged items).
hipError_t launch_rand_init(const FitBatch &f, int c, Ptr Ybase,
                            hipStream_t st);
// Clear bytes (a multiple of 4) at p with a fill kernel.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// Set slot (per item) to the 1x1x1 unit tensor.
hipError_t launch_set_unit(const FitBatch &f, Ptr slot, hipStream_t st);
// Normalise the end slot Y0 to unit norm; nu[item*W + c] = its norm.
hipError_t launch_normalize(const FitBatch &f, int c, Ptr Y0, hipStream_t st);

// Message gathering / extraction / overlap.  Each rotated incoming side
// (top, right, bottom) is made of up to two message segments (two for the
// union of two blocks), already listed in rotated order.
struct GatherSrc {
  const double *src[3][2];  // site-0 slot of each segment
  int32_t n[3][2];          // sites per segment (0: unused)
  int32_t rev[3][2];        // segment read in reverse site order
  int32_t ksrc;             // bond cap of the source slots
  int32_t pad_;
};
hipError_t launch_gather(const FitBatch &f, const GatherSrc *srcs,
                         hipStream_t st);
// Final boundary of column 0 -> message of H sites at dst[item].
hipError_t launch_extract(const FitBatch &f, double *const *dst,
                          const int32_t *rev, hipStream_t st);
// Copy of one slot-shaped tensor: mode 0 copy n doubles, 1 transpose an
// inner site [a][q][b] -> [b][q][a] (bond cap K, P), 2 transpose a K x K end
// site.
struct CopyJob {
  const double *src;
  double *dst;
  int64_t n;
  int32_t mode;
  int32_t pad_;
};
hipError_t launch_copy_jobs(const CopyJob *jobs, int njobs, int K, int P,
                            hipStream_t st);
// out[i] = sum_k a_i[k] b_i[k] over n doubles.
hipError_t launch_dots(int items, const double *const *a,
                       const double *const *b, size_t n, double *out,
                       hipStream_t st);
// out[i] = <a_i | b_i> for items i, each an L-site padded MPS.
hipError_t launch_overlap(int items, int K, int P, int L, const double *const *a,
                          const double *const *b, double *E, double *U,
                          double *out, hipStream_t st);

// Per-kernel-class launch timing (process-wide; enabled by the "timing"
// option).  Each timed launch records a pair of HIP events on its stream and
// the algorithmic floating-point operations and bytes it processes.
enum KernelClass : int {
  KC_VISIT = 0,  // fused F.X -> ket -> bra (-> local update) on MFMA
  KC_T1 = 1,     // F . X            (generic chain)
  KC_KET = 2,    // T1 . A ket layer (generic chain)
  KC_BRA = 3,    // T2 . A bra layer (generic chain)
  KC_LOCAL = 4,  // T3 . G  local update (generic chain)
  KC_ENV = 5,    // Y . T3  environment update
  KC_END = 6,    // end-site contractions
  KC_QR = 7,     // Householder QR / LQ
  KC_OTHER = 8,  // gather, extract, normalise, overlaps, copies
  KC_COUNT = 9
};
void timing_enable(bool on);
bool timing_enabled();
void timing_reset();
// Synchronises the recorded events and returns the totals of one class.
// flops/bytes: the algorithmic counts on every item's true bond dimensions;
// pflops/pbytes: the same contractions counted at the padded bond cap K and
// the bytes the kernels' own data flow moves (padded operands, T3 spills).
hipError_t timing_query(int cls, const char **name, long long *launches,
                        double *ms, double *flops, double *bytes,
                        double *pflops = nullptr, double *pbytes = nullptr);

// Continuous batching across contexts (the request server): a set of
// shared batches that sweeps many contexts at once, every message of every
// context in the batch of its shape.  A context must be put in engine mode
// before its tensors are set (it then holds no message batches of its own
// and bbp_sweep rejects it).  sweepset_run makes one synchronous sweep of
// each of the n contexts, writing each one's residual and status; contexts
// that leave or join between calls make the affected batches be rebuilt,
// keeping the warm starts of the items that stay.
struct SweepSet;
SweepSet *sweepset_create(hipStream_t st);
void sweepset_destroy(SweepSet *s);
// Device memory of the shared batches through the given allocator.
void sweepset_set_allocator(SweepSet *s, bbp_alloc_fn alloc, bbp_free_fn free_, void *user);
bbp_status ctx_set_engine(bbp_ctx *c);
bbp_status sweepset_run(SweepSet *s, bbp_ctx *const *cs, int n, double *res,
                        bbp_status *status, std::string *err);

// What the blockBP update (bbp_ite_step) needs of a context: its problem,
// options, stream and host copy of the tensors, and its error slot.
struct CtxInfo {
  int infinite, Lx, Ly, bx, by, D, chi, d, chi_env, n_fit, sx, sy, single_layer;
  uint64_t seed;
  hipStream_t stream;
  bbp_alloc_fn alloc_fn;  // the caller's allocator (null: hipMalloc)
  bbp_free_fn free_fn;
  void *alloc_user;
  size_t hbm_budget;  // 0: no limit
};
bbp_status ctx_info(bbp_ctx *c, CtxInfo *out);
bbp_status ctx_fail(bbp_ctx *c, bbp_status s, const std::string &m);
const double *ctx_tensors(bbp_ctx *c, size_t *n);
// bbp_rdm_bonds restricted to what the n bonds need: each region in its
// bond's frame only, the bond's line and its two sites' unit steps; nothing
// is kept for later queries.  Same values as bbp_rdm_bonds.
bbp_status rdm_bonds_only(bbp_ctx *c, int n, const int32_t *x0, const int32_t *y0,
                          const int32_t *x1, const int32_t *y1, double *rho);
// Keep the boundary stacks of bond-only contractions for later calls (reused
// while the columns a later call needs are unchanged).  For a context whose
// messages and settings stay fixed after its first contraction.
void ctx_keep_stacks(bbp_ctx *c);
// Replace the host tensors of n sites (lattice site indices, site layout of
// bbp_set_tensors) for the observables only: regions are contracted from
// them, the sweeps' rotated copies are not rebuilt, so a context updated
// this way must not be swept.
bbp_status ctx_replace_sites(bbp_ctx *c, int n, const int *site, const double *A);

}  // namespace bbp
