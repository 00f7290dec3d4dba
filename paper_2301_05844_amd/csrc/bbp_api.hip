// libbbp host side: the C ABI of include/bbp.h, the block partition and
// message bookkeeping of block BP (Sec. II, Eq. (1)), and the launch sequence
// of one synchronous sweep (App. A column absorptions as variational fits).
//
// Nothing here touches the GPU before bbp_set_tensors has validated its
// input, so argument checking works on machines without a GPU.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <tuple>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bbp.h"
#include "bbp_internal.h"

using namespace bbp;

namespace {

const char kDirs[4] = {'L', 'R', 'U', 'D'};
int dir_index(char d) { return d == 'L' ? 0 : d == 'R' ? 1 : d == 'U' ? 2 : 3; }
char opposite(char d) {
  return d == 'L' ? 'R' : d == 'R' ? 'L' : d == 'U' ? 'D' : 'U';
}
// Leg permutation from A[s,u,l,d,r] to the frame with side `d` on the left:
// L identity, R half turn, U quarter turn counter-clockwise, D clockwise.
void rot_perm(char d, int perm[5]) {
  static const int P[4][5] = {{0, 1, 2, 3, 4},
                              {0, 3, 4, 1, 2},
                              {0, 4, 1, 2, 3},
                              {0, 2, 3, 4, 1}};
  std::memcpy(perm, P[dir_index(d)], sizeof(int) * 5);
}
bool out_reversed(char d) { return d == 'R' || d == 'U'; }

// Device bytes a context holds now and at most (every API entry that may
// allocate names its context's account for the calling thread), and the
// allocator the context's device memory comes from (hipMalloc/hipFree unless
// the caller supplied one; its memory is handed back only after the
// context's stream has drained).  When an allocation fails, `evict` frees
// what the context only keeps for reuse and the allocation is tried once
// more.
struct MemAcct {
  size_t now = 0, peak = 0;
  size_t budget = 0;  // bytes the owner may hold (0: no limit)
  bbp_alloc_fn alloc_fn = nullptr;
  bbp_free_fn free_fn = nullptr;
  void *user = nullptr;
  const hipStream_t *stream = nullptr;
  void (*evict)(void *) = nullptr;
  void *evict_user = nullptr;
};
thread_local MemAcct *tl_acct = nullptr;
struct AcctScope {
  MemAcct *prev;
  explicit AcctScope(MemAcct *a) : prev(tl_acct) { tl_acct = a; }
  ~AcctScope() { tl_acct = prev; }
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  MemAcct *acct = nullptr;
  bool borrowed = false;  // memory owned elsewhere (a caller's workspace): never freed here
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), acct(o.acct), borrowed(o.borrowed) {
    o.p = nullptr;
    o.bytes = 0;
    o.acct = nullptr;
    o.borrowed = false;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      acct = o.acct;
      borrowed = o.borrowed;
      o.p = nullptr;
      o.bytes = 0;
      o.acct = nullptr;
      o.borrowed = false;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  // Points at b bytes of memory that someone else owns.
  void borrow(void *q, size_t b) {
    release();
    p = q;
    bytes = b;
    borrowed = true;
  }
  void release() {
    if (p && !borrowed) {
      if (acct && acct->free_fn) {
        if (acct->stream) (void)hipStreamSynchronize(*acct->stream);
        acct->free_fn(p, acct->user);
      } else {
        (void)hipFree(p);
      }
      if (acct) acct->now -= bytes;
    }
    p = nullptr;
    bytes = 0;
    acct = nullptr;
    borrowed = false;
  }
  // (Re)allocates b bytes; an existing allocation of exactly b bytes is kept
  // (its contents are not cleared).
  hipError_t alloc(size_t b) {
    if (p && b == bytes && acct == tl_acct) return hipSuccess;
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = raw_alloc(b);
    if (e != hipSuccess && tl_acct && tl_acct->evict) {
      (void)hipGetLastError();  // the failed attempt's error is not a launch error
      tl_acct->evict(tl_acct->evict_user);
      e = raw_alloc(b);
    }
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return e;
    }
    bytes = b;
    acct = tl_acct;
    if (acct) {
      acct->now += b;
      acct->peak = std::max(acct->peak, acct->now);
    }
    return hipSuccess;
  }
  double *d() const { return (double *)p; }

 private:
  hipError_t raw_alloc(size_t b) {
    if (tl_acct && tl_acct->budget && tl_acct->now + b > tl_acct->budget)
      return hipErrorOutOfMemory;  // beyond the context's byte budget
    if (tl_acct && tl_acct->alloc_fn) {
      p = tl_acct->alloc_fn(b, tl_acct->user);
      return p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(&p, b);
  }
};

// Page-locked host staging for transfers that must not wait on the device:
// a copy from pageable memory is carried out synchronously, behind the
// work already queued on its stream.  Blocks are kept by the context and
// handed out in order; a call that stages through them resets the pool at
// its start and synchronises before it returns, so the next call may reuse
// every block.  A pageable pool (the request server's contexts, whose
// calls run while another thread captures the shared sweeps into a graph,
// which a page-locked allocation would break) gives the same results with
// transfers that wait.
struct PinnedPool {
  struct Block {
    char *p;
    size_t size;
  };
  std::vector<Block> blocks;
  size_t bi = 0, off = 0;
  bool pageable = false;
  PinnedPool() = default;
  PinnedPool(const PinnedPool &) = delete;
  PinnedPool &operator=(const PinnedPool &) = delete;
  void reset() {
    bi = 0;
    off = 0;
  }
  // `bytes` of staging (256-byte aligned), or nullptr when none can be had.
  void *get(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    while (bi < blocks.size() && off + bytes > blocks[bi].size) {
      ++bi;
      off = 0;
    }
    if (bi == blocks.size()) {
      void *q = nullptr;
      const size_t sz = std::max(bytes, (size_t)8 << 20);
      if (pageable) {
        q = std::malloc(sz);
        if (!q) return nullptr;
      } else if (hipHostMalloc(&q, sz, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      blocks.push_back(Block{(char *)q, sz});
      off = 0;
    }
    void *r = blocks[bi].p + off;
    off += bytes;
    return r;
  }
  ~PinnedPool() {
    for (Block &b : blocks)
      if (pageable) std::free(b.p);
      else (void)hipHostFree(b.p);
  }
};

struct Message {
  int bi, bj;
  char dir;
  int n;                    // sites
  std::vector<int> bonds;   // n + 1 entries, ends 1
};

// Incoming message on `side` of a block: message id or -1 (trivial).
struct Incoming {
  int id;
  int n;
};

struct Group {
  int W = 0, H = 0;
  std::vector<int> ids;  // message ids in this batch
  FitBatch fb;
  std::vector<DevBuf> bufs;
  DevBuf gather, dst, rev;
  DevBuf t3r;  // line batches: the right environment chain's own T3 scratch
  std::vector<FitDims> dims;  // [items][W], host copy
  std::vector<int> have;      // [items*W] warm start valid
  // host staging of the per-sweep tables (kept alive until the stream syncs)
  std::vector<double> host;  // rotated region tensors of a boundary-stack batch
  std::vector<GatherSrc> gs;
  std::vector<double *> dsts;
  std::vector<int32_t> revs;
  std::vector<int32_t> flags;  // [W][items]
  DevBuf flagbuf;              // [W][items]
  int cache_gen = 0;           // observables call that last used this batch
  // a message batch's column absorptions as a HIP graph, replayed in later
  // sweeps while the launch sequence and its arguments stay the same
  hipGraphExec_t graph = nullptr;
  FitBatch graph_fb;  // the batch the graph was captured with
  int graph_nfit = 0;
  Group() = default;
  Group(const Group &) = delete;
  Group &operator=(const Group &) = delete;
  ~Group() {
    if (graph) (void)hipGraphExecDestroy(graph);
  }
};

// Reduced density matrices of one region (block or union of two blocks)
// computed from its boundary stacks; NaN where not computed.
struct RegionResult {
  int H = 0, W = 0;
  bool has_row = false, has_col = false;
  std::vector<double> zrow, lsrow;  // per row: line value and log scale
  std::vector<double> site;         // [H][W][d*d]  unit (s',s) at s'*d+s
  std::vector<double> hbond;        // [H][W-1][d^2][d^2]
  std::vector<double> zcol, lscol;  // per column
  std::vector<double> vbond;        // [W][H-1][d^2][d^2]
};

}  // namespace

struct bbp_ctx {
  MemAcct mem;  // first member: outlives every buffer below
  // problem
  int infinite = 0, Lx = 0, Ly = 0, ucx = 1, ucy = 1, bx = 1, by = 1, D = 1,
      chi = 1, d = 2;
  int sx = 0, sy = 0;  // partition shift: trivial columns left, rows on top
  int gx = 1, gy = 1;
  int chi_env = -1, n_fit = 2;
  int precision = 64;  // 64; 32: fit contractions on FP32 MFMA; 16: on BF16 MFMA
  int lanes = 3;       // streams that independent fit batches spread over
  int graphs = 1;      // 1: message batches replay their column absorptions as HIP graphs
  int skip_pad = 1;    // 1: the column absorptions' kernels stop at the true bond extents
  int msg_split = 2;   // message batches of one shape split into this many (one per lane)
  bool engine = false; // messages swept by a shared SweepSet (no message batches of its own)
  int single_layer = 0; // 1: the network is sum_s A[s] (bra layer fixed at index 0)
  int init = 0;         // initial messages: 0 identity product MPDO, 1 random product MPDO
  DevBuf delta;         // single layer: the bra tensor, [s][0][0][0][0] = 1
  DevBuf rot;                   // engine mode: rotated block tensors of every message
  std::vector<size_t> rot_off;  // doubles from rot's start to message i's block
  uint64_t serial = 0; // unique per context of the process (identifies it across sweeps)
  int64_t sweeps_done = 0;  // sweeps since the tensors were set
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  std::vector<hipStream_t> aux;     // lanes 1.. (lane 0 is `stream`)
  std::vector<hipEvent_t> lane_ev;  // fork event, then one join event per aux lane
  std::vector<hipEvent_t> dep_ev;   // ordering events between lanes within one call
  PinnedPool pin;                   // host staging of the observables' transfers
  hipStream_t cap = nullptr;        // stream HIP graphs are captured on (never run)
  bool tensors_set = false;
  bool device_ready = false;
  std::string err;
  std::vector<double> A;  // host copy of the input tensors
  std::vector<Message> msgs;
  int P = 1, K = 1, Lmax = 1;
  size_t S = 0;
  DevBuf msgbuf[2], trivial, ovE, ovU, ovOut, ovA, ovB, errflag;
  int cur = 0;
  std::vector<std::unique_ptr<Group>> groups;
  // observables' boundary-stack, line and unit-output buffers of earlier
  // calls, kept for the next call with the same shapes
  // (entries tagged with the observables call that last used them; only the
  // last two calls' entries are kept)
  std::vector<std::unique_ptr<Group>> batch_cache;
  std::vector<std::pair<int, DevBuf>> unit_out_cache;
  std::vector<std::unique_ptr<Group>> unit_groups;  // matrix-unit step batches
  // Boundary stacks kept from earlier bond-only region contractions (the
  // blockBP update's environment context, stack_reuse on): each with the
  // rotated tensors of every column it absorbed, reused by a later call
  // while the columns that call needs are unchanged.
  struct KeptStack {
    Group *g;
    int item;
    std::vector<double> cols;  // [H][W][site] in the stack's canonical frame
    std::vector<double> nu;    // [W] column scales
  };
  bool stack_reuse = false;
  std::map<std::tuple<int, int, int, char>, KeptStack> kept_stacks;
  std::vector<std::unique_ptr<Group>> kept_groups;
  int obs_call = 0;
  double last_flops = 0.0;
  std::map<std::tuple<int, int, int>, RegionResult> obs;  // (kind, bi, bj)

  bbp_status fail(bbp_status s, const std::string &m) {
    err = m;
    return s;
  }
  bbp_status hip_fail(hipError_t e, const char *where) {
    err = std::string(where) + ": " + hipGetErrorString(e);
    return BBP_EDEVICE;
  }

  // ---- lattice ----------------------------------------------------------
  bool neighbour(int bi, int bj, char dr, int *ni, int *nj) const {
    if (infinite) {
      *ni = bi;
      *nj = bj;
      return true;
    }
    int dx = dr == 'L' ? -1 : dr == 'R' ? 1 : 0;
    int dy = dr == 'U' ? -1 : dr == 'D' ? 1 : 0;
    *ni = bi + dx;
    *nj = bj + dy;
    return *ni >= 0 && *ni < gx && *nj >= 0 && *nj < gy;
  }
  int msg_id(int bi, int bj, char dr) const {
    for (size_t i = 0; i < msgs.size(); ++i)
      if (msgs[i].bi == bi && msgs[i].bj == bj && msgs[i].dir == dr)
        return (int)i;
    return -1;
  }
  Incoming incoming(int bi, int bj, char side) const {
    int ni, nj;
    int n = (side == 'L' || side == 'R') ? by : bx;
    if (!neighbour(bi, bj, side, &ni, &nj)) return Incoming{-1, n};
    return Incoming{msg_id(ni, nj, opposite(side)), n};
  }
  // Site tensor (original orientation) at lattice coordinates; nullptr for a
  // trivial padding site.
  const double *site(int x, int y) const {
    const size_t ss = (size_t)d * D * D * D * D;
    if (infinite) {
      int cx = ((x % ucx) + ucx) % ucx, cy = ((y % ucy) + ucy) % ucy;
      return A.data() + (size_t)(cy * ucx + cx) * ss;
    }
    x -= sx;
    y -= sy;
    if (x >= 0 && y >= 0 && x < Lx && y < Ly) return A.data() + (size_t)(y * Lx + x) * ss;
    return nullptr;
  }
};

namespace {

// Rotated copy of one site tensor into dst (d*D^4 doubles).
void rotate_site(const bbp_ctx *c, const double *src, char dir, double *dst) {
  const int D = c->D, d = c->d;
  const size_t ss = (size_t)d * D * D * D * D;
  if (!src) {
    std::fill(dst, dst + ss, 0.0);
    dst[0] = 1.0;  // trivial site: A[0,0,0,0,0] = 1
    return;
  }
  int perm[5];
  rot_perm(dir, perm);
  int in[5], o[5];
  for (o[0] = 0; o[0] < d; ++o[0])
    for (o[1] = 0; o[1] < D; ++o[1])
      for (o[2] = 0; o[2] < D; ++o[2])
        for (o[3] = 0; o[3] < D; ++o[3])
          for (o[4] = 0; o[4] < D; ++o[4]) {
            for (int t = 0; t < 5; ++t) in[perm[t]] = o[t];
            size_t si = ((((size_t)in[0] * D + in[1]) * D + in[2]) * D + in[3]) *
                            D + in[4];
            size_t di = ((((size_t)o[0] * D + o[1]) * D + o[2]) * D + o[3]) * D +
                        o[4];
            dst[di] = src[si];
          }
}

// Region (rows H x cols W) coordinates of canonical (y', x') in frame `dir`.
void canon_to_region(char dir, int H, int W, int yc, int xc, int *y, int *x) {
  switch (dir) {
    case 'L': *y = yc; *x = xc; break;
    case 'R': *y = H - 1 - yc; *x = W - 1 - xc; break;
    case 'U': *y = xc; *x = W - 1 - yc; break;
    default: *y = H - 1 - xc; *x = yc; break;  // 'D'
  }
}

// Canonical top/right/bottom incoming messages for orientation dir, given
// the region's natural top/bottom/left/right: which side and reversal.
void canon_sources(char dir, char src_side[3], int rev[3]) {
  switch (dir) {
    case 'L':
      src_side[0] = 'U'; src_side[1] = 'R'; src_side[2] = 'D';
      rev[0] = rev[1] = rev[2] = 0;
      break;
    case 'R':
      src_side[0] = 'D'; src_side[1] = 'L'; src_side[2] = 'U';
      rev[0] = rev[1] = rev[2] = 1;
      break;
    case 'U':
      src_side[0] = 'R'; src_side[1] = 'D'; src_side[2] = 'L';
      rev[0] = 0; rev[1] = 1; rev[2] = 0;
      break;
    default:  // 'D'
      src_side[0] = 'L'; src_side[1] = 'U'; src_side[2] = 'R';
      rev[0] = 1; rev[1] = 0; rev[2] = 1;
      break;
  }
}

std::vector<int> reversed(const std::vector<int> &v) {
  return std::vector<int>(v.rbegin(), v.rend());
}

// Bond caps of the fit result for every column, right to left.  mt/mb: bond
// lists (W+1) of the rotated top/bottom messages, mr: bond list (H+1) of the
// rotated right message.  Y site j of column c is (bl, p, br).
void column_dims(int W, int H, int K, int P, const std::vector<int> &mt,
                 const std::vector<int> &mb, const std::vector<int> &mr,
                 std::vector<FitDims> &out) {
  const int N = H + 2;
  out.assign(W, FitDims{});
  std::vector<int> xb(mr.begin(), mr.end());  // X bonds j = 0..N-2
  for (int c = W - 1; c >= 0; --c) {
    FitDims &f = out[c];
    std::vector<int> p(N, P), b(N - 1);
    p[0] = mt[c];
    p[N - 1] = mb[c];
    for (int j = 0; j < N - 1; ++j) b[j] = std::min(K, xb[j] * P);
    for (int j = 0; j < N - 1; ++j)
      b[j] = std::min(b[j], (j ? b[j - 1] : 1) * p[j]);
    for (int j = N - 1; j >= 1; --j)
      b[j - 1] = std::min(b[j - 1], p[j] * (j < N - 1 ? b[j] : 1));
    for (int j = 0; j < N; ++j) {
      f.p[j] = p[j];
      f.bl[j] = j ? b[j - 1] : 1;
      f.br[j] = j < N - 1 ? b[j] : 1;
    }
    for (int j = 0; j < N - 1; ++j) f.xb[j] = xb[j];
    xb = b;
  }
}

}  // namespace

// Host <-> device transfers are ordered on the context's stream (a server
// worker's stream is non-blocking, so the null stream would not wait for it);
// the stream is synchronised before the host buffer is read or released.
static hipError_t copy_sync(bbp_ctx *c, void *dst, const void *src, size_t bytes,
                            hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}
static hipError_t zero_sync(bbp_ctx *c, void *p, size_t bytes) {
  hipError_t e = hipMemsetAsync(p, 0, bytes, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}

// ---- lanes: independent batches on several streams ------------------------
// Lane 0 is the context stream; lanes 1.. are the context's own non-blocking
// streams (default priority), created on first use.  Batches of different
// messages (or boundary stacks) share no buffers, so they may run
// concurrently; every kernel's result depends only on its own inputs, so the
// results do not depend on the lane count.
static hipError_t make_lanes(bbp_ctx *c, int n) {
  while ((int)c->aux.size() < n - 1) {
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    c->aux.push_back(s);
  }
  while ((int)c->lane_ev.size() < n) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    c->lane_ev.push_back(ev);
  }
  return hipSuccess;
}
static hipStream_t lane_stream(const bbp_ctx *c, int l) {
  return l == 0 ? c->stream : c->aux[l - 1];
}

// Work enqueued on lanes 1..n-1 after fork() is ordered after everything
// enqueued on the context stream before it; after join() (also run by the
// destructor, so an early error return still joins) the context stream
// waits for all of it.
struct LaneFork {
  bbp_ctx *c;
  int n = 1;
  explicit LaneFork(bbp_ctx *ctx) : c(ctx) {}
  hipError_t fork(int want) {
    hipError_t e = make_lanes(c, want);
    if (e != hipSuccess) return e;
    e = hipEventRecord(c->lane_ev[0], c->stream);
    for (int l = 1; e == hipSuccess && l < want; ++l)
      e = hipStreamWaitEvent(c->aux[l - 1], c->lane_ev[0], 0);
    if (e == hipSuccess) n = want;
    return e;
  }
  hipError_t join() {
    hipError_t e = hipSuccess;
    for (int l = 1; l < n; ++l) {
      hipError_t e1 = hipEventRecord(c->lane_ev[l], c->aux[l - 1]);
      if (e1 == hipSuccess) e1 = hipStreamWaitEvent(c->stream, c->lane_ev[l], 0);
      if (e == hipSuccess) e = e1;
    }
    n = 1;
    return e;
  }
  ~LaneFork() { (void)join(); }
};

// Work enqueued on `dst` after this call is ordered after the work enqueued
// on `src` before it; `k` counts the context's dependency events used so far
// by the current call (each wait gets an event of its own).
static hipError_t lane_after(bbp_ctx *c, hipStream_t dst, hipStream_t src, size_t &k) {
  if (dst == src) return hipSuccess;
  while (c->dep_ev.size() <= k) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    c->dep_ev.push_back(ev);
  }
  hipEvent_t ev = c->dep_ev[k++];
  hipError_t e = hipEventRecord(ev, src);
  if (e == hipSuccess) e = hipStreamWaitEvent(dst, ev, 0);
  return e;
}

// Copies `bytes` from host memory to the device on `st` through the pinned
// pool, so that the call returns without waiting for the stream.
static hipError_t upload_pinned(bbp_ctx *c, void *dst, const void *src, size_t bytes,
                                hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  void *h = c->pin.get(bytes);
  if (!h) return hipErrorOutOfMemory;
  std::memcpy(h, src, bytes);
  return hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, st);
}

// Splits a batch of ids into up to `parts` contiguous batches of at least
// `min_items` each.
static std::vector<std::vector<int>> split_batch(const std::vector<int> &ids, int parts,
                                                 int min_items) {
  const int n = (int)ids.size();
  const int k = std::max(1, std::min(parts, n / std::max(1, min_items)));
  std::vector<std::vector<int>> out(k);
  for (int p = 0; p < k; ++p)
    out[p].assign(ids.begin() + (size_t)n * p / k, ids.begin() + (size_t)n * (p + 1) / k);
  return out;
}
constexpr int kLaneMinItems = 8;

// A batch of the given shape from the context's cache (the one set up last
// time for the same W, H and item count keeps its device buffers), else new.
static std::unique_ptr<Group> take_batch(bbp_ctx *c, int W, int H, int items) {
  for (auto it = c->batch_cache.begin(); it != c->batch_cache.end(); ++it)
    if ((*it)->W == W && (*it)->H == H && (*it)->fb.items == items) {
      std::unique_ptr<Group> g = std::move(*it);
      c->batch_cache.erase(it);
      g->ids.clear();
      return g;
    }
  std::unique_ptr<Group> g(new Group);
  g->W = W;
  g->H = H;
  return g;
}
// Returns batches to the cache when the call that used them ends (also on an
// early error return).
struct BatchReturn {
  bbp_ctx *c;
  std::vector<std::unique_ptr<Group>> *v;
  ~BatchReturn() {
    for (auto &g : *v)
      if (g) {
        g->cache_gen = c->obs_call;
        c->batch_cache.push_back(std::move(g));
      }
    v->clear();
  }
};
// Kept boundary stacks: groups no stack refers to any more go back to the
// batch cache; release_kept drops every kept stack.
static void gc_kept(bbp_ctx *c) {
  std::set<const Group *> used;
  for (auto &kv : c->kept_stacks) used.insert(kv.second.g);
  auto &v = c->kept_groups;
  for (auto &g : v)
    if (g && !used.count(g.get())) {
      g->cache_gen = c->obs_call;
      c->batch_cache.push_back(std::move(g));
    }
  v.erase(std::remove(v.begin(), v.end(), nullptr), v.end());
}
static void release_kept(bbp_ctx *c) {
  c->kept_stacks.clear();
  gc_kept(c);
}

// A device buffer of exactly `bytes` from the context's cache, else new.
static DevBuf take_unit_out(bbp_ctx *c, size_t bytes) {
  for (auto it = c->unit_out_cache.begin(); it != c->unit_out_cache.end(); ++it)
    if (it->second.bytes == bytes) {
      DevBuf b = std::move(it->second);
      c->unit_out_cache.erase(it);
      return b;
    }
  return DevBuf();
}
// At the end of an observables call (also on an early error return): drop
// the cached entries no call since the previous one has used.
struct CacheTrim {
  bbp_ctx *c;
  ~CacheTrim() {
    const int keep = c->obs_call - 1;
    auto &b = c->batch_cache;
    b.erase(std::remove_if(b.begin(), b.end(),
                           [&](const std::unique_ptr<Group> &g) { return g->cache_gen < keep; }),
            b.end());
    auto &u = c->unit_out_cache;
    u.erase(std::remove_if(u.begin(), u.end(),
                           [&](const std::pair<int, DevBuf> &e) { return e.first < keep; }),
            u.end());
    auto &ug = c->unit_groups;
    ug.erase(std::remove_if(ug.begin(), ug.end(),
                            [&](const std::unique_ptr<Group> &g) { return g->cache_gen < keep; }),
             ug.end());
  }
};

// Frees the observables' kept buffers (every entry belongs to a call that
// has returned, so no device work uses them).
static void evict_caches(void *ctx) {
  bbp_ctx *c = static_cast<bbp_ctx *>(ctx);
  c->batch_cache.clear();
  c->unit_out_cache.clear();
  c->unit_groups.clear();
}

// ---------------------------------------------------------------------------
static bbp_status ensure_device(bbp_ctx *c) {
  if (c->device_ready) return BBP_OK;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0)
    return c->fail(BBP_EDEVICE, "no HIP device available");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, 0);
  if (e != hipSuccess) return c->hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return c->fail(BBP_EDEVICE,
                   std::string("libbbp is built for gfx950, device is ") +
                       prop.gcnArchName);
  c->device_ready = true;
  return BBP_OK;
}

// Buffers a batch needs (bit mask for alloc_batch).
enum : unsigned {
  NEED_FIT = 1u,      // store, xin, mt, mb, lenv, renv, tmp, acan, rbuf, nu
  NEED_SCRATCH = 2u,  // t3, and t1/t2 when the generic chain or QR needs them
};

// With `pinned`, the slot table goes up through the context's pinned pool
// and the call returns without waiting for the device (the clears and the
// upload are queued on the context stream).
static bbp_status alloc_batch(bbp_ctx *c, Group &g, int items, int bond_cap,
                              const std::vector<uint64_t> &slots,
                              unsigned need = NEED_FIT | NEED_SCRATCH, bool pinned = false) {
  FitBatch &f = g.fb;
  f.items = items;
  f.tile_items = items;
  f.K = bond_cap;
  f.P = c->P;
  f.D = c->D;
  f.d = c->d;
  f.H = g.H;
  f.W = g.W;
  f.N = g.H + 2;
  f.S = (size_t)bond_cap * c->P * bond_cap;
  f.seed = c->seed;
  f.prec = c->precision;
  f.bra_one = c->single_layer ? c->delta.d() : nullptr;
  const size_t it = f.items, S = f.S, K = f.K, P = f.P;
  const bool fused = visit_fused_fits(f);
  const bool fit = (need & NEED_FIT) != 0, scr = (need & NEED_SCRATCH) != 0;
  struct Req {
    double **dst;
    size_t n;
    bool zero;  // cleared: zero padding of MPS slots is relied upon
  };
  std::vector<Req> reqs = {
      {&f.store, fit ? it * f.W * f.N * S : 0, true},
      {&f.xin, fit ? it * f.N * S : 0, true},
      {&f.mt, fit ? it * f.W * S : 0, true},
      {&f.mb, fit ? it * f.W * S : 0, true},
      {&f.lenv, fit ? it * f.N * S : 0, true},
      {&f.renv, fit ? it * f.N * S : 0, true},
      {&f.t1, scr && (!fused || qr_needs_scratch(f)) ? it * K * P * P * K : 0,
       false},
      {&f.t2, scr && !fused ? it * (size_t)f.d * K * K * P * P : 0, false},
      {&f.t3, scr ? it * K * P * P * K : 0, false},
      {&f.tmp, fit ? it * S : 0, false},
      {&f.acan, fit ? it * f.H * f.W * (size_t)f.d * P * P : 0, true},
      {&f.rbuf, fit ? it * K * K : 0, false},
      {&f.nu, fit ? it * f.W : 0, true},
  };
  // a batch set up again with the same shapes keeps its allocations
  if (g.bufs.size() != reqs.size() + 4) {
    g.bufs.clear();
    g.bufs.resize(reqs.size() + 4);
  }
  hipError_t e;
  for (size_t i = 0; i < reqs.size(); ++i) {
    *reqs[i].dst = nullptr;
    if (reqs[i].n == 0) {
      g.bufs[i].release();
      continue;
    }
    e = g.bufs[i].alloc(reqs[i].n * 8);
    if (e != hipSuccess) return c->fail(BBP_ENOMEM, "device allocation failed");
    *reqs[i].dst = g.bufs[i].d();
    if (reqs[i].zero) {
      e = hipMemsetAsync(g.bufs[i].p, 0, g.bufs[i].bytes, c->stream);
      if (e != hipSuccess) return c->hip_fail(e, "clear buffers");
    }
  }
  size_t k = reqs.size();
  if (g.bufs[k].alloc(it * 4) != hipSuccess ||
      g.bufs[k + 1].alloc(sizeof(FitDims) * it * f.W) != hipSuccess ||
      g.bufs[k + 2].alloc(8 * it) != hipSuccess ||
      g.gather.alloc(sizeof(GatherSrc) * it) != hipSuccess ||
      g.dst.alloc(sizeof(double *) * it) != hipSuccess ||
      g.rev.alloc(4 * it) != hipSuccess ||
      g.flagbuf.alloc(4 * it * f.W) != hipSuccess)
    return c->fail(BBP_ENOMEM, "device allocation failed");
  f.flag = (int32_t *)g.bufs[k].p;
  f.dims = (FitDims *)g.bufs[k + 1].p;
  f.slot = (uint64_t *)g.bufs[k + 2].p;
  f.err = (int32_t *)c->errflag.p;
  g.dims.assign(it * f.W, FitDims{});
  g.have.assign(it * f.W, 0);
  e = pinned ? upload_pinned(c, f.slot, slots.data(), 8 * it, c->stream)
             : copy_sync(c, f.slot, slots.data(), 8 * it, hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "upload slots");
  return BBP_OK;
}

// Upload rotated block tensors of every message of a group.
static bbp_status upload_rotated(bbp_ctx *c, Group &g) {
  FitBatch &f = g.fb;
  const size_t ss = (size_t)c->d * c->P * c->P;
  std::vector<double> host((size_t)f.items * f.H * f.W * ss);
  for (int i = 0; i < f.items; ++i) {
    const Message &m = c->msgs[g.ids[i]];
    for (int yc = 0; yc < f.H; ++yc)
      for (int xc = 0; xc < f.W; ++xc) {
        int y, x;
        canon_to_region(m.dir, c->by, c->bx, yc, xc, &y, &x);
        const double *src = c->site(m.bi * c->bx + x, m.bj * c->by + y);
        rotate_site(c, src, m.dir,
                    host.data() + (((size_t)i * f.H + yc) * f.W + xc) * ss);
      }
  }
  hipError_t e = copy_sync(c, f.acan, host.data(), host.size() * 8,
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "upload tensors");
  return BBP_OK;
}

// Uniform value in [-1, 1) number i of the counter-based stream of (seed,
// slot, site): SplitMix64 (Steele, Lea, Flood 2014) chained over the
// counters, the top 53 bits scaled; the same values the fit's random starts
// draw (k_rand_init).
static double host_counter_uniform(uint64_t seed, uint64_t slot, uint64_t site, uint64_t i) {
  auto sm = [](uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const uint64_t h = sm(sm(sm(sm(seed) ^ slot) ^ site) ^ i);
  return (double)(h >> 11) * 0x1p-52 - 1.0;
}

static bbp_status init_messages(bbp_ctx *c) {
  // init 0: identity product MPDO, m[(k,k')] = delta_kk' / sqrt(D), bonds 1.
  // init 1: random product MPDO (App. A), per site m[(k,k')] = sum_a
  // R[k][a] R[k'][a] with R the D x D counter-based uniform values of (seed,
  // 2^41 + message, site), scaled to unit 2-norm; bonds 1.
  const size_t per = (size_t)c->Lmax * c->S;
  std::vector<double> host(per * c->msgs.size(), 0.0);
  const int D = c->D;
  const double v = 1.0 / std::sqrt((double)D);
  std::vector<double> R((size_t)D * D), M((size_t)D * D);
  for (size_t e = 0; e < c->msgs.size(); ++e) {
    Message &m = c->msgs[e];
    m.bonds.assign(m.n + 1, 1);
    for (int s = 0; s < m.n; ++s) {
      double *site = &host[e * per + (size_t)s * c->S];
      if (c->init == 0) {
        for (int k = 0; k < D; ++k) site[(size_t)(k * D + k) * c->K] = v;
        continue;
      }
      for (int i = 0; i < D * D; ++i)
        R[i] = host_counter_uniform(c->seed, (1ull << 41) + e, (uint64_t)s, (uint64_t)i);
      double nrm = 0.0;
      for (int k = 0; k < D; ++k)
        for (int kp = 0; kp < D; ++kp) {
          double x = 0.0;
          for (int a = 0; a < D; ++a) x += R[k * D + a] * R[kp * D + a];
          M[k * D + kp] = x;
          nrm += x * x;
        }
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0)) return c->fail(BBP_ENUMERIC, "zero random initial message");
      for (int q = 0; q < D * D; ++q) site[(size_t)q * c->K] = M[q] / nrm;
    }
  }
  hipError_t err = copy_sync(c, c->msgbuf[c->cur].p, host.data(), host.size() * 8,
                             hipMemcpyHostToDevice);
  if (err != hipSuccess) return c->hip_fail(err, "upload messages");
  for (auto &g : c->groups) std::fill(g->have.begin(), g->have.end(), 0);
  return BBP_OK;
}

// Multiply-adds of the fit contractions of one column absorption, counted
// with the true bond dimensions on the split-layer schedule.
static double column_macs(const FitDims &f, const std::vector<int> &xb_bonds,
                          int xp0, int xpN, int N, int P, int D, int d,
                          int n_fit) {
  const double D6 = std::pow((double)D, 6);
  auto xb = [&](int j) { return (double)xb_bonds[j]; };  // X bond j|j+1
  auto xl = [&](int j) { return j ? xb(j - 1) : 1.0; };
  auto xr = [&](int j) { return j < N - 1 ? xb(j) : 1.0; };
  // inner site j: T1 (yf*P*xf*P*xb) + ket + bra (2*yf*xb*d*D^6) + local
  // (yf*P*xb*P*yb) + env (yb*P*xb*yf*P); LR front = left.
  auto inner = [&](int j, bool rl, bool local, bool env) {
    double yf = rl ? f.br[j] : f.bl[j], yb = rl ? f.bl[j] : f.br[j];
    double xf = rl ? xr(j) : xl(j), xbk = rl ? xl(j) : xr(j);
    double m = yf * P * xf * P * xbk + 2.0 * yf * xbk * d * D6;
    if (local) m += yf * P * xbk * P * yb;
    if (env) m += yb * P * xbk * yf * P;
    return m;
  };
  auto endsite = [&](int j, bool local, bool env) {
    double a = f.p[j], xe = (j == 0) ? xr(0) : xl(N - 1);
    double ye = (j == 0) ? f.br[0] : f.bl[N - 1];
    double xp = (j == 0) ? xp0 : xpN;  // X end site's physical dimension
    double m = a * P * xp * xe;
    if (local) m += a * P * xe * ye;
    if (env) m += ye * a * P * xe;
    return m;
  };
  double t = 0.0;
  for (int j = N - 1; j >= 1; --j)
    t += (j == N - 1) ? endsite(j, false, true) : inner(j, true, false, true);
  for (int s = 0; s < n_fit; ++s) {
    for (int j = 0; j < N - 1; ++j)
      t += j == 0 ? endsite(0, true, true) : inner(j, false, true, true);
    for (int j = N - 1; j >= 1; --j)
      t += j == N - 1 ? endsite(j, true, true) : inner(j, true, true, true);
  }
  t += endsite(0, true, false);
  return t;
}

static bbp_status enqueue_columns(bbp_ctx *c, Group &g, int col_lo, hipStream_t st,
                                  const std::vector<int> &any_rnd, int col_hi = -1);
static bool same_batch(const FitBatch &a, const FitBatch &b);

// Absorb canonical columns W-1 .. col_lo of every item of a batch (App. A:
// each column is an MPO x MPS variational fit), or col_hi .. col_lo when
// col_hi >= 0 (the batch's store then holds column col_hi + 1's result).
// Uses g.dims (uploaded here) for the bond caps and the random-start flags.  A message batch
// (graph = true) whose columns all start warm has the same launch sequence,
// with the same arguments, in every sweep: it is captured as a HIP graph
// once and replayed, one launch instead of one per kernel.  Timing brackets
// (a process-wide switch) are not captured.
static bbp_status absorb_columns(bbp_ctx *c, Group &g, int col_lo, hipStream_t st,
                                 bool graph = false, int col_hi = -1, bool pinned = false) {
  FitBatch &f = g.fb;
  const int W = f.W;
  hipError_t e;
  std::vector<int> any_rnd(W, 0);
  for (int i = 0; i < f.items; ++i)
    for (int col = 0; col < W; ++col)
      any_rnd[col] |= g.dims[(size_t)i * W + col].rnd;
  // the kernels that skip zero padding read the true extents (f.dims) only
  // while the batch's dims describe what is being absorbed: during this call
  struct TrueDims {
    FitBatch &f;
    ~TrueDims() {
      f.hdims = nullptr;
      f.bounded = 0;
    }
  } true_dims{f};
  f.hdims = g.dims.data();
  f.bounded = c->skip_pad;
  e = pinned ? upload_pinned(c, f.dims, g.dims.data(), sizeof(FitDims) * g.dims.size(), st)
             : hipMemcpyAsync(f.dims, g.dims.data(), sizeof(FitDims) * g.dims.size(),
                              hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return c->hip_fail(e, "upload dims");
  g.flags.assign((size_t)W * f.items, 0);
  for (int col = 0; col < W; ++col)
    for (int i = 0; i < f.items; ++i)
      g.flags[(size_t)col * f.items + i] = g.dims[(size_t)i * W + col].rnd;
  e = pinned ? upload_pinned(c, g.flagbuf.p, g.flags.data(), 4 * g.flags.size(), st)
             : hipMemcpyAsync(g.flagbuf.p, g.flags.data(), 4 * g.flags.size(),
                              hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return c->hip_fail(e, "upload flags");
  bool warm = true;
  for (int col = col_lo; col < W; ++col) warm = warm && !any_rnd[col];
  if (!graph || !c->graphs || !warm || bbp::timing_enabled() || col_hi >= 0)
    return enqueue_columns(c, g, col_lo, st, any_rnd, col_hi);
  if (g.graph && (g.graph_nfit != c->n_fit || !same_batch(g.graph_fb, f))) {
    (void)hipGraphExecDestroy(g.graph);
    g.graph = nullptr;
  }
  if (!g.graph) {
    // captured on a stream of its own (the context stream may be the null
    // stream, which cannot be captured); the graph is then launched on st
    if (!c->cap && (e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking)) != hipSuccess)
      return c->hip_fail(e, "capture stream");
    hipGraph_t gr = nullptr;
    if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed)) != hipSuccess)
      return c->hip_fail(e, "begin capture");
    bbp_status bs = enqueue_columns(c, g, col_lo, c->cap, any_rnd);
    e = hipStreamEndCapture(c->cap, &gr);
    if (bs != BBP_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return bs;
    }
    if (e != hipSuccess) return c->hip_fail(e, "end capture");
    e = hipGraphInstantiate(&g.graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
      g.graph = nullptr;
      return c->hip_fail(e, "instantiate graph");
    }
    g.graph_fb = f;
    g.graph_nfit = c->n_fit;
  }
  if ((e = hipGraphLaunch(g.graph, st)) != hipSuccess) return c->hip_fail(e, "graph launch");
  return BBP_OK;
}

static bool same_batch(const FitBatch &a, const FitBatch &b) {
  return a.items == b.items && a.tile_items == b.tile_items && a.K == b.K && a.P == b.P &&
         a.D == b.D && a.d == b.d && a.H == b.H && a.W == b.W && a.N == b.N && a.S == b.S &&
         a.store == b.store && a.xin == b.xin && a.mt == b.mt && a.mb == b.mb &&
         a.lenv == b.lenv && a.renv == b.renv && a.t1 == b.t1 && a.t2 == b.t2 &&
         a.t3 == b.t3 && a.tmp == b.tmp && a.acan == b.acan && a.abra == b.abra &&
         a.rbuf == b.rbuf && a.nu == b.nu && a.flag == b.flag && a.err == b.err &&
         a.dims == b.dims && a.slot == b.slot && a.seed == b.seed && a.prec == b.prec &&
         a.bounded == b.bounded && a.bra_one == b.bra_one;
}

// The launches of absorb_columns, enqueued on st.
static bbp_status enqueue_columns(bbp_ctx *c, Group &g, int col_lo, hipStream_t st,
                                  const std::vector<int> &any_rnd, int col_hi) {
  FitBatch &f = g.fb;
  const int W = f.W, N = f.N;
  hipError_t e;
  const size_t sN = (size_t)N * f.S, sWN = (size_t)W * N * f.S;
  for (int col = col_hi >= 0 ? col_hi : W - 1; col >= col_lo; --col) {
    Ptr X = col == W - 1 ? Ptr{f.xin, sN}
                         : Ptr{f.store + slot_store(f, col + 1, 0), sWN};
    auto Xs = [&](int j) { return Ptr{X.p + (size_t)j * f.S, X.stride}; };
    auto Ys = [&](int j) { return Ptr{f.store + slot_store(f, col, j), sWN}; };
    auto Le = [&](int j) { return Ptr{f.lenv + (size_t)j * f.S, sN}; };
    auto Re = [&](int j) { return Ptr{f.renv + (size_t)j * f.S, sN}; };
    Ptr MT{f.mt + (size_t)col * f.S, (size_t)W * f.S};
    Ptr MB{f.mb + (size_t)col * f.S, (size_t)W * f.S};
    if (any_rnd[col]) {
      f.flag = (int32_t *)g.flagbuf.p + (size_t)col * f.items;
      if ((e = launch_rand_init(f, col, Ys(0), st)) != hipSuccess)
        return c->hip_fail(e, "rand_init");
      for (int j = N - 1; j >= 1; --j) {
        e = launch_qr(f, col, j, j == N - 1 ? RL_BOT : RL_INNER, Ys(j), true,
                      true, st);
        if (e == hipSuccess) e = launch_apply_l(f, j - 1 == 0, Ys(j - 1), st);
        if (e != hipSuccess) return c->hip_fail(e, "canonicalise");
      }
    }
    if ((e = launch_set_unit(f, Le(0), st)) != hipSuccess ||
        (e = launch_set_unit(f, Re(N - 1), st)) != hipSuccess)
      return c->hip_fail(e, "set_unit");
    for (int j = N - 1; j >= 1; --j) {
      if (j == N - 1) {
        e = launch_end_chain(f, col, true, MB, Xs(N - 1), st);
        if (e == hipSuccess) e = launch_end_env(f, col, true, Ys(N - 1), Re(N - 2), st);
      } else {
        e = launch_inner_chain(f, col, j, true, Xs(j), Re(j), st);
        if (e == hipSuccess) e = launch_inner_env(f, col, j, true, Ys(j), Re(j - 1), st);
      }
      if (e != hipSuccess) return c->hip_fail(e, "right environments");
    }
    for (int sw = 0; sw < c->n_fit; ++sw) {
      for (int j = 0; j < N - 1; ++j) {
        if (j == 0) {
          e = launch_end_chain(f, col, false, MT, Xs(0), st);
          if (e == hipSuccess) e = launch_end_local(f, col, false, Re(0), Ys(0), st);
          if (e == hipSuccess) e = launch_qr(f, col, 0, LR_TOP, Ys(0), false, false, st);
          if (e == hipSuccess) e = launch_end_env(f, col, false, Ys(0), Le(1), st);
        } else {
          e = launch_inner_visit(f, col, j, false, Xs(j), Le(j), Re(j), Ys(j), st);
          if (e == hipSuccess) e = launch_qr(f, col, j, LR_INNER, Ys(j), false, false, st);
          if (e == hipSuccess) e = launch_inner_env(f, col, j, false, Ys(j), Le(j + 1), st);
        }
        if (e != hipSuccess) return c->hip_fail(e, "left-to-right visit");
      }
      for (int j = N - 1; j >= 1; --j) {
        if (j == N - 1) {
          e = launch_end_chain(f, col, true, MB, Xs(N - 1), st);
          if (e == hipSuccess) e = launch_end_local(f, col, true, Le(N - 1), Ys(N - 1), st);
          if (e == hipSuccess) e = launch_qr(f, col, N - 1, RL_BOT, Ys(N - 1), false, false, st);
          if (e == hipSuccess) e = launch_end_env(f, col, true, Ys(N - 1), Re(N - 2), st);
        } else {
          e = launch_inner_visit(f, col, j, true, Xs(j), Re(j), Le(j), Ys(j), st);
          if (e == hipSuccess) e = launch_qr(f, col, j, RL_INNER, Ys(j), false, false, st);
          if (e == hipSuccess) e = launch_inner_env(f, col, j, true, Ys(j), Re(j - 1), st);
        }
        if (e != hipSuccess) return c->hip_fail(e, "right-to-left visit");
      }
    }
    e = launch_end_chain(f, col, false, MT, Xs(0), st);
    if (e == hipSuccess) e = launch_end_local(f, col, false, Re(0), Ys(0), st);
    if (e == hipSuccess) e = launch_normalize(f, col, Ys(0), st);
    if (e != hipSuccess) return c->hip_fail(e, "final visit");
  }
  return BBP_OK;
}

// Sweep tables of item i of batch g for message `id` of context c: its
// three gather sources in the previous sweep's buffer `cur`, its destination
// in `nb`, the bond caps of every column (g.dims, with the random-start flag
// where the warm start's shapes no longer agree), and the new message's bond
// list.  Returns the item's fit FLOPs on the true bonds.
static double prepare_item(bbp_ctx *c, int id, double *cur, double *nb, Group &g, int i,
                           GatherSrc &gs, double *&dst, int32_t &rev,
                           std::vector<int> &new_bonds) {
  const FitBatch &f = g.fb;
  const int W = f.W, H = f.H, N = f.N;
  const size_t per = (size_t)c->Lmax * c->S;
  const Message &m = c->msgs[id];
  char side[3];
  int rv[3];
  canon_sources(m.dir, side, rv);
  std::vector<int> bl[3];
  gs = GatherSrc{};
  gs.ksrc = c->K;
  for (int k = 0; k < 3; ++k) {
    Incoming in = c->incoming(m.bi, m.bj, side[k]);
    if (in.id < 0) {
      gs.src[k][0] = c->trivial.d();
      bl[k].assign(in.n + 1, 1);
    } else {
      gs.src[k][0] = cur + (size_t)in.id * per;
      bl[k] = c->msgs[in.id].bonds;
    }
    gs.n[k][0] = in.n;
    gs.rev[k][0] = rv[k];
    if (rv[k]) bl[k] = reversed(bl[k]);
  }
  dst = nb + (size_t)id * per;
  rev = out_reversed(m.dir) ? 1 : 0;
  std::vector<FitDims> cd;
  column_dims(W, H, f.K, f.P, bl[0], bl[2], bl[1], cd);
  std::vector<int> xbonds = bl[1];
  double flops = 0.0;
  for (int col = W - 1; col >= 0; --col) {
    FitDims &nd = cd[col];
    FitDims &od = g.dims[(size_t)i * W + col];
    bool same = g.have[(size_t)i * W + col] &&
                std::memcmp(nd.bl, od.bl, sizeof(nd.bl)) == 0 &&
                std::memcmp(nd.br, od.br, sizeof(nd.br)) == 0 &&
                std::memcmp(nd.p, od.p, sizeof(nd.p)) == 0;
    nd.rnd = same ? 0 : 1;
    od = nd;
    g.have[(size_t)i * W + col] = 1;
    const int xp0 = col == W - 1 ? 1 : cd[col + 1].p[0];
    const int xpN = col == W - 1 ? 1 : cd[col + 1].p[N - 1];
    flops += 2.0 * column_macs(nd, xbonds, xp0, xpN, N, f.P, f.D, f.d, c->n_fit);
    xbonds.assign(N - 1, 1);
    for (int j = 0; j < N - 1; ++j) xbonds[j] = nd.br[j];
  }
  const FitDims &c0 = cd[0];
  std::vector<int> cb(H + 1, 1);
  for (int s2 = 0; s2 + 1 < H; ++s2) cb[s2 + 1] = c0.br[s2 + 1];
  new_bonds = rev ? reversed(cb) : cb;
  return flops;
}

static bbp_status run_sweep(bbp_ctx *c, double *residual) {
  hipStream_t st = c->stream;
  const int nxt = 1 - c->cur;
  const size_t per = (size_t)c->Lmax * c->S;
  double *cur = c->msgbuf[c->cur].d(), *nb = c->msgbuf[nxt].d();
  hipError_t e = hipMemsetAsync(c->errflag.p, 0, 4, st);
  if (e != hipSuccess) return c->hip_fail(e, "memset");
  std::vector<std::vector<int>> new_bonds(c->msgs.size());
  double flops = 0.0;
  const int nl = std::max(1, std::min(c->lanes, (int)c->groups.size()));
  LaneFork lanes(c);
  if ((e = lanes.fork(nl)) != hipSuccess) return c->hip_fail(e, "fork lanes");
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    Group &g = *c->groups[gi];
    st = lane_stream(c, (int)(gi % nl));
    FitBatch &f = g.fb;
    const int W = f.W, H = f.H, N = f.N;
    std::vector<GatherSrc> &gs = g.gs;
    std::vector<double *> &dsts = g.dsts;
    std::vector<int32_t> &revs = g.revs;
    gs.assign(f.items, GatherSrc{});
    dsts.assign(f.items, nullptr);
    revs.assign(f.items, 0);
    for (int i = 0; i < f.items; ++i)
      flops += prepare_item(c, g.ids[i], cur, nb, g, i, gs[i], dsts[i], revs[i],
                            new_bonds[g.ids[i]]);
    e = hipMemcpyAsync(g.gather.p, gs.data(), sizeof(GatherSrc) * f.items,
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.dst.p, dsts.data(), sizeof(double *) * f.items,
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.rev.p, revs.data(), 4 * f.items,
                         hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return c->hip_fail(e, "upload sweep tables");
    e = launch_gather(f, (const GatherSrc *)g.gather.p, st);
    if (e != hipSuccess) return c->hip_fail(e, "gather");

    bbp_status bs = absorb_columns(c, g, 0, st, true);
    if (bs != BBP_OK) return bs;
    e = launch_extract(f, (double *const *)g.dst.p, (const int32_t *)g.rev.p, st);
    if (e != hipSuccess) return c->hip_fail(e, "extract");
  }
  st = c->stream;
  if ((e = lanes.join()) != hipSuccess) return c->hip_fail(e, "join lanes");
  // residual: overlaps of new and old messages, grouped by length
  const int nm = (int)c->msgs.size();
  std::vector<double> ov(nm, 0.0);
  std::map<int, std::vector<int>> by_len;
  for (int i = 0; i < nm; ++i) by_len[c->msgs[i].n].push_back(i);
  // every length group's overlaps go to their own part of the output, read
  // back with the error flag after one synchronisation (the groups share the
  // overlap kernel's scratch, in stream order)
  std::vector<const double *> pa(nm), pb(nm);
  std::vector<double> out(nm, 0.0);
  int off = 0;
  for (auto &kv : by_len) {
    const std::vector<int> &ids = kv.second;
    for (size_t i = 0; i < ids.size(); ++i) {
      pa[off + i] = nb + (size_t)ids[i] * per;
      pb[off + i] = cur + (size_t)ids[i] * per;
    }
    off += (int)ids.size();
  }
  e = hipMemcpyAsync(c->ovA.p, pa.data(), 8 * (size_t)nm, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ovB.p, pb.data(), 8 * (size_t)nm, hipMemcpyHostToDevice, st);
  off = 0;
  for (auto &kv : by_len) {
    if (e != hipSuccess) break;
    const int n = (int)kv.second.size();
    e = launch_overlap(n, c->K, c->P, kv.first, (const double *const *)c->ovA.p + off,
                       (const double *const *)c->ovB.p + off, c->ovE.d(), c->ovU.d(),
                       c->ovOut.d() + off, st);
    off += n;
  }
  int32_t errv = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(out.data(), c->ovOut.p, 8 * (size_t)nm, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&errv, c->errflag.p, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return c->hip_fail(e, "overlap");
  off = 0;
  for (auto &kv : by_len)
    for (int id : kv.second) ov[id] = out[off++];
  double sum = 0.0;
  bool finite = true;
  for (int i = 0; i < nm; ++i) {
    if (!std::isfinite(ov[i])) finite = false;
    sum += std::max(0.0, 2.0 - 2.0 * std::fabs(ov[i]));
  }
  if (errv || !finite) {
    for (auto &g : c->groups) std::fill(g->have.begin(), g->have.end(), 0);
    return c->fail(BBP_ENUMERIC, "zero-norm or non-finite boundary in sweep");
  }
  for (int i = 0; i < nm; ++i) c->msgs[i].bonds = new_bonds[i];
  c->cur = nxt;
  c->obs.clear();
  release_kept(c);
  c->last_flops = flops;
  if (residual) *residual = nm ? sum / nm : 0.0;
  return BBP_OK;
}

// ---------------------------------------------------------------------------
// Observables (Sec. II; App. A second paragraph; App. B): a region (a block,
// or the union of two neighbouring blocks for a bond crossing them) with its
// incoming messages.  Boundary MPSs are absorbed from each side at bond
// chi_env (the same fit engine as the messages), then every line of the
// region is contracted exactly between its two boundaries: left and right
// environment chains, and environment steps with a matrix unit |s'><s| on
// one site, whose contractions are the one- and two-site reduced density
// matrices.
// ---------------------------------------------------------------------------
namespace {

struct Seg {
  int id;  // message id, -1 for a trivial message
  int n;   // sites
};

// A bond whose two-site values are wanted: frame, line and the position of
// its first site along the line (region coordinates).
struct Target {
  bool row;
  int line, pos;
};

struct RegionSpec {
  int kind, bi, bj;  // 0 block, 1 block + right neighbour, 2 block + lower
  int H, W;
  std::vector<Seg> side[4];  // incoming on 'U','D','L','R', natural order
  bool row, col;             // frames needed
  // empty: every line of the frames and every site and bond on it;
  // otherwise only the lines and bonds listed
  std::vector<Target> targets;
  bool wants_line(bool r, int k) const {
    if (targets.empty()) return true;
    for (const Target &t : targets)
      if (t.row == r && t.line == k) return true;
    return false;
  }
};

int side_slot(char s) { return s == 'U' ? 0 : s == 'D' ? 1 : s == 'L' ? 2 : 3; }

struct StackItem {
  int region;
  char orient;
  int Wc, Hc;  // canonical width (columns absorbed from) and height
};

struct LineItem {
  int region;
  bool row;     // row frame ('D' stack as X, 'U' stack as Y) or column frame
  int k;        // row (row frame) or column (column frame) in the region
  int xs, ys;   // stack item indices of the X and Y boundaries
  int cx, cy;   // canonical column of the line in the X / Y frames
  double ls;    // log scale of the two boundaries
};

// Where a boundary stack's results live: its batch, its item there and its
// column scales.
struct StackRef {
  Group *g = nullptr;
  int item = 0;
  const double *nu = nullptr;
};

struct UnitItem {
  int line;  // index in the line batch
  int j;     // canonical site (1..H)
  int u;     // matrix unit s'*d + s
};

}  // namespace

static RegionSpec region_spec(const bbp_ctx *c, int kind, int bi, int bj) {
  RegionSpec r;
  r.kind = kind;
  r.bi = bi;
  r.bj = bj;
  r.row = r.col = false;
  auto inc = [&](int i, int j, char sd) {
    Incoming in = c->incoming(i, j, sd);
    return Seg{in.id, in.n};
  };
  if (kind == 0) {
    r.H = c->by;
    r.W = c->bx;
    for (char sd : {'U', 'D', 'L', 'R'}) r.side[side_slot(sd)] = {inc(bi, bj, sd)};
  } else if (kind == 1) {
    int ni, nj;
    c->neighbour(bi, bj, 'R', &ni, &nj);
    r.H = c->by;
    r.W = 2 * c->bx;
    r.side[0] = {inc(bi, bj, 'U'), inc(ni, nj, 'U')};
    r.side[1] = {inc(bi, bj, 'D'), inc(ni, nj, 'D')};
    r.side[2] = {inc(bi, bj, 'L')};
    r.side[3] = {inc(ni, nj, 'R')};
  } else {
    int ni, nj;
    c->neighbour(bi, bj, 'D', &ni, &nj);
    r.H = 2 * c->by;
    r.W = c->bx;
    r.side[0] = {inc(bi, bj, 'U')};
    r.side[1] = {inc(ni, nj, 'D')};
    r.side[2] = {inc(bi, bj, 'L'), inc(ni, nj, 'L')};
    r.side[3] = {inc(bi, bj, 'R'), inc(ni, nj, 'R')};
  }
  return r;
}

static uint64_t region_slot(int kind, int bi, int bj, char orient) {
  return (2ull << 40) | ((uint64_t)kind << 36) | ((uint64_t)bj << 24) |
         ((uint64_t)bi << 12) | ((uint64_t)dir_index(orient) << 8);
}

// Gather table and bond lists of one rotated side made of message segments.
static void side_source(const bbp_ctx *c, const std::vector<Seg> &segs,
                        bool rev, GatherSrc &g, int k, std::vector<int> &bonds) {
  std::vector<Seg> order = segs;
  if (rev) std::reverse(order.begin(), order.end());
  const size_t per = (size_t)c->Lmax * c->S;
  const double *cur = c->msgbuf[c->cur].d();
  bonds.assign(1, 1);
  for (size_t t = 0; t < 2; ++t) {
    g.src[k][t] = nullptr;
    g.n[k][t] = 0;
    g.rev[k][t] = 0;
  }
  for (size_t t = 0; t < order.size(); ++t) {
    const Seg &sg = order[t];
    g.src[k][t] = sg.id < 0 ? c->trivial.d() : cur + (size_t)sg.id * per;
    g.n[k][t] = sg.n;
    g.rev[k][t] = rev ? 1 : 0;
    std::vector<int> b = sg.id < 0 ? std::vector<int>(sg.n + 1, 1)
                                   : c->msgs[sg.id].bonds;
    if (rev) b = reversed(b);
    bonds.insert(bonds.end(), b.begin() + 1, b.end());
  }
}

// Lattice coordinates of region cell (y, x).
static const double *region_site(const bbp_ctx *c, const RegionSpec &r, int y,
                                 int x) {
  return c->site(r.bi * c->bx + x, r.bj * c->by + y);
}

// The regions' contractions are planned, and their device memory taken,
// before any of them is enqueued; then the boundary stacks of every shape
// run on lanes of their own, each line batch follows on the lane of its
// stacks (its matrix-unit steps and contractions behind it), and the host
// synchronises once at the end.  A shape's column absorptions are a chain of
// dependent launches whose length does not depend on its item count, so
// shapes side by side (the blocks' stacks beside the two-block unions')
// shorten the whole; every transfer in between goes through pinned staging,
// so enqueueing never waits on the device.
static bbp_status compute_regions(bbp_ctx *c, std::vector<RegionSpec> &regs) {
  ++c->obs_call;
  CacheTrim trim{c};  // declared first: runs after every batch has been returned
  hipStream_t st = c->stream;
  hipError_t e = hipMemsetAsync(c->errflag.p, 0, 4, st);
  if (e != hipSuccess) return c->hip_fail(e, "memset");
  c->pin.reset();
  size_t nev = 0;  // dependency events this call has used
  const int Kenv = c->chi_env, P = c->P, d = c->d, d2 = d * d;
  const size_t asite = (size_t)d * P * P;
  const int nl = std::max(1, c->lanes);
  // ---- 1. boundary stacks, batched by rotated shape -----------------------
  std::vector<StackItem> stacks;
  std::vector<std::array<int, 4>> stack_of(regs.size(), {-1, -1, -1, -1});
  for (size_t r = 0; r < regs.size(); ++r) {
    const RegionSpec &R = regs[r];
    std::vector<char> ors;
    if (R.row) ors.insert(ors.end(), {'D', 'U'});
    if (R.col) ors.insert(ors.end(), {'L', 'R'});
    for (char o : ors) {
      StackItem it{(int)r, o, 0, 0};
      if (o == 'D' || o == 'U') {
        it.Wc = R.H;
        it.Hc = R.W;
      } else {
        it.Wc = R.W;
        it.Hc = R.H;
      }
      stack_of[r][dir_index(o)] = (int)stacks.size();
      stacks.push_back(it);
    }
  }
  // Reuse of kept stacks (bond-only contractions with stack_reuse on): a
  // line at canonical column cx reads its stack after the absorption of
  // columns W-1..cx+1, so a kept stack serves while those columns' rotated
  // tensors are unchanged; its boundary messages and fit settings are fixed
  // while stacks are kept.
  bool reuse = c->stack_reuse;
  for (const RegionSpec &R : regs) reuse = reuse && !R.targets.empty();
  std::vector<std::vector<double>> rot(reuse ? stacks.size() : 0);
  std::vector<char> reused(stacks.size(), 0);
  std::vector<int> need_lo(stacks.size(), 1), redo_hi(stacks.size(), -1);
  std::vector<StackRef> where(stacks.size());  // group, item, column scales
  if (reuse)
    for (size_t sidx = 0; sidx < stacks.size(); ++sidx) {
      const StackItem &it = stacks[sidx];
      const RegionSpec &R = regs[it.region];
      std::vector<double> &t = rot[sidx];
      t.assign((size_t)it.Hc * it.Wc * asite, 0.0);
      for (int yc = 0; yc < it.Hc; ++yc)
        for (int xc = 0; xc < it.Wc; ++xc) {
          int y, x;
          canon_to_region(it.orient, R.H, R.W, yc, xc, &y, &x);
          rotate_site(c, region_site(c, R, y, x), it.orient,
                      t.data() + ((size_t)yc * it.Wc + xc) * asite);
        }
      int lo = it.Wc;  // lowest canonical column any of its lines needs absorbed
      for (const Target &tg : R.targets) {
        int cx = -1;
        if (tg.row && it.orient == 'D') cx = R.H - 1 - tg.line;
        if (tg.row && it.orient == 'U') cx = tg.line;
        if (!tg.row && it.orient == 'L') cx = tg.line;
        if (!tg.row && it.orient == 'R') cx = R.W - 1 - tg.line;
        if (cx >= 0) lo = std::min(lo, cx + 1);
      }
      need_lo[sidx] = lo;
      auto kv = c->kept_stacks.find(std::make_tuple(R.kind, R.bi, R.bj, it.orient));
      if (kv == c->kept_stacks.end() || kv->second.cols.size() != t.size()) continue;
      // the first column in absorption order (W-1 first) whose tensors changed
      int c0 = -1;
      for (int xc = it.Wc - 1; xc >= lo && c0 < 0; --xc)
        for (int yc = 0; yc < it.Hc; ++yc) {
          const size_t o = ((size_t)yc * it.Wc + xc) * asite;
          if (std::memcmp(t.data() + o, kv->second.cols.data() + o, asite * 8) != 0) {
            c0 = xc;
            break;
          }
        }
      if (c0 >= 0 && kv->second.g->fb.items != 1) continue;  // recomputed whole
      reused[sidx] = 1;
      redo_hi[sidx] = c0;  // >= 0: columns c0..lo re-absorbed in the kept batch
      where[sidx] = StackRef{kv->second.g, kv->second.item, kv->second.nu.data()};
    }
  std::map<std::pair<int, int>, std::vector<int>> sgroups;
  for (size_t i = 0; i < stacks.size(); ++i)
    if (!reused[i]) sgroups[{stacks[i].Wc, stacks[i].Hc}].push_back((int)i);
  std::vector<std::vector<int>> batches;
  std::vector<int> shape_items;  // items of the shape each batch belongs to
  std::vector<int> batch_lane;
  if (reuse) {  // kept stacks are updated in place, one per batch
    for (auto &kv : sgroups)
      for (int id : kv.second) {
        batches.push_back({id});
        shape_items.push_back(1);
        batch_lane.push_back((int)(batch_lane.size() % nl));
      }
  } else {
    // One lane per shape; lanes left over split the shapes with the longest
    // chains (one part's QRs then run beside another part's visits).  The
    // parts, longest chains first, go to the lane with the least work so
    // far.  A chain's length is its absorbed columns times its fit steps.
    struct Shape {
      const std::vector<int> *ids;
      double cost;
      int parts;
    };
    std::vector<Shape> shapes;
    for (auto &kv : sgroups)
      shapes.push_back(Shape{&kv.second,
                             (double)std::max(1, kv.first.first - 1) * (kv.first.second + 1), 1});
    for (int extra = nl - (int)shapes.size(); extra > 0; --extra) {
      int best = -1;
      for (size_t i = 0; i < shapes.size(); ++i)
        if ((int)shapes[i].ids->size() >= (shapes[i].parts + 1) * kLaneMinItems &&
            (best < 0 ||
             shapes[i].cost / shapes[i].parts > shapes[best].cost / shapes[best].parts))
          best = (int)i;
      if (best < 0) break;
      ++shapes[best].parts;
    }
    std::vector<double> cost;
    for (const Shape &sh : shapes)
      for (auto &part : split_batch(*sh.ids, sh.parts, kLaneMinItems)) {
        batches.push_back(part);
        shape_items.push_back((int)sh.ids->size());
        cost.push_back(sh.cost);
      }
    std::vector<int> order(batches.size());
    for (size_t b = 0; b < order.size(); ++b) order[b] = (int)b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<double> load(nl, 0.0);
    batch_lane.assign(batches.size(), 0);
    for (int b : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      batch_lane[b] = l;
      load[l] += cost[b];
    }
  }
  std::vector<std::unique_ptr<Group>> sg;
  BatchReturn sg_return{c, &sg};
  std::vector<double *> sg_host;  // pinned rotated tensors of every batch
  // allocate and stage every batch first: allocation waits on the context
  // stream, which must not yet hold absorption work
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const std::vector<int> &ids = batches[bi];
    std::unique_ptr<Group> gp =
        take_batch(c, stacks[ids[0]].Wc, stacks[ids[0]].Hc, (int)ids.size());
    Group &g = *gp;
    std::vector<uint64_t> slots(ids.size());
    for (size_t i = 0; i < ids.size(); ++i) {
      const StackItem &it = stacks[ids[i]];
      const RegionSpec &R = regs[it.region];
      slots[i] = region_slot(R.kind, R.bi, R.bj, it.orient);
      where[ids[i]] = StackRef{gp.get(), (int)i, nullptr};
    }
    bbp_status bs = alloc_batch(c, g, (int)ids.size(), Kenv, slots, NEED_FIT | NEED_SCRATCH,
                                true);
    if (bs != BBP_OK) return bs;
    FitBatch &f = g.fb;
    f.tile_items = shape_items[bi];
    // rotated tensors (every site written), gather tables and bond caps
    double *hst = (double *)c->pin.get((size_t)f.items * f.H * f.W * asite * 8);
    if (!hst) return c->fail(BBP_ENOMEM, "pinned host allocation failed");
    g.gs.assign(f.items, GatherSrc{});
    for (int i = 0; i < f.items; ++i) {
      const StackItem &it = stacks[ids[i]];
      const RegionSpec &R = regs[it.region];
      for (int yc = 0; yc < f.H; ++yc)
        for (int xc = 0; xc < f.W; ++xc) {
          int y, x;
          canon_to_region(it.orient, R.H, R.W, yc, xc, &y, &x);
          rotate_site(c, region_site(c, R, y, x), it.orient,
                      hst + (((size_t)i * f.H + yc) * f.W + xc) * asite);
        }
      char side[3];
      int rv[3];
      canon_sources(it.orient, side, rv);
      std::vector<int> bl[3];
      g.gs[i].ksrc = c->K;
      for (int k = 0; k < 3; ++k)
        side_source(c, R.side[side_slot(side[k])], rv[k] != 0, g.gs[i], k, bl[k]);
      std::vector<FitDims> cd;
      column_dims(f.W, f.H, Kenv, P, bl[0], bl[2], bl[1], cd);
      for (int col = 0; col < f.W; ++col) {
        cd[col].rnd = 1;
        g.dims[(size_t)i * f.W + col] = cd[col];
      }
    }
    g.ids = ids;
    sg.push_back(std::move(gp));
    sg_host.push_back(hst);
  }
  // kept stacks whose columns from redo_hi down changed: those columns are
  // re-absorbed in place (their batch holds the earlier columns' results)
  std::vector<int> redo;
  for (size_t sidx = 0; sidx < stacks.size(); ++sidx)
    if (reused[sidx] && redo_hi[sidx] >= 0) redo.push_back((int)sidx);
  // the lane each stack is computed on (-1: kept and unchanged)
  std::vector<int> stack_lane(stacks.size(), -1);
  for (size_t b = 0; b < sg.size(); ++b)
    for (int id : sg[b]->ids) stack_lane[id] = batch_lane[b];
  for (size_t r = 0; r < redo.size(); ++r)
    stack_lane[redo[r]] = (int)((sg.size() + r) % nl);

  // boundary after absorbing canonical columns W-1..col+1 (col = W-1: none)
  auto boundary = [&](int sidx, int col, size_t j) -> const double * {
    const FitBatch &f = where[sidx].g->fb;
    const int i = where[sidx].item;
    if (col == f.W - 1) return f.xin + ((size_t)i * f.N + j) * f.S;
    return f.store + ((size_t)i * f.W * f.N) * f.S + slot_store(f, col + 1, (int)j);
  };
  auto logscale = [&](int sidx, int col) {
    const int W = where[sidx].g->fb.W;
    double t = 0.0;
    for (int cc = col + 1; cc < W; ++cc) t += std::log(where[sidx].nu[cc]);
    return t;
  };

  // ---- 2. lines, batched by length (planned here, enqueued below) ---------
  std::vector<LineItem> lines;
  for (size_t r = 0; r < regs.size(); ++r) {
    const RegionSpec &R = regs[r];
    if (R.row)
      for (int k = 0; k < R.H; ++k) {
        if (!R.wants_line(true, k)) continue;
        lines.push_back(LineItem{(int)r, true, k, stack_of[r][dir_index('D')],
                                 stack_of[r][dir_index('U')], R.H - 1 - k, k, 0.0});
      }
    if (R.col)
      for (int k = 0; k < R.W; ++k) {
        if (!R.wants_line(false, k)) continue;
        lines.push_back(LineItem{(int)r, false, k, stack_of[r][dir_index('L')],
                                 stack_of[r][dir_index('R')], k, R.W - 1 - k, 0.0});
      }
  }
  std::map<int, std::vector<int>> lgroups;
  for (size_t i = 0; i < lines.size(); ++i) {
    const int Hc = stacks[lines[i].xs].Hc;
    lgroups[Hc].push_back((int)i);
  }
  // buffers the enqueued work uses, alive until the final synchronisation
  // and then kept by the context for the next call
  std::deque<DevBuf> keep;
  std::vector<std::unique_ptr<Group>> unit_groups;
  std::vector<DevBuf> outs;
  struct OutReturn {  // device buffers and unit batches back to the context's caches
    bbp_ctx *c;
    std::vector<DevBuf> &o;
    std::deque<DevBuf> &k;
    std::vector<std::unique_ptr<Group>> &u;
    ~OutReturn() {
      for (DevBuf &b : o)
        if (b.p) c->unit_out_cache.emplace_back(c->obs_call, std::move(b));
      for (DevBuf &b : k)
        if (b.p) c->unit_out_cache.emplace_back(c->obs_call, std::move(b));
      for (auto &g : u)
        if (g) {
          g->cache_gen = c->obs_call;
          c->unit_groups.push_back(std::move(g));
        }
    }
  } out_return{c, outs, keep, unit_groups};
  // a device buffer of `bytes` kept until the end of the call (from the
  // context's cache when one of that size is there)
  auto keep_buf = [&](size_t bytes) -> DevBuf * {
    keep.push_back(take_unit_out(c, bytes));
    return keep.back().alloc(bytes) == hipSuccess ? &keep.back() : nullptr;
  };
  std::vector<std::unique_ptr<Group>> lgs;
  BatchReturn lg_return{c, &lgs};
  struct Tag {
    int kind, line, j, u, v;
  };
  struct LinePlan {
    const std::vector<int> *lids = nullptr;
    int Hc = 0, lane = 0, rlane = 0;
    Group *lg = nullptr;
    std::vector<CopyJob> jobs;
    DevBuf *djobs = nullptr;
    double *fresh = nullptr;  // reuse: the lines' current tensors (pinned)
    std::vector<UnitItem> units[2];
    int CH = 0;
    size_t chmax = 0;
    Group *ug = nullptr;
    DevBuf *kets = nullptr, *bras = nullptr, *tabs = nullptr, *ujobs = nullptr;
    double *outp[2] = {nullptr, nullptr};
    std::vector<const double *> pa, pb;
    std::vector<Tag> tags;
    DevBuf *da = nullptr, *db = nullptr, *dout = nullptr;
    double *vals = nullptr;  // pinned
  };
  std::vector<LinePlan> plans;
  plans.reserve(lgroups.size());
  for (auto &kv : lgroups) {
    plans.emplace_back();
    LinePlan &pl = plans.back();
    const int Hc = kv.first;
    const std::vector<int> &lids = kv.second;
    pl.lids = &lids;
    pl.Hc = Hc;
    lgs.push_back(take_batch(c, 1, Hc, (int)lids.size()));
    Group &lg = *lgs.back();
    pl.lg = &lg;
    std::vector<uint64_t> slots(lids.size(), 0);
    bbp_status bs = alloc_batch(c, lg, (int)lids.size(), Kenv, slots, NEED_FIT | NEED_SCRATCH,
                                true);
    if (bs != BBP_OK) return bs;
    FitBatch &f = lg.fb;
    pl.lane = std::max(0, stack_lane[lines[lids[0]].xs]);
    // the left and right environment chains are independent: the right one
    // takes a lane of its own (with a T3 scratch of its own) where the visit
    // is fused (T3 is then the only buffer the two would share; the unfused
    // contractions also stage T1 and T2): another lane of its stacks, which
    // the batch waits for anyway, else, for the only line batch, the next
    // lane; otherwise both keep to the batch's lane
    pl.rlane = pl.lane;
    if (nl >= 2 && visit_fused_fits(f)) {
      for (int li : lids)
        for (int sidx : {lines[li].xs, lines[li].ys})
          if (pl.rlane == pl.lane && stack_lane[sidx] >= 0 && stack_lane[sidx] != pl.lane)
            pl.rlane = stack_lane[sidx];
      if (pl.rlane == pl.lane && lgroups.size() == 1) pl.rlane = (pl.lane + 1) % nl;
    }
    if (pl.rlane != pl.lane &&
        lg.t3r.alloc((size_t)f.items * f.K * f.P * f.P * f.K * 8) != hipSuccess)
      return c->fail(BBP_ENOMEM, "device allocation failed");
    // ---- 3. matrix-unit steps ------------------------------------------
    // needed (line, j, direction): sites and the first site of a bond take
    // a left-to-right step; the second site of a bond a right-to-left step.
    for (size_t li = 0; li < lids.size(); ++li) {
      const LineItem &L = lines[lids[li]];
      const RegionSpec &R = regs[L.region];
      std::vector<int> lr, rl;
      if (!R.targets.empty()) {  // the listed bonds (j, j+1), j = pos + 1
        for (const Target &t : R.targets)
          if (t.row == L.row && t.line == L.k) {
            lr.push_back(t.pos + 1);
            rl.push_back(t.pos + 2);
          }
      } else if (L.row) {
        if (R.kind == 0) {
          for (int j = 1; j <= Hc; ++j) lr.push_back(j);
          for (int j = 2; j <= Hc; ++j) rl.push_back(j);
        } else {  // union: the bond crossing the two blocks
          lr.push_back(c->bx);
          rl.push_back(c->bx + 1);
        }
      } else {
        if (R.kind == 0) {
          for (int j = 1; j < Hc; ++j) lr.push_back(j);
          for (int j = 2; j <= Hc; ++j) rl.push_back(j);
        } else {
          lr.push_back(c->by);
          rl.push_back(c->by + 1);
        }
      }
      for (int j : lr)
        for (int u = 0; u < d2; ++u) pl.units[0].push_back(UnitItem{(int)li, j, u});
      for (int j : rl)
        for (int u = 0; u < d2; ++u) pl.units[1].push_back(UnitItem{(int)li, j, u});
    }
    // units per chunk: 256, fewer where the units' contraction scratch (T1,
    // T2, T3: up to (2 + d) K^2 P^2 doubles a unit) of the line batches,
    // which run side by side, would pass 16 GiB together
    const size_t unit_scratch = 8ull * (2 + d) * Kenv * Kenv * (size_t)P * P;
    pl.CH = (int)std::max<size_t>(
        8, std::min<size_t>(256, (16ull << 30) / lgroups.size() / unit_scratch));
    // chunk buffers, allocated once for the largest chunk and reused (stream
    // order keeps a chunk's uploads behind the previous chunk's kernels)
    const size_t chmax =
        std::min<size_t>(pl.CH, std::max(pl.units[0].size(), pl.units[1].size()));
    pl.chmax = chmax;
    if (chmax > 0) {
      std::unique_ptr<Group> ugp;
      for (auto it = c->unit_groups.begin(); it != c->unit_groups.end(); ++it)
        if ((*it)->fb.items == (int)chmax && (*it)->fb.K == Kenv) {
          ugp = std::move(*it);
          c->unit_groups.erase(it);
          break;
        }
      if (!ugp) ugp.reset(new Group);
      unit_groups.push_back(std::move(ugp));
      pl.ug = unit_groups.back().get();
      pl.ug->W = 1;
      pl.ug->H = 1;
      bbp_status bs2 = alloc_batch(c, *pl.ug, (int)chmax, Kenv,
                                   std::vector<uint64_t>(chmax, 0), NEED_SCRATCH, true);
      if (bs2 != BBP_OK) return bs2;
    }
  }

  // The host tables of a line batch (copy jobs, matrix-unit buffers, the
  // contraction pointers), built while the GPU works on the stacks.
  auto plan_tables = [&](LinePlan &pl) -> bbp_status {
    const std::vector<int> &lids = *pl.lids;
    const int Hc = pl.Hc;
    FitBatch &f = pl.lg->fb;
    const int N = f.N;
    if (reuse) {
      pl.fresh = (double *)c->pin.get(lids.size() * (size_t)Hc * asite * 8);
      if (!pl.fresh) return c->fail(BBP_ENOMEM, "pinned host allocation failed");
    }
    for (size_t li = 0; li < lids.size(); ++li) {
      const LineItem &L = lines[lids[li]];
      const Group &gx = *where[L.xs].g;
      const int ix = where[L.xs].item;
      for (int j = 0; j < N; ++j) {
        pl.jobs.push_back(CopyJob{boundary(L.xs, L.cx, j), f.xin + (li * N + j) * f.S,
                                  (int64_t)f.S, 0, 0});
        const bool endsite = (j == 0 || j == N - 1);
        pl.jobs.push_back(CopyJob{boundary(L.ys, L.cy, N - 1 - j),
                                  f.store + (li * N + j) * f.S, (int64_t)f.S,
                                  endsite ? 2 : 1, 0});
      }
      for (int j = 0; j < Hc; ++j)
        if (reuse)  // a kept stack's tensors may be older than the line's
          std::memcpy(pl.fresh + (li * Hc + j) * asite,
                      rot[L.xs].data() + ((size_t)j * gx.fb.W + L.cx) * asite, asite * 8);
        else
          pl.jobs.push_back(CopyJob{
              gx.fb.acan + (((size_t)ix * gx.fb.H + j) * gx.fb.W + L.cx) * asite,
              f.acan + (li * Hc + j) * asite, (int64_t)asite, 0, 0});
      pl.jobs.push_back(CopyJob{gx.fb.mt + ((size_t)ix * gx.fb.W + L.cx) * gx.fb.S,
                                f.mt + li * f.S, (int64_t)f.S, 0, 0});
      pl.jobs.push_back(CopyJob{gx.fb.mb + ((size_t)ix * gx.fb.W + L.cx) * gx.fb.S,
                                f.mb + li * f.S, (int64_t)f.S, 0, 0});
    }
    if (!(pl.djobs = keep_buf(sizeof(CopyJob) * pl.jobs.size())))
      return c->fail(BBP_ENOMEM, "device allocation failed");
    std::vector<double *> out_ptr[2];
    if (pl.chmax > 0) {
      DevBuf *bufs[4];
      const size_t sizes[4] = {pl.chmax * asite * 8, pl.chmax * asite * 8,
                               pl.chmax * 3 * sizeof(double *), sizeof(CopyJob) * 2 * pl.chmax};
      for (int k = 0; k < 4; ++k)
        if (!(bufs[k] = keep_buf(sizes[k])))
          return c->fail(BBP_ENOMEM, "device allocation failed");
      pl.kets = bufs[0];
      pl.bras = bufs[1];
      pl.tabs = bufs[2];
      pl.ujobs = bufs[3];
    }
    for (int dir = 0; dir < 2; ++dir) {
      const std::vector<UnitItem> &U = pl.units[dir];
      if (U.empty()) continue;
      outs.push_back(take_unit_out(c, U.size() * f.S * 8));
      if (outs.back().alloc(U.size() * f.S * 8) != hipSuccess)
        return c->fail(BBP_ENOMEM, "device allocation failed");
      pl.outp[dir] = outs.back().d();
      out_ptr[dir].resize(U.size());
      for (size_t i = 0; i < U.size(); ++i) out_ptr[dir][i] = pl.outp[dir] + i * f.S;
    }
    // ---- 4. contractions: line values, site and bond density matrices -----
    for (size_t li = 0; li < lids.size(); ++li) {
      pl.pa.push_back(f.lenv + (li * N + 1) * f.S);
      pl.pb.push_back(f.renv + (li * N + 0) * f.S);
      pl.tags.push_back(Tag{0, (int)li, 0, 0, 0});
    }
    std::map<std::tuple<int, int, int>, int> lr_index, rl_index;
    for (size_t i = 0; i < pl.units[0].size(); ++i)
      lr_index[{pl.units[0][i].line, pl.units[0][i].j, pl.units[0][i].u}] = (int)i;
    for (size_t i = 0; i < pl.units[1].size(); ++i)
      rl_index[{pl.units[1][i].line, pl.units[1][i].j, pl.units[1][i].u}] = (int)i;
    for (auto &kv2 : lr_index) {
      const int li = std::get<0>(kv2.first), j = std::get<1>(kv2.first),
                u = std::get<2>(kv2.first);
      // site: <L^u_{j+1}, R_j>
      pl.pa.push_back(out_ptr[0][kv2.second]);
      pl.pb.push_back(f.renv + ((size_t)li * N + j) * f.S);
      pl.tags.push_back(Tag{1, li, j, u, 0});
      // bond (j, j+1): <L^u_{j+1}, R^v_j> with R^v_j the step at site j+1
      for (int v = 0; v < d2; ++v) {
        auto it = rl_index.find({li, j + 1, v});
        if (it == rl_index.end()) continue;
        pl.pa.push_back(out_ptr[0][kv2.second]);
        pl.pb.push_back(out_ptr[1][it->second]);
        pl.tags.push_back(Tag{2, li, j, u, v});
      }
    }
    DevBuf *bufs[3];
    for (int k = 0; k < 3; ++k)
      if (!(bufs[k] = keep_buf(pl.pa.size() * 8)))
        return c->fail(BBP_ENOMEM, "device allocation failed");
    pl.da = bufs[0];
    pl.db = bufs[1];
    pl.dout = bufs[2];
    pl.vals = (double *)c->pin.get(pl.pa.size() * 8);
    if (!pl.vals) return c->fail(BBP_ENOMEM, "pinned host allocation failed");
      return BBP_OK;
  };

  // ---- enqueue: stacks, then each line batch behind its stacks ------------
  LaneFork lanes(c);
  if ((e = lanes.fork(nl)) != hipSuccess) return c->hip_fail(e, "fork lanes");
  // every exit waits for the enqueued work before any buffer it uses goes
  struct Drain {
    LaneFork &l;
    hipStream_t s;
    ~Drain() {
      (void)l.join();
      (void)hipStreamSynchronize(s);
    }
  } drain{lanes, st};
  for (size_t r = 0; r < redo.size(); ++r) {
    const int sidx = redo[r];
    Group &g = *where[sidx].g;
    const hipStream_t sb = lane_stream(c, stack_lane[sidx]);
    e = upload_pinned(c, g.fb.acan, rot[sidx].data(), rot[sidx].size() * 8, sb);
    if (e != hipSuccess) return c->hip_fail(e, "region setup");
    bbp_status bs = absorb_columns(c, g, need_lo[sidx], sb, false, redo_hi[sidx], true);
    if (bs != BBP_OK) return bs;
  }
  std::vector<double *> nu_h(sg.size(), nullptr), redo_nu(redo.size(), nullptr);
  for (size_t b = 0; b < sg.size(); ++b) {
    Group &g = *sg[b];
    FitBatch &f = g.fb;
    const hipStream_t sb = lane_stream(c, batch_lane[b]);
    e = hipMemcpyAsync(f.acan, sg_host[b], (size_t)f.items * f.H * f.W * asite * 8,
                       hipMemcpyHostToDevice, sb);
    if (e == hipSuccess) e = upload_pinned(c, g.gather.p, g.gs.data(),
                                           sizeof(GatherSrc) * f.items, sb);
    if (e == hipSuccess) e = launch_gather(f, (const GatherSrc *)g.gather.p, sb);
    if (e != hipSuccess) return c->hip_fail(e, "region setup");
    nu_h[b] = (double *)c->pin.get((size_t)f.items * f.W * 8);
    if (!nu_h[b]) return c->fail(BBP_ENOMEM, "pinned host allocation failed");
    if (f.W > 1) {
      // with kept stacks only the columns the lines need now: later calls
      // extend a kept stack in place
      bbp_status bs = absorb_columns(c, g, reuse ? std::max(1, need_lo[g.ids[0]]) : 1, sb,
                                     false, -1, true);
      if (bs != BBP_OK) return bs;
      e = hipMemcpyAsync(nu_h[b], f.nu, (size_t)f.items * f.W * 8, hipMemcpyDeviceToHost, sb);
      if (e != hipSuccess) return c->hip_fail(e, "region stacks");
    } else {
      std::fill_n(nu_h[b], (size_t)f.items * f.W, 1.0);
    }
  }
  for (size_t r = 0; r < redo.size(); ++r) {  // the kept entry's new column scales
    const FitBatch &f = where[redo[r]].g->fb;
    redo_nu[r] = (double *)c->pin.get((size_t)f.items * f.W * 8);
    if (!redo_nu[r]) return c->fail(BBP_ENOMEM, "pinned host allocation failed");
    e = hipMemcpyAsync(redo_nu[r], f.nu, (size_t)f.items * f.W * 8, hipMemcpyDeviceToHost,
                       lane_stream(c, stack_lane[redo[r]]));
    if (e != hipSuccess) return c->hip_fail(e, "region stacks");
  }
  for (size_t b = 0; b < sg.size(); ++b)  // column scales of the computed stacks
    for (size_t i = 0; i < sg[b]->ids.size(); ++i)
      where[sg[b]->ids[i]].nu = nu_h[b] + i * sg[b]->fb.W;
  if (reuse) {
    // keep the computed stacks (and their batches) for later calls: their
    // column scales are read now
    if ((e = lanes.join()) != hipSuccess) return c->hip_fail(e, "join lanes");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return c->hip_fail(e, "region stacks");
    for (size_t r = 0; r < redo.size(); ++r) {
      const int sidx = redo[r];
      const RegionSpec &R = regs[stacks[sidx].region];
      bbp_ctx::KeptStack &k =
          c->kept_stacks.at(std::make_tuple(R.kind, R.bi, R.bj, stacks[sidx].orient));
      const FitBatch &f = k.g->fb;
      std::copy(redo_nu[r] + (size_t)k.item * f.W, redo_nu[r] + (size_t)(k.item + 1) * f.W,
                k.nu.begin());
      k.cols = rot[sidx];
      const StackItem &it = stacks[sidx];
      for (int yc = 0; yc < it.Hc; ++yc)  // columns below need_lo: not absorbed now
        for (int xc = 0; xc < need_lo[sidx]; ++xc)
          std::fill_n(k.cols.data() + ((size_t)yc * it.Wc + xc) * asite, asite, std::nan(""));
    }
    for (size_t sidx = 0; sidx < stacks.size(); ++sidx) {
      if (reused[sidx]) continue;
      const RegionSpec &R = regs[stacks[sidx].region];
      const StackRef &w = where[sidx];
      bbp_ctx::KeptStack &k =
          c->kept_stacks[std::make_tuple(R.kind, R.bi, R.bj, stacks[sidx].orient)];
      k = bbp_ctx::KeptStack{w.g, w.item, rot[sidx],
                             std::vector<double>(w.nu, w.nu + w.g->fb.W)};
      const StackItem &it = stacks[sidx];
      for (int yc = 0; yc < it.Hc; ++yc)  // columns below need_lo: not absorbed
        for (int xc = 0; xc < need_lo[sidx]; ++xc)
          std::fill_n(k.cols.data() + ((size_t)yc * it.Wc + xc) * asite, asite, std::nan(""));
      where[sidx].nu = k.nu.data();
    }
    for (auto &gp : sg) c->kept_groups.push_back(std::move(gp));
    sg.clear();
    gc_kept(c);
    if ((e = lanes.fork(nl)) != hipSuccess) return c->hip_fail(e, "fork lanes");
  }

  for (LinePlan &pl : plans) {
    bbp_status tb = plan_tables(pl);
    if (tb != BBP_OK) return tb;
    const std::vector<int> &lids = *pl.lids;
    const int Hc = pl.Hc;
    Group &lg = *pl.lg;
    FitBatch &f = lg.fb;
    const int N = f.N;
    const hipStream_t sl = lane_stream(c, pl.lane);
    // its boundary stacks on other lanes come first
    std::set<int> deps;
    for (int li : lids)
      for (int sidx : {lines[li].xs, lines[li].ys})
        if (stack_lane[sidx] >= 0 && stack_lane[sidx] != pl.lane) deps.insert(stack_lane[sidx]);
    for (int l : deps)
      if ((e = lane_after(c, sl, lane_stream(c, l), nev)) != hipSuccess)
        return c->hip_fail(e, "line dependencies");
    e = upload_pinned(c, pl.djobs->p, pl.jobs.data(), sizeof(CopyJob) * pl.jobs.size(), sl);
    if (e == hipSuccess && reuse)
      e = hipMemcpyAsync(f.acan, pl.fresh, lids.size() * (size_t)Hc * asite * 8,
                         hipMemcpyHostToDevice, sl);
    for (size_t o = 0; e == hipSuccess && o < pl.jobs.size(); o += 60000)
      e = launch_copy_jobs((const CopyJob *)pl.djobs->p + o,
                           (int)std::min<size_t>(60000, pl.jobs.size() - o), Kenv, P, sl);
    if (e != hipSuccess) return c->hip_fail(e, "line setup");
    const size_t sN = (size_t)N * f.S;
    auto Xs = [&](int j) { return Ptr{f.xin + (size_t)j * f.S, sN}; };
    auto Ys = [&](int j) { return Ptr{f.store + (size_t)j * f.S, sN}; };
    auto Le = [&](int j) { return Ptr{f.lenv + (size_t)j * f.S, sN}; };
    auto Re = [&](int j) { return Ptr{f.renv + (size_t)j * f.S, sN}; };
    Ptr MT{f.mt, f.S}, MB{f.mb, f.S};
    if ((e = launch_set_unit(f, Le(0), sl)) != hipSuccess ||
        (e = launch_set_unit(f, Re(N - 1), sl)) != hipSuccess)
      return c->hip_fail(e, "set_unit");
    {
      FitBatch fr = f;
      const hipStream_t sr = lane_stream(c, pl.rlane);
      if (sr != sl) {
        fr.t3 = lg.t3r.d();
        if ((e = lane_after(c, sr, sl, nev)) != hipSuccess) return c->hip_fail(e, "fork lanes");
      }
      for (int j = 0; j < N - 1; ++j) {
        if (j == 0) {
          e = launch_end_chain(f, 0, false, MT, Xs(0), sl);
          if (e == hipSuccess) e = launch_end_env(f, 0, false, Ys(0), Le(1), sl);
        } else {
          e = launch_inner_chain(f, 0, j, false, Xs(j), Le(j), sl);
          if (e == hipSuccess) e = launch_inner_env(f, 0, j, false, Ys(j), Le(j + 1), sl);
        }
        if (e != hipSuccess) return c->hip_fail(e, "line left environments");
      }
      for (int j = N - 1; j >= 1; --j) {
        if (j == N - 1) {
          e = launch_end_chain(fr, 0, true, MB, Xs(N - 1), sr);
          if (e == hipSuccess) e = launch_end_env(fr, 0, true, Ys(N - 1), Re(N - 2), sr);
        } else {
          e = launch_inner_chain(fr, 0, j, true, Xs(j), Re(j), sr);
          if (e == hipSuccess) e = launch_inner_env(fr, 0, j, true, Ys(j), Re(j - 1), sr);
        }
        if (e != hipSuccess) return c->hip_fail(e, "line right environments");
      }
      if (sr != sl && (e = lane_after(c, sl, sr, nev)) != hipSuccess)
        return c->hip_fail(e, "join lanes");
    }
    for (int dir = 0; dir < 2; ++dir) {
      const std::vector<UnitItem> &U = pl.units[dir];
      if (U.empty()) continue;
      for (size_t o = 0; o < U.size(); o += pl.CH) {
        const int n = (int)std::min<size_t>(pl.CH, U.size() - o);
        FitBatch &fu = pl.ug->fb;
        fu.items = n;
        e = hipMemsetAsync(pl.kets->p, 0, (size_t)n * asite * 8, sl);
        CopyJob *uj = (CopyJob *)c->pin.get(sizeof(CopyJob) * 2 * n);
        double **tab = (double **)c->pin.get(sizeof(double *) * 3 * n);
        if (!uj || !tab) return c->fail(BBP_ENOMEM, "pinned host allocation failed");
        const size_t slice = asite / d;
        for (int i = 0; i < n; ++i) {
          const UnitItem &ui = U[o + i];
          const double *A = f.acan + ((size_t)ui.line * Hc + (ui.j - 1)) * asite;
          const int sp = ui.u / d, s0 = ui.u % d;
          // bra: A; ket: only physical index s' present, equal to A[s]
          uj[2 * i] = CopyJob{A, pl.bras->d() + (size_t)i * asite, (int64_t)asite, 0, 0};
          uj[2 * i + 1] = CopyJob{A + s0 * slice, pl.kets->d() + (size_t)i * asite + sp * slice,
                                  (int64_t)slice, 0, 0};
          tab[i] = f.xin + ((size_t)ui.line * N + ui.j) * f.S;
          tab[n + i] = (dir == 0 ? f.lenv : f.renv) + ((size_t)ui.line * N + ui.j) * f.S;
          tab[2 * n + i] = f.store + ((size_t)ui.line * N + ui.j) * f.S;
        }
        if (e == hipSuccess)
          e = hipMemcpyAsync(pl.ujobs->p, uj, sizeof(CopyJob) * 2 * n, hipMemcpyHostToDevice,
                             sl);
        if (e == hipSuccess)
          e = hipMemcpyAsync(pl.tabs->p, tab, sizeof(double *) * 3 * n, hipMemcpyHostToDevice,
                             sl);
        if (e == hipSuccess)
          e = launch_copy_jobs((const CopyJob *)pl.ujobs->p, 2 * n, Kenv, P, sl);
        if (e != hipSuccess) return c->hip_fail(e, "unit setup");
        fu.acan = pl.kets->d();
        fu.abra = pl.bras->d();
        double *const *tp = (double *const *)pl.tabs->p;
        Ptr X{nullptr, 0, tp}, F{nullptr, 0, tp + n}, Y{nullptr, 0, tp + 2 * n};
        e = launch_inner_chain(fu, 0, 1, dir == 1, X, F, sl);
        if (e == hipSuccess)
          e = launch_inner_env(fu, 0, 1, dir == 1, Y, Ptr{pl.outp[dir] + o * f.S, f.S}, sl);
        if (e != hipSuccess) return c->hip_fail(e, "unit steps");
      }
    }
    e = upload_pinned(c, pl.da->p, pl.pa.data(), pl.pa.size() * 8, sl);
    if (e == hipSuccess) e = upload_pinned(c, pl.db->p, pl.pb.data(), pl.pb.size() * 8, sl);
    if (e == hipSuccess)
      e = launch_dots((int)pl.pa.size(), (const double *const *)pl.da->p,
                      (const double *const *)pl.db->p, f.S, pl.dout->d(), sl);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pl.vals, pl.dout->p, pl.pa.size() * 8, hipMemcpyDeviceToHost, sl);
    if (e != hipSuccess) return c->hip_fail(e, "line contractions");
  }
  if ((e = lanes.join()) != hipSuccess) return c->hip_fail(e, "join lanes");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return c->hip_fail(e, "region contractions");
  int32_t errv = 0;
  e = copy_sync(c, &errv, c->errflag.p, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return c->hip_fail(e, "error flag");
  if (errv) return c->fail(BBP_ENUMERIC, "zero or non-finite boundary norm");
  for (LineItem &L : lines) L.ls = logscale(L.xs, L.cx) + logscale(L.ys, L.cy);
  // results per line
  std::vector<double> lz(lines.size(), 0.0);
  // unit results: (line, j, u) -> LR step value maps keyed in host tables
  std::map<std::tuple<int, int, int>, double> site_rho;        // (line,j,u)
  std::map<std::tuple<int, int, int, int>, double> bond_rho;   // (line,j,u,v)
  for (const LinePlan &pl : plans)
    for (size_t t = 0; t < pl.tags.size(); ++t) {
      const Tag &tg = pl.tags[t];
      const int line = (*pl.lids)[tg.line];
      if (tg.kind == 0) lz[line] = pl.vals[t];
      else if (tg.kind == 1) site_rho[{line, tg.j, tg.u}] = pl.vals[t];
      else bond_rho[{line, tg.j, tg.u, tg.v}] = pl.vals[t];
    }
  // ---- 5. results per region ----------------------------------------------
  const double nan = std::nan("");
  for (size_t r = 0; r < regs.size(); ++r) {
    const RegionSpec &R = regs[r];
    RegionResult &res = c->obs[std::make_tuple(R.kind, R.bi, R.bj)];
    res.H = R.H;
    res.W = R.W;
    if (R.row) {
      res.has_row = true;
      res.zrow.assign(R.H, nan);
      res.lsrow.assign(R.H, nan);
      res.site.assign((size_t)R.H * R.W * d2, nan);
      res.hbond.assign((size_t)R.H * std::max(R.W - 1, 0) * d2 * d2, nan);
    }
    if (R.col) {
      res.has_col = true;
      res.zcol.assign(R.W, nan);
      res.lscol.assign(R.W, nan);
      res.vbond.assign((size_t)R.W * std::max(R.H - 1, 0) * d2 * d2, nan);
    }
  }
  for (size_t li = 0; li < lines.size(); ++li) {
    const LineItem &L = lines[li];
    const RegionSpec &R = regs[L.region];
    RegionResult &res = c->obs[std::make_tuple(R.kind, R.bi, R.bj)];
    if (L.row) {
      res.zrow[L.k] = lz[li];
      res.lsrow[L.k] = L.ls;
    } else {
      res.zcol[L.k] = lz[li];
      res.lscol[L.k] = L.ls;
    }
  }
  for (auto &kv : site_rho) {
    const LineItem &L = lines[std::get<0>(kv.first)];
    const RegionSpec &R = regs[L.region];
    if (!L.row) continue;
    RegionResult &res = c->obs[std::make_tuple(R.kind, R.bi, R.bj)];
    const int x = std::get<1>(kv.first) - 1;
    res.site[((size_t)L.k * R.W + x) * d2 + std::get<2>(kv.first)] = kv.second;
  }
  for (auto &kv : bond_rho) {
    const LineItem &L = lines[std::get<0>(kv.first)];
    const RegionSpec &R = regs[L.region];
    RegionResult &res = c->obs[std::make_tuple(R.kind, R.bi, R.bj)];
    const int p0 = std::get<1>(kv.first) - 1, u = std::get<2>(kv.first),
              v = std::get<3>(kv.first);
    if (L.row)
      res.hbond[(((size_t)L.k * (R.W - 1) + p0) * d2 + u) * d2 + v] = kv.second;
    else
      res.vbond[(((size_t)L.k * (R.H - 1) + p0) * d2 + u) * d2 + v] = kv.second;
  }
  return BBP_OK;
}

// Region-local position of lattice site (x, y): block indices and offsets.
// Infinite lattices use the unit-cell copy nearest the centre of the block.
static void locate(const bbp_ctx *c, int x, int y, int *bi, int *bj, int *lx,
                   int *ly) {
  if (c->infinite) {
    const int ox = (c->bx - c->ucx) / 2, oy = (c->by - c->ucy) / 2;
    x = ox + (((x - ox) % c->ucx) + c->ucx) % c->ucx;
    y = oy + (((y - oy) % c->ucy) + c->ucy) % c->ucy;
  }
  *bi = x / c->bx;
  *bj = y / c->by;
  *lx = x % c->bx;
  *ly = y % c->by;
}

struct Query {
  int kind, bi, bj;
  bool row;   // row frame (sites, horizontal bonds) or column frame
  int line, pos;
  bool bond;
};

static bbp_status make_query(bbp_ctx *c, int x0, int y0, int x1, int y1,
                             bool bond, Query &q) {
  if (!c->infinite) {
    const bool in0 = x0 >= 0 && y0 >= 0 && x0 < c->Lx && y0 < c->Ly;
    const bool in1 = x1 >= 0 && y1 >= 0 && x1 < c->Lx && y1 < c->Ly;
    if (!in0 || (bond && !in1)) return c->fail(BBP_EINVAL, "site outside the lattice");
  }
  int bi, bj, lx, ly;
  if (!c->infinite) {  // lattice coordinates in the shifted partition
    x0 += c->sx;
    y0 += c->sy;
    x1 += c->sx;
    y1 += c->sy;
  }
  locate(c, x0, y0, &bi, &bj, &lx, &ly);
  q.bi = bi;
  q.bj = bj;
  q.bond = bond;
  if (!bond) {
    q.kind = 0;
    q.row = true;
    q.line = ly;
    q.pos = lx;
    return BBP_OK;
  }
  if (x1 == x0 + 1 && y1 == y0) {
    q.row = true;
    q.line = ly;
    if (lx + 1 < c->bx) {
      q.kind = 0;
      q.pos = lx;
    } else {
      q.kind = 1;
      q.pos = c->bx - 1;
    }
  } else if (x1 == x0 && y1 == y0 + 1) {
    q.row = false;
    q.line = lx;
    if (ly + 1 < c->by) {
      q.kind = 0;
      q.pos = ly;
    } else {
      q.kind = 2;
      q.pos = c->by - 1;
    }
  } else {
    return c->fail(BBP_EINVAL, "bond must join (x,y) to (x+1,y) or (x,y+1)");
  }
  return BBP_OK;
}

static bbp_status ensure_regions(bbp_ctx *c, const std::vector<Query> &qs) {
  std::map<std::tuple<int, int, int>, std::pair<bool, bool>> need;
  for (const Query &q : qs) {
    auto key = std::make_tuple(q.kind, q.bi, q.bj);
    auto it = c->obs.find(key);
    const bool have_row = it != c->obs.end() && it->second.has_row;
    const bool have_col = it != c->obs.end() && it->second.has_col;
    auto &n = need[key];
    if (q.row && !have_row) n.first = true;
    if (!q.row && !have_col) n.second = true;
    if (q.kind == 0 && q.row && !have_col) n.second = true;  // whole block
    if (q.kind == 0 && !q.row && !have_row) n.first = true;
  }
  std::vector<RegionSpec> regs;
  for (auto &kv : need) {
    if (!kv.second.first && !kv.second.second) continue;
    RegionSpec r = region_spec(c, std::get<0>(kv.first), std::get<1>(kv.first),
                               std::get<2>(kv.first));
    r.row = kv.second.first;
    r.col = kv.second.second;
    regs.push_back(r);
    c->obs.erase(kv.first);
  }
  if (regs.empty()) return BBP_OK;
  return compute_regions(c, regs);
}

static bbp_status answer(bbp_ctx *c, const Query &q, const double *op,
                         double *out) {
  const RegionResult &res = c->obs.at(std::make_tuple(q.kind, q.bi, q.bj));
  const int d = c->d, d2 = d * d;
  double num = 0.0, den = 0.0;
  if (!q.bond) {
    const double *rho = &res.site[((size_t)q.line * res.W + q.pos) * d2];
    for (int sp = 0; sp < d; ++sp)
      for (int s = 0; s < d; ++s) num += op[sp * d + s] * rho[sp * d + s];
    for (int s = 0; s < d; ++s) den += rho[s * d + s];
  } else {
    const double *rho =
        q.row ? &res.hbond[((size_t)q.line * (res.W - 1) + q.pos) * d2 * d2]
              : &res.vbond[((size_t)q.line * (res.H - 1) + q.pos) * d2 * d2];
    for (int s0p = 0; s0p < d; ++s0p)
      for (int s1p = 0; s1p < d; ++s1p)
        for (int s0 = 0; s0 < d; ++s0)
          for (int s1 = 0; s1 < d; ++s1) {
            const double o = op[(s0p * d + s1p) * d2 + s0 * d + s1];
            num += o * rho[(s0p * d + s0) * d2 + s1p * d + s1];
          }
    for (int s0 = 0; s0 < d; ++s0)
      for (int s1 = 0; s1 < d; ++s1) den += rho[(s0 * d + s0) * d2 + s1 * d + s1];
  }
  if (!std::isfinite(num) || !std::isfinite(den) || den == 0.0)
    return c->fail(BBP_ENUMERIC, "vanishing or non-finite region contraction");
  *out = num / den;
  return BBP_OK;
}

// Block grid and directed messages of the (shifted) partition.
static void partition(bbp_ctx *c) {
  if (c->infinite) {
    c->gx = c->gy = 1;
  } else {
    c->gx = (c->Lx + c->sx + c->bx - 1) / c->bx;
    c->gy = (c->Ly + c->sy + c->by - 1) / c->by;
  }
  c->msgs.clear();
  for (int bj = 0; bj < c->gy; ++bj)
    for (int bi = 0; bi < c->gx; ++bi)
      for (char dr : kDirs) {
        int ni, nj;
        if (c->neighbour(bi, bj, dr, &ni, &nj)) {
          Message m{bi, bj, dr, (dr == 'L' || dr == 'R') ? c->by : c->bx, {}};
          m.bonds.assign(m.n + 1, 1);
          c->msgs.push_back(m);
        }
      }
}

// Normalised reduced density matrices of n sites (d x d) or bonds
// (d^2 x d^2), rho[a][b] with <O> = Tr(rho O), from the same region
// contractions as the expectation values.
static bbp_status rdm_many(bbp_ctx *c, int n, const int32_t *x0, const int32_t *y0,
                           const int32_t *x1, const int32_t *y1, bool bond, double *out) {
  if (!c) return BBP_EINVAL;
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  if (n < 0 || (n > 0 && (!x0 || !y0 || !out || (bond && (!x1 || !y1)))))
    return c->fail(BBP_EINVAL, "null argument");
  if (c->chi_env < c->chi) return c->fail(BBP_EINVAL, "chi_env must be at least chi");
  std::vector<Query> qs(n);
  for (int i = 0; i < n; ++i) {
    bbp_status s = make_query(c, x0[i], y0[i], bond ? x1[i] : 0, bond ? y1[i] : 0, bond, qs[i]);
    if (s != BBP_OK) return s;
  }
  bbp_status s = ensure_regions(c, qs);
  if (s != BBP_OK) return s;
  const int d = c->d, d2 = d * d, m = bond ? d2 : d;
  for (int i = 0; i < n; ++i) {
    const Query &q = qs[i];
    const RegionResult &res = c->obs.at(std::make_tuple(q.kind, q.bi, q.bj));
    double *rho = out + (size_t)i * m * m;
    double den = 0.0;
    if (!q.bond) {
      // unit (s', s) at s' d + s is the expectation of |s'><s|: rho[s][s']
      const double *u = &res.site[((size_t)q.line * res.W + q.pos) * d2];
      for (int s0 = 0; s0 < d; ++s0) den += u[s0 * d + s0];
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) rho[a * d + b] = u[b * d + a];
    } else {
      const double *u = q.row ? &res.hbond[((size_t)q.line * (res.W - 1) + q.pos) * d2 * d2]
                              : &res.vbond[((size_t)q.line * (res.H - 1) + q.pos) * d2 * d2];
      for (int s0 = 0; s0 < d; ++s0)
        for (int s1 = 0; s1 < d; ++s1) den += u[(s0 * d + s0) * d2 + s1 * d + s1];
      // unit ((s0',s1'),(s0,s1)) at (s0' d + s0) d^2 + s1' d + s1
      for (int s0 = 0; s0 < d; ++s0)
        for (int s1 = 0; s1 < d; ++s1)
          for (int s0p = 0; s0p < d; ++s0p)
            for (int s1p = 0; s1p < d; ++s1p)
              rho[(s0 * d + s1) * d2 + s0p * d + s1p] =
                  u[(s0p * d + s0) * d2 + s1p * d + s1];
    }
    if (!std::isfinite(den) || den == 0.0)
      return c->fail(BBP_ENUMERIC, "vanishing or non-finite region contraction");
    for (int k = 0; k < m * m; ++k) rho[k] /= den;
  }
  return BBP_OK;
}

// Two-site reduced density matrices of n bonds computed on their own: the
// region of each bond contracted in the bond's frame only (two boundary
// stacks), its line only, and the matrix-unit steps of its two sites only.
// The partial region results are dropped afterwards, so that later queries
// recompute whole regions.
static bbp_status rdm_bonds_only(bbp_ctx *c, int n, const int32_t *x0, const int32_t *y0,
                                 const int32_t *x1, const int32_t *y1, double *out) {
  if (!c) return BBP_EINVAL;
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  if (n < 0 || (n > 0 && (!x0 || !y0 || !x1 || !y1 || !out)))
    return c->fail(BBP_EINVAL, "null argument");
  if (c->chi_env < c->chi) return c->fail(BBP_EINVAL, "chi_env must be at least chi");
  std::vector<Query> qs(n);
  std::map<std::tuple<int, int, int>, RegionSpec> want;
  for (int i = 0; i < n; ++i) {
    bbp_status s = make_query(c, x0[i], y0[i], x1[i], y1[i], true, qs[i]);
    if (s != BBP_OK) return s;
    const Query &q = qs[i];
    auto key = std::make_tuple(q.kind, q.bi, q.bj);
    auto it = want.find(key);
    if (it == want.end()) {
      RegionSpec r = region_spec(c, q.kind, q.bi, q.bj);
      r.row = r.col = false;
      it = want.emplace(key, r).first;
    }
    (q.row ? it->second.row : it->second.col) = true;
    it->second.targets.push_back(Target{q.row, q.line, q.pos});
  }
  std::vector<RegionSpec> regs;
  for (auto &kv : want) {
    c->obs.erase(kv.first);
    regs.push_back(kv.second);
  }
  struct Drop {  // partial results never serve a later query
    bbp_ctx *c;
    const std::map<std::tuple<int, int, int>, RegionSpec> &w;
    ~Drop() {
      for (auto &kv : w) c->obs.erase(kv.first);
    }
  } drop{c, want};
  if (!regs.empty()) {
    bbp_status s = compute_regions(c, regs);
    if (s != BBP_OK) return s;
  }
  const int d = c->d, d2 = d * d;
  for (int i = 0; i < n; ++i) {
    const Query &q = qs[i];
    const RegionResult &res = c->obs.at(std::make_tuple(q.kind, q.bi, q.bj));
    const double *u = q.row ? &res.hbond[((size_t)q.line * (res.W - 1) + q.pos) * d2 * d2]
                            : &res.vbond[((size_t)q.line * (res.H - 1) + q.pos) * d2 * d2];
    double *rho = out + (size_t)i * d2 * d2;
    double den = 0.0;
    for (int s0 = 0; s0 < d; ++s0)
      for (int s1 = 0; s1 < d; ++s1) den += u[(s0 * d + s0) * d2 + s1 * d + s1];
    for (int s0 = 0; s0 < d; ++s0)
      for (int s1 = 0; s1 < d; ++s1)
        for (int s0p = 0; s0p < d; ++s0p)
          for (int s1p = 0; s1p < d; ++s1p)
            rho[(s0 * d + s1) * d2 + s0p * d + s1p] = u[(s0p * d + s0) * d2 + s1p * d + s1];
    if (!std::isfinite(den) || den == 0.0)
      return c->fail(BBP_ENUMERIC, "vanishing or non-finite region contraction");
    for (int k = 0; k < d2 * d2; ++k) rho[k] /= den;
  }
  return BBP_OK;
}

// Queries of n sites (bond false) or bonds, checked, appended to qs.
static bool null_args(int n, const int32_t *x0, const int32_t *y0, const int32_t *x1,
                      const int32_t *y1, bool bond, const double *op, const double *out) {
  return n < 0 || (n > 0 && (!x0 || !y0 || !op || !out || (bond && (!x1 || !y1))));
}
static bbp_status expect_queries(bbp_ctx *c, int n, const int32_t *x0, const int32_t *y0,
                                 const int32_t *x1, const int32_t *y1, bool bond,
                                 const double *op, std::vector<Query> &qs) {
  const int m = bond ? c->d * c->d : c->d;
  for (int i = 0; n > 0 && i < m * m; ++i)
    if (!std::isfinite(op[i])) return c->fail(BBP_EINVAL, "non-finite operator");
  for (int i = 0; i < n; ++i) {
    Query q;
    bbp_status s = make_query(c, x0[i], y0[i], bond ? x1[i] : 0, bond ? y1[i] : 0, bond, q);
    if (s != BBP_OK) return s;
    qs.push_back(q);
  }
  return BBP_OK;
}

// ns sites with op_site, then nb bonds with op_bond, from one contraction of
// every region they need.
static bbp_status expect_terms(bbp_ctx *c, int ns, const int32_t *xs, const int32_t *ys,
                               const double *op_site, int nb, const int32_t *x0,
                               const int32_t *y0, const int32_t *x1, const int32_t *y1,
                               const double *op_bond, double *out_sites, double *out_bonds) {
  if (!c) return BBP_EINVAL;
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  if (null_args(ns, xs, ys, nullptr, nullptr, false, op_site, out_sites) ||
      null_args(nb, x0, y0, x1, y1, true, op_bond, out_bonds))
    return c->fail(BBP_EINVAL, "null argument");
  if (c->chi_env < c->chi)
    return c->fail(BBP_EINVAL, "chi_env must be at least chi");
  std::vector<Query> qs;
  bbp_status s = expect_queries(c, ns, xs, ys, nullptr, nullptr, false, op_site, qs);
  if (s == BBP_OK) s = expect_queries(c, nb, x0, y0, x1, y1, true, op_bond, qs);
  if (s == BBP_OK) s = ensure_regions(c, qs);
  if (s != BBP_OK) return s;
  for (int i = 0; i < ns + nb; ++i)
    if ((s = answer(c, qs[i], i < ns ? op_site : op_bond,
                    i < ns ? &out_sites[i] : &out_bonds[i - ns])) != BBP_OK)
      return s;
  return BBP_OK;
}

static bbp_status expect_many(bbp_ctx *c, int n, const int32_t *x0,
                              const int32_t *y0, const int32_t *x1,
                              const int32_t *y1, bool bond, const double *op,
                              double *out) {
  return bond ? expect_terms(c, 0, nullptr, nullptr, nullptr, n, x0, y0, x1, y1, op, nullptr, out)
              : expect_terms(c, n, x0, y0, op, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                             out, nullptr);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

bbp_status bbp_create(bbp_ctx **out, int32_t infinite, int32_t Lx, int32_t Ly,
                      int32_t ucx, int32_t ucy, int32_t bx, int32_t by,
                      int32_t D, int32_t chi) {
  if (!out) return BBP_EINVAL;
  *out = nullptr;
  if (bx <= 0 || by <= 0 || D <= 0 || chi <= 0) return BBP_EINVAL;
  if (bx + 2 > NMAX || by + 2 > NMAX || 2 * bx + 2 > NMAX || 2 * by + 2 > NMAX)
    return BBP_EINVAL;
  if (chi > 128) return BBP_EINVAL;
  if (infinite) {
    if (ucx <= 0 || ucy <= 0 || bx % ucx || by % ucy) return BBP_EINVAL;
  } else if (Lx <= 0 || Ly <= 0) {
    return BBP_EINVAL;
  }
  bbp_ctx *c = new (std::nothrow) bbp_ctx;
  if (!c) return BBP_ENOMEM;
  c->mem.evict = evict_caches;
  c->mem.evict_user = c;
  static std::atomic<uint64_t> next_serial{1};
  c->serial = next_serial++;
  c->infinite = infinite ? 1 : 0;
  c->Lx = infinite ? 0 : Lx;
  c->Ly = infinite ? 0 : Ly;
  c->ucx = infinite ? ucx : Lx;
  c->ucy = infinite ? ucy : Ly;
  c->bx = bx;
  c->by = by;
  c->D = D;
  c->chi = chi;
  partition(c);
  *out = c;
  return BBP_OK;
}

bbp_status bbp_set_option(bbp_ctx *c, const char *key, double v) {
  if (!c || !key) return BBP_EINVAL;
  std::string k(key);
  const bool late_ok = (k == "n_fit" || k == "chi_env" || k == "timing" || k == "precision" ||
                        k == "graphs" || k == "skip_padding" || k == "hbm_budget");
  if (c->tensors_set && !late_ok)
    return c->fail(BBP_ESTATE, "option must be set before bbp_set_tensors");
  if (!std::isfinite(v)) return c->fail(BBP_EINVAL, "non-finite option value");
  if (k == "d") {
    if (v < 1 || v > 8 || v != std::floor(v)) return c->fail(BBP_EINVAL, "d");
    c->d = (int)v;
  } else if (k == "chi_env") {
    if (v < 1 || v > 128 || v != std::floor(v))
      return c->fail(BBP_EINVAL, "chi_env must be an integer in [1,128]");
    c->chi_env = (int)v;
    c->obs.clear();
    release_kept(c);
  } else if (k == "n_fit") {
    if (v < 1 || v > 64 || v != std::floor(v))
      return c->fail(BBP_EINVAL, "n_fit must be an integer in [1,64]");
    c->n_fit = (int)v;
    c->obs.clear();
    release_kept(c);
  } else if (k == "timing") {
    bbp::timing_enable(v != 0.0);
    bbp::timing_reset();
  } else if (k == "precision") {
    if (v != 64 && v != 32 && v != 16)
      return c->fail(BBP_EINVAL, "precision must be 64, 32 or 16");
    c->precision = (int)v;
    for (auto &g : c->groups) g->fb.prec = c->precision;
    c->obs.clear();
    release_kept(c);
  } else if (k == "graphs") {
    if (v != 0 && v != 1) return c->fail(BBP_EINVAL, "graphs must be 0 or 1");
    c->graphs = (int)v;
  } else if (k == "single_layer") {
    if (v != 0 && v != 1) return c->fail(BBP_EINVAL, "single_layer must be 0 or 1");
    c->single_layer = (int)v;
  } else if (k == "shift_x" || k == "shift_y") {
    const int b = k == "shift_x" ? c->bx : c->by;
    if (c->infinite) return c->fail(BBP_EINVAL, "partition shifts are for finite lattices");
    if (v < 0 || v >= b || v != std::floor(v))
      return c->fail(BBP_EINVAL, "a partition shift must be an integer in [0, block size)");
    (k == "shift_x" ? c->sx : c->sy) = (int)v;
    partition(c);
  } else if (k == "message_split") {
    if (v < 0 || v > 4 || v != std::floor(v))
      return c->fail(BBP_EINVAL, "message_split must be an integer in [0,4]");
    c->msg_split = (int)v;
  } else if (k == "skip_padding") {
    if (v != 0 && v != 1) return c->fail(BBP_EINVAL, "skip_padding must be 0 or 1");
    c->skip_pad = (int)v;
  } else if (k == "lanes") {
    if (v < 1 || v > 4 || v != std::floor(v))
      return c->fail(BBP_EINVAL, "lanes must be an integer in [1,4]");
    c->lanes = (int)v;
  } else if (k == "seed") {
    if (v < 0 || v != std::floor(v) || v > 9007199254740992.0)
      return c->fail(BBP_EINVAL, "seed must be a non-negative integer");
    c->seed = (uint64_t)v;
  } else if (k == "init") {
    if (v != 0 && v != 1) return c->fail(BBP_EINVAL, "init must be 0 or 1");
    c->init = (int)v;
  } else if (k == "hbm_budget") {
    if (v < 0 || v != std::floor(v) || v > 1e18)
      return c->fail(BBP_EINVAL, "hbm_budget must be a non-negative integer (bytes)");
    c->mem.budget = (size_t)v;
  } else {
    return c->fail(BBP_EINVAL, "unknown option " + k);
  }
  return BBP_OK;
}

bbp_status bbp_set_stream(bbp_ctx *c, void *s) {
  if (!c) return BBP_EINVAL;
  c->stream = (hipStream_t)s;
  return BBP_OK;
}

bbp_status bbp_set_allocator(bbp_ctx *c, bbp_alloc_fn alloc, bbp_free_fn free_, void *user) {
  if (!c) return BBP_EINVAL;
  if ((alloc == nullptr) != (free_ == nullptr))
    return c->fail(BBP_EINVAL, "allocator needs both functions, or neither");
  if (c->device_ready)
    return c->fail(BBP_ESTATE, "allocator must be set before bbp_set_tensors");
  c->mem.alloc_fn = alloc;
  c->mem.free_fn = free_;
  c->mem.user = user;
  c->mem.stream = &c->stream;
  return BBP_OK;
}

// Canonical (W, H) of a message's fit: columns absorbed and sites per column.
static std::pair<int, int> message_shape(const bbp_ctx *c, const Message &m) {
  const bool lr = m.dir == 'L' || m.dir == 'R';
  return {lr ? c->bx : c->by, lr ? c->by : c->bx};
}

bbp_status bbp_get_tensors(bbp_ctx *c, double *A, size_t n) {
  if (!c || !A) return BBP_EINVAL;
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  if (n != c->A.size()) return c->fail(BBP_EINVAL, "tensor size does not match the lattice");
  std::copy(c->A.begin(), c->A.end(), A);
  return BBP_OK;
}

bbp_status bbp_set_tensors(bbp_ctx *c, const double *A, size_t n) {
  if (!c || !A) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  const int D = c->D, d = c->d;
  const size_t ss = (size_t)d * D * D * D * D;
  const size_t nsites = (size_t)c->ucx * c->ucy;
  if (n != nsites * ss)
    return c->fail(BBP_EINVAL, "tensor size does not match the lattice");
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(A[i])) return c->fail(BBP_EINVAL, "non-finite tensor entry");
  if (!c->infinite) {
    for (int y = 0; y < c->Ly; ++y)
      for (int x = 0; x < c->Lx; ++x) {
        const double *t = A + (size_t)(y * c->Lx + x) * ss;
        for (int s = 0; s < d; ++s)
          for (int u = 0; u < D; ++u)
            for (int l = 0; l < D; ++l)
              for (int dd = 0; dd < D; ++dd)
                for (int r = 0; r < D; ++r) {
                  bool pad = (y == 0 && u > 0) || (x == 0 && l > 0) ||
                             (y == c->Ly - 1 && dd > 0) ||
                             (x == c->Lx - 1 && r > 0);
                  double v = t[((((size_t)s * D + u) * D + l) * D + dd) * D + r];
                  if (pad && v != 0.0)
                    return c->fail(BBP_EINVAL,
                                   "nonzero entry on an open-edge leg index > 0");
                }
      }
  }
  bbp_status s = ensure_device(c);
  if (s != BBP_OK) return s;
  c->A.assign(A, A + n);
  c->P = D * D;
  c->K = c->chi;
  c->S = (size_t)c->K * c->P * c->K;
  c->Lmax = std::max(c->bx, c->by);
  if (c->chi_env < 0) c->chi_env = std::min(128, 2 * D * D + 10);
  const size_t per = (size_t)c->Lmax * c->S;
  const size_t nm = std::max<size_t>(c->msgs.size(), 1);
  if (c->msgbuf[0].alloc(per * nm * 8) != hipSuccess ||
      c->msgbuf[1].alloc(per * nm * 8) != hipSuccess ||
      c->trivial.alloc(per * 8) != hipSuccess ||
      c->ovE.alloc(nm * c->K * c->K * 8) != hipSuccess ||
      c->ovU.alloc(nm * c->S * 8) != hipSuccess ||
      c->ovOut.alloc(nm * 8) != hipSuccess || c->ovA.alloc(nm * 8) != hipSuccess ||
      c->ovB.alloc(nm * 8) != hipSuccess || c->errflag.alloc(64) != hipSuccess)
    return c->fail(BBP_ENOMEM, "device allocation failed");
  if (c->single_layer) {
    const size_t ss1 = (size_t)c->d * c->P * c->P;
    std::vector<double> dl(ss1, 0.0);
    for (int s1 = 0; s1 < c->d; ++s1) dl[(size_t)s1 * c->P * c->P] = 1.0;
    if (c->delta.alloc(ss1 * 8) != hipSuccess)
      return c->fail(BBP_ENOMEM, "device allocation failed");
    if (copy_sync(c, c->delta.p, dl.data(), ss1 * 8, hipMemcpyHostToDevice) != hipSuccess)
      return c->fail(BBP_EDEVICE, "upload single-layer bra");
  }
  if (zero_sync(c, c->errflag.p, c->errflag.bytes) != hipSuccess ||
      zero_sync(c, c->msgbuf[0].p, c->msgbuf[0].bytes) != hipSuccess ||
      zero_sync(c, c->msgbuf[1].p, c->msgbuf[1].bytes) != hipSuccess)
    return c->fail(BBP_EDEVICE, "clear message buffers");
  {
    std::vector<double> triv(per, 0.0);
    for (int s2 = 0; s2 < c->Lmax; ++s2) triv[(size_t)s2 * c->S] = 1.0;
    if (copy_sync(c, c->trivial.p, triv.data(), per * 8, hipMemcpyHostToDevice) !=
        hipSuccess)
      return c->fail(BBP_EDEVICE, "upload trivial message");
  }
  c->cur = 0;
  // groups by canonical (W, H), each split into message_split parts of at
  // least kLaneMinItems messages, one per lane in turn: one part's QR and
  // environment updates, which hold few CUs, then overlap the other part's
  // visits (16x16 D=4 chi=32: 8 sweeps 107 -> 102 ms with two parts; three
  // parts gain nothing more); message_split 0: one group per message (the
  // kernels stay those of the whole shape, so results are the same bits);
  // the groups of an earlier call are kept (with their device buffers) when
  // the partition is the same
  std::vector<std::unique_ptr<Group>> groups;
  std::vector<int> shape_items;  // items of the shape each group belongs to
  if (c->engine) {  // the shared batches copy each message's rotated block from here
    const size_t ssite = (size_t)c->d * c->P * c->P;
    std::vector<double> host;
    c->rot_off.assign(c->msgs.size(), 0);
    for (size_t i = 0; i < c->msgs.size(); ++i) {
      const Message &m = c->msgs[i];
      const auto sh = message_shape(c, m);
      c->rot_off[i] = host.size();
      host.resize(host.size() + (size_t)sh.first * sh.second * ssite);
      for (int yc = 0; yc < sh.second; ++yc)
        for (int xc = 0; xc < sh.first; ++xc) {
          int y, x;
          canon_to_region(m.dir, c->by, c->bx, yc, xc, &y, &x);
          rotate_site(c, c->site(m.bi * c->bx + x, m.bj * c->by + y), m.dir,
                      host.data() + c->rot_off[i] + ((size_t)yc * sh.first + xc) * ssite);
        }
    }
    if (c->rot.alloc(std::max<size_t>(host.size(), 1) * 8) != hipSuccess)
      return c->fail(BBP_ENOMEM, "device allocation failed");
    if (!host.empty() &&
        copy_sync(c, c->rot.p, host.data(), host.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return c->fail(BBP_EDEVICE, "upload rotated tensors");
  } else {
    std::map<std::pair<int, int>, std::vector<int>> by_shape;
    for (size_t i = 0; i < c->msgs.size(); ++i)
      by_shape[message_shape(c, c->msgs[i])].push_back((int)i);
    for (auto &kv : by_shape)
      for (auto &part : c->msg_split == 0
                            ? split_batch(kv.second, (int)kv.second.size(), 1)
                            : split_batch(kv.second, c->msg_split, kLaneMinItems)) {
        groups.emplace_back(new Group);
        groups.back()->W = kv.first.first;
        groups.back()->H = kv.first.second;
        groups.back()->ids = part;
        shape_items.push_back((int)kv.second.size());
      }
  }
  bool same = groups.size() == c->groups.size();
  for (size_t i = 0; same && i < groups.size(); ++i)
    same = groups[i]->W == c->groups[i]->W && groups[i]->H == c->groups[i]->H &&
           groups[i]->ids == c->groups[i]->ids;
  if (!same) c->groups.swap(groups);
  for (auto &g : c->groups) {
    // random-state slot bases: message e, column c -> (1<<40)|(e<<8)|c
    std::vector<uint64_t> slots(g->ids.size());
    for (size_t i = 0; i < slots.size(); ++i)
      slots[i] = (1ull << 40) | ((uint64_t)g->ids[i] << 8);
    if ((s = alloc_batch(c, *g, (int)g->ids.size(), c->K, slots)) != BBP_OK)
      return s;
    g->fb.tile_items = shape_items[&g - &c->groups[0]];
    if ((s = upload_rotated(c, *g)) != BBP_OK) return s;
  }
  if ((s = init_messages(c)) != BBP_OK) return s;
  c->obs.clear();
  release_kept(c);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hip_fail(e, "set_tensors");
  c->tensors_set = true;
  c->sweeps_done = 0;
  return BBP_OK;
}

// One JSON line per sweep, appended to the file the environment variable
// BBP_SWEEP_LOG names (nothing when it is unset or empty).
static void log_sweep(const bbp_ctx *c, double r, double ms) {
  const char *path = std::getenv("BBP_SWEEP_LOG");
  if (!path || !*path) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"ctx\": %llu, \"sweep\": %lld, \"residual\": %.17g, \"ms\": %.6f, "
               "\"fit_flops\": %.17g, \"messages\": %zu}\n",
               (unsigned long long)c->serial, (long long)c->sweeps_done, r, ms, c->last_flops,
               c->msgs.size());
  std::fclose(f);
}

bbp_status bbp_sweep(bbp_ctx *c, int32_t n, double *residual) {
  if (!c) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  if (c->engine) return c->fail(BBP_ESTATE, "this context is swept by a shared sweep set");
  if (n < 0) return c->fail(BBP_EINVAL, "negative sweep count");
  double r = 0.0;
  for (int i = 0; i < n; ++i) {
    const auto t0 = std::chrono::steady_clock::now();
    bbp_status s = run_sweep(c, &r);
    if (s != BBP_OK) return s;
    ++c->sweeps_done;
    log_sweep(c, r, std::chrono::duration<double, std::milli>(
                        std::chrono::steady_clock::now() - t0).count());
  }
  if (residual) *residual = r;
  return BBP_OK;
}

bbp_status bbp_get_messages(bbp_ctx *c, double *buf, size_t n, size_t *needed) {
  if (!c) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  const size_t per = (size_t)c->Lmax * c->S;
  size_t total = 0;
  for (const Message &m : c->msgs) {
    total += 1 + m.n + 1;
    for (int s = 0; s < m.n; ++s)
      total += (size_t)m.bonds[s] * c->P * m.bonds[s + 1];
  }
  if (needed) *needed = total;
  if (!buf) return BBP_OK;
  if (n < total) return c->fail(BBP_EINVAL, "buffer too small");
  std::vector<double> host(per * c->msgs.size());
  hipError_t e = copy_sync(c, host.data(), c->msgbuf[c->cur].p, host.size() * 8,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return c->hip_fail(e, "download messages");
  size_t o = 0;
  for (size_t i = 0; i < c->msgs.size(); ++i) {
    const Message &m = c->msgs[i];
    buf[o++] = m.n;
    for (int s = 0; s <= m.n; ++s) buf[o++] = m.bonds[s];
    for (int s = 0; s < m.n; ++s) {
      const double *src = host.data() + i * per + (size_t)s * c->S;
      for (int a = 0; a < m.bonds[s]; ++a)
        for (int q = 0; q < c->P; ++q)
          for (int b = 0; b < m.bonds[s + 1]; ++b)
            buf[o++] = src[((size_t)a * c->P + q) * c->K + b];
    }
  }
  return BBP_OK;
}

bbp_status bbp_set_messages(bbp_ctx *c, const double *buf, size_t n) {
  if (!c || !buf) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  const size_t per = (size_t)c->Lmax * c->S;
  std::vector<double> host(per * c->msgs.size(), 0.0);
  std::vector<std::vector<int>> bonds(c->msgs.size());
  size_t o = 0;
  for (size_t i = 0; i < c->msgs.size(); ++i) {
    const Message &m = c->msgs[i];
    if (o + 1 + m.n + 1 > n) return c->fail(BBP_EINVAL, "message buffer too short");
    if ((int)buf[o] != m.n) return c->fail(BBP_EINVAL, "message length mismatch");
    ++o;
    bonds[i].resize(m.n + 1);
    for (int s = 0; s <= m.n; ++s) {
      double v = buf[o++];
      if (v < 1 || v > c->K || v != std::floor(v))
        return c->fail(BBP_EINVAL, "bond dimension out of range");
      bonds[i][s] = (int)v;
    }
    if (bonds[i][0] != 1 || bonds[i][m.n] != 1)
      return c->fail(BBP_EINVAL, "message end bonds must be 1");
    for (int s = 0; s < m.n; ++s) {
      double *dst = host.data() + i * per + (size_t)s * c->S;
      for (int a = 0; a < bonds[i][s]; ++a)
        for (int q = 0; q < c->P; ++q)
          for (int b = 0; b < bonds[i][s + 1]; ++b) {
            if (o >= n) return c->fail(BBP_EINVAL, "message buffer too short");
            double v = buf[o++];
            if (!std::isfinite(v)) return c->fail(BBP_EINVAL, "non-finite message");
            dst[((size_t)a * c->P + q) * c->K + b] = v;
          }
    }
  }
  if (o != n) return c->fail(BBP_EINVAL, "message buffer has trailing data");
  hipError_t e = copy_sync(c, c->msgbuf[c->cur].p, host.data(), host.size() * 8,
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "upload messages");
  for (size_t i = 0; i < c->msgs.size(); ++i) c->msgs[i].bonds = bonds[i];
  for (auto &g : c->groups) std::fill(g->have.begin(), g->have.end(), 0);
  c->obs.clear();
  release_kept(c);
  return BBP_OK;
}

bbp_status bbp_stats(bbp_ctx *c, int32_t *n_messages, double *sweep_flops) {
  if (!c) return BBP_EINVAL;
  if (n_messages) *n_messages = (int32_t)c->msgs.size();
  if (sweep_flops) *sweep_flops = c->last_flops;
  return BBP_OK;
}

bbp_status bbp_expect_site(bbp_ctx *c, int32_t x, int32_t y, const double *op,
                           double *out) {
  if (!c) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  return expect_many(c, 1, &x, &y, nullptr, nullptr, false, op, out);
}

bbp_status bbp_expect_bond(bbp_ctx *c, int32_t x0, int32_t y0, int32_t x1,
                           int32_t y1, const double *op, double *out) {
  if (!c) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  return expect_many(c, 1, &x0, &y0, &x1, &y1, true, op, out);
}

bbp_status bbp_expect_sites(bbp_ctx *c, int32_t n, const int32_t *xs,
                            const int32_t *ys, const double *op, double *out) {
  if (!c) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  return expect_many(c, n, xs, ys, nullptr, nullptr, false, op, out);
}

bbp_status bbp_expect_bonds(bbp_ctx *c, int32_t n, const int32_t *x0,
                            const int32_t *y0, const int32_t *x1,
                            const int32_t *y1, const double *op, double *out) {
  if (!c) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  return expect_many(c, n, x0, y0, x1, y1, true, op, out);
}

bbp_status bbp_expect_terms(bbp_ctx *c, int32_t ns, const int32_t *xs, const int32_t *ys,
                            const double *op_site, int32_t nb, const int32_t *x0,
                            const int32_t *y0, const int32_t *x1, const int32_t *y1,
                            const double *op_bond, double *out_sites, double *out_bonds) {
  if (!c) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  return expect_terms(c, ns, xs, ys, op_site, nb, x0, y0, x1, y1, op_bond, out_sites,
                      out_bonds);
}
bbp_status bbp_rdm_sites(bbp_ctx *c, int32_t n, const int32_t *xs, const int32_t *ys,
                         double *rho) {
  return rdm_many(c, n, xs, ys, nullptr, nullptr, false, rho);
}

bbp_status bbp_rdm_bonds(bbp_ctx *c, int32_t n, const int32_t *x0, const int32_t *y0,
                         const int32_t *x1, const int32_t *y1, double *rho) {
  return rdm_many(c, n, x0, y0, x1, y1, true, rho);
}

bbp_status bbp_trace_distance(int32_t m, const double *rho, const double *sigma,
                              double *out) {
  if (m < 1 || m > 64 || !rho || !sigma || !out) return BBP_EINVAL;
  // Tr|Z| / 2 = half the sum of the singular values of Z = rho - sigma, by
  // one-sided Jacobi rotations of Z's columns (Hestenes): once every column
  // pair is orthogonal, the column norms are the singular values.
  std::vector<double> z((size_t)m * m);
  for (int i = 0; i < m * m; ++i) {
    z[i] = rho[i] - sigma[i];
    if (!std::isfinite(z[i])) return BBP_EINVAL;
  }
  auto col = [&](int r, int cidx) -> double & { return z[(size_t)r * m + cidx]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        double a = 0.0, b = 0.0, g = 0.0;
        for (int r = 0; r < m; ++r) {
          a += col(r, p) * col(r, p);
          b += col(r, q) * col(r, q);
          g += col(r, p) * col(r, q);
        }
        if (g == 0.0 || std::fabs(g) <= 1e-300) continue;
        off = std::max(off, std::fabs(g) / std::sqrt(a * b));
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int r = 0; r < m; ++r) {
          const double u = col(r, p), w = col(r, q);
          col(r, p) = cs * u - sn * w;
          col(r, q) = sn * u + cs * w;
        }
      }
    if (off < 1e-15) break;
  }
  double tr = 0.0;
  for (int cidx = 0; cidx < m; ++cidx) {
    double nrm = 0.0;
    for (int r = 0; r < m; ++r) nrm += col(r, cidx) * col(r, cidx);
    tr += std::sqrt(nrm);
  }
  *out = 0.5 * tr;
  return BBP_OK;
}

bbp_status bbp_log_norm(bbp_ctx *c, double *log_abs, int32_t *sign) {
  if (!c || !log_abs) return BBP_EINVAL;
  AcctScope acct_scope(&c->mem);
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  if (c->chi_env < c->chi)
    return c->fail(BBP_EINVAL, "chi_env must be at least chi");
  // Z_A of every block: line 0 of its row frame
  std::vector<Query> qs;
  for (int bj = 0; bj < c->gy; ++bj)
    for (int bi = 0; bi < c->gx; ++bi)
      qs.push_back(Query{0, bi, bj, true, 0, 0, false});
  bbp_status s = ensure_regions(c, qs);
  if (s != BBP_OK) return s;
  double total = 0.0;
  int sg = 1;
  for (const Query &q : qs) {
    const RegionResult &res = c->obs.at(std::make_tuple(0, q.bi, q.bj));
    const double z = res.zrow[0];
    if (!(std::isfinite(z) && z != 0.0))
      return c->fail(BBP_ENUMERIC, "vanishing block contraction");
    total += std::log(std::fabs(z)) + res.lsrow[0];
    if (z < 0) sg = -sg;
  }
  // Z_AB = <m_{A->B}, m_{B->A}> over edges (messages to the right / down)
  std::vector<int> ea, eb;
  for (size_t i = 0; i < c->msgs.size(); ++i) {
    const Message &m = c->msgs[i];
    if (m.dir != 'R' && m.dir != 'D') continue;
    int ni, nj;
    c->neighbour(m.bi, m.bj, m.dir, &ni, &nj);
    ea.push_back((int)i);
    eb.push_back(c->msg_id(ni, nj, opposite(m.dir)));
  }
  const size_t per = (size_t)c->Lmax * c->S;
  double *cur = c->msgbuf[c->cur].d();
  std::map<int, std::vector<int>> by_len;
  for (size_t t = 0; t < ea.size(); ++t) by_len[c->msgs[ea[t]].n].push_back((int)t);
  for (auto &kv : by_len) {
    std::vector<const double *> pa, pb;
    for (int t : kv.second) {
      pa.push_back(cur + (size_t)ea[t] * per);
      pb.push_back(cur + (size_t)eb[t] * per);
    }
    std::vector<double> ov(pa.size());
    hipError_t e = copy_sync(c, c->ovA.p, pa.data(), 8 * pa.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = copy_sync(c, c->ovB.p, pb.data(), 8 * pb.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = launch_overlap((int)pa.size(), c->K, c->P, kv.first,
                         (const double *const *)c->ovA.p,
                         (const double *const *)c->ovB.p, c->ovE.d(), c->ovU.d(),
                         c->ovOut.d(), c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ov.data(), c->ovOut.p, 8 * ov.size(), hipMemcpyDeviceToHost,
                         c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "edge overlaps");
    for (double z : ov) {
      if (!(std::isfinite(z) && z != 0.0))
        return c->fail(BBP_ENUMERIC, "vanishing edge overlap");
      total -= std::log(std::fabs(z));
      if (z < 0) sg = -sg;
    }
  }
  *log_abs = total;
  if (sign) *sign = sg;
  return BBP_OK;
}

bbp_status bbp_memory(const bbp_ctx *c, size_t *now, size_t *peak) {
  if (!c) return BBP_EINVAL;
  if (now) *now = c->mem.now;
  if (peak) *peak = c->mem.peak;
  return BBP_OK;
}

bbp_status bbp_kernel_stats(bbp_ctx *c, int32_t cls, const char **name,
                            int64_t *launches, double *ms, double *flops,
                            double *bytes) {
  if (!c) return BBP_EINVAL;
  if (cls < 0 || cls >= bbp::KC_COUNT)
    return c->fail(BBP_EINVAL, "kernel class out of range");
  long long n = 0;
  hipError_t e = bbp::timing_query(cls, name, &n, ms, flops, bytes);
  if (e != hipSuccess) return c->hip_fail(e, "kernel timing");
  if (launches) *launches = n;
  return BBP_OK;
}

bbp_status bbp_kernel_stats_padded(bbp_ctx *c, int32_t cls, double *flops,
                                   double *bytes) {
  if (!c) return BBP_EINVAL;
  if (cls < 0 || cls >= bbp::KC_COUNT)
    return c->fail(BBP_EINVAL, "kernel class out of range");
  hipError_t e = bbp::timing_query(cls, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   flops, bytes);
  if (e != hipSuccess) return c->hip_fail(e, "kernel timing");
  return BBP_OK;
}

bbp_status bbp_kernel_stats_reset(bbp_ctx *c) {
  if (!c) return BBP_EINVAL;
  bbp::timing_reset();
  return BBP_OK;
}

const char *bbp_last_error(const bbp_ctx *c) {
  return c ? c->err.c_str() : "null context";
}

void bbp_destroy(bbp_ctx *c) {
  if (!c) return;
  if (c->device_ready) (void)hipStreamSynchronize(c->stream);
  for (hipStream_t s : c->aux) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  for (hipEvent_t ev : c->lane_ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : c->dep_ev) (void)hipEventDestroy(ev);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One directed message update outside a context (Eq. (1); App. A): a block
// of H x W tensors in the canonical frame (the receiver on its left), its
// incoming top, right and bottom messages, column absorptions W-1 .. 0 as
// variational fits, the two dimension-1 end sites contracted into the
// message.  The same batch engine as a sweep, with one item whose buffers
// are carved from one workspace allocated per call.
// ---------------------------------------------------------------------------
namespace {

thread_local std::string tl_update_err;

bbp_status update_fail(bbp_status s, const std::string &m) {
  tl_update_err = m;
  return s;
}

// Workspace of bbp_update_message_noalloc, for callers that cannot
// allocate device memory.  Each GPU holds its own copy until the process
// ends; every call on a GPU shares it, so calls that overlap on one GPU race.
constexpr size_t kUpdateScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kUpdateScratchBytes];

// Device address of `scratch` on the current device, taken once per device
// with that device current (in host code the array's name is a host-side
// stand-in, not a device address).
std::mutex scratch_mu;
std::map<int, void *> scratch_ptr;

hipError_t device_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(scratch_mu);
  auto it = scratch_ptr.find(dev);
  if (it != scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void *ptr = nullptr;
  e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  scratch_ptr[dev] = ptr;
  *out = ptr;
  return hipSuccess;
}

// Byte layout of one update's workspace (256-byte aligned pieces).
struct UpdateLayout {
  size_t store, xin, mt, mb, lenv, renv, t1, t2, t3, tmp, rbuf, nu, triv, err, flag,
      dims, slot, gather, dst, rev, total;
  size_t zero_end;  // [0, zero_end) is cleared before the update
};

UpdateLayout update_layout(const FitBatch &f) {
  UpdateLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) / 256 * 256;
    return at;
  };
  const size_t S = f.S, K = f.K, P = f.P;
  const bool fused = visit_fused_fits(f);
  L.store = take(8 * f.W * f.N * S);
  L.xin = take(8 * f.N * S);
  L.mt = take(8 * f.W * S);
  L.mb = take(8 * f.W * S);
  L.lenv = take(8 * f.N * S);
  L.renv = take(8 * f.N * S);
  L.nu = take(8 * f.W);
  L.err = take(4);
  L.zero_end = off;
  L.triv = take(8 * std::max(f.W, f.H) * S);
  L.t1 = (!fused || qr_needs_scratch(f)) ? take(8 * K * P * P * K) : 0;
  L.t2 = !fused ? take(8 * (size_t)f.d * K * K * P * P) : 0;
  L.t3 = take(8 * K * P * P * K);
  L.tmp = take(8 * S);
  L.rbuf = take(8 * K * K);
  L.flag = take(4 * f.W);
  L.dims = take(sizeof(FitDims) * f.W);
  L.slot = take(8);
  L.gather = take(sizeof(GatherSrc));
  L.dst = take(sizeof(double *));
  L.rev = take(4);
  L.total = off;
  return L;
}

bool valid_bonds(const int32_t *b, int n, int chi, std::vector<int> &out) {
  out.assign(n + 1, 1);
  if (!b) return true;
  if (b[0] != 1 || b[n] != 1) return false;
  for (int i = 0; i <= n; ++i) {
    if (b[i] < 1 || b[i] > chi) return false;
    out[i] = b[i];
  }
  return true;
}

// The batch of one update: shapes from the spec, no buffers yet.
bbp_status update_batch(const bbp_update_spec *sp, FitBatch &f) {
  if (!sp) return update_fail(BBP_EINVAL, "null spec");
  if (sp->H < 1 || sp->W < 1 || sp->H + 2 > NMAX)
    return update_fail(BBP_EINVAL, "H must be in [1, " + std::to_string(NMAX - 2) +
                                       "] and W >= 1");
  if (sp->D < 1 || sp->D > 8 || sp->d < 1 || sp->d > 8)
    return update_fail(BBP_EINVAL, "D and d must be in [1, 8]");
  if (sp->chi < 1 || sp->chi > 128) return update_fail(BBP_EINVAL, "chi must be in [1, 128]");
  if (sp->n_fit < 1 || sp->n_fit > 64) return update_fail(BBP_EINVAL, "n_fit must be in [1, 64]");
  f = FitBatch{};
  f.items = f.tile_items = 1;
  f.K = sp->chi;
  f.D = sp->D;
  f.P = sp->D * sp->D;
  f.d = sp->d;
  f.H = sp->H;
  f.W = sp->W;
  f.N = sp->H + 2;
  f.S = (size_t)f.K * f.P * f.K;
  f.seed = sp->seed;
  f.prec = 64;
  return BBP_OK;
}

// workspace: null to allocate one for the call, else ws_bytes of device
// memory the caller provides (checked against the layout's size).
bbp_status update_message(const bbp_update_spec *sp, const double *A, const double *mt,
                          const int32_t *mt_bonds, const double *mr,
                          const int32_t *mr_bonds, const double *mb,
                          const int32_t *mb_bonds, double *out, int32_t *out_bonds,
                          double *log_scale, void *stream, void *workspace,
                          size_t ws_bytes) {
  FitBatch f;
  bbp_status bs = update_batch(sp, f);
  if (bs != BBP_OK) return bs;
  if (!A || !out || !out_bonds || !log_scale)
    return update_fail(BBP_EINVAL, "null tensor, output, bonds or log-scale pointer");
  std::vector<int> bt, br, bb;
  if (!valid_bonds(mt ? mt_bonds : nullptr, f.W, f.K, bt) ||
      !valid_bonds(mr ? mr_bonds : nullptr, f.H, f.K, br) ||
      !valid_bonds(mb ? mb_bonds : nullptr, f.W, f.K, bb))
    return update_fail(BBP_EINVAL, "message bonds must be 1 at both ends and in [1, chi]");
  if ((mt && !mt_bonds) || (mr && !mr_bonds) || (mb && !mb_bonds))
    return update_fail(BBP_EINVAL, "a message needs its bond list");
  const UpdateLayout L = update_layout(f);
  hipStream_t st = (hipStream_t)stream;
  unsigned char *ws = (unsigned char *)workspace;
  DevBuf owned;
  hipError_t e;
  if (!ws) {
    if ((e = owned.alloc(L.total)) != hipSuccess)
      return update_fail(BBP_ENOMEM, "device allocation failed");
    ws = (unsigned char *)owned.p;
  } else if (L.total > ws_bytes) {
    return update_fail(BBP_EINVAL, "update needs " + std::to_string(L.total) +
                                       " bytes of workspace, " + std::to_string(ws_bytes) +
                                       " given");
  }
  // nothing returns before the stream is done with the workspace
  struct Drain {
    hipStream_t st;
    ~Drain() { (void)hipStreamSynchronize(st); }
  } drain{st};
  auto at = [&](size_t off) { return (double *)(ws + off); };
  f.store = at(L.store);
  f.xin = at(L.xin);
  f.mt = at(L.mt);
  f.mb = at(L.mb);
  f.lenv = at(L.lenv);
  f.renv = at(L.renv);
  f.t1 = L.t1 ? at(L.t1) : nullptr;
  f.t2 = L.t2 ? at(L.t2) : nullptr;
  f.t3 = at(L.t3);
  f.tmp = at(L.tmp);
  f.acan = const_cast<double *>(A);
  f.rbuf = at(L.rbuf);
  f.nu = at(L.nu);
  f.err = (int32_t *)(ws + L.err);
  f.dims = (FitDims *)(ws + L.dims);
  f.slot = (uint64_t *)(ws + L.slot);
  // the fit engine's bookkeeping (no device memory of its own)
  bbp_ctx host;
  host.n_fit = sp->n_fit;
  host.stream = st;
  Group g;
  g.W = f.W;
  g.H = f.H;
  g.fb = f;
  g.flagbuf.borrow(ws + L.flag, 4 * f.W);
  g.fb.flag = (int32_t *)(ws + L.flag);
  std::vector<FitDims> cd;
  column_dims(f.W, f.H, f.K, f.P, bt, bb, br, cd);
  for (auto &x : cd) x.rnd = 1;
  g.dims = cd;
  g.have.assign(f.W, 0);
  // workspace: zero padding, trivial message sites, tables
  double *triv = at(L.triv);
  GatherSrc gs{};
  gs.ksrc = f.K;
  const double *src[3] = {mt, mr, mb};
  const int nsite[3] = {f.W, f.H, f.W};
  for (int k = 0; k < 3; ++k) {
    gs.src[k][0] = src[k] ? src[k] : triv;
    gs.n[k][0] = nsite[k];
  }
  double *dst_tab = out;
  const int32_t rev0 = 0;
  const uint64_t slot0 = sp->slot;
  FitBatch ft = f;
  ft.items = std::max(f.W, f.H);
  if ((e = launch_zero(ws, L.zero_end, st)) != hipSuccess ||
      (e = launch_set_unit(ft, Ptr{triv, f.S}, st)) != hipSuccess ||
      (e = hipMemcpyAsync(ws + L.slot, &slot0, 8, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(ws + L.gather, &gs, sizeof gs, hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(ws + L.dst, &dst_tab, sizeof dst_tab, hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(ws + L.rev, &rev0, 4, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = launch_gather(g.fb, (const GatherSrc *)(ws + L.gather), st)) != hipSuccess)
    return update_fail(BBP_EDEVICE, std::string("update setup: ") + hipGetErrorString(e));
  bs = absorb_columns(&host, g, 0, st, false);
  if (bs != BBP_OK) return update_fail(bs, host.err);
  if ((e = launch_extract(g.fb, (double *const *)(ws + L.dst), (const int32_t *)(ws + L.rev),
                          st)) != hipSuccess)
    return update_fail(BBP_EDEVICE, std::string("extract: ") + hipGetErrorString(e));
  std::vector<double> nu(f.W, 0.0);
  int32_t errv = 0;
  if ((e = hipMemcpyAsync(nu.data(), f.nu, 8 * f.W, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(&errv, f.err, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return update_fail(BBP_EDEVICE, std::string("update: ") + hipGetErrorString(e));
  if (errv) return update_fail(BBP_ENUMERIC, "zero or non-finite boundary norm");
  double ls = 0.0;
  for (double v : nu) ls += std::log(v);
  *log_scale = ls;
  const FitDims &c0 = cd[0];
  out_bonds[0] = out_bonds[f.H] = 1;
  for (int s2 = 0; s2 + 1 < f.H; ++s2) out_bonds[s2 + 1] = c0.br[s2 + 1];
  return BBP_OK;
}

}  // namespace

extern "C" {

bbp_status bbp_update_workspace(const bbp_update_spec *spec, size_t *bytes) {
  FitBatch f;
  bbp_status bs = update_batch(spec, f);
  if (bs != BBP_OK) return bs;
  if (!bytes) return update_fail(BBP_EINVAL, "null bytes pointer");
  *bytes = update_layout(f).total;
  return BBP_OK;
}

bbp_status bbp_update_message(const bbp_update_spec *spec, const double *A, const double *mt,
                              const int32_t *mt_bonds, const double *mr,
                              const int32_t *mr_bonds, const double *mb,
                              const int32_t *mb_bonds, double *out, int32_t *out_bonds,
                              double *log_scale, void *hip_stream) {
  return update_message(spec, A, mt, mt_bonds, mr, mr_bonds, mb, mb_bonds, out, out_bonds,
                        log_scale, hip_stream, nullptr, 0);
}

bbp_status bbp_update_message_noalloc(const bbp_update_spec *spec, const double *A,
                                      const double *mt, const int32_t *mt_bonds,
                                      const double *mr, const int32_t *mr_bonds,
                                      const double *mb, const int32_t *mb_bonds, double *out,
                                      int32_t *out_bonds, double *log_scale,
                                      void *hip_stream) {
  FitBatch f;
  bbp_status bs = update_batch(spec, f);
  if (bs != BBP_OK) return bs;
  const size_t need = update_layout(f).total;
  if (need > kUpdateScratchBytes)
    return update_fail(BBP_EINVAL, "update needs " + std::to_string(need) +
                                       " bytes of workspace; the static workspace holds " +
                                       std::to_string(kUpdateScratchBytes));
  void *ws = nullptr;
  hipError_t e = device_scratch(&ws);
  if (e != hipSuccess)
    return update_fail(BBP_EDEVICE, std::string("static workspace: ") + hipGetErrorString(e));
  return update_message(spec, A, mt, mt_bonds, mr, mr_bonds, mb, mb_bonds, out, out_bonds,
                        log_scale, hip_stream, ws, kUpdateScratchBytes);
}

const char *bbp_update_last_error(void) { return tl_update_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Continuous batching across contexts (the request server): one synchronous
// sweep of many contexts at once, every message of every context in shared
// batches of one shape (W, H, bond cap, D, d), so that one launch of each
// fit kernel covers every resident solve's messages of that shape.  A
// batch is rebuilt when the set of contexts sweeping changes; the items that
// stay keep their fit results (warm starts) and bond caps, copied to their
// new positions.  Each item reads its context's messages and writes its
// context's next messages, so the results are those of the context alone
// (the visit tiling is fixed per shape, not chosen from the item count).
// ---------------------------------------------------------------------------
namespace bbp {

struct SharedItem {
  bbp_ctx *c;
  uint64_t serial;
  int id;
  bool operator==(const SharedItem &o) const { return serial == o.serial && id == o.id; }
};

struct SweepSet {
  bbp_ctx eng;  // host context of the shared batches: streams, lanes, error flag
  std::map<std::tuple<int, int, int, int, int>, std::vector<SharedItem>> items;
  std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<Group>> groups;
  // the previous batch of each shape, kept with its buffers: a rebuild fills
  // it (when its capacity suffices) and the two swap
  std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<Group>> spare;
  DevBuf ovE, ovU, ovOut, ovA, ovB;
  DevBuf jobs;                      // copy jobs of a rebuild
  std::vector<CopyJob> jobs_host;
};

// Items the visit tiling of a shared batch is chosen for (a fixed count, so
// that a context's results do not depend on who shares its batches).
constexpr int kSharedTileItems = 1024;

SweepSet *sweepset_create(hipStream_t st) {
  SweepSet *s = new (std::nothrow) SweepSet;
  if (!s) return nullptr;
  s->eng.stream = st;
  s->eng.lanes = 3;
  return s;
}

void sweepset_destroy(SweepSet *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->eng.stream);
  for (hipStream_t a : s->eng.aux) {
    (void)hipStreamSynchronize(a);
    (void)hipStreamDestroy(a);
  }
  for (hipEvent_t ev : s->eng.lane_ev) (void)hipEventDestroy(ev);
  if (s->eng.cap) (void)hipStreamDestroy(s->eng.cap);
  delete s;
}

void sweepset_set_allocator(SweepSet *s, bbp_alloc_fn alloc, bbp_free_fn free_, void *user) {
  s->eng.mem.alloc_fn = alloc;
  s->eng.mem.free_fn = free_;
  s->eng.mem.user = user;
  s->eng.mem.stream = &s->eng.stream;
}

bbp_status ctx_set_engine(bbp_ctx *c) {
  if (!c) return BBP_EINVAL;
  if (c->tensors_set) return c->fail(BBP_ESTATE, "engine mode must be set before the tensors");
  c->engine = true;
  c->pin.pageable = true;
  return BBP_OK;
}

static bbp_status rebuild_group(SweepSet *s, const std::tuple<int, int, int, int, int> &key,
                                const std::vector<SharedItem> &its) {
  bbp_ctx &eng = s->eng;
  const int W = std::get<0>(key), H = std::get<1>(key), K = std::get<2>(key);
  const int D = std::get<3>(key), d = std::get<4>(key);
  const int n = (int)its.size();
  int cap = 8;
  while (cap < n) cap *= 2;
  Group *old = s->groups.count(key) ? s->groups[key].get() : nullptr;
  const std::vector<SharedItem> *old_items = s->items.count(key) ? &s->items[key] : nullptr;
  std::unique_ptr<Group> g = std::move(s->spare[key]);
  if (!g) {
    g.reset(new Group);
    g->W = W;
    g->H = H;
  }
  eng.D = D;
  eng.d = d;
  eng.P = D * D;
  eng.precision = 64;
  eng.seed = 0;
  // buffers for `cap` items (kept from the spare when its capacity is the
  // same; cleared again), the first n in use
  std::vector<uint64_t> slots(cap, 0);
  for (int i = 0; i < n; ++i) slots[i] = (1ull << 40) | ((uint64_t)its[i].id << 8);
  bbp_status bs = alloc_batch(&eng, *g, cap, K, slots);
  if (bs != BBP_OK) return bs;
  FitBatch &f = g->fb;
  f.items = n;
  f.tile_items = kSharedTileItems;
  // each item's rotated block from its context; the fit results (warm
  // starts) and bond caps of the items that stay from the previous batch
  const size_t ablock = (size_t)H * W * d * D * D * D * D;
  const size_t fslot = (size_t)W * f.N * f.S;
  s->jobs_host.clear();
  for (int i = 0; i < n; ++i) {
    const bbp_ctx *c = its[i].c;
    s->jobs_host.push_back(CopyJob{c->rot.d() + c->rot_off[its[i].id], f.acan + i * ablock,
                                   (int64_t)ablock, 0, 0});
    if (!old || !old_items) continue;
    auto pos = std::find(old_items->begin(), old_items->end(), its[i]);
    if (pos == old_items->end()) continue;
    const size_t o = (size_t)(pos - old_items->begin());
    s->jobs_host.push_back(CopyJob{old->fb.store + o * fslot, f.store + i * fslot,
                                   (int64_t)fslot, 0, 0});
    for (int col = 0; col < W; ++col) {
      g->dims[(size_t)i * W + col] = old->dims[o * W + col];
      g->have[(size_t)i * W + col] = old->have[o * W + col];
    }
  }
  hipError_t e = hipSuccess;
  const size_t nj = s->jobs_host.size();
  if (s->jobs.bytes < nj * sizeof(CopyJob) &&
      s->jobs.alloc(nj * sizeof(CopyJob) * 2) != hipSuccess)
    return eng.fail(BBP_ENOMEM, "device allocation failed");
  e = copy_sync(&eng, s->jobs.p, s->jobs_host.data(), nj * sizeof(CopyJob),
                hipMemcpyHostToDevice);
  for (size_t o = 0; e == hipSuccess && o < nj; o += 60000)
    e = launch_copy_jobs((const CopyJob *)s->jobs.p + o, (int)std::min<size_t>(60000, nj - o),
                         K, D * D, eng.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(eng.stream);
  if (e != hipSuccess) return eng.hip_fail(e, "shared batch setup");
  if (s->groups.count(key)) s->spare[key] = std::move(s->groups[key]);
  s->groups[key] = std::move(g);
  s->items[key] = its;
  return BBP_OK;
}

bbp_status sweepset_run(SweepSet *s, bbp_ctx *const *cs, int n, double *res,
                        bbp_status *status, std::string *err) {
  bbp_ctx &eng = s->eng;
  AcctScope acct_scope(&eng.mem);
  for (int k = 0; k < n; ++k) status[k] = BBP_OK;
  // 1. the shared batches this sweep needs
  std::map<std::tuple<int, int, int, int, int>, std::vector<SharedItem>> want;
  for (int k = 0; k < n; ++k) {
    bbp_ctx *c = cs[k];
    if (!c || !c->tensors_set || !c->engine) {
      if (err) *err = "context not ready for a shared sweep";
      return BBP_ESTATE;
    }
    for (size_t i = 0; i < c->msgs.size(); ++i) {
      const auto sh = message_shape(c, c->msgs[i]);
      want[std::make_tuple(sh.first, sh.second, c->K, c->D, c->d)].push_back(
          SharedItem{c, c->serial, (int)i});
    }
  }
  for (auto it = s->groups.begin(); it != s->groups.end();) {
    if (!want.count(it->first)) {
      s->items.erase(it->first);
      s->spare.erase(it->first);
      it = s->groups.erase(it);
    } else {
      ++it;
    }
  }
  for (auto &kv : want) {
    auto have = s->items.find(kv.first);
    if (have != s->items.end() && have->second == kv.second) continue;
    bbp_status bs = rebuild_group(s, kv.first, kv.second);
    if (bs != BBP_OK) {
      if (err) *err = eng.err;
      return bs;
    }
    // fresh pointers to each item's context (a context keeps its serial)
  }
  for (auto &kv : want) s->items[kv.first] = kv.second;
  hipError_t e;
  if (!eng.errflag.p && eng.errflag.alloc(64) != hipSuccess) {
    if (err) *err = "device allocation failed";
    return BBP_ENOMEM;
  }
  if ((e = launch_zero(eng.errflag.p, 64, eng.stream)) != hipSuccess) {
    if (err) *err = hipGetErrorString(e);
    return BBP_EDEVICE;
  }
  // every context's streams are synchronised with the engine's: each call on
  // a context ends with its stream synchronised, and the engine stream runs
  // everything below
  std::map<uint64_t, std::vector<std::vector<int>>> new_bonds;
  std::map<uint64_t, double> flops;
  for (int k = 0; k < n; ++k) {
    new_bonds[cs[k]->serial].assign(cs[k]->msgs.size(), {});
    flops[cs[k]->serial] = 0.0;
  }
  // 2. gather, column absorptions and extraction, one batch per lane
  const int nl = std::max(1, std::min(eng.lanes, (int)s->groups.size()));
  {
    LaneFork lanes(&eng);
    if ((e = lanes.fork(nl)) != hipSuccess) {
      if (err) *err = hipGetErrorString(e);
      return BBP_EDEVICE;
    }
    int gi = 0;
    for (auto &kv : s->groups) {
      Group &g = *kv.second;
      const std::vector<SharedItem> &its = s->items[kv.first];
      FitBatch &f = g.fb;
      f.err = (int32_t *)eng.errflag.p;
      const hipStream_t st = lane_stream(&eng, gi++ % nl);
      g.gs.assign(f.items, GatherSrc{});
      g.dsts.assign(f.items, nullptr);
      g.revs.assign(f.items, 0);
      for (int i = 0; i < f.items; ++i) {
        bbp_ctx *c = its[i].c;
        double *cur = c->msgbuf[c->cur].d(), *nb = c->msgbuf[1 - c->cur].d();
        flops[c->serial] += prepare_item(c, its[i].id, cur, nb, g, i, g.gs[i], g.dsts[i],
                                         g.revs[i], new_bonds[c->serial][its[i].id]);
      }
      e = hipMemcpyAsync(g.gather.p, g.gs.data(), sizeof(GatherSrc) * f.items,
                         hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(g.dst.p, g.dsts.data(), sizeof(double *) * f.items,
                           hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(g.rev.p, g.revs.data(), 4 * f.items, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = launch_gather(f, (const GatherSrc *)g.gather.p, st);
      if (e != hipSuccess) {
        if (err) *err = std::string("shared gather: ") + hipGetErrorString(e);
        return BBP_EDEVICE;
      }
      bbp_status bs = absorb_columns(&eng, g, 0, st, true);
      if (bs != BBP_OK) {
        if (err) *err = eng.err;
        return bs;
      }
      e = launch_extract(f, (double *const *)g.dst.p, (const int32_t *)g.rev.p, st);
      if (e != hipSuccess) {
        if (err) *err = std::string("shared extract: ") + hipGetErrorString(e);
        return BBP_EDEVICE;
      }
    }
    if ((e = lanes.join()) != hipSuccess) {
      if (err) *err = hipGetErrorString(e);
      return BBP_EDEVICE;
    }
  }
  // 3. overlaps of new and old messages of every context, batched by shape
  struct Ov {
    int k, i;
  };
  std::map<std::tuple<int, int, int>, std::vector<Ov>> by;  // (K, P, L)
  size_t total = 0;
  for (int k = 0; k < n; ++k)
    for (size_t i = 0; i < cs[k]->msgs.size(); ++i) {
      by[std::make_tuple(cs[k]->K, cs[k]->P, cs[k]->msgs[i].n)].push_back(Ov{k, (int)i});
      ++total;
    }
  std::vector<std::vector<double>> ov(n);
  for (int k = 0; k < n; ++k) ov[k].assign(cs[k]->msgs.size(), 0.0);
  std::vector<double> part(total);
  std::vector<std::vector<const double *>> keep_a, keep_b;
  size_t off = 0;
  std::vector<std::pair<size_t, std::vector<Ov>>> order;
  for (auto &kv : by) {
    const int K = std::get<0>(kv.first), P = std::get<1>(kv.first), L = std::get<2>(kv.first);
    const std::vector<Ov> &v = kv.second;
    const size_t S = (size_t)K * P * K;
    keep_a.emplace_back(v.size());
    keep_b.emplace_back(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
      bbp_ctx *c = cs[v[i].k];
      const size_t per = (size_t)c->Lmax * c->S;
      keep_a.back()[i] = c->msgbuf[1 - c->cur].d() + (size_t)v[i].i * per;
      keep_b.back()[i] = c->msgbuf[c->cur].d() + (size_t)v[i].i * per;
    }
    if (s->ovE.alloc(std::max<size_t>(s->ovE.bytes, v.size() * K * K * 8)) != hipSuccess ||
        s->ovU.alloc(std::max<size_t>(s->ovU.bytes, v.size() * S * 8)) != hipSuccess ||
        s->ovOut.alloc(std::max<size_t>(s->ovOut.bytes, total * 8)) != hipSuccess ||
        s->ovA.alloc(std::max<size_t>(s->ovA.bytes, v.size() * 8)) != hipSuccess ||
        s->ovB.alloc(std::max<size_t>(s->ovB.bytes, v.size() * 8)) != hipSuccess) {
      if (err) *err = "device allocation failed";
      return BBP_ENOMEM;
    }
    e = hipMemcpyAsync(s->ovA.p, keep_a.back().data(), 8 * v.size(), hipMemcpyHostToDevice,
                       eng.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->ovB.p, keep_b.back().data(), 8 * v.size(), hipMemcpyHostToDevice,
                         eng.stream);
    if (e == hipSuccess)
      e = launch_overlap((int)v.size(), K, P, L, (const double *const *)s->ovA.p,
                         (const double *const *)s->ovB.p, s->ovE.d(), s->ovU.d(),
                         s->ovOut.d() + off, eng.stream);
    // the pointer tables are rewritten by the next shape: wait for this one
    if (e == hipSuccess) e = hipStreamSynchronize(eng.stream);
    if (e != hipSuccess) {
      if (err) *err = std::string("shared overlaps: ") + hipGetErrorString(e);
      return BBP_EDEVICE;
    }
    order.emplace_back(off, v);
    off += v.size();
  }
  int32_t errv = 0;
  e = hipMemcpyAsync(part.data(), s->ovOut.p, 8 * total, hipMemcpyDeviceToHost, eng.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&errv, eng.errflag.p, 4, hipMemcpyDeviceToHost, eng.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(eng.stream);
  if (e != hipSuccess) {
    if (err) *err = std::string("shared residual: ") + hipGetErrorString(e);
    return BBP_EDEVICE;
  }
  for (auto &o : order)
    for (size_t i = 0; i < o.second.size(); ++i)
      ov[o.second[i].k][o.second[i].i] = part[o.first + i];
  // 4. per context: residual, or a numeric failure (the shared error flag
  // cannot tell which context's fit failed: every context of this sweep
  // reports it and keeps its previous messages)
  for (int k = 0; k < n; ++k) {
    bbp_ctx *c = cs[k];
    const int nm = (int)c->msgs.size();
    double sum = 0.0;
    bool finite = true;
    for (int i = 0; i < nm; ++i) {
      if (!std::isfinite(ov[k][i])) finite = false;
      sum += std::max(0.0, 2.0 - 2.0 * std::fabs(ov[k][i]));
    }
    if (errv || !finite) {
      status[k] = c->fail(BBP_ENUMERIC, "zero-norm or non-finite boundary in a shared sweep");
      res[k] = std::nan("");
      continue;
    }
    for (int i = 0; i < nm; ++i) c->msgs[i].bonds = new_bonds[c->serial][i];
    c->cur = 1 - c->cur;
    c->obs.clear();
    release_kept(c);
    c->last_flops = flops[c->serial];
    res[k] = nm ? sum / nm : 0.0;
  }
  if (errv) {  // warm starts of every shared batch are no longer trusted
    for (auto &kv : s->groups) std::fill(kv.second->have.begin(), kv.second->have.end(), 0);
  }
  return BBP_OK;
}

bbp_status ctx_info(bbp_ctx *c, CtxInfo *o) {
  if (!c || !o) return BBP_EINVAL;
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  *o = CtxInfo{c->infinite, c->Lx, c->Ly, c->bx, c->by, c->D, c->chi, c->d,
               c->chi_env, c->n_fit, c->sx, c->sy, c->single_layer, c->seed,
               c->stream, c->mem.alloc_fn, c->mem.free_fn, c->mem.user, c->mem.budget};
  return BBP_OK;
}

bbp_status ctx_fail(bbp_ctx *c, bbp_status s, const std::string &m) { return c->fail(s, m); }

bbp_status rdm_bonds_only(bbp_ctx *c, int n, const int32_t *x0, const int32_t *y0,
                          const int32_t *x1, const int32_t *y1, double *rho) {
  return ::rdm_bonds_only(c, n, x0, y0, x1, y1, rho);
}

void ctx_keep_stacks(bbp_ctx *c) { c->stack_reuse = true; }

bbp_status ctx_replace_sites(bbp_ctx *c, int n, const int *site, const double *A) {
  if (!c || n < 0 || (n > 0 && (!site || !A))) return BBP_EINVAL;
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  const size_t ss = (size_t)c->d * c->D * c->D * c->D * c->D;
  const int nsites = c->ucx * c->ucy;
  for (int i = 0; i < n; ++i) {
    if (site[i] < 0 || site[i] >= nsites) return c->fail(BBP_EINVAL, "site out of range");
    std::copy(A + (size_t)i * ss, A + (size_t)(i + 1) * ss, c->A.begin() + (size_t)site[i] * ss);
  }
  c->obs.clear();  // kept stacks stay: each is checked against the tensors it absorbed
  return BBP_OK;
}

const double *ctx_tensors(bbp_ctx *c, size_t *n) {
  *n = c->A.size();
  return c->A.data();
}

}  // namespace bbp
