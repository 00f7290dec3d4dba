// libbbp host side: the C ABI of include/bbp.h, the block partition and
// message bookkeeping of block BP (Sec. II, Eq. (1)), and the launch sequence
// of one synchronous sweep (App. A column absorptions as variational fits).
//
// Nothing here touches the GPU before bbp_set_tensors has validated its
// input, so argument checking works on machines without a GPU.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
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

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t b) {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = b;
    if (b == 0) return hipSuccess;
    return hipMalloc(&p, b);
  }
  double *d() const { return (double *)p; }
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
  DevBuf gather, dst, rev, dims_host_unused;
  std::vector<FitDims> dims;  // [items][W], host copy
  std::vector<int> have;      // [items*W] warm start valid
  // host staging of the per-sweep tables (kept alive until the stream syncs)
  std::vector<GatherSrc> gs;
  std::vector<double *> dsts;
  std::vector<int32_t> revs;
  std::vector<int32_t> flags;  // [W][items]
  DevBuf flagbuf;              // [W][items]
};

}  // namespace

struct bbp_ctx {
  // problem
  int infinite = 0, Lx = 0, Ly = 0, ucx = 1, ucy = 1, bx = 1, by = 1, D = 1,
      chi = 1, d = 2;
  int gx = 1, gy = 1;
  int chi_env = -1, n_fit = 2;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
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
  double last_flops = 0.0;

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
    if (x < Lx && y < Ly) return A.data() + (size_t)(y * Lx + x) * ss;
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
    xb = b;
  }
}

}  // namespace

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

static bbp_status alloc_group(bbp_ctx *c, Group &g) {
  FitBatch &f = g.fb;
  f.items = (int)g.ids.size();
  f.K = c->K;
  f.P = c->P;
  f.D = c->D;
  f.d = c->d;
  f.H = g.H;
  f.W = g.W;
  f.N = g.H + 2;
  f.S = c->S;
  f.seed = c->seed;
  const size_t it = f.items, S = f.S, K = f.K, P = f.P;
  struct Req {
    double **dst;
    size_t n;
  };
  std::vector<Req> reqs = {
      {&f.store, it * f.W * f.N * S},
      {&f.xin, it * f.N * S},
      {&f.mt, it * f.W * S},
      {&f.mb, it * f.W * S},
      {&f.lenv, it * f.N * S},
      {&f.renv, it * f.N * S},
      {&f.t1, it * K * P * P * K},
      {&f.t2, it * (size_t)f.d * K * K * P * P},
      {&f.t3, it * K * P * P * K},
      {&f.tmp, it * S},
      {&f.acan, it * f.H * f.W * (size_t)f.d * P * P},
      {&f.rbuf, it * K * K},
      {&f.nu, it},
  };
  g.bufs.resize(reqs.size() + 4);
  for (size_t i = 0; i < reqs.size(); ++i) {
    hipError_t e = g.bufs[i].alloc(std::max<size_t>(reqs[i].n, 1) * 8);
    if (e != hipSuccess) return c->fail(BBP_ENOMEM, "device allocation failed");
    *reqs[i].dst = g.bufs[i].d();
    e = hipMemsetAsync(g.bufs[i].p, 0, g.bufs[i].bytes, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "clear buffers");
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
  // random-state slot bases: message e, column c -> (1<<40)|(e<<8)|c
  std::vector<uint64_t> slots(it);
  for (size_t i = 0; i < it; ++i)
    slots[i] = (1ull << 40) | ((uint64_t)g.ids[i] << 8);
  hipError_t e = hipMemcpy(f.slot, slots.data(), 8 * it, hipMemcpyHostToDevice);
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
  hipError_t e = hipMemcpy(f.acan, host.data(), host.size() * 8,
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "upload tensors");
  return BBP_OK;
}

static bbp_status init_messages(bbp_ctx *c) {
  // identity product MPDO: m[(k,k')] = delta_kk' / sqrt(D), bonds 1
  const size_t per = (size_t)c->Lmax * c->S;
  std::vector<double> host(per * c->msgs.size(), 0.0);
  const double v = 1.0 / std::sqrt((double)c->D);
  for (size_t e = 0; e < c->msgs.size(); ++e) {
    Message &m = c->msgs[e];
    m.bonds.assign(m.n + 1, 1);
    for (int s = 0; s < m.n; ++s)
      for (int k = 0; k < c->D; ++k)
        host[e * per + (size_t)s * c->S + (size_t)(k * c->D + k) * c->K] = v;
  }
  hipError_t err = hipMemcpy(c->msgbuf[c->cur].p, host.data(), host.size() * 8,
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

static bbp_status run_sweep(bbp_ctx *c, double *residual) {
  hipStream_t st = c->stream;
  const int nxt = 1 - c->cur;
  const size_t per = (size_t)c->Lmax * c->S;
  double *cur = c->msgbuf[c->cur].d(), *nb = c->msgbuf[nxt].d();
  hipError_t e = hipMemsetAsync(c->errflag.p, 0, 4, st);
  if (e != hipSuccess) return c->hip_fail(e, "memset");
  std::vector<std::vector<int>> new_bonds(c->msgs.size());
  double flops = 0.0;
  for (auto &gp : c->groups) {
    Group &g = *gp;
    FitBatch &f = g.fb;
    const int W = f.W, H = f.H, N = f.N;
    std::vector<GatherSrc> &gs = g.gs;
    std::vector<double *> &dsts = g.dsts;
    std::vector<int32_t> &revs = g.revs;
    gs.assign(f.items, GatherSrc{});
    dsts.assign(f.items, nullptr);
    revs.assign(f.items, 0);
    std::vector<int> any_rnd(W, 0);
    std::vector<std::vector<int>> xb0(f.items);
    for (int i = 0; i < f.items; ++i) {
      const Message &m = c->msgs[g.ids[i]];
      char side[3];
      int rv[3];
      canon_sources(m.dir, side, rv);
      std::vector<int> bl[3];
      for (int k = 0; k < 3; ++k) {
        Incoming in = c->incoming(m.bi, m.bj, side[k]);
        if (in.id < 0) {
          gs[i].src[k] = c->trivial.d();
          bl[k].assign(in.n + 1, 1);
        } else {
          gs[i].src[k] = cur + (size_t)in.id * per;
          bl[k] = c->msgs[in.id].bonds;
        }
        gs[i].rev[k] = rv[k];
        if (rv[k]) bl[k] = reversed(bl[k]);
      }
      dsts[i] = nb + (size_t)g.ids[i] * per;
      revs[i] = out_reversed(m.dir) ? 1 : 0;
      std::vector<FitDims> cd;
      column_dims(W, H, f.K, f.P, bl[0], bl[2], bl[1], cd);
      std::vector<int> xbonds = bl[1];
      for (int col = W - 1; col >= 0; --col) {
        FitDims &nd = cd[col];
        FitDims &od = g.dims[(size_t)i * W + col];
        bool same = g.have[(size_t)i * W + col] &&
                    std::memcmp(nd.bl, od.bl, sizeof(nd.bl)) == 0 &&
                    std::memcmp(nd.br, od.br, sizeof(nd.br)) == 0 &&
                    std::memcmp(nd.p, od.p, sizeof(nd.p)) == 0;
        nd.rnd = same ? 0 : 1;
        any_rnd[col] |= nd.rnd;
        od = nd;
        g.have[(size_t)i * W + col] = 1;
        const int xp0 = col == W - 1 ? 1 : cd[col + 1].p[0];
        const int xpN = col == W - 1 ? 1 : cd[col + 1].p[N - 1];
        flops += 2.0 * column_macs(nd, xbonds, xp0, xpN, N, f.P, f.D, f.d,
                                   c->n_fit);
        xbonds.assign(N - 1, 1);
        for (int j = 0; j < N - 1; ++j) xbonds[j] = nd.br[j];
      }
      const FitDims &c0 = cd[0];
      std::vector<int> cb(H + 1, 1);
      for (int s = 0; s + 1 < H; ++s) cb[s + 1] = c0.br[s + 1];
      new_bonds[g.ids[i]] = revs[i] ? reversed(cb) : cb;
    }
    e = hipMemcpyAsync(g.gather.p, gs.data(), sizeof(GatherSrc) * f.items,
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.dst.p, dsts.data(), sizeof(double *) * f.items,
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(g.rev.p, revs.data(), 4 * f.items,
                         hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(f.dims, g.dims.data(), sizeof(FitDims) * g.dims.size(),
                         hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return c->hip_fail(e, "upload sweep tables");
    e = launch_gather(f, (const GatherSrc *)g.gather.p, st);
    if (e != hipSuccess) return c->hip_fail(e, "gather");

    const size_t sN = (size_t)N * f.S, sWN = (size_t)W * N * f.S;
    g.flags.assign((size_t)W * f.items, 0);
    for (int col = 0; col < W; ++col)
      for (int i = 0; i < f.items; ++i)
        g.flags[(size_t)col * f.items + i] = g.dims[(size_t)i * W + col].rnd;
    e = hipMemcpyAsync(g.flagbuf.p, g.flags.data(), 4 * g.flags.size(),
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return c->hip_fail(e, "upload flags");
    for (int col = W - 1; col >= 0; --col) {
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
          e = launch_end_chain(f, true, MB, Xs(N - 1), st);
          if (e == hipSuccess) e = launch_end_env(f, true, Ys(N - 1), Re(N - 2), st);
        } else {
          e = launch_inner_chain(f, col, j, true, Xs(j), Re(j), st);
          if (e == hipSuccess) e = launch_inner_env(f, true, Ys(j), Re(j - 1), st);
        }
        if (e != hipSuccess) return c->hip_fail(e, "right environments");
      }
      for (int sw = 0; sw < c->n_fit; ++sw) {
        for (int j = 0; j < N - 1; ++j) {
          if (j == 0) {
            e = launch_end_chain(f, false, MT, Xs(0), st);
            if (e == hipSuccess) e = launch_end_local(f, false, Re(0), Ys(0), st);
            if (e == hipSuccess) e = launch_qr(f, col, 0, LR_TOP, Ys(0), false, false, st);
            if (e == hipSuccess) e = launch_end_env(f, false, Ys(0), Le(1), st);
          } else {
            e = launch_inner_chain(f, col, j, false, Xs(j), Le(j), st);
            if (e == hipSuccess) e = launch_inner_local(f, false, Re(j), Ys(j), st);
            if (e == hipSuccess) e = launch_qr(f, col, j, LR_INNER, Ys(j), false, false, st);
            if (e == hipSuccess) e = launch_inner_env(f, false, Ys(j), Le(j + 1), st);
          }
          if (e != hipSuccess) return c->hip_fail(e, "left-to-right visit");
        }
        for (int j = N - 1; j >= 1; --j) {
          if (j == N - 1) {
            e = launch_end_chain(f, true, MB, Xs(N - 1), st);
            if (e == hipSuccess) e = launch_end_local(f, true, Le(N - 1), Ys(N - 1), st);
            if (e == hipSuccess) e = launch_qr(f, col, N - 1, RL_BOT, Ys(N - 1), false, false, st);
            if (e == hipSuccess) e = launch_end_env(f, true, Ys(N - 1), Re(N - 2), st);
          } else {
            e = launch_inner_chain(f, col, j, true, Xs(j), Re(j), st);
            if (e == hipSuccess) e = launch_inner_local(f, true, Le(j), Ys(j), st);
            if (e == hipSuccess) e = launch_qr(f, col, j, RL_INNER, Ys(j), false, false, st);
            if (e == hipSuccess) e = launch_inner_env(f, true, Ys(j), Re(j - 1), st);
          }
          if (e != hipSuccess) return c->hip_fail(e, "right-to-left visit");
        }
      }
      e = launch_end_chain(f, false, MT, Xs(0), st);
      if (e == hipSuccess) e = launch_end_local(f, false, Re(0), Ys(0), st);
      if (e == hipSuccess) e = launch_normalize(f, Ys(0), st);
      if (e != hipSuccess) return c->hip_fail(e, "final visit");
    }
    e = launch_extract(f, (double *const *)g.dst.p, (const int32_t *)g.rev.p, st);
    if (e != hipSuccess) return c->hip_fail(e, "extract");
  }
  // residual: overlaps of new and old messages, grouped by length
  const int nm = (int)c->msgs.size();
  std::vector<double> ov(nm, 0.0);
  std::map<int, std::vector<int>> by_len;
  for (int i = 0; i < nm; ++i) by_len[c->msgs[i].n].push_back(i);
  for (auto &kv : by_len) {
    const std::vector<int> &ids = kv.second;
    std::vector<const double *> pa(ids.size()), pb(ids.size());
    for (size_t i = 0; i < ids.size(); ++i) {
      pa[i] = nb + (size_t)ids[i] * per;
      pb[i] = cur + (size_t)ids[i] * per;
    }
    e = hipMemcpyAsync(c->ovA.p, pa.data(), 8 * ids.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->ovB.p, pb.data(), 8 * ids.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = launch_overlap((int)ids.size(), c->K, c->P, kv.first,
                         (const double *const *)c->ovA.p,
                         (const double *const *)c->ovB.p, c->ovE.d(),
                         c->ovU.d(), c->ovOut.d(), st);
    std::vector<double> part(ids.size());
    if (e == hipSuccess)
      e = hipMemcpyAsync(part.data(), c->ovOut.p, 8 * ids.size(),
                         hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return c->hip_fail(e, "overlap");
    for (size_t i = 0; i < ids.size(); ++i) ov[ids[i]] = part[i];
  }
  int32_t errv = 0;
  e = hipMemcpy(&errv, c->errflag.p, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return c->hip_fail(e, "error flag");
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
  c->last_flops = flops;
  if (residual) *residual = nm ? sum / nm : 0.0;
  return BBP_OK;
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
  c->infinite = infinite ? 1 : 0;
  c->Lx = infinite ? 0 : Lx;
  c->Ly = infinite ? 0 : Ly;
  c->ucx = infinite ? ucx : Lx;
  c->ucy = infinite ? ucy : Ly;
  c->bx = bx;
  c->by = by;
  c->D = D;
  c->chi = chi;
  if (infinite) {
    c->gx = c->gy = 1;
  } else {
    c->gx = (Lx + bx - 1) / bx;
    c->gy = (Ly + by - 1) / by;
  }
  for (int bj = 0; bj < c->gy; ++bj)
    for (int bi = 0; bi < c->gx; ++bi)
      for (char dr : kDirs) {
        int ni, nj;
        if (c->neighbour(bi, bj, dr, &ni, &nj)) {
          Message m{bi, bj, dr, (dr == 'L' || dr == 'R') ? by : bx, {}};
          m.bonds.assign(m.n + 1, 1);
          c->msgs.push_back(m);
        }
      }
  *out = c;
  return BBP_OK;
}

bbp_status bbp_set_option(bbp_ctx *c, const char *key, double v) {
  if (!c || !key) return BBP_EINVAL;
  std::string k(key);
  const bool late_ok = (k == "n_fit" || k == "chi_env");
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
  } else if (k == "n_fit") {
    if (v < 1 || v > 64 || v != std::floor(v))
      return c->fail(BBP_EINVAL, "n_fit must be an integer in [1,64]");
    c->n_fit = (int)v;
  } else if (k == "seed") {
    if (v < 0 || v != std::floor(v) || v > 9007199254740992.0)
      return c->fail(BBP_EINVAL, "seed must be a non-negative integer");
    c->seed = (uint64_t)v;
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

bbp_status bbp_set_tensors(bbp_ctx *c, const double *A, size_t n) {
  if (!c || !A) return BBP_EINVAL;
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
  if (hipMemset(c->msgbuf[0].p, 0, c->msgbuf[0].bytes) != hipSuccess ||
      hipMemset(c->msgbuf[1].p, 0, c->msgbuf[1].bytes) != hipSuccess)
    return c->fail(BBP_EDEVICE, "clear message buffers");
  {
    std::vector<double> triv(per, 0.0);
    for (int s2 = 0; s2 < c->Lmax; ++s2) triv[(size_t)s2 * c->S] = 1.0;
    if (hipMemcpy(c->trivial.p, triv.data(), per * 8, hipMemcpyHostToDevice) !=
        hipSuccess)
      return c->fail(BBP_EDEVICE, "upload trivial message");
  }
  c->cur = 0;
  // groups by canonical (W, H)
  c->groups.clear();
  std::map<std::pair<int, int>, int> gid;
  for (size_t i = 0; i < c->msgs.size(); ++i) {
    const Message &m = c->msgs[i];
    int W = (m.dir == 'L' || m.dir == 'R') ? c->bx : c->by;
    int H = (m.dir == 'L' || m.dir == 'R') ? c->by : c->bx;
    auto key = std::make_pair(W, H);
    if (!gid.count(key)) {
      gid[key] = (int)c->groups.size();
      c->groups.emplace_back(new Group);
      c->groups.back()->W = W;
      c->groups.back()->H = H;
    }
    c->groups[gid[key]]->ids.push_back((int)i);
  }
  for (auto &g : c->groups) {
    if ((s = alloc_group(c, *g)) != BBP_OK) return s;
    if ((s = upload_rotated(c, *g)) != BBP_OK) return s;
  }
  if ((s = init_messages(c)) != BBP_OK) return s;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return c->hip_fail(e, "set_tensors");
  c->tensors_set = true;
  return BBP_OK;
}

bbp_status bbp_sweep(bbp_ctx *c, int32_t n, double *residual) {
  if (!c) return BBP_EINVAL;
  if (!c->tensors_set) return c->fail(BBP_ESTATE, "bbp_set_tensors first");
  if (n < 0) return c->fail(BBP_EINVAL, "negative sweep count");
  double r = 0.0;
  for (int i = 0; i < n; ++i) {
    bbp_status s = run_sweep(c, &r);
    if (s != BBP_OK) return s;
  }
  if (residual) *residual = r;
  return BBP_OK;
}

bbp_status bbp_get_messages(bbp_ctx *c, double *buf, size_t n, size_t *needed) {
  if (!c) return BBP_EINVAL;
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
  hipError_t e = hipMemcpy(host.data(), c->msgbuf[c->cur].p, host.size() * 8,
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
  hipError_t e = hipMemcpy(c->msgbuf[c->cur].p, host.data(), host.size() * 8,
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return c->hip_fail(e, "upload messages");
  for (size_t i = 0; i < c->msgs.size(); ++i) c->msgs[i].bonds = bonds[i];
  for (auto &g : c->groups) std::fill(g->have.begin(), g->have.end(), 0);
  return BBP_OK;
}

bbp_status bbp_stats(bbp_ctx *c, int32_t *n_messages, double *sweep_flops) {
  if (!c) return BBP_EINVAL;
  if (n_messages) *n_messages = (int32_t)c->msgs.size();
  if (sweep_flops) *sweep_flops = c->last_flops;
  return BBP_OK;
}

bbp_status bbp_expect_site(bbp_ctx *c, int32_t, int32_t, const double *,
                           double *) {
  return c ? c->fail(BBP_ESTATE, "observables not available") : BBP_EINVAL;
}
bbp_status bbp_expect_bond(bbp_ctx *c, int32_t, int32_t, int32_t, int32_t,
                           const double *, double *) {
  return c ? c->fail(BBP_ESTATE, "observables not available") : BBP_EINVAL;
}
bbp_status bbp_expect_sites(bbp_ctx *c, int32_t, const int32_t *,
                            const int32_t *, const double *, double *) {
  return c ? c->fail(BBP_ESTATE, "observables not available") : BBP_EINVAL;
}
bbp_status bbp_expect_bonds(bbp_ctx *c, int32_t, const int32_t *,
                            const int32_t *, const int32_t *, const int32_t *,
                            const double *, double *) {
  return c ? c->fail(BBP_ESTATE, "observables not available") : BBP_EINVAL;
}
bbp_status bbp_log_norm(bbp_ctx *c, double *, int32_t *) {
  return c ? c->fail(BBP_ESTATE, "observables not available") : BBP_EINVAL;
}

const char *bbp_last_error(const bbp_ctx *c) {
  return c ? c->err.c_str() : "null context";
}

void bbp_destroy(bbp_ctx *c) {
  if (!c) return;
  if (c->device_ready) (void)hipDeviceSynchronize();
  delete c;
}

}  // extern "C"
