// libbbp request server: many block-BP solves (open lattices of different
// size, D and chi) served on one GPU with continuous batching.
//
// One engine thread admits queued requests first-in first-out while a slot
// is free and their device-memory estimate fits in what the byte budget
// leaves, and sweeps every resident request together: each sweep is one set
// of shared batches, every message of every resident request in the batch of
// its shape (block width and height, bond cap, D, d), so that one launch of
// each fit kernel covers all of them (bbp::SweepSet).  Requests join and
// leave between sweeps, their messages stay resident in their own buffers,
// and the items that stay keep their warm starts when a batch is rebuilt.  A
// request whose residual drops below its tolerance (or that reaches its
// sweep cap) goes to a finisher thread, which evaluates its outputs on the
// request's own stream while the others keep sweeping, then frees its
// memory.  Each item of a shared batch is computed from its own request's
// inputs only, with the tiling fixed per shape, so a result is the same
// (bitwise) whether its request ran alone or in a mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bbp.h"
#include "bbp_internal.h"

namespace {

struct Request {
  int64_t id = 0;
  bbp_request r{};
  std::vector<double> A;
  std::vector<double> ops;  // n_site_ops d x d, then n_bond_ops d^2 x d^2 operators
  size_t estimate = 0;
  int32_t state = BBP_REQ_QUEUED;
  bool cancel = false;     // asked for (under the server lock)
  bool cancelled = false;  // taken effect (engine thread)
  bool ok = true;
  std::vector<double> out;
  std::string err;
  double t_submit = 0.0, t_admit = 0.0, t_finish = 0.0;
  // while resident: its context (engine mode) and stream, sweeps so far
  bbp_ctx *c = nullptr;
  hipStream_t st = nullptr;
  int32_t sweeps = 0;
  double res = 1.0;
};

// Device bytes of one fit batch item (mirrors the buffers a batch item
// holds: stored fits, boundary, top/bottom rows, environments, scratch,
// rotated tensors), with bond cap Kc over W columns of height H.
size_t item_doubles(int W, int H, int Kc, int D) {
  const size_t P = (size_t)D * D, N = (size_t)H + 2;
  const size_t S = (size_t)Kc * P * Kc, T = (size_t)Kc * Kc * P * P;
  bbp::FitBatch f{};
  f.K = Kc;
  f.P = (int)P;
  f.D = D;
  f.d = 2;
  f.items = 1;
  f.W = W;
  f.H = H;
  f.N = (int)N;
  const bool fused = bbp::visit_fused_fits(f);
  const bool qscr = bbp::qr_needs_scratch(f);
  return ((size_t)W * N + 4 * N + 2 * (size_t)W + 1) * S + T * (1 + (qscr || !fused) + 2 * !fused) +
         (size_t)H * W * 2 * P * P + (size_t)Kc * Kc + (size_t)W + 64;
}

// Device memory of the server's contexts and shared batches: a block freed
// by one request is kept for the next allocation of about its size, so that
// admissions and departures (every few sweeps) call neither hipMalloc nor
// hipFree, whose device-wide synchronisation would stall the resident
// requests' work.  Beyond `limit` cached bytes the largest blocks are
// released; everything is released when the server is destroyed.
struct BlockCache {
  std::mutex mu;
  std::multimap<size_t, void *> free_blocks;  // size -> block
  std::map<void *, size_t> size_of;           // every live or cached block
  size_t cached = 0, limit = 0;

  void release_all_cached() {
    for (auto &kv : free_blocks) {
      (void)hipFree(kv.second);
      size_of.erase(kv.second);
    }
    free_blocks.clear();
    cached = 0;
  }
  ~BlockCache() {
    release_all_cached();
    for (auto &kv : size_of) (void)hipFree(kv.first);
  }
};

void *cache_alloc(size_t bytes, void *user) {
  BlockCache *bc = (BlockCache *)user;
  std::lock_guard<std::mutex> lk(bc->mu);
  auto it = bc->free_blocks.lower_bound(bytes);
  if (it != bc->free_blocks.end() && it->first <= bytes + bytes / 4) {
    void *p = it->second;
    bc->cached -= it->first;
    bc->free_blocks.erase(it);
    return p;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    bc->release_all_cached();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  bc->size_of[p] = bytes;
  return p;
}

void cache_free(void *p, void *user) {
  BlockCache *bc = (BlockCache *)user;
  std::lock_guard<std::mutex> lk(bc->mu);
  auto it = bc->size_of.find(p);
  if (it == bc->size_of.end()) return;
  bc->free_blocks.insert({it->second, p});
  bc->cached += it->second;
  while (bc->cached > bc->limit && !bc->free_blocks.empty()) {
    auto big = std::prev(bc->free_blocks.end());
    (void)hipFree(big->second);
    bc->cached -= big->first;
    bc->size_of.erase(big->second);
    bc->free_blocks.erase(big);
  }
}

}  // namespace

struct bbp_server {
  size_t budget = 0, used = 0;
  int32_t slots = 1, running = 0, max_running = 0;
  int64_t shared_sweeps = 0, request_sweeps = 0;  // sweeps run, and their requests summed
  int32_t max_together = 0;                       // most requests in one shared sweep
  double t_sweep = 0.0, t_admit_s = 0.0, t_finish_s = 0.0;  // busy seconds: shared sweeps,
                                                            // admissions, output evaluation
  bool stop = false;
  int64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv;   // admission, finishing, stop
  std::deque<std::shared_ptr<Request>> queue;
  std::deque<std::shared_ptr<Request>> finishing;
  std::map<int64_t, std::shared_ptr<Request>> all;
  std::thread engine;
  std::vector<std::thread> finishers;
  BlockCache cache;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void engine_loop();
  void finisher_loop();
  bool setup(Request &q);
  void outputs(Request &q);
  void done(const std::shared_ptr<Request> &q);
};

namespace {

int64_t n_sites(const bbp_request &r) { return (int64_t)r.Lx * r.Ly; }
int64_t n_bonds(const bbp_request &r) {
  return (int64_t)(r.Lx - 1) * r.Ly + (int64_t)r.Lx * (r.Ly - 1);
}
size_t result_len(const bbp_request &r) {
  size_t n = 6;
  if (r.outputs & BBP_OUT_SZ) n += (size_t)n_sites(r);
  if (r.outputs & BBP_OUT_SS) n += (size_t)n_bonds(r);
  n += (size_t)r.n_site_ops * n_sites(r) + (size_t)r.n_bond_ops * n_bonds(r);
  return n;
}
size_t ops_len(const bbp_request &r) { return (size_t)r.n_site_ops * 4 + (size_t)r.n_bond_ops * 16; }
int chi_env_of(const bbp_request &r) {
  return std::max(r.chi, std::min(128, 2 * r.D * r.D + 10));
}

bbp_status check_request(const bbp_request *r) {
  if (!r) return BBP_EINVAL;
  if (r->Lx <= 0 || r->Ly <= 0 || r->bx <= 0 || r->by <= 0 || r->D <= 0 || r->chi <= 0 ||
      r->chi > 128 || r->max_sweeps <= 0 || !(r->tol >= 0.0) ||
      (r->outputs & ~(BBP_OUT_SZ | BBP_OUT_SS | BBP_OUT_LOGNORM)) != 0 ||
      r->n_site_ops < 0 || r->n_site_ops > 16 || r->n_bond_ops < 0 || r->n_bond_ops > 16)
    return BBP_EINVAL;
  if (r->bx + 2 > bbp::NMAX || r->by + 2 > bbp::NMAX || 2 * r->bx + 2 > bbp::NMAX ||
      2 * r->by + 2 > bbp::NMAX)
    return BBP_EINVAL;
  return BBP_OK;
}

}  // namespace

// A request's context (in engine mode: its messages are swept by the shared
// batches) and stream, tensors uploaded.  False (with q.err set under the
// lock) when any step fails.
bool bbp_server::setup(Request &q) {
  const bbp_request &r = q.r;
  std::string why;
  bbp_status s = bbp_create(&q.c, 0, r.Lx, r.Ly, 0, 0, r.bx, r.by, r.D, r.chi);
  if (s != BBP_OK) why = "bbp_create (status " + std::to_string((int)s) + ")";
  // its own calls (uploads, observables) on one stream of its own
  if (why.empty() && (s = bbp_set_option(q.c, "lanes", 1)) != BBP_OK) why = "lanes";
  if (why.empty() && (s = bbp_set_option(q.c, "chi_env", chi_env_of(r))) != BBP_OK)
    why = "chi_env";
  if (why.empty() && (s = bbp::ctx_set_engine(q.c)) != BBP_OK) why = "engine mode";
  if (why.empty() && (s = bbp_set_allocator(q.c, cache_alloc, cache_free, &cache)) != BBP_OK)
    why = "allocator";
  if (why.empty()) {
    if (hipSetDevice(0) == hipSuccess &&
        hipStreamCreateWithFlags(&q.st, hipStreamNonBlocking) == hipSuccess)
      (void)bbp_set_stream(q.c, q.st);
    else
      q.st = nullptr;  // no device: set_tensors reports it below
  }
  if (why.empty() && (s = bbp_set_tensors(q.c, q.A.data(), q.A.size())) != BBP_OK)
    why = std::string("bbp_set_tensors (status ") + std::to_string((int)s) + "): " +
          bbp_last_error(q.c);
  if (why.empty()) return true;
  std::lock_guard<std::mutex> lk(mu);
  q.err = why;
  return false;
}

// The requested outputs from a request's converged (or capped) messages.
void bbp_server::outputs(Request &q) {
  const bbp_request &r = q.r;
  std::vector<double> out(result_len(r), 0.0);
  bbp_ctx *c = q.c;
  bool ok = true;
  std::string why;
  auto fail = [&](bbp_status s, const char *what) {
    const char *m = bbp_last_error(c);
    why = std::string(what) + " (status " + std::to_string((int)s) + ")" +
          (m && *m ? std::string(": ") + m : std::string());
    ok = false;
  };
  out[0] = q.res < r.tol ? 1.0 : 0.0;
  out[1] = q.sweeps;
  out[2] = q.res;
  const int64_t ns = n_sites(r), nb = n_bonds(r);
  std::vector<int32_t> xs(ns), ys(ns), x0, y0, x1, y1;
  for (int y = 0; y < r.Ly; ++y)
    for (int x = 0; x < r.Lx; ++x) {
      xs[(size_t)y * r.Lx + x] = x;
      ys[(size_t)y * r.Lx + x] = y;
    }
  for (int y = 0; y < r.Ly; ++y)
    for (int x = 0; x + 1 < r.Lx; ++x) {
      x0.push_back(x); y0.push_back(y); x1.push_back(x + 1); y1.push_back(y);
    }
  for (int y = 0; y + 1 < r.Ly; ++y)
    for (int x = 0; x < r.Lx; ++x) {
      x0.push_back(x); y0.push_back(y); x1.push_back(x); y1.push_back(y + 1);
    }
  size_t o = 6;
  bbp_status s;
  auto site_op = [&](const double *op) {
    if (ok && (s = bbp_expect_sites(c, (int32_t)ns, xs.data(), ys.data(), op, &out[o])) != BBP_OK)
      fail(s, "bbp_expect_sites");
    o += (size_t)ns;
  };
  auto bond_op = [&](const double *op) {
    if (ok && (s = bbp_expect_bonds(c, (int32_t)nb, x0.data(), y0.data(), x1.data(), y1.data(),
                                    op, &out[o])) != BBP_OK)
      fail(s, "bbp_expect_bonds");
    o += (size_t)nb;
  };
  if (r.outputs & BBP_OUT_SZ) {
    const double sz[4] = {1.0, 0.0, 0.0, -1.0};
    site_op(sz);
  }
  if (r.outputs & BBP_OUT_SS) {
    // S.S = (sx sx + sy sy + sz sz) / 4 on (s0, s1), s0 the major index
    const double ss[16] = {0.25, 0, 0, 0, 0, -0.25, 0.5, 0, 0, 0.5, -0.25, 0, 0, 0, 0, 0.25};
    bond_op(ss);
  }
  for (int k = 0; k < r.n_site_ops; ++k) site_op(q.ops.data() + 4 * k);
  for (int k = 0; k < r.n_bond_ops; ++k) bond_op(q.ops.data() + 4 * r.n_site_ops + 16 * k);
  if (ok && (r.outputs & BBP_OUT_LOGNORM)) {
    int32_t sign = 0;
    if ((s = bbp_log_norm(c, &out[3], &sign)) != BBP_OK) fail(s, "bbp_log_norm");
    out[4] = sign;
  }
  size_t cur = 0, peak = 0;
  (void)bbp_memory(c, &cur, &peak);
  out[5] = (double)peak;
  std::lock_guard<std::mutex> lk(mu);
  if (ok) q.out.swap(out);
  else q.err = why;
  q.ok = ok;
}

// Releases a request's context, stream and budget and publishes its state.
void bbp_server::done(const std::shared_ptr<Request> &q) {
  if (q->c) bbp_destroy(q->c);
  q->c = nullptr;
  if (q->st) (void)hipStreamDestroy(q->st);
  q->st = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu);
    q->t_finish = now();
    if (q->cancelled) q->state = BBP_REQ_CANCELLED;
    else if (!q->ok) q->state = BBP_REQ_FAILED;
    else q->state = BBP_REQ_DONE;
    q->A.clear();
    q->A.shrink_to_fit();
    used -= q->estimate;
    --running;
  }
  cv.notify_all();
}

// Admission and the shared sweeps: between sweeps, queued requests are
// admitted first-in first-out while a slot is free and their estimate fits
// in what the budget leaves; every resident request then takes one more
// synchronous sweep in the shared batches (one launch set per shape for all
// of them); a request whose residual falls below its tolerance, or that has
// made its sweep cap, goes to the finishers, which evaluate its outputs on
// its own stream while the sweeps of the others go on.
void bbp_server::engine_loop() {
  hipStream_t est = nullptr;
  if (hipSetDevice(0) != hipSuccess || hipStreamCreateWithFlags(&est, hipStreamNonBlocking) != hipSuccess)
    est = nullptr;
  bbp::SweepSet *set = bbp::sweepset_create(est);
  if (set) bbp::sweepset_set_allocator(set, cache_alloc, cache_free, &cache);
  std::vector<std::shared_ptr<Request>> resident;
  for (;;) {
    std::vector<std::shared_ptr<Request>> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        return stop || !resident.empty() ||
               (!queue.empty() && running < slots && used + queue.front()->estimate <= budget);
      });
      if (stop) break;
      while (!queue.empty() && running < slots && used + queue.front()->estimate <= budget) {
        std::shared_ptr<Request> q = queue.front();
        queue.pop_front();
        used += q->estimate;
        ++running;
        max_running = std::max(max_running, running);
        q->state = BBP_REQ_RUNNING;
        q->t_admit = now();
        admit.push_back(q);
      }
    }
    const double ta = now();
    for (auto &q : admit) {
      if (setup(*q) && set) {
        resident.push_back(q);
      } else {
        if (!set) {
          std::lock_guard<std::mutex> lk(mu);
          q->err = "no device for the shared sweeps";
        }
        q->ok = false;
        done(q);
      }
    }
    // cancellations take effect before the next sweep
    {
      std::lock_guard<std::mutex> lk(mu);
      t_admit_s += now() - ta;
      for (auto &q : resident) q->cancelled = q->cancel;
    }
    for (auto it = resident.begin(); it != resident.end();) {
      if ((*it)->cancelled) {
        done(*it);
        it = resident.erase(it);
      } else {
        ++it;
      }
    }
    if (resident.empty()) continue;
    std::vector<bbp_ctx *> cs;
    for (auto &q : resident) cs.push_back(q->c);
    std::vector<double> res(cs.size(), 0.0);
    std::vector<bbp_status> st(cs.size(), BBP_OK);
    std::string why;
    const double ts = now();
    bbp_status bs = bbp::sweepset_run(set, cs.data(), (int)cs.size(), res.data(), st.data(), &why);
    {
      std::lock_guard<std::mutex> lk(mu);
      t_sweep += now() - ts;
      ++shared_sweeps;
      request_sweeps += (int64_t)resident.size();
      max_together = std::max(max_together, (int32_t)resident.size());
    }
    std::vector<std::shared_ptr<Request>> keep, finished;
    for (size_t k = 0; k < resident.size(); ++k) {
      auto &q = resident[k];
      if (bs != BBP_OK || st[k] != BBP_OK) {
        std::lock_guard<std::mutex> lk(mu);
        q->err = "shared sweep (status " +
                 std::to_string((int)(bs != BBP_OK ? bs : st[k])) + "): " +
                 (bs != BBP_OK ? why : std::string(bbp_last_error(q->c)));
        q->ok = false;
        finished.push_back(q);
        continue;
      }
      ++q->sweeps;
      q->res = res[k];
      if (q->res < q->r.tol || q->sweeps >= q->r.max_sweeps)
        finished.push_back(q);
      else
        keep.push_back(q);
    }
    resident.swap(keep);
    for (auto &q : finished) {
      if (!q->ok) {
        done(q);
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        finishing.push_back(q);
      }
      cv.notify_all();
    }
  }
  for (auto &q : resident) {
    q->cancelled = true;
    done(q);
  }
  bbp::sweepset_destroy(set);
  if (est) (void)hipStreamDestroy(est);
}

void bbp_server::finisher_loop() {
  for (;;) {
    std::shared_ptr<Request> q;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !finishing.empty(); });
      if (finishing.empty()) return;  // stopping with nothing left to finish
      q = finishing.front();
      finishing.pop_front();
    }
    const double tf = now();
    outputs(*q);
    {
      std::lock_guard<std::mutex> lk(mu);
      t_finish_s += now() - tf;
    }
    done(q);
  }
}

extern "C" {

bbp_status bbp_server_estimate(const bbp_request *r, size_t *bytes) {
  if (!bytes) return BBP_EINVAL;
  bbp_status s = check_request(r);
  if (s != BBP_OK) return s;
  const int D = r->D, K = r->chi, P = D * D;
  const int gx = (r->Lx + r->bx - 1) / r->bx, gy = (r->Ly + r->by - 1) / r->by;
  const int Lm = std::max(r->bx, r->by);
  const size_t S = (size_t)K * P * K;
  const size_t nh = (size_t)(gx - 1) * gy, nv = (size_t)gx * (gy - 1), nm = 2 * (nh + nv);
  size_t dbl = (2 * nm + 1) * Lm * S + nm * ((size_t)K * K + S);
  // sweep batches: horizontal messages absorb bx columns of height by, and
  // vertical ones by columns of height bx
  dbl += 2 * nh * item_doubles(r->bx, r->by, K, D) + 2 * nv * item_doubles(r->by, r->bx, K, D);
  // observables: up to four boundary stacks per region (block or union of
  // two blocks), the line batches, and one chunk of matrix-unit items
  const int Ke = chi_env_of(*r);
  const size_t Se = (size_t)Ke * P * Ke;
  const size_t R = (size_t)gx * gy + nh + nv;
  dbl += 4 * R * item_doubles(2 * Lm, 2 * Lm, Ke, D);
  dbl += 2 * R * item_doubles(1, 2 * Lm, Ke, D);
  dbl += 2 * (2 * R * (2 * (size_t)Lm + 2) * 4) * Se;
  dbl += 256 * (item_doubles(1, 1, Ke, D) + 2 * 2 * (size_t)P * P);
  *bytes = dbl * 8 + ((size_t)64 << 20);
  return BBP_OK;
}

bbp_status bbp_server_create(bbp_server **out, size_t budget_bytes, int32_t max_slots) {
  if (!out || budget_bytes == 0 || max_slots <= 0 || max_slots > 64) return BBP_EINVAL;
  *out = nullptr;
  bbp_server *s = new (std::nothrow) bbp_server;
  if (!s) return BBP_ENOMEM;
  s->budget = budget_bytes;
  s->slots = max_slots;
  s->cache.limit = budget_bytes / 4;
  try {
    s->engine = std::thread([s] { s->engine_loop(); });
    for (int i = 0; i < 3; ++i) s->finishers.emplace_back([s] { s->finisher_loop(); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    if (s->engine.joinable()) s->engine.join();
    for (auto &t : s->finishers) t.join();
    delete s;
    return BBP_ENOMEM;
  }
  *out = s;
  return BBP_OK;
}

bbp_status bbp_server_submit(bbp_server *s, const bbp_request *r, const double *A, size_t n,
                             const double *ops, int64_t *ticket) {
  if (!s || !A || !ticket) return BBP_EINVAL;
  bbp_status st = check_request(r);
  if (st != BBP_OK) return st;
  const size_t nops = ops_len(*r);
  if (nops > 0 && !ops) return BBP_EINVAL;
  for (size_t i = 0; i < nops; ++i)
    if (!std::isfinite(ops[i])) return BBP_EINVAL;
  const size_t need = (size_t)r->Lx * r->Ly * 2 * r->D * r->D * r->D * r->D;
  if (n != need) return BBP_EINVAL;
  size_t est = 0;
  if ((st = bbp_server_estimate(r, &est)) != BBP_OK) return st;
  if (est > s->budget) return BBP_ENOMEM;  // could never be admitted
  std::shared_ptr<Request> q;
  try {
    q = std::make_shared<Request>();
    q->r = *r;
    q->A.assign(A, A + n);
    if (nops) q->ops.assign(ops, ops + nops);
  } catch (...) {
    return BBP_ENOMEM;
  }
  q->estimate = est;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return BBP_ESTATE;
    q->id = s->next_id++;
    q->t_submit = s->now();
    s->queue.push_back(q);
    s->all[q->id] = q;
    *ticket = q->id;
  }
  s->cv.notify_all();
  return BBP_OK;
}

bbp_status bbp_server_poll(bbp_server *s, int64_t ticket, int32_t *state, double *out, size_t n,
                           size_t *needed, double *times) {
  if (!s || !state) return BBP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return BBP_EINVAL;
  const Request &q = *it->second;
  *state = q.state;
  const size_t len = result_len(q.r);
  if (needed) *needed = len;
  if (times) {
    times[0] = q.t_submit;
    times[1] = q.t_admit;
    times[2] = q.t_finish;
  }
  if (q.state == BBP_REQ_DONE && out) {
    if (n < len) return BBP_EINVAL;
    std::memcpy(out, q.out.data(), len * sizeof(double));
  }
  return BBP_OK;
}

bbp_status bbp_server_cancel(bbp_server *s, int64_t ticket) {
  if (!s) return BBP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return BBP_EINVAL;
  Request &q = *it->second;
  q.cancel = true;
  if (q.state == BBP_REQ_QUEUED) {
    for (auto i = s->queue.begin(); i != s->queue.end(); ++i)
      if ((*i)->id == ticket) {
        s->queue.erase(i);
        break;
      }
    q.state = BBP_REQ_CANCELLED;
    q.t_finish = s->now();
  }
  return BBP_OK;
}

bbp_status bbp_server_stats(bbp_server *s, int32_t *running, int32_t *queued,
                            size_t *bytes_in_use, int32_t *max_running) {
  if (!s) return BBP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (running) *running = s->running;
  if (queued) *queued = (int32_t)s->queue.size();
  if (bytes_in_use) *bytes_in_use = s->used;
  if (max_running) *max_running = s->max_running;
  return BBP_OK;
}

bbp_status bbp_server_sweeps(bbp_server *s, int64_t *sweeps, int64_t *request_sweeps,
                             int32_t *max_together, double *busy) {
  if (!s) return BBP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (sweeps) *sweeps = s->shared_sweeps;
  if (request_sweeps) *request_sweeps = s->request_sweeps;
  if (max_together) *max_together = s->max_together;
  if (busy) {
    busy[0] = s->t_sweep;
    busy[1] = s->t_admit_s;
    busy[2] = s->t_finish_s;
  }
  return BBP_OK;
}

const char *bbp_server_error(bbp_server *s, int64_t ticket) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return "unknown ticket";
  return it->second->err.c_str();
}

void bbp_server_destroy(bbp_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto &kv : s->all) kv.second->cancel = true;
    for (auto &q : s->queue) {
      q->state = BBP_REQ_CANCELLED;
      q->t_finish = s->now();
    }
    s->queue.clear();
  }
  s->cv.notify_all();
  if (s->engine.joinable()) s->engine.join();
  for (auto &t : s->finishers) t.join();
  delete s;
}

}  // extern "C"
