// libbbp request server: many block-BP solves (open lattices of different
// size, D and chi) served concurrently on one GPU.
//
// A fixed pool of worker threads takes requests first-in first-out, each only
// once its device-memory estimate fits in what the byte budget leaves free.
// A worker owns one context and one HIP stream per request: it sweeps until
// the message residual is below the request's tolerance (or its sweep cap),
// then evaluates the requested observables (every <sigma_z>, every nearest-
// neighbour <S.S>, the log-norm) and releases the memory.  Requests join and
// leave between sweeps; while several are resident their kernels run
// concurrently on their streams.  No state is shared between requests, so a
// result is the same whether its request ran alone or in a mix.
#include <algorithm>
#include <chrono>
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
  size_t estimate = 0;
  int32_t state = BBP_REQ_QUEUED;
  bool cancel = false;
  std::vector<double> out;
  std::string err;
  double t_submit = 0.0, t_admit = 0.0, t_finish = 0.0;
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

}  // namespace

struct bbp_server {
  size_t budget = 0, used = 0;
  int32_t slots = 1, running = 0, max_running = 0;
  bool stop = false;
  int64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<int64_t, std::shared_ptr<Request>> all;
  std::vector<std::thread> pool;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker();
  void serve(Request &q);
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
  return n;
}

bbp_status check_request(const bbp_request *r) {
  if (!r) return BBP_EINVAL;
  if (r->Lx <= 0 || r->Ly <= 0 || r->bx <= 0 || r->by <= 0 || r->D <= 0 || r->chi <= 0 ||
      r->chi > 128 || r->max_sweeps <= 0 || !(r->tol >= 0.0) ||
      (r->outputs & ~(BBP_OUT_SZ | BBP_OUT_SS | BBP_OUT_LOGNORM)) != 0)
    return BBP_EINVAL;
  return BBP_OK;
}

}  // namespace

void bbp_server::serve(Request &q) {
  const bbp_request &r = q.r;
  std::vector<double> out(result_len(r), 0.0);
  bbp_ctx *c = nullptr;
  hipStream_t st = nullptr;
  auto fail = [&](bbp_status s, const char *what) {
    const char *m = c ? bbp_last_error(c) : "";
    q.err = std::string(what) + " (status " + std::to_string((int)s) + ")" +
            (m && *m ? std::string(": ") + m : std::string());
  };
  bbp_status s = bbp_create(&c, 0, r.Lx, r.Ly, 0, 0, r.bx, r.by, r.D, r.chi);
  bool ok = s == BBP_OK;
  if (!ok) fail(s, "bbp_create");
  // requests overlap on their own streams; each keeps to its one stream
  if (ok && (s = bbp_set_option(c, "lanes", 1)) != BBP_OK) {
    fail(s, "bbp_set_option");
    ok = false;
  }
  if (ok && hipSetDevice(0) == hipSuccess &&
      hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess) {
    (void)bbp_set_stream(c, st);
  } else if (ok) {
    st = nullptr;  // no device: set_tensors reports it below
  }
  if (ok && (s = bbp_set_tensors(c, q.A.data(), q.A.size())) != BBP_OK) {
    fail(s, "bbp_set_tensors");
    ok = false;
  }
  int32_t sweeps = 0;
  double res = 1.0;
  bool cancelled = false;
  while (ok && sweeps < r.max_sweeps) {
    {
      std::lock_guard<std::mutex> lk(mu);
      cancelled = q.cancel;
    }
    if (cancelled) break;
    if ((s = bbp_sweep(c, 1, &res)) != BBP_OK) {
      fail(s, "bbp_sweep");
      ok = false;
      break;
    }
    ++sweeps;
    if (res < r.tol) break;
  }
  size_t o = 6;
  if (ok && !cancelled) {
    out[0] = res < r.tol ? 1.0 : 0.0;
    out[1] = sweeps;
    out[2] = res;
    if (r.outputs & BBP_OUT_SZ) {
      const int64_t n = n_sites(r);
      std::vector<int32_t> xs(n), ys(n);
      for (int y = 0; y < r.Ly; ++y)
        for (int x = 0; x < r.Lx; ++x) {
          xs[(size_t)y * r.Lx + x] = x;
          ys[(size_t)y * r.Lx + x] = y;
        }
      const double sz[4] = {1.0, 0.0, 0.0, -1.0};
      if ((s = bbp_expect_sites(c, (int32_t)n, xs.data(), ys.data(), sz, &out[o])) != BBP_OK) {
        fail(s, "bbp_expect_sites");
        ok = false;
      }
      o += (size_t)n;
    }
    if (ok && (r.outputs & BBP_OUT_SS)) {
      // S.S = (sx sx + sy sy + sz sz) / 4 on (s0, s1), s0 the major index
      const double ss[16] = {0.25, 0, 0, 0, 0, -0.25, 0.5, 0, 0, 0.5, -0.25, 0, 0, 0, 0, 0.25};
      const int64_t n = n_bonds(r);
      std::vector<int32_t> x0, y0, x1, y1;
      for (int y = 0; y < r.Ly; ++y)
        for (int x = 0; x + 1 < r.Lx; ++x) {
          x0.push_back(x); y0.push_back(y); x1.push_back(x + 1); y1.push_back(y);
        }
      for (int y = 0; y + 1 < r.Ly; ++y)
        for (int x = 0; x < r.Lx; ++x) {
          x0.push_back(x); y0.push_back(y); x1.push_back(x); y1.push_back(y + 1);
        }
      if ((s = bbp_expect_bonds(c, (int32_t)n, x0.data(), y0.data(), x1.data(), y1.data(), ss,
                                &out[o])) != BBP_OK) {
        fail(s, "bbp_expect_bonds");
        ok = false;
      }
      o += (size_t)n;
    }
    if (ok && (r.outputs & BBP_OUT_LOGNORM)) {
      int32_t sign = 0;
      if ((s = bbp_log_norm(c, &out[3], &sign)) != BBP_OK) {
        fail(s, "bbp_log_norm");
        ok = false;
      }
      out[4] = sign;
    }
    size_t now = 0, peak = 0;
    (void)bbp_memory(c, &now, &peak);
    out[5] = (double)peak;
  }
  if (c) bbp_destroy(c);
  if (st) (void)hipStreamDestroy(st);
  std::lock_guard<std::mutex> lk(mu);
  q.t_finish = now();
  if (cancelled || (q.cancel && !ok)) {
    q.state = BBP_REQ_CANCELLED;
  } else if (!ok) {
    q.state = BBP_REQ_FAILED;
  } else {
    q.out.swap(out);
    q.state = BBP_REQ_DONE;
  }
  q.A.clear();
  q.A.shrink_to_fit();
}

void bbp_server::worker() {
  for (;;) {
    std::shared_ptr<Request> q;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        return stop || (!queue.empty() && used + queue.front()->estimate <= budget);
      });
      if (stop) return;
      q = queue.front();
      queue.pop_front();
      used += q->estimate;
      ++running;
      max_running = std::max(max_running, running);
      q->state = BBP_REQ_RUNNING;
      q->t_admit = now();
    }
    serve(*q);
    {
      std::lock_guard<std::mutex> lk(mu);
      used -= q->estimate;
      --running;
    }
    cv.notify_all();
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
  const int Ke = std::min(128, 2 * D * D + 10);
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
  try {
    for (int i = 0; i < max_slots; ++i) s->pool.emplace_back([s] { s->worker(); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    for (auto &t : s->pool) t.join();
    delete s;
    return BBP_ENOMEM;
  }
  *out = s;
  return BBP_OK;
}

bbp_status bbp_server_submit(bbp_server *s, const bbp_request *r, const double *A, size_t n,
                             int64_t *ticket) {
  if (!s || !A || !ticket) return BBP_EINVAL;
  bbp_status st = check_request(r);
  if (st != BBP_OK) return st;
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
  for (auto &t : s->pool) t.join();
  delete s;
}

}  // extern "C"
