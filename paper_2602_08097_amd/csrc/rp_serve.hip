// rp_serve.hip -- the request loop of include/rp_serve.h: continuous batching
// of prune sweeps and search batches over HIP streams, pruned graphs in a
// device arena admitted by budget with least-recently-used eviction.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/rp_serve.h"
#include "rp_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

uint32_t gcd_u32(uint32_t a, uint32_t b) {
  while (b) {
    const uint32_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

constexpr size_t kAlign = 256;
constexpr int64_t kMaxReqQueries = 65536;

enum GState { ABSENT = 0, PRUNING = 1, READY = 2 };

struct Graph {
  uint32_t num = 0, den = 0;  // alpha in lowest terms; {0, 0} for the base graph
  int32_t R = 0;
  bool is_base = false;
  GState state = ABSENT;
  size_t off = 0, bytes = 0;  // arena block
  int32_t* nbr = nullptr;
  int32_t* deg = nullptr;
  int users = 0;              // in-flight launches that read or write it
  int64_t wanted = 0;         // pending requests that need it
  uint64_t last_use = 0;
  rp::GraphView view{};
};

struct Req {
  rp_request r{};
  Graph* g = nullptr;
  double t_submit = 0, t_start = 0, t_done = 0;
  int32_t status = RP_OK;
  int32_t batch = 1;
  uint64_t seq = 0;
};

struct Launch {
  int stream = 0;
  hipEvent_t ev = nullptr;
  std::vector<Req*> reqs;
  std::vector<Graph*> graphs;  // users to release at completion
  bool sweep = false;
};

}  // namespace

struct rp_server {
  rp_graph* base = nullptr;
  int device = 0;
  int fifo = 0;  // 0: batching; 1: one request at a time; 2: same, prunes on the plain kernel
  int n_streams = 0;
  int32_t max_batch = 0;
  std::vector<hipStream_t> streams;
  std::vector<bool> busy;           // a launch is in flight on the stream
  std::vector<rp::SearchJob*> jobs_host;  // pinned, per stream
  std::vector<rp::SearchJob*> jobs_dev;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> length
  rp::DevCounters* ctr = nullptr;
  Graph base_graph;
  std::map<uint64_t, Graph*> graphs;     // (num, den, R) -> pruned graph
  uint64_t clock = 0, seq = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> incoming;       // submitted, not yet seen by the worker
  std::deque<Req*> pending;        // seen, not launched (arrival order)
  std::vector<Launch> inflight;
  std::deque<rp_completion> done;
  bool shutdown = false;
  std::thread worker;
  rp_server_stats stats{};
  int64_t unfinished = 0;          // submitted and not completed
};

namespace {

uint64_t graph_key(uint32_t num, uint32_t den, int32_t R) {
  return ((uint64_t)num << 40) | ((uint64_t)den << 20) | (uint64_t)R;
}

size_t graph_bytes(const rp_server* s, int32_t R) {
  const size_t b = (size_t)s->base->view.n * ((size_t)R + 1) * 4;
  return (b + kAlign - 1) & ~(kAlign - 1);
}

// ---- arena (first fit, coalescing) -----------------------------------------

bool arena_alloc(rp_server* s, size_t bytes, size_t* off) {
  for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      s->free_blocks.erase(it);
      if (rest) s->free_blocks[roff] = rest;
      return true;
    }
  }
  return false;
}

void arena_free(rp_server* s, size_t off, size_t bytes) {
  auto it = s->free_blocks.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_blocks.erase(nx);
  }
  if (it != s->free_blocks.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_blocks.erase(it);
    }
  }
}

void evict(rp_server* s, Graph* g) {
  arena_free(s, g->off, g->bytes);
  g->state = ABSENT;
  g->nbr = g->deg = nullptr;
  s->stats.evictions++;
  s->stats.resident_graphs--;
  s->stats.resident_bytes -= (int64_t)g->bytes;
}

// Place g in the arena, evicting idle graphs from the least recently used on
// (in FIFO mode also graphs that only later requests want: they are pruned
// again when their turn comes).
bool admit(rp_server* s, Graph* g) {
  const size_t bytes = graph_bytes(s, g->R);
  size_t off = 0;
  while (!arena_alloc(s, bytes, &off)) {
    Graph* victim = nullptr;
    for (auto& kv : s->graphs) {
      Graph* c = kv.second;
      if (c->state == READY && c->users == 0 && (c->wanted == 0 || s->fifo) && c != g &&
          (!victim || c->last_use < victim->last_use))
        victim = c;
    }
    if (!victim) return false;
    evict(s, victim);
  }
  g->off = off;
  g->bytes = bytes;
  g->nbr = (int32_t*)(s->arena + off);
  g->deg = (int32_t*)(s->arena + off + (size_t)s->base->view.n * g->R * 4);
  g->view = s->base->view;
  g->view.nbr = g->nbr;
  g->view.deg = g->deg;
  g->view.r_max = g->R;
  g->view.frame_e = nullptr;  // the base's exponents belong to the base lists
  s->stats.resident_graphs++;
  s->stats.resident_bytes += (int64_t)bytes;
  return true;
}

void finish(rp_server* s, Req* q, int32_t status, double t_done) {
  q->status = status;
  q->t_done = t_done;
  rp_completion c;
  c.tag = q->r.tag;
  c.status = q->status;
  c.batch = q->batch;
  c.t_submit = q->t_submit;
  c.t_start = q->t_start;
  c.t_done = q->t_done;
  s->done.push_back(c);
  s->unfinished--;
  if (q->g) q->g->wanted--;
  delete q;
}

// ---- launches (worker thread, lock held) -----------------------------------

bool record(rp_server* s, Launch& L) {
  if (hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(L.ev, s->streams[L.stream]) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  s->busy[L.stream] = true;
  s->inflight.push_back(std::move(L));
  return true;
}

void fail_launch(rp_server* s, Launch& L, const char* what) {
  rp::fail(RP_EDEVICE, "%s", what);
  const double t = now_s();
  for (Req* q : L.reqs) finish(s, q, RP_EDEVICE, t);
  for (Graph* g : L.graphs) {
    g->users--;
    if (g->state == PRUNING) {
      evict(s, g);
      s->stats.evictions--;  // not an eviction by budget
    }
  }
}

// Copy a ready graph into a prune request's outputs, on stream `st`.
bool enqueue_copy(rp_server* s, Req* q, hipStream_t st) {
  const size_t n = (size_t)s->base->view.n;
  if (q->r.out_ids &&
      hipMemcpyAsync(q->r.out_ids, q->g->nbr, n * q->g->R * 4, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return false;
  if (q->r.out_hops &&
      hipMemcpyAsync(q->r.out_hops, q->g->deg, n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return false;
  return true;
}

// One sweep over up to kMaxAlphas graphs of the same R (stream 0).
void launch_sweep(rp_server* s, std::vector<Graph*>& gs, std::vector<Req*>& reqs) {
  Launch L;
  L.stream = 0;
  L.sweep = true;
  hipStream_t st = s->streams[0];
  bool okl = true;
  if (s->fifo == 2) {
    Graph* g = gs[0];
    okl = rp::launch_prune_plain(s->base->view, g->num * g->num, g->den * g->den, g->R, g->nbr,
                                 g->deg, s->ctr, st) == hipSuccess;
  } else {
    rp::SweepArgs a = {};
    a.n_alpha = (int32_t)gs.size();
    a.n_out = a.n_alpha;
    for (int i = 0; i < a.n_alpha; ++i) {
      a.num2[i] = gs[i]->num * gs[i]->num;
      a.den2[i] = gs[i]->den * gs[i]->den;
      a.ratio[i] = (double)a.den2[i] / (double)a.num2[i];
      a.out[i] = {gs[i]->nbr, gs[i]->deg, gs[i]->R, i};
    }
    okl = rp::launch_prune_batched(s->base->view, a, s->ctr, st) == hipSuccess;
  }
  const double t = now_s();
  for (Graph* g : gs) {
    g->state = PRUNING;
    g->users++;
    g->last_use = ++s->clock;
    L.graphs.push_back(g);
  }
  for (Req* q : reqs) {
    q->t_start = t;
    q->batch = (int32_t)reqs.size();
    if (okl) okl = enqueue_copy(s, q, st);
    L.reqs.push_back(q);
  }
  s->stats.sweeps++;
  s->stats.swept_alphas += (int64_t)gs.size();
  if (!okl || !record(s, L)) {
    (void)hipGetLastError();
    fail_launch(s, L, "sweep launch failed");
  }
}

// One search launch of the queries of `reqs` (same graph, k, L) on stream si.
void launch_queries(rp_server* s, int si, Graph* g, std::vector<Req*>& reqs) {
  Launch L;
  L.stream = si;
  hipStream_t st = s->streams[si];
  rp::SearchJob* jh = s->jobs_host[si];
  const size_t esz = rp::elem_size(s->base->view.dtype);
  const int d = s->base->view.d;
  int64_t nj = 0;
  const double t = now_s();
  for (Req* q : reqs) {
    const rp_request& r = q->r;
    for (int64_t i = 0; i < r.nq; ++i, ++nj) {
      jh[nj].q = (const char*)r.queries + (size_t)i * d * esz;
      jh[nj].ids = r.out_ids + i * r.k;
      jh[nj].dist = r.out_dist ? r.out_dist + i * r.k : nullptr;
      jh[nj].hops = r.out_hops ? r.out_hops + i : nullptr;
    }
    q->t_start = t;
    q->batch = (int32_t)reqs.size();
    L.reqs.push_back(q);
  }
  g->users++;
  g->last_use = ++s->clock;
  L.graphs.push_back(g);
  const rp_request& r0 = reqs[0]->r;
  bool okl = hipMemcpyAsync(s->jobs_dev[si], jh, nj * sizeof(rp::SearchJob),
                            hipMemcpyHostToDevice, st) == hipSuccess;
  if (okl)
    okl = rp::launch_search_jobs(g->view, s->jobs_dev[si], nj, r0.k, r0.L, st) == hipSuccess;
  s->stats.searches++;
  s->stats.searched_queries += nj;
  if (!okl || !record(s, L)) {
    (void)hipGetLastError();
    fail_launch(s, L, "search launch failed");
  }
}

void retire(rp_server* s) {
  for (size_t i = 0; i < s->inflight.size();) {
    Launch& L = s->inflight[i];
    const hipError_t e = hipEventQuery(L.ev);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    const double t = now_s();
    const int32_t st = e == hipSuccess ? RP_OK : RP_EDEVICE;
    if (e != hipSuccess) (void)hipGetLastError();
    for (Graph* g : L.graphs) {
      g->users--;
      if (g->state == PRUNING) g->state = READY;
    }
    for (Req* q : L.reqs) finish(s, q, st, t);
    (void)hipEventDestroy(L.ev);
    s->busy[L.stream] = false;
    s->inflight.erase(s->inflight.begin() + (long)i);
    s->cv_done.notify_all();
  }
}

// Launch what can run now (lock held).
void schedule(rp_server* s) {
  if (s->fifo) {
    if (!s->inflight.empty() || s->pending.empty()) return;
    Req* q = s->pending.front();
    Graph* g = q->g;
    if (g->state == ABSENT) {
      if (!admit(s, g)) return;  // cannot happen once the arena is idle
      std::vector<Graph*> gs{g};
      std::vector<Req*> rs;
      if (q->r.type == RP_REQ_PRUNE) {
        s->pending.pop_front();
        rs.push_back(q);
      }
      launch_sweep(s, gs, rs);
      return;
    }
    s->pending.pop_front();
    std::vector<Req*> rs{q};
    if (q->r.type == RP_REQ_PRUNE) {
      Launch L;
      L.stream = 0;
      q->t_start = now_s();
      L.reqs.push_back(q);
      g->users++;
      L.graphs.push_back(g);
      if (!enqueue_copy(s, q, s->streams[0]) || !record(s, L)) {
        (void)hipGetLastError();
        fail_launch(s, L, "copy failed");
      }
    } else {
      launch_queries(s, 1, g, rs);
    }
    return;
  }

  // prune requests whose graph is resident: copy on the sweep stream
  if (!s->busy[0]) {
    std::vector<Req*> copies;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
      Req* q = *it;
      if (q->r.type == RP_REQ_PRUNE && q->g->state == READY) {
        copies.push_back(q);
        it = s->pending.erase(it);
      } else {
        ++it;
      }
    }
    if (!copies.empty()) {
      Launch L;
      L.stream = 0;
      const double t = now_s();
      bool okl = true;
      for (Req* q : copies) {
        q->t_start = t;
        q->batch = (int32_t)copies.size();
        if (okl) okl = enqueue_copy(s, q, s->streams[0]);
        L.reqs.push_back(q);
        q->g->users++;
        q->g->last_use = ++s->clock;
        L.graphs.push_back(q->g);
      }
      if (!okl || !record(s, L)) {
        (void)hipGetLastError();
        fail_launch(s, L, "copy failed");
      }
    }
  }

  // graphs needed by pending requests: one sweep of up to 8 alphas, same R,
  // oldest need first
  if (!s->busy[0]) {
    std::vector<Graph*> gs;
    int32_t R = -1;
    for (Req* q : s->pending) {
      Graph* g = q->g;
      if (g->state != ABSENT || g->is_base) continue;
      if (R < 0) R = g->R;
      if (g->R != R || std::find(gs.begin(), gs.end(), g) != gs.end()) continue;
      if (!admit(s, g)) break;
      gs.push_back(g);
      if ((int)gs.size() == rp::kMaxAlphas) break;
    }
    if (!gs.empty()) {
      std::vector<Req*> rs;
      for (auto it = s->pending.begin(); it != s->pending.end();) {
        Req* q = *it;
        if (q->r.type == RP_REQ_PRUNE && std::find(gs.begin(), gs.end(), q->g) != gs.end()) {
          rs.push_back(q);
          it = s->pending.erase(it);
        } else {
          ++it;
        }
      }
      launch_sweep(s, gs, rs);
    }
  }

  // query batches on every idle query stream
  for (int si = 1; si < s->n_streams; ++si) {
    if (s->busy[si]) continue;
    Req* first = nullptr;
    for (Req* q : s->pending)
      if (q->r.type == RP_REQ_QUERY && q->g->state == READY) {
        first = q;
        break;
      }
    if (!first) break;
    std::vector<Req*> rs;
    int64_t nq = 0;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
      Req* q = *it;
      if (q->r.type == RP_REQ_QUERY && q->g == first->g && q->r.k == first->r.k &&
          q->r.L == first->r.L && (rs.empty() || nq + q->r.nq <= s->max_batch)) {
        rs.push_back(q);
        nq += q->r.nq;
        it = s->pending.erase(it);
      } else {
        ++it;
      }
    }
    launch_queries(s, si, first->g, rs);
  }
}

void worker_main(rp_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->incoming.empty() && !s->shutdown) {
      if (s->inflight.empty())
        s->cv_work.wait(lk, [&] { return !s->incoming.empty() || s->shutdown; });
      else
        s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
    while (!s->incoming.empty()) {
      s->pending.push_back(s->incoming.front());
      s->incoming.pop_front();
    }
    retire(s);
    schedule(s);
    if (s->shutdown && s->pending.empty() && s->inflight.empty() && s->incoming.empty()) break;
  }
}

rp_status check_request(const rp_server* s, const rp_request* r) {
  const rp::GraphView& v = s->base->view;
  const bool on_base = r->type == RP_REQ_QUERY && r->alpha.num == 0 && r->alpha.den == 0;
  if (r->type != RP_REQ_PRUNE && r->type != RP_REQ_QUERY)
    return rp::fail(RP_EINVAL, "unknown request type %d", r->type);
  if (!on_base) {
    rp_status st = rp::check_alpha(r->alpha);
    if (st != RP_OK) return st;
    if (r->R < 1 || r->R > v.r_max)
      return rp::fail(RP_EINVAL, "R must be in [1, %d] (got %d)", v.r_max, r->R);
    if (graph_bytes(s, r->R) > s->arena_bytes)
      return rp::fail(RP_ENOMEM, "a graph with R=%d does not fit the budget", r->R);
  }
  if (r->type == RP_REQ_PRUNE) {
    if (r->out_ids && !rp::device_range(r->out_ids, (size_t)v.n * r->R * 4))
      return rp::fail(RP_EINVAL, "out_ids is not a device array of n*R int32");
    if (r->out_hops && !rp::device_range(r->out_hops, (size_t)v.n * 4))
      return rp::fail(RP_EINVAL, "out_hops is not a device array of n int32");
    return RP_OK;
  }
  if (r->nq < 1 || r->nq > kMaxReqQueries)
    return rp::fail(RP_EINVAL, "nq must be in [1, %lld]", (long long)kMaxReqQueries);
  if (r->k < 1 || r->L < r->k || r->L > rp::kMaxL)
    return rp::fail(RP_EINVAL, "need 1 <= k <= L <= %d", rp::kMaxL);
  if (!rp::device_range(r->queries, (size_t)r->nq * v.d * rp::elem_size(v.dtype)))
    return rp::fail(RP_EINVAL, "queries is not a device array of nq*d elements");
  if (!rp::device_range(r->out_ids, (size_t)r->nq * r->k * 4))
    return rp::fail(RP_EINVAL, "out_ids is not a device array of nq*k int32");
  if (r->out_dist && !rp::device_range(r->out_dist, (size_t)r->nq * r->k * 8))
    return rp::fail(RP_EINVAL, "out_dist is not a device array of nq*k double");
  if (r->out_hops && !rp::device_range(r->out_hops, (size_t)r->nq * 4))
    return rp::fail(RP_EINVAL, "out_hops is not a device array of nq int32");
  return RP_OK;
}

}  // namespace

extern "C" {

rp_status rp_server_create(rp_graph_t base, int64_t budget_bytes, int32_t n_streams,
                           int32_t max_query_batch, int32_t fifo, rp_server_t* out) {
  if (!out) return rp::fail(RP_EINVAL, "out is null");
  *out = nullptr;
  if (!base) return rp::fail(RP_ESTATE, "base is null");
  if (base->base) return rp::fail(RP_EINVAL, "the server needs a base handle, not a derived one");
  if (n_streams < 2 || n_streams > 8) return rp::fail(RP_EINVAL, "n_streams must be in [2, 8]");
  if (max_query_batch < 1 || max_query_batch > kMaxReqQueries)
    return rp::fail(RP_EINVAL, "max_query_batch must be in [1, %lld]", (long long)kMaxReqQueries);
  if (budget_bytes < (int64_t)kAlign) return rp::fail(RP_EINVAL, "budget_bytes too small");
  if (fifo < 0 || fifo > 2) return rp::fail(RP_EINVAL, "fifo must be 0, 1 or 2");
  rp_server* s = new (std::nothrow) rp_server();
  if (!s) return rp::fail(RP_ENOMEM, "host allocation failed");
  s->base = base;
  s->device = base->device;
  s->fifo = fifo;
  s->n_streams = n_streams;
  s->max_batch = max_query_batch;
  s->arena_bytes = (size_t)budget_bytes & ~(kAlign - 1);
  auto cleanup = [&](rp_status st, const char* what) {
    (void)hipGetLastError();
    for (hipStream_t st_ : s->streams) (void)hipStreamDestroy(st_);
    for (auto* p : s->jobs_host) (void)hipHostFree(p);
    for (auto* p : s->jobs_dev) (void)hipFree(p);
    if (s->arena) (void)hipFree(s->arena);
    if (s->ctr) (void)hipFree(s->ctr);
    delete s;
    return rp::fail(st, "%s", what);
  };
  if (hipSetDevice(s->device) != hipSuccess) return cleanup(RP_EDEVICE, "hipSetDevice failed");
  if (hipMalloc((void**)&s->arena, s->arena_bytes) != hipSuccess)
    return cleanup(RP_ENOMEM, "hipMalloc of the graph arena failed");
  if (hipMalloc((void**)&s->ctr, sizeof(rp::DevCounters)) != hipSuccess ||
      hipMemset(s->ctr, 0, sizeof(rp::DevCounters)) != hipSuccess)
    return cleanup(RP_ENOMEM, "hipMalloc of counters failed");
  s->free_blocks[0] = s->arena_bytes;
  for (int i = 0; i < n_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      return cleanup(RP_EDEVICE, "hipStreamCreate failed");
    s->streams.push_back(st);
    s->busy.push_back(false);
    rp::SearchJob* h = nullptr;
    rp::SearchJob* d = nullptr;
    const size_t jb = (size_t)kMaxReqQueries * sizeof(rp::SearchJob);
    if (hipHostMalloc((void**)&h, jb, hipHostMallocDefault) != hipSuccess)
      return cleanup(RP_ENOMEM, "hipHostMalloc of job descriptors failed");
    s->jobs_host.push_back(h);
    if (hipMalloc((void**)&d, jb) != hipSuccess)
      return cleanup(RP_ENOMEM, "hipMalloc of job descriptors failed");
    s->jobs_dev.push_back(d);
  }
  s->base_graph.is_base = true;
  s->base_graph.state = READY;
  s->base_graph.R = base->view.r_max;
  s->base_graph.nbr = (int32_t*)base->view.nbr;
  s->base_graph.deg = (int32_t*)base->view.deg;
  s->base_graph.view = base->view;
  s->worker = std::thread(worker_main, s);
  *out = s;
  return rp::ok();
}

rp_status rp_server_submit(rp_server_t s, const rp_request* req) {
  if (!s) return rp::fail(RP_ESTATE, "server is null");
  if (!req) return rp::fail(RP_EINVAL, "request is null");
  rp_status st = check_request(s, req);
  if (st != RP_OK) return st;
  Req* q = new (std::nothrow) Req();
  if (!q) return rp::fail(RP_ENOMEM, "host allocation failed");
  q->r = *req;
  q->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->shutdown) {
      delete q;
      return rp::fail(RP_ESTATE, "server is shutting down");
    }
    if (req->type == RP_REQ_QUERY && req->alpha.num == 0 && req->alpha.den == 0) {
      q->g = &s->base_graph;
    } else {
      const uint32_t gd = gcd_u32((uint32_t)req->alpha.num, (uint32_t)req->alpha.den);
      const uint32_t num = (uint32_t)req->alpha.num / gd, den = (uint32_t)req->alpha.den / gd;
      const uint64_t key = graph_key(num, den, req->R);
      auto it = s->graphs.find(key);
      if (it == s->graphs.end()) {
        Graph* g = new Graph();
        g->num = num;
        g->den = den;
        g->R = req->R;
        it = s->graphs.emplace(key, g).first;
      }
      q->g = it->second;
    }
    q->g->wanted++;
    q->seq = ++s->seq;
    s->unfinished++;
    s->incoming.push_back(q);
  }
  s->cv_work.notify_one();
  return rp::ok();
}

int32_t rp_server_poll(rp_server_t s, rp_completion* out, int32_t max, int32_t wait_ms) {
  if (!s || !out) return -1;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
  int32_t n = 0;
  while (n < max && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.pop_front();
  }
  return n;
}

rp_status rp_server_replay(rp_server_t s, const rp_request* reqs, const double* arrival_s,
                           int32_t n, rp_completion* out) {
  if (!s) return rp::fail(RP_ESTATE, "server is null");
  if (n < 0 || (n > 0 && (!reqs || !arrival_s || !out))) return rp::fail(RP_EINVAL, "bad arrays");
  for (int32_t i = 0; i < n; ++i) {
    rp_status st = check_request(s, &reqs[i]);
    if (st != RP_OK) return st;
  }
  std::vector<int64_t> tags(n);
  const double t0 = now_s();
  for (int32_t i = 0; i < n; ++i) {
    const double due = t0 + arrival_s[i];
    double t = now_s();
    if (due - t > 2e-3)
      std::this_thread::sleep_for(std::chrono::duration<double>(due - t - 1e-3));
    while (now_s() < due) {
    }
    rp_request r = reqs[i];
    r.tag = i;
    rp_status st = rp_server_submit(s, &r);
    if (st != RP_OK) return st;
  }
  int32_t got = 0;
  std::vector<rp_completion> buf(256);
  while (got < n) {
    const int32_t m = rp_server_poll(s, buf.data(), (int32_t)buf.size(), 100);
    for (int32_t j = 0; j < m; ++j) {
      const int64_t i = buf[j].tag;
      if (i < 0 || i >= n) continue;
      out[i] = buf[j];
      out[i].tag = reqs[i].tag;
      ++got;
    }
  }
  return rp::ok();
}

rp_status rp_server_stats_get(rp_server_t s, rp_server_stats* out) {
  if (!s) return rp::fail(RP_ESTATE, "server is null");
  if (!out) return rp::fail(RP_EINVAL, "out is null");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return rp::ok();
}

void rp_server_destroy(rp_server_t s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->shutdown = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto* p : s->jobs_host) (void)hipHostFree(p);
  for (auto* p : s->jobs_dev) (void)hipFree(p);
  (void)hipFree(s->arena);
  (void)hipFree(s->ctr);
  for (auto& kv : s->graphs) delete kv.second;
  for (Req* q : s->pending) delete q;
  delete s;
}

}  // extern "C"
