// rp_api.hip -- the C-ABI (include/rp.h): argument checks, handle lifetime,
// dispatch to the kernels.  Every device array is checked on the host to lie
// inside a device allocation large enough for the sizes given, so that a
// wrong size or a host pointer becomes RP_EINVAL instead of a GPU fault.
#include <algorithm>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "rp_internal.h"

namespace rp {

namespace {
thread_local char g_err[512];
}  // namespace

rp_status fail(rp_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

rp_status ok() {
  g_err[0] = 0;
  return RP_OK;
}

const char* last_error() { return g_err; }

// Is [p, p + bytes) inside one device allocation?
bool device_range(const void* p, size_t bytes) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return false;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const char* b = (const char*)base;
  const char* q = (const char*)p;
  return q >= b && (size_t)(q - b) + bytes <= size;
}

size_t elem_size(int32_t dt) { return dt == RP_U8 ? 1 : 4; }

rp_status check_alpha(rp_alpha a) {
  if (a.den < 1 || a.num < a.den || a.num > 65535)
    return fail(RP_EINVAL, "alpha must be num/den with 1 <= den <= num <= 65535 (got %d/%d)",
                a.num, a.den);
  return RP_OK;
}

}  // namespace rp

using rp::check_alpha;
using rp::device_range;
using rp::elem_size;
using rp::fail;
using rp::ok;

namespace {

rp_status check_launch(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(RP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return RP_OK;
}

rp_status validate_adjacency(const rp::GraphView& v, rp::DevCounters* ctr, hipStream_t s) {
  if (!device_range(v.nbr, (size_t)v.n * v.r_max * 4))
    return fail(RP_EINVAL, "nbr is not a device array of n*r_max int32");
  if (!device_range(v.deg, (size_t)v.n * 4))
    return fail(RP_EINVAL, "deg is not a device array of n int32");
  rp::DevCounters zero = {};
  hipError_t e = hipMemcpyAsync(ctr, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return check_launch(e, "counter reset");
  rp_status st = check_launch(rp::launch_validate(v, ctr, s), "validate");
  if (st != RP_OK) return st;
  rp::DevCounters host = {};
  e = hipMemcpyAsync(&host, ctr, sizeof(host), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return check_launch(e, "validate readback");
  // leave the counters at zero for the graph's own use
  e = hipMemcpyAsync(ctr, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return check_launch(e, "counter reset");
  if (host.errors)
    return fail(RP_ERANGE, "%llu vertices have a degree outside [0, r_max] or an id outside [0, n)",
                (unsigned long long)host.errors);
  return RP_OK;
}

// The per-point max |x_k| of a float32 point set; a point with a NaN or
// infinite coordinate makes the load fail (synchronous: reads the count back).
rp_status add_maxabs(rp_graph* g, hipStream_t s) {
  rp_status st =
      check_launch(rp::launch_maxabs_f32(g->view, (float*)g->aux, g->ctr, s), "maxabs");
  if (st != RP_OK) return st;
  rp::DevCounters host = {}, zero = {};
  hipError_t e = hipMemcpyAsync(&host, g->ctr, sizeof(host), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->ctr, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return check_launch(e, "maxabs readback");
  if (host.errors)
    return fail(RP_EINVAL, "%llu points have a NaN or infinite coordinate",
                (unsigned long long)host.errors);
  return RP_OK;
}

// Float32 graphs that the batched prune serves (lists of at most 128 ids) get
// the frame exponent of every vertex once, so a sweep reads one byte per
// vertex instead of max|x| of every candidate.
rp_status add_frame_exponents(rp_graph* g, hipStream_t stream) {
  g->frame_e = nullptr;
  if (g->view.dtype != RP_F32 || !rp::prune_f32_shape_ok(g->view)) return RP_OK;
  if (hipMalloc(&g->frame_e, (size_t)g->view.n) != hipSuccess) {
    (void)hipGetLastError();
    g->frame_e = nullptr;
    return fail(RP_ENOMEM, "hipMalloc of the frame exponents failed");
  }
  rp_status st = check_launch(
      rp::launch_frame_exponents_f32(g->view, (int8_t*)g->frame_e, stream), "frame exponents");
  if (st == RP_OK) g->view.frame_e = (const int8_t*)g->frame_e;
  return st;
}

rp_status check_outputs(const rp_graph* g, int32_t R, const int32_t* out_nbr,
                        const int32_t* out_deg) {
  if (R < 1) return fail(RP_EINVAL, "R must be >= 1 (got %d)", R);
  if (!device_range(out_nbr, (size_t)g->view.n * R * 4))
    return fail(RP_EINVAL, "out_nbr is not a device array of n*R int32");
  if (!device_range(out_deg, (size_t)g->view.n * 4))
    return fail(RP_EINVAL, "out_deg is not a device array of n int32");
  const char* a = (const char*)out_nbr;
  const char* b = (const char*)g->view.nbr;
  size_t la = (size_t)g->view.n * R * 4, lb = (size_t)g->view.n * g->view.r_max * 4;
  if (a < b + lb && b < a + la) return fail(RP_EINVAL, "out_nbr overlaps the graph's nbr");
  return RP_OK;
}

}  // namespace

namespace rp {

// Argument checks shared by the K-NN entry points.
rp_status knn_args(const uint8_t* points, int64_t n, int32_t d, const int32_t* query_ids,
                   int64_t nq, const int32_t* cand_ids, int64_t nc, int32_t K,
                   const int32_t* out_ids) {
  if (n < 1 || n >= (1ll << 31)) return fail(RP_EINVAL, "n must be in [1, 2^31)");
  if (!rp::knn_u8_supported(d))
    return fail(RP_EINVAL, "d must be a multiple of 16 in [16, 256] (got %d)", d);
  if (K < 1 || K > 128) return fail(RP_EINVAL, "K must be in [1, 128] (got %d)", K);
  if (nq < 0 || nq >= (1ll << 31) || nc < 0 || nc >= (1ll << 31))
    return fail(RP_EINVAL, "nq and nc must be in [0, 2^31)");
  if (!query_ids && nq > n) return fail(RP_EINVAL, "nq > n without query_ids");
  if (!cand_ids && nc > n) return fail(RP_EINVAL, "nc > n without cand_ids");
  if (!device_range(points, (size_t)n * d)) return fail(RP_EINVAL, "points is not a device array of n*d bytes");
  if (((uintptr_t)points & 15) != 0) return fail(RP_EINVAL, "points must be 16-byte aligned");
  if (nq == 0) return RP_OK;
  if (query_ids && !device_range(query_ids, (size_t)nq * 4))
    return fail(RP_EINVAL, "query_ids is not a device array of nq int32");
  if (cand_ids && nc > 0 && !device_range(cand_ids, (size_t)nc * 4))
    return fail(RP_EINVAL, "cand_ids is not a device array of nc int32");
  if (!device_range(out_ids, (size_t)nq * K * 4))
    return fail(RP_EINVAL, "out_ids is not a device array of nq*K int32");
  return RP_OK;
}

}  // namespace rp

extern "C" {

const char* rp_last_error(void) { return rp::last_error(); }

rp_status rp_load_graph(const void* points, int32_t dtype, int64_t n, int32_t d,
                        const int32_t* nbr, const int32_t* deg, int32_t r_max, int32_t start,
                        void* stream, rp_graph_t* out) {
  if (!out) return fail(RP_EINVAL, "out is null");
  *out = nullptr;
  if (dtype != RP_U8 && dtype != RP_F32) return fail(RP_EINVAL, "dtype must be RP_U8 or RP_F32");
  if (n < 1 || n >= (1ll << 31)) return fail(RP_EINVAL, "n must be in [1, 2^31)");
  if (d < 1 || d > rp::kMaxDim) return fail(RP_EINVAL, "d must be in [1, %d]", rp::kMaxDim);
  if (r_max < 1 || r_max > rp::kMaxRmax)
    return fail(RP_EINVAL, "r_max must be in [1, %d]", rp::kMaxRmax);
  if (start < 0 || (int64_t)start >= n) return fail(RP_ERANGE, "start outside [0, n)");
  if (!device_range(points, (size_t)n * d * elem_size(dtype)))
    return fail(RP_EINVAL, "points is not a device array of n*d elements");
  rp_graph* g = new (std::nothrow) rp_graph();
  if (!g) return fail(RP_ENOMEM, "host allocation failed");
  g->view = {points, dtype, n, d, nbr, deg, r_max, start, nullptr, nullptr, nullptr};
  g->base = nullptr;
  g->aux = nullptr;
  if (hipGetDevice(&g->device) != hipSuccess) {
    delete g;
    return fail(RP_EDEVICE, "hipGetDevice failed");
  }
  if (hipMalloc((void**)&g->ctr, sizeof(rp::DevCounters)) != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    return fail(RP_ENOMEM, "hipMalloc of counters failed");
  }
  rp_status st = validate_adjacency(g->view, g->ctr, (hipStream_t)stream);
  if (st == RP_OK) {
    if (hipMalloc(&g->aux, (size_t)n * 4) != hipSuccess) {
      (void)hipGetLastError();
      g->aux = nullptr;
      st = fail(RP_ENOMEM, "hipMalloc of the per-point array failed");
    } else if (dtype == RP_U8) {
      g->view.norms = (const uint32_t*)g->aux;
      st = check_launch(rp::launch_norms_u8(g->view, (uint32_t*)g->aux, (hipStream_t)stream),
                        "norms");
    } else {
      g->view.maxabs = (const float*)g->aux;
      st = add_maxabs(g, (hipStream_t)stream);
      if (st == RP_OK) st = add_frame_exponents(g, (hipStream_t)stream);
    }
  }
  // the per-point arrays are complete when the call returns, so work on any
  // other stream (a server's) may read them
  if (st == RP_OK) st = check_launch(hipStreamSynchronize((hipStream_t)stream), "load sync");
  if (st != RP_OK) {
    if (g->frame_e) (void)hipFree(g->frame_e);
    if (g->aux) (void)hipFree(g->aux);
    (void)hipFree(g->ctr);
    delete g;
    return st;
  }
  *out = g;
  return ok();
}

rp_status rp_graph_derive(rp_graph_t base, const int32_t* nbr, const int32_t* deg, int32_t r_max,
                          void* stream, rp_graph_t* out) {
  if (!out) return fail(RP_EINVAL, "out is null");
  *out = nullptr;
  if (!base) return fail(RP_ESTATE, "base is null");
  if (r_max < 1 || r_max > rp::kMaxRmax)
    return fail(RP_EINVAL, "r_max must be in [1, %d]", rp::kMaxRmax);
  rp_graph* g = new (std::nothrow) rp_graph();
  if (!g) return fail(RP_ENOMEM, "host allocation failed");
  g->view = base->view;
  g->view.nbr = nbr;
  g->view.deg = deg;
  g->view.r_max = r_max;
  g->base = base;
  g->device = base->device;
  g->aux = nullptr;  // the view points at the base's per-point array
  if (hipMalloc((void**)&g->ctr, sizeof(rp::DevCounters)) != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    return fail(RP_ENOMEM, "hipMalloc of counters failed");
  }
  g->view.frame_e = nullptr;
  g->frame_e = nullptr;
  rp_status st = validate_adjacency(g->view, g->ctr, (hipStream_t)stream);
  if (st == RP_OK) st = add_frame_exponents(g, (hipStream_t)stream);
  if (st == RP_OK) st = check_launch(hipStreamSynchronize((hipStream_t)stream), "derive sync");
  if (st != RP_OK) {
    if (g->frame_e) (void)hipFree(g->frame_e);
    (void)hipFree(g->ctr);
    delete g;
    return st;
  }
  *out = g;
  return ok();
}

rp_status rp_prune_plain(rp_graph_t g, rp_alpha alpha, int32_t R, int32_t* out_nbr,
                         int32_t* out_deg, void* stream) {
  if (!g) return fail(RP_ESTATE, "graph is null");
  rp_status st = check_alpha(alpha);
  if (st != RP_OK) return st;
  st = check_outputs(g, R, out_nbr, out_deg);
  if (st != RP_OK) return st;
  st = check_launch(rp::launch_prune_plain(g->view, (uint32_t)alpha.num * alpha.num,
                                           (uint32_t)alpha.den * alpha.den, R, out_nbr, out_deg,
                                           g->ctr, (hipStream_t)stream),
                    "prune_plain");
  if (st != RP_OK) return st;
  g->nodes += g->view.n;
  return ok();
}

struct rp_plan {
  rp_graph* g;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int64_t nodes;  // vertex-prunes per launch
};

namespace {

rp_status sweep_args(rp_graph_t g, const rp_alpha* alphas, int32_t n_a, const int32_t* Rs,
                     int32_t n_R, int32_t* const* out_nbr, int32_t* const* out_deg,
                     rp::SweepArgs* a_out, bool unsorted = false) {
  if (!g) return fail(RP_ESTATE, "graph is null");
  if (!alphas || !Rs || !out_nbr || !out_deg) return fail(RP_EINVAL, "null host array");
  if (n_a < 1 || n_a > rp::kMaxAlphas)
    return fail(RP_EINVAL, "n_a must be in [1, %d]", rp::kMaxAlphas);
  if (n_R < 1 || n_R > rp::kMaxRs) return fail(RP_EINVAL, "n_R must be in [1, %d]", rp::kMaxRs);
  rp::SweepArgs a = {};
  a.n_alpha = n_a;
  a.n_out = n_a * n_R;
  a.unsorted = unsorted ? 1 : 0;
  for (int i = 0; i < n_a; ++i) {
    rp_status st = check_alpha(alphas[i]);
    if (st != RP_OK) return st;
    a.num2[i] = (uint32_t)alphas[i].num * alphas[i].num;
    a.den2[i] = (uint32_t)alphas[i].den * alphas[i].den;
    a.ratio[i] = (double)a.den2[i] / (double)a.num2[i];
  }
  for (int ia = 0; ia < n_a; ++ia)
    for (int ir = 0; ir < n_R; ++ir) {
      const int o = ia * n_R + ir;
      rp_status st = check_outputs(g, Rs[ir], out_nbr[o], out_deg[o]);
      if (st != RP_OK) return st;
      a.out[o] = {out_nbr[o], out_deg[o], Rs[ir], ia};
    }
  *a_out = a;
  return RP_OK;
}

}  // namespace

rp_status rp_plan_sweep(rp_graph_t g, const rp_alpha* alphas, int32_t n_a, const int32_t* Rs,
                        int32_t n_R, int32_t* const* out_nbr, int32_t* const* out_deg,
                        void* stream, rp_plan_t* out) {
  if (!out) return fail(RP_EINVAL, "out is null");
  *out = nullptr;
  rp::SweepArgs a;
  rp_status st = sweep_args(g, alphas, n_a, Rs, n_R, out_nbr, out_deg, &a);
  if (st != RP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(RP_EINVAL, "capture needs a non-default stream");
  rp_plan* p = new (std::nothrow) rp_plan();
  if (!p) return fail(RP_ENOMEM, "host allocation failed");
  p->g = g;
  p->nodes = g->view.n * a.n_out;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = rp::launch_prune_batched(g->view, a, g->ctr, s);
    e = hipStreamEndCapture(s, &p->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return fail(RP_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  }
  *out = p;
  return ok();
}

rp_status rp_plan_launch(rp_plan_t p, void* stream) {
  if (!p) return fail(RP_ESTATE, "plan is null");
  rp_status st = check_launch(hipGraphLaunch(p->exec, (hipStream_t)stream), "graph launch");
  if (st != RP_OK) return st;
  p->g->nodes += p->nodes;
  return ok();
}

void rp_plan_free(rp_plan_t p) {
  if (!p) return;
  (void)hipGraphExecDestroy(p->exec);
  (void)hipGraphDestroy(p->graph);
  delete p;
}

rp_status rp_gram_error(rp_graph_t g, const int32_t* nodes, int64_t n_nodes, double* out,
                        void* stream) {
  if (!g) return fail(RP_ESTATE, "graph is null");
  if (!out) return fail(RP_EINVAL, "out is null");
  const rp::GraphView& v = g->view;
  if (v.dtype != RP_F32 || !rp::prune_f32_supported(v))
    return fail(RP_EINVAL, "needs a float32 graph that the batched kernel serves");
  if (n_nodes < 0 || n_nodes >= (1ll << 31)) return fail(RP_EINVAL, "bad n_nodes");
  for (int i = 0; i < 4; ++i) out[i] = 0.0;
  if (n_nodes == 0) return ok();
  if (!device_range(nodes, (size_t)n_nodes * 4))
    return fail(RP_EINVAL, "nodes is not a device array of n_nodes int32");
  hipStream_t s = (hipStream_t)stream;
  rp::GramErrorStats* d = nullptr;
  if (hipMalloc((void**)&d, sizeof(*d)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RP_ENOMEM, "hipMalloc failed");
  }
  rp::GramErrorStats h = {};
  hipError_t e = hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = rp::launch_gram_error_f32(v, nodes, n_nodes, d, g->ctr, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) return check_launch(e, "gram error");
  out[0] = h.max_rel;
  out[1] = h.pairs ? h.sum_rel / (double)h.pairs : 0.0;
  out[2] = (double)h.pairs;
  out[3] = h.max_band;
  return ok();
}

rp_status rp_tune_set(rp_graph_t g, int32_t n_a, int32_t n_R, int32_t waves) {
  if (!g) return fail(RP_ESTATE, "graph is null");
  if (n_a < 1 || n_a > rp::kMaxAlphas || n_R < 1 || n_R > rp::kMaxRs)
    return fail(RP_EINVAL, "bad sweep shape");
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(RP_EINVAL, "waves must be 0, 1, 2, 4 or 8");
  const rp::GraphView& v = g->view;
  rp::set_tuned_waves(rp::TuneKey{rp::batched_kernel(v), v.dtype, v.d, v.r_max, n_a, n_a * n_R},
                      waves);
  return ok();
}

rp_status rp_tune_get(rp_graph_t g, int32_t n_a, int32_t n_R, int32_t* waves) {
  if (!g) return fail(RP_ESTATE, "graph is null");
  if (!waves) return fail(RP_EINVAL, "waves is null");
  const rp::GraphView& v = g->view;
  *waves = rp::tuned_waves(
      rp::TuneKey{rp::batched_kernel(v), v.dtype, v.d, v.r_max, n_a, n_a * n_R});
  return ok();
}

rp_status rp_autotune_sweep(rp_graph_t g, const rp_alpha* alphas, int32_t n_a, const int32_t* Rs,
                            int32_t n_R, int32_t* const* out_nbr, int32_t* const* out_deg,
                            void* stream, int32_t* waves, float* ms) {
  if (!waves) return fail(RP_EINVAL, "waves is null");
  rp::SweepArgs a;
  rp_status st = sweep_args(g, alphas, n_a, Rs, n_R, out_nbr, out_deg, &a);
  if (st != RP_OK) return st;
  const rp::GraphView& v = g->view;
  const rp::TuneKey key{rp::batched_kernel(v), v.dtype, v.d, v.r_max, n_a, a.n_out};
  hipStream_t s = (hipStream_t)stream;
  static const int kCand[4] = {1, 2, 4, 8};
  if (ms)
    for (int i = 0; i < 4; ++i) ms[i] = 0.f;
  if (key.kernel == 0) {
    *waves = 1;
    return check_launch(rp::launch_prune_batched(v, a, g->ctr, s), "prune_batched") == RP_OK
               ? ok()
               : RP_EDEVICE;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return check_launch(hipGetLastError(), "event create");
  int best = 1;
  float best_ms = 0.f;
  int64_t launches = 0;
  const int before = rp::tuned_waves(key);
  hipError_t err = hipSuccess;
  for (int c = 0; c < 4 && err == hipSuccess; ++c) {
    const int w = kCand[c];
    if ((size_t)w * rp::batched_wave_lds(v) > (size_t)rp::max_lds_per_group()) continue;
    rp::set_tuned_waves(key, w);
    float t[3];
    err = rp::launch_prune_batched(v, a, g->ctr, s);  // warm-up
    ++launches;
    for (int r = 0; r < 3 && err == hipSuccess; ++r) {
      err = hipEventRecord(e0, s);
      ++launches;
      if (err == hipSuccess) err = rp::launch_prune_batched(v, a, g->ctr, s);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      if (err == hipSuccess) err = hipEventElapsedTime(&t[r], e0, e1);
    }
    if (err != hipSuccess) break;
    std::sort(t, t + 3);
    if (ms) ms[c] = t[1];
    if (c == 0 || t[1] < best_ms) {
      best = w;
      best_ms = t[1];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) {
    rp::set_tuned_waves(key, before);
    return check_launch(err, "autotune");
  }
  rp::set_tuned_waves(key, best);
  // the outputs end with the chosen configuration's result
  st = check_launch(rp::launch_prune_batched(v, a, g->ctr, s), "prune_batched");
  if (st == RP_OK) st = check_launch(hipStreamSynchronize(s), "autotune sync");
  if (st != RP_OK) return st;
  g->nodes += v.n * a.n_out * (launches + 1);
  *waves = best;
  return ok();
}

rp_status rp_prune_sweep(rp_graph_t g, const rp_alpha* alphas, int32_t n_a, const int32_t* Rs,
                         int32_t n_R, int32_t* const* out_nbr, int32_t* const* out_deg,
                         void* stream) {
  rp::SweepArgs a;
  rp_status st0 = sweep_args(g, alphas, n_a, Rs, n_R, out_nbr, out_deg, &a);
  if (st0 != RP_OK) return st0;
  rp_status st = check_launch(rp::launch_prune_batched(g->view, a, g->ctr, (hipStream_t)stream),
                              "prune_batched");
  if (st != RP_OK) return st;
  g->nodes += g->view.n * a.n_out;
  return ok();
}

rp_status rp_prune_sweep_unsorted(rp_graph_t g, const rp_alpha* alphas, int32_t n_a,
                                  const int32_t* Rs, int32_t n_R, int32_t* const* out_nbr,
                                  int32_t* const* out_deg, void* stream) {
  rp::SweepArgs a;
  rp_status st0 = sweep_args(g, alphas, n_a, Rs, n_R, out_nbr, out_deg, &a, true);
  if (st0 != RP_OK) return st0;
  rp_status st = check_launch(rp::launch_prune_batched(g->view, a, g->ctr, (hipStream_t)stream),
                              "prune_batched");
  if (st != RP_OK) return st;
  g->nodes += g->view.n * a.n_out;
  return ok();
}

rp_status rp_prune(rp_graph_t g, rp_alpha alpha, int32_t R, int32_t* out_nbr, int32_t* out_deg,
                   void* stream) {
  return rp_prune_sweep(g, &alpha, 1, &R, 1, &out_nbr, &out_deg, stream);
}

rp_status rp_search(rp_graph_t g, const void* queries, int64_t nq, int32_t k, int32_t L,
                    int32_t* out_ids, double* out_dist, int32_t* out_hops, void* stream) {
  if (!g) return fail(RP_ESTATE, "graph is null");
  if (nq < 0 || nq >= (1ll << 31)) return fail(RP_EINVAL, "nq must be in [0, 2^31)");
  if (k < 1 || L < k || L > rp::kMaxL)
    return fail(RP_EINVAL, "need 1 <= k <= L <= %d (got k=%d, L=%d)", rp::kMaxL, k, L);
  if (nq == 0) return ok();
  const rp::GraphView& v = g->view;
  if (!device_range(queries, (size_t)nq * v.d * elem_size(v.dtype)))
    return fail(RP_EINVAL, "queries is not a device array of nq*d elements");
  if (!device_range(out_ids, (size_t)nq * k * 4))
    return fail(RP_EINVAL, "out_ids is not a device array of nq*k int32");
  if (out_dist && !device_range(out_dist, (size_t)nq * k * 8))
    return fail(RP_EINVAL, "out_dist is not a device array of nq*k double");
  if (out_hops && !device_range(out_hops, (size_t)nq * 4))
    return fail(RP_EINVAL, "out_hops is not a device array of nq int32");
  rp_status st = check_launch(
      rp::launch_search(v, queries, nq, k, L, out_ids, out_dist, out_hops, (hipStream_t)stream),
      "search");
  return st == RP_OK ? ok() : st;
}


rp_status rp_knn_u8(const uint8_t* points, int64_t n, int32_t d, const int32_t* query_ids,
                    int64_t nq, const int32_t* cand_ids, int64_t nc, int32_t K,
                    int32_t* out_ids, void* stream) {
  rp_status st = rp::knn_args(points, n, d, query_ids, nq, cand_ids, nc, K, out_ids);
  if (st != RP_OK || nq == 0) return st == RP_OK ? ok() : st;
  hipStream_t s = (hipStream_t)stream;
  const int slices = rp::knn_u8_slices(nq, nc);
  const size_t ws_bytes = rp::knn_u8_workspace_bytes(nq, slices);
  void* ws = nullptr;
  if (ws_bytes && hipMallocAsync(&ws, ws_bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RP_ENOMEM, "workspace of %zu bytes could not be allocated", ws_bytes);
  }
  const hipError_t e = rp::launch_knn_u8(points, n, d, query_ids, nq, cand_ids, nc, K, out_ids,
                                         (uint64_t*)ws, slices, s);
  if (ws) (void)hipFreeAsync(ws, s);
  st = check_launch(e, "knn_u8");
  return st == RP_OK ? ok() : st;
}

rp_status rp_build_slow(const void* points, int32_t dtype, int64_t n, int32_t d, rp_alpha alpha,
                        int32_t R, int32_t* out_nbr, int32_t* out_deg, void* stream) {
  if (dtype != RP_U8 && dtype != RP_F32) return fail(RP_EINVAL, "dtype must be RP_U8 or RP_F32");
  if (n < 1 || n >= (1ll << 31)) return fail(RP_EINVAL, "n must be in [1, 2^31)");
  if (d < 1 || d > rp::kMaxDim) return fail(RP_EINVAL, "d must be in [1, %d]", rp::kMaxDim);
  if (R < 1) return fail(RP_EINVAL, "R must be >= 1 (got %d)", R);
  rp_status st = check_alpha(alpha);
  if (st != RP_OK) return st;
  if (!device_range(points, (size_t)n * d * elem_size(dtype)))
    return fail(RP_EINVAL, "points is not a device array of n*d elements");
  if (!device_range(out_nbr, (size_t)n * R * 4))
    return fail(RP_EINVAL, "out_nbr is not a device array of n*R int32");
  if (!device_range(out_deg, (size_t)n * 4))
    return fail(RP_EINVAL, "out_deg is not a device array of n int32");
  hipStream_t s = (hipStream_t)stream;
  const int groups = rp::slow_build_groups(n);
  const size_t bytes = rp::slow_build_workspace_bytes(n, groups);
  void* ws = nullptr;
  if (hipMallocAsync(&ws, bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RP_ENOMEM, "workspace of %zu bytes could not be allocated", bytes);
  }
  const hipError_t e = rp::launch_slow_build(
      points, dtype, n, d, (uint32_t)alpha.num * alpha.num, (uint32_t)alpha.den * alpha.den, R,
      out_nbr, out_deg, ws, groups, s);
  (void)hipFreeAsync(ws, s);
  st = check_launch(e, "slow build");
  return st == RP_OK ? ok() : st;
}

rp_status rp_f32_band(int32_t d, double* out) {
  if (!out) return fail(RP_EINVAL, "out is null");
  if (d < 1 || d > rp::kMaxDim) return fail(RP_EINVAL, "d must be in [1, %d]", rp::kMaxDim);
  rp::f32_band(d, out);
  return ok();
}

rp_status rp_read_counters(rp_graph_t g, rp_counters* out, int32_t reset, void* stream) {
  if (!g) return fail(RP_ESTATE, "graph is null");
  if (!out) return fail(RP_EINVAL, "out is null");
  rp::DevCounters host = {};
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&host, g->ctr, sizeof(host), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return check_launch(e, "counter readback");
  out->nodes = g->nodes;
  out->rechecks = (int64_t)host.rechecks;
  if (reset) {
    rp::DevCounters zero = {};
    e = hipMemcpyAsync(g->ctr, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return check_launch(e, "counter reset");
    g->nodes = 0;
  }
  return ok();
}

void rp_free_graph(rp_graph_t g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(g->ctr);
  if (g->aux) (void)hipFree(g->aux);
  if (g->frame_e) (void)hipFree(g->frame_e);
  delete g;
}

}  // extern "C"
