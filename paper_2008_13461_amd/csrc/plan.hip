// Batched execution plans (one hipGraph per step) and kernel timing.
//
// A plan owns its workspace and a private capture stream.  The first run --
// and any run whose buffers or sizes differ from the captured ones --
// records the whole step (doublets, links, n-tuplets, fit and optionally its
// adjoint) into a hipGraph; every run then launches the graph on the
// caller's stream.  None of the captured calls uses hipMemsetAsync.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pt_internal.h"

namespace pt {

pt_err launch_doublets(const pt_hits& h, const DevCfg& k, pt_cells& cells, uint32_t* status, pt_workspace ws,
                       hipStream_t s);
pt_err launch_links(const pt_hits& h, const DevCfg& k, const pt_cells& cells, pt_links& L, uint32_t* status,
                    pt_workspace ws, hipStream_t s, int block);
pt_err launch_ntuplets(const pt_hits& h, const DevCfg& k, const pt_cells& cells, const pt_links& L,
                       pt_ntuplets& T, uint32_t* status, pt_workspace ws, hipStream_t s);
pt_err launch_fit(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, const float* offsets, int precision,
                  pt_tracks& out, uint32_t* status, pt_workspace ws, hipStream_t s);
pt_err launch_fit_bwd(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, const float* offsets,
                      int precision, const void* g_params, const void* g_chi2, void* grad_hits,
                      double* grad_offsets, int n_max, uint32_t* status, pt_workspace ws, hipStream_t s);
pt_err launch_ambiguity(const pt_hits& h, const pt_cells& cells, const pt_ntuplets& T, int precision,
                        const pt_tracks& tracks, int32_t* selected, int32_t* n_selected, pt_workspace ws,
                        hipStream_t s);
pt_err launch_vertices(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, int precision,
                       const pt_tracks& tracks, const int32_t* selected, const int32_t* n_selected,
                       pt_vertices& out, uint32_t* status, pt_workspace ws, hipStream_t s);

// ---------------------------------------------------------------------------
// kernel timing

namespace {
struct TimingState {
  std::mutex mu;
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
  };
  std::map<std::string, std::vector<Rec>> recs;
};
TimingState& timing() {
  static TimingState t;
  return t;
}
}  // namespace

thread_local bool g_capturing = false;
thread_local bool g_no_timing = false;

void* timing_begin(hipStream_t s) {
  if (!timing().on || g_capturing || g_no_timing) return nullptr;
  hipEvent_t* ev = new hipEvent_t[2];
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    delete[] ev;
    return nullptr;
  }
  if (hipEventRecord(ev[0], s) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    delete[] ev;
    return nullptr;
  }
  return ev;
}

void timing_end(void* tok, const char* name, hipStream_t s) {
  if (!tok) return;
  hipEvent_t* ev = static_cast<hipEvent_t*>(tok);
  if (hipEventRecord(ev[1], s) != hipSuccess) {  // no record for this launch
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    delete[] ev;
    return;
  }
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  t.recs[name].push_back({ev[0], ev[1]});
  delete[] ev;
}

// ---------------------------------------------------------------------------
// plans

struct Plan {
  pt_config cfg;
  DevCfg dev;
  int32_t n_hits_max, n_events_max, cells_cap, links_cap, tuplets_cap, precision, stages;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint8_t> key;  // bytes of everything the captured graph depends on
};

}  // namespace pt

using namespace pt;

extern "C" {

void pt_timing_enable(int32_t on) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  t.on = on != 0;
}

void pt_timing_reset(void) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto& kv : t.recs)
    for (auto& r : kv.second) {
      (void)hipEventDestroy(r.a);  // cleanup: nothing to recover
      (void)hipEventDestroy(r.b);
    }
  t.recs.clear();
}

int32_t pt_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  auto it = t.recs.find(kernel);
  if (it == t.recs.end()) {
    if (total_ms) *total_ms = 0.0;
    if (launches) *launches = 0;
    return PT_ERR_ARG;
  }
  double sum = 0.0;
  for (auto& r : it->second) {
    PT_HIP_CHECK(hipEventSynchronize(r.b));
    float ms = 0.f;
    PT_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    sum += ms;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = static_cast<int64_t>(it->second.size());
  return PT_OK;
}

pt_err pt_plan_create(const pt_config* cfg, int32_t n_hits_max, int32_t n_events_max, int32_t cells_cap,
                      int32_t links_cap, int32_t tuplets_cap, int32_t precision, int32_t stages,
                      pt_plan* out) {
  if (!cfg || !out || n_hits_max < 0 || n_events_max < 0 || cells_cap < 0 || links_cap < 0 || tuplets_cap < 0)
    return PT_ERR_ARG;
  if (precision != PT_FIT_F64 && precision != PT_FIT_F32 && precision != PT_FIT_F32_F64SOLVE) return PT_ERR_ARG;
  if (stages & ~(PT_STAGE_ADJOINT | PT_STAGE_AMBIGUITY | PT_STAGE_VERTICES)) return PT_ERR_ARG;
  Plan* p = new Plan();
  p->cfg = *cfg;
  if (!derive_config(*cfg, &p->dev)) {
    delete p;
    return PT_ERR_ARG;
  }
  p->n_hits_max = n_hits_max;
  p->n_events_max = n_events_max;
  p->cells_cap = cells_cap;
  p->links_cap = links_cap;
  p->tuplets_cap = tuplets_cap;
  p->precision = precision;
  p->stages = stages;
  p->ws_bytes = pt_workspace_size(cfg, n_hits_max, n_events_max, cells_cap, links_cap, tuplets_cap);
  if (p->ws_bytes == 0) {
    delete p;
    return PT_ERR_ARG;
  }
  if (p->dev.fishbone_theta2 > 0.0) fishbone_prepare();
  hipError_t he = hipMalloc(&p->ws, p->ws_bytes);
  if (he == hipSuccess) he = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (he != hipSuccess) {
    if (p->ws) (void)hipFree(p->ws);
    delete p;
    return device_error(he);
  }
  *out = reinterpret_cast<pt_plan>(p);
  return PT_OK;
}

void pt_plan_destroy(pt_plan plan) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return;
  // teardown: errors here have no recovery
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->ws) (void)hipFree(p->ws);
  delete p;
}

static pt_err enqueue_step(Plan* p, const pt_hits* hits, pt_cells* cells, pt_links* links, pt_ntuplets* tuplets,
                           pt_tracks* tracks, const float* offsets, const void* g_params, const void* g_chi2,
                           void* grad_hits, double* grad_offsets, int32_t* selected, int32_t* n_selected,
                           pt_vertices* vertices, uint32_t* status, hipStream_t s) {
  pt_workspace ws{p->ws, p->ws_bytes};
  pt_err e = launch_doublets(*hits, p->dev, *cells, status, ws, s);
  if (e == PT_OK) e = launch_links(*hits, p->dev, *cells, *links, status, ws, s, p->cfg.block_links);
  if (e == PT_OK) e = launch_ntuplets(*hits, p->dev, *cells, *links, *tuplets, status, ws, s);
  if (e == PT_OK) e = launch_fit(*hits, p->dev, *tuplets, offsets, p->precision, *tracks, status, ws, s);
  if (e == PT_OK && (p->stages & PT_STAGE_ADJOINT))
    e = launch_fit_bwd(*hits, p->dev, *tuplets, offsets, p->precision, g_params, g_chi2, grad_hits, grad_offsets,
                       std::min(tuplets->cap, tracks->cap), status, ws, s);
  if (e == PT_OK && (p->stages & PT_STAGE_AMBIGUITY))
    e = launch_ambiguity(*hits, *cells, *tuplets, p->precision, *tracks, selected, n_selected, ws, s);
  if (e == PT_OK && (p->stages & PT_STAGE_VERTICES)) {
    const bool sel = (p->stages & PT_STAGE_AMBIGUITY) != 0;
    e = launch_vertices(*hits, p->dev, *tuplets, p->precision, *tracks, sel ? selected : nullptr,
                        sel ? n_selected : nullptr, *vertices, status, ws, s);
  }
  return e;
}

pt_err pt_plan_run(pt_plan plan, const pt_hits* hits, pt_cells* cells, pt_links* links, pt_ntuplets* tuplets,
                   pt_tracks* tracks, const float* module_offsets, const void* g_params, const void* g_chi2,
                   void* grad_hits, double* grad_offsets, int32_t* selected, int32_t* n_selected,
                   pt_vertices* vertices, uint32_t* status, pt_stream stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p || !hits || !cells || !links || !tuplets || !tracks) return PT_ERR_ARG;
  if (hits->n_hits > p->n_hits_max || hits->n_events > p->n_events_max || cells->cap > p->cells_cap ||
      links->cap > p->links_cap || tuplets->cap > p->tuplets_cap || tracks->cap < tuplets->cap)
    return PT_ERR_ARG;
  if ((p->stages & PT_STAGE_ADJOINT) && !g_params) return PT_ERR_ARG;
  if ((p->stages & PT_STAGE_AMBIGUITY) && (!selected || !n_selected || !tuplets->cells)) return PT_ERR_ARG;
  if ((p->stages & PT_STAGE_VERTICES) &&
      (!vertices || !tracks->cov || !vertices->event_first || !vertices->count || !vertices->track_vertex ||
       (vertices->cap > 0 && (!vertices->z || !vertices->var || !vertices->chi2 || !vertices->ndf ||
                              !vertices->n_tracks || !vertices->sum_pt2))))
    return PT_ERR_ARG;
  if ((module_offsets || grad_offsets) && !hits->module) return PT_ERR_ARG;
  // everything the captured graph depends on
  std::vector<uint8_t> key;
  auto add = [&key](const void* v, size_t n) {
    const uint8_t* b = static_cast<const uint8_t*>(v);
    key.insert(key.end(), b, b + n);
  };
  add(hits, sizeof(*hits));
  add(cells, sizeof(*cells));
  add(links, sizeof(*links));
  add(tuplets, sizeof(*tuplets));
  add(tracks, sizeof(*tracks));
  const void* ptrs[] = {module_offsets, g_params, g_chi2, grad_hits, grad_offsets, selected, n_selected, status};
  add(ptrs, sizeof(ptrs));
  if (vertices) add(vertices, sizeof(*vertices));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  clear_stale_error();
  if (!p->exec || key != p->key) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    PT_HIP_CHECK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    g_capturing = true;
    pt_err e = enqueue_step(p, hits, cells, links, tuplets, tracks, module_offsets, g_params, g_chi2, grad_hits,
                            grad_offsets, selected, n_selected, vertices, status, p->cap_stream);
    g_capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
    if (e != PT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    if (ce != hipSuccess || !g) return device_error(ce != hipSuccess ? ce : hipErrorStreamCaptureInvalidated);
    p->graph = g;
    PT_HIP_CHECK(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->key = key;
  }
  PT_HIP_CHECK(hipGraphLaunch(p->exec, s));
  return PT_OK;
}

}  // extern "C"
