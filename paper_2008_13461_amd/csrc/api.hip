// The C interface declared in include/pixeltrack.h: argument checks, the
// host-side derivation of the cut constants, workspace sizing, and dispatch
// to the kernels of each step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

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
pt_err launch_fit_noalloc(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, const float* offsets,
                          int precision, pt_tracks& out, uint32_t* status, hipStream_t s);
pt_err launch_ambiguity(const pt_hits& h, const pt_cells& cells, const pt_ntuplets& T, int precision,
                        const pt_tracks& tracks, int32_t* selected, int32_t* n_selected, pt_workspace ws,
                        hipStream_t s);
pt_err launch_vertices(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, int precision,
                       const pt_tracks& tracks, const int32_t* selected, const int32_t* n_selected,
                       pt_vertices& out, uint32_t* status, pt_workspace ws, hipStream_t s);

// The derived constants, with the expressions documented in pixeltrack.h.
// Evaluated without contraction so that they are reproducible.
#pragma clang fp contract(off)
bool derive_config(const pt_config& c, DevCfg* d) {
  std::memset(d, 0, sizeof(*d));
  if (c.n_pairs < 1 || c.n_pairs > kMaxPairs) return false;
  if (!(c.pt_min > 0.0) || !(c.bfield > 0.0)) return false;
  if (c.min_hits < 3 || c.max_hits > kMaxHits || c.min_hits > c.max_hits) return false;
  if (c.n_modules < 1) return false;
  const int B = c.n_phi_bins > 0 ? c.n_phi_bins : 128;
  if (B < 4 || B > 65536) return false;
  d->n_pairs = c.n_pairs;
  d->n_bins = B;
  d->bin_shift = -1;
  for (int sh = 0; sh < 31; ++sh)
    if ((1 << sh) == B) d->bin_shift = sh;
  d->bin_scale = static_cast<float>(B / (2.0 * M_PI));
  d->cut_mask = c.cut_mask;
  d->z0_max = c.z0_max;
  const double kappa_max = (0.299792458 * c.bfield) / (100.0 * c.pt_min);
  d->kappa_max2 = kappa_max * kappa_max;
  const double bin_w = 2.0 * M_PI / B;
  for (int l = 0; l < kLayers; ++l) d->n_inner_pairs[l] = 0;
  for (int p = 0; p < c.n_pairs; ++p) {
    const int li = c.pair_inner[p], lo = c.pair_outer[p];
    if (li >= kLayers || lo >= kLayers || li == lo) return false;
    if (!(c.pair_dphi[p] > 0.0 && c.pair_dphi[p] < 0.5 * M_PI)) return false;
    d->pair_inner[p] = li;
    d->pair_outer[p] = lo;
    d->tan_dphi[p] = std::tan(c.pair_dphi[p]);
    d->zlo[p] = c.pair_zlo[p];
    d->zhi[p] = c.pair_zhi[p];
    // Azimuth half-window in bins.  A passing pair differs by at most dphi in
    // azimuth; one extra bin absorbs the rounding of the single-precision bin
    // assignment, so the binned search never misses a doublet.
    int w = B;
    if (c.cut_mask & PT_CUT_PHIW) w = static_cast<int>(std::ceil(c.pair_dphi[p] / bin_w)) + 1;
    d->pair_wbins[p] = std::min(w, B);
    if (d->n_inner_pairs[li] >= kMaxPairsPerLayer) return false;
    d->inner_pairs[li][d->n_inner_pairs[li]++] = p;
  }
  d->theta2_barrel = c.ca_theta_barrel * c.ca_theta_barrel;
  d->theta2_endcap = c.ca_theta_endcap * c.ca_theta_endcap;
  // The link search bins the out-cells of a hit by the direction of their R-Z
  // segment into buckets at least as wide as the largest cut angle, with a
  // margin far above the rounding of the keys: a pair that passes the R-Z
  // test then lies in the same or a neighbouring bucket.
  {
    const double th = std::max(std::fabs(c.ca_theta_barrel), std::fabs(c.ca_theta_endcap));
    d->rz_buckets = 0;
    if (th < 0.5) {  // NaN fails
      const double b = std::floor(2.0 / (std::asin(th) + 1e-4));
      d->rz_buckets = b >= 4.0 ? static_cast<int32_t>(std::min(b, static_cast<double>(kRzBuckets))) : 0;
    }
  }
  d->rmax_bpix1 = c.ca_rmax_bpix1;
  d->rmax_other = c.ca_rmax_other;
  for (int l = 0; l < kLayers; ++l) d->layer_barrel[l] = c.layer_barrel[l] ? 1 : 0;
  for (int p = 0; p < c.n_pairs; ++p)
    if (!d->layer_barrel[d->pair_outer[p]]) d->endcap_pairs |= 1u << p;
  d->root_always_mask = c.root_always_mask;
  d->root_if_free_mask = c.root_if_free_mask;
  d->min_hits = c.min_hits;
  d->max_hits = c.max_hits;
  d->K = 0.299792458 * c.bfield / 100.0;
  d->x_over_x0 = c.x_over_x0;
  d->highland_a = c.highland_a;
  d->highland_b = c.highland_b;
  d->VT = c.sigma_rphi * c.sigma_rphi;
  d->VZ_barrel = c.sigma_z * c.sigma_z;
  d->VR_disk = c.sigma_r * c.sigma_r;
  d->p_cap = c.p_cap;
  d->f64_threshold = c.f64_solve_threshold > 0.0 ? c.f64_solve_threshold : 1024.0;
  d->n_modules = c.n_modules;
  d->block_doublets = c.block_doublets;
  if (!(c.vtx_dz_cut > 0.0) || c.vtx_kmeans_iter < 1) return false;
  d->vtx_min_hits = c.vtx_min_hits;
  d->vtx_kmeans_iter = c.vtx_kmeans_iter;
  d->vtx_pt_min = c.vtx_pt_min;
  d->vtx_err_max = c.vtx_err_max;
  d->vtx_dz_cut = c.vtx_dz_cut;
  d->vtx_chi2_max = c.vtx_chi2_max;
  d->vtx_split_chi2_ndf = c.vtx_split_chi2_ndf;
  d->vtx_pt_cap = c.vtx_pt_cap;
  if (!(c.fishbone_theta >= 0.0)) return false;
  d->fishbone_theta2 = c.fishbone_theta * c.fishbone_theta;
  if (c.exclusive_hits != 0 && c.exclusive_hits != 1) return false;
  d->exclusive_hits = c.exclusive_hits;
  return true;
}
#pragma clang fp contract(on)

namespace {

bool hits_ok(const pt_hits* h) {
  if (!h || h->n_hits < 0 || h->n_events < 0) return false;
  if (h->dtype != PT_F32 && h->dtype != PT_F64) return false;
  if (h->n_events > 0 && !h->event_offsets) return false;
  if (h->n_hits > 0 && (!h->x || !h->y || !h->z || !h->layer)) return false;
  return true;
}

bool ws_ok(const pt_workspace& ws, size_t need) {
  return need == 0 || (ws.ptr && ws.bytes >= need && (reinterpret_cast<uintptr_t>(ws.ptr) & 255) == 0);
}

thread_local hipError_t g_last_device_error = hipSuccess;
thread_local char g_last_device_text[256];

}  // namespace

pt_err device_error(hipError_t e) {
  g_last_device_error = e;
  return PT_ERR_DEVICE;
}

}  // namespace pt

using namespace pt;

extern "C" {

int32_t pt_abi_version(void) { return PT_ABI_VERSION; }

const char* pt_err_string(pt_err e) {
  switch (e) {
    case PT_OK: return "ok";
    case PT_ERR_ARG: return "invalid argument";
    case PT_ERR_DEVICE: return "HIP runtime or kernel launch failure";
    case PT_ERR_UNSUPPORTED: return "unsupported request";
    case PT_ERR_WORKSPACE: return "workspace too small or misaligned";
    case PT_ERR_TOO_LARGE: return "more tracks than the fixed scratch of the allocation-free fit holds";
  }
  return "unknown error";
}

const char* pt_last_device_error(void) {
  if (g_last_device_error == hipSuccess) return "";
  std::snprintf(g_last_device_text, sizeof(g_last_device_text), "%s: %s", hipGetErrorName(g_last_device_error),
                hipGetErrorString(g_last_device_error));
  return g_last_device_text;
}

size_t pt_workspace_size(const pt_config* cfg, int32_t n_hits, int32_t n_events, int32_t cells_cap,
                         int32_t links_cap, int32_t tuplets_cap) {
  (void)links_cap;
  if (!cfg || n_hits < 0 || n_events < 0 || cells_cap < 0 || tuplets_cap < 0) return 0;
  DevCfg d;
  if (!derive_config(*cfg, &d)) return 0;
  size_t s = ws_doublets(n_hits, n_events, d.n_bins);
  if (d.fishbone_theta2 > 0.0) s = std::max(s, ws_fishbone(n_hits, cells_cap));
  s = std::max(s, ws_links(n_hits, cells_cap));
  s = std::max(s, ws_ntuplets(cells_cap, tuplets_cap));
  s = std::max(s, ws_fit(tuplets_cap, d.n_modules));
  s = std::max(s, ws_ambiguity(n_hits, cells_cap, tuplets_cap));
  s = std::max(s, ws_vertices(n_events, tuplets_cap));
  return s;
}

pt_err pt_build_doublets(const pt_hits* hits, const pt_config* cfg, pt_cells* cells, uint32_t* status,
                         pt_workspace ws, pt_stream stream) {
  DevCfg d;
  if (!hits_ok(hits) || !cfg || !cells || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (cells->cap < 0 || !cells->count || (hits->n_hits > 0 && (!cells->inner_first || !cells->inner_count)))
    return PT_ERR_ARG;
  if (cells->cap > 0 && (!cells->inner || !cells->outer || !cells->pair)) return PT_ERR_ARG;
  size_t need = ws_doublets(hits->n_hits, hits->n_events, d.n_bins);
  if (d.fishbone_theta2 > 0.0) need = std::max(need, ws_fishbone(hits->n_hits, cells->cap));
  if (!ws_ok(ws, need)) return PT_ERR_WORKSPACE;
  clear_stale_error();
  return launch_doublets(*hits, d, *cells, status, ws, reinterpret_cast<hipStream_t>(stream));
}

pt_err pt_link_cells(const pt_hits* hits, const pt_config* cfg, const pt_cells* cells, pt_links* links,
                     uint32_t* status, pt_workspace ws, pt_stream stream) {
  DevCfg d;
  if (!hits_ok(hits) || !cfg || !cells || !links || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (cells->cap < 0 || links->cap < 0 || !cells->count || !links->count) return PT_ERR_ARG;
  if (cells->cap > 0 && (!cells->inner || !cells->outer || !cells->pair ||
                         !links->out_start || !links->out_count || !links->has_inner))
    return PT_ERR_ARG;
  if (hits->n_hits > 0 && (!cells->inner_first || !cells->inner_count)) return PT_ERR_ARG;
  if (links->cap > 0 && (!links->in_cell || !links->out_cell)) return PT_ERR_ARG;
  if (!ws_ok(ws, ws_links(hits->n_hits, cells->cap))) return PT_ERR_WORKSPACE;
  clear_stale_error();
  return launch_links(*hits, d, *cells, *links, status, ws, reinterpret_cast<hipStream_t>(stream),
                      cfg->block_links);
}

pt_err pt_find_ntuplets(const pt_hits* hits, const pt_config* cfg, const pt_cells* cells, const pt_links* links,
                        pt_ntuplets* tuplets, uint32_t* status, pt_workspace ws, pt_stream stream) {
  DevCfg d;
  if (!hits_ok(hits) || !cfg || !cells || !links || !tuplets || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (tuplets->cap < 0 || !tuplets->count || !tuplets->count_raw) return PT_ERR_ARG;
  if (tuplets->cap > 0 && (!tuplets->hits || !tuplets->cells || !tuplets->n || !tuplets->kept)) return PT_ERR_ARG;
  if (cells->cap < 0 || !cells->count || links->cap < 0 || !links->count) return PT_ERR_ARG;
  if (cells->cap > 0 && (!cells->inner || !cells->outer || !cells->pair || !links->out_start ||
                         !links->out_count || !links->has_inner))
    return PT_ERR_ARG;
  if (links->cap > 0 && !links->out_cell) return PT_ERR_ARG;
  if (!ws_ok(ws, ws_ntuplets(cells->cap, tuplets->cap))) return PT_ERR_WORKSPACE;
  clear_stale_error();
  return launch_ntuplets(*hits, d, *cells, *links, *tuplets, status, ws, reinterpret_cast<hipStream_t>(stream));
}

pt_err pt_fit_broken_line(const pt_hits* hits, const pt_config* cfg, const pt_ntuplets* tuplets,
                          const float* module_offsets, int32_t precision, pt_tracks* tracks, uint32_t* status,
                          pt_workspace ws, pt_stream stream) {
  DevCfg d;
  if (!hits_ok(hits) || !cfg || !tuplets || !tracks || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (precision != PT_FIT_F64 && precision != PT_FIT_F32 && precision != PT_FIT_F32_F64SOLVE) return PT_ERR_ARG;
  if (tuplets->cap < 0 || tracks->cap < 0 || !tuplets->count) return PT_ERR_ARG;
  if (module_offsets && !hits->module) return PT_ERR_ARG;
  const int n_max = std::min(tuplets->cap, tracks->cap);
  if (n_max > 0 && (!tuplets->hits || !tuplets->n || !tracks->params || !tracks->chi2 || !tracks->status))
    return PT_ERR_ARG;
  if (!ws_ok(ws, ws_fit(n_max, d.n_modules))) return PT_ERR_WORKSPACE;
  clear_stale_error();
  return launch_fit(*hits, d, *tuplets, module_offsets, precision, *tracks, status, ws,
                    reinterpret_cast<hipStream_t>(stream));
}

pt_err pt_resolve_ambiguities(const pt_hits* hits, const pt_config* cfg, const pt_cells* cells,
                              const pt_ntuplets* tuplets, int32_t precision, const pt_tracks* tracks,
                              int32_t* selected, int32_t* n_selected, uint32_t* status, pt_workspace ws,
                              pt_stream stream) {
  DevCfg d;
  (void)status;
  if (!hits_ok(hits) || !cfg || !cells || !tuplets || !tracks || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (precision != PT_FIT_F64 && precision != PT_FIT_F32 && precision != PT_FIT_F32_F64SOLVE) return PT_ERR_ARG;
  if (cells->cap < 0 || tuplets->cap < 0 || tracks->cap < 0 || !tuplets->count || !n_selected) return PT_ERR_ARG;
  const int n_max = std::min(tuplets->cap, tracks->cap);
  if (n_max > 0 && (!tuplets->hits || !tuplets->cells || !tuplets->n || !tracks->params || !tracks->chi2 ||
                    !selected))
    return PT_ERR_ARG;
  if (!ws_ok(ws, ws_ambiguity(hits->n_hits, cells->cap, n_max))) return PT_ERR_WORKSPACE;
  clear_stale_error();
  return launch_ambiguity(*hits, *cells, *tuplets, precision, *tracks, selected, n_selected, ws,
                          reinterpret_cast<hipStream_t>(stream));
}

pt_err pt_find_vertices(const pt_hits* hits, const pt_config* cfg, const pt_ntuplets* tuplets, int32_t precision,
                        const pt_tracks* tracks, const int32_t* selected, const int32_t* n_selected,
                        pt_vertices* out, uint32_t* status, pt_workspace ws, pt_stream stream) {
  DevCfg d;
  if (!hits_ok(hits) || !cfg || !tuplets || !tracks || !out || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (precision != PT_FIT_F64 && precision != PT_FIT_F32 && precision != PT_FIT_F32_F64SOLVE) return PT_ERR_ARG;
  if (tuplets->cap < 0 || tracks->cap < 0 || !tuplets->count || out->cap < 0) return PT_ERR_ARG;
  if ((selected == nullptr) != (n_selected == nullptr)) return PT_ERR_ARG;
  if (!out->event_first || !out->count) return PT_ERR_ARG;
  if (out->cap > 0 && (!out->z || !out->var || !out->chi2 || !out->ndf || !out->n_tracks || !out->sum_pt2))
    return PT_ERR_ARG;
  const int n_max = std::min(tuplets->cap, tracks->cap);
  if (n_max > 0 && (!tuplets->hits || !tuplets->n || !tracks->params || !tracks->cov || !out->track_vertex))
    return PT_ERR_ARG;
  if (hits->n_events > 0 && !hits->event_offsets) return PT_ERR_ARG;
  if (!ws_ok(ws, ws_vertices(hits->n_events, n_max))) return PT_ERR_WORKSPACE;
  clear_stale_error();
  return launch_vertices(*hits, d, *tuplets, precision, *tracks, selected, n_selected, *out, status, ws,
                         reinterpret_cast<hipStream_t>(stream));
}

pt_err pt_fit_broken_line_noalloc(const pt_hits* hits, const pt_config* cfg, const pt_ntuplets* tuplets,
                                  const float* module_offsets, int32_t precision, pt_tracks* tracks,
                                  uint32_t* status, pt_stream stream) {
  DevCfg d;
  if (!hits_ok(hits) || !cfg || !tuplets || !tracks || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (precision != PT_FIT_F64 && precision != PT_FIT_F32 && precision != PT_FIT_F32_F64SOLVE) return PT_ERR_ARG;
  if (tuplets->cap < 0 || tracks->cap < 0 || !tuplets->count) return PT_ERR_ARG;
  if (module_offsets && !hits->module) return PT_ERR_ARG;
  const int n_max = std::min(tuplets->cap, tracks->cap);
  if (n_max > 0 && (!tuplets->hits || !tuplets->n || !tracks->params || !tracks->chi2 || !tracks->status))
    return PT_ERR_ARG;
  if (n_max > PT_NOALLOC_FIT_MAX_TRACKS) return PT_ERR_TOO_LARGE;
  clear_stale_error();
  return launch_fit_noalloc(*hits, d, *tuplets, module_offsets, precision, *tracks, status,
                            reinterpret_cast<hipStream_t>(stream));
}

pt_err pt_fit_broken_line_bwd(const pt_hits* hits, const pt_config* cfg, const pt_ntuplets* tuplets,
                              const float* module_offsets, int32_t precision, const void* g_params,
                              const void* g_chi2, void* grad_hits, double* grad_offsets, uint32_t* status,
                              pt_workspace ws, pt_stream stream) {
  DevCfg d;
  if (!hits_ok(hits) || !cfg || !tuplets || !derive_config(*cfg, &d)) return PT_ERR_ARG;
  if (precision != PT_FIT_F64 && precision != PT_FIT_F32 && precision != PT_FIT_F32_F64SOLVE) return PT_ERR_ARG;
  if (tuplets->cap < 0 || !tuplets->count) return PT_ERR_ARG;
  if ((module_offsets || grad_offsets) && !hits->module) return PT_ERR_ARG;
  const int n_max = tuplets->cap;
  if (n_max > 0 && (!tuplets->hits || !tuplets->n || !g_params)) return PT_ERR_ARG;
  if (!ws_ok(ws, ws_fit(n_max, d.n_modules))) return PT_ERR_WORKSPACE;
  clear_stale_error();
  return launch_fit_bwd(*hits, d, *tuplets, module_offsets, precision, g_params, g_chi2, grad_hits, grad_offsets,
                        n_max, status, ws, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
