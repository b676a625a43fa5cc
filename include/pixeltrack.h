/*
 * pixeltrack.h -- C interface of the MI355X pixel-track library.
 *
 * The library reconstructs pixel tracks from hits with the method of Bocci,
 * Kortelainen, Innocente, Pantaleo and Rovere, "Heterogeneous reconstruction
 * of tracks and primary vertices with the CMS pixel tracker": doublets
 * between hits of chosen layer pairs, Cellular Automaton links between
 * doublets, n-tuplets by depth-first search with duplicate removal
 * (section 3.2, section 3.3) and the broken-line fit of each n-tuplet
 * (section 3.4), plus the gradient of that fit with respect to hit positions
 * and per-module alignment translations.
 *
 * Conventions shared by every call
 *  - Memory: every array pointer is a DEVICE pointer owned by the caller;
 *    struct arguments themselves (pt_hits, pt_config, ...) live in HOST
 *    memory and are read before the call returns.  No call allocates or frees
 *    memory.  Scratch space comes from the caller's pt_workspace.
 *  - Streams: every call enqueues its kernels on `stream` (a hipStream_t,
 *    NULL = the null stream) and returns without synchronising.  Outputs are
 *    valid once the stream has reached the end of the call.  Calls are
 *    re-entrant on distinct streams with distinct workspaces.  The plain
 *    calls do not use hipMemsetAsync, so they may be captured in a graph.
 *  - Errors: argument errors return PT_ERR_ARG synchronously and enqueue
 *    nothing.  A failed kernel launch or HIP runtime call returns
 *    PT_ERR_DEVICE; pt_last_device_error names the HIP error.  Every call
 *    clears the calling thread's HIP error state (hipGetLastError) before it
 *    launches, so an error left there by other code on the thread is neither
 *    reported by the call nor kept for the caller.  Conditions that
 *    are only known on the device (capacity overflow, non-finite hits, layer
 *    ids out of range, truncated searches, fit failures) set bits and
 *    counters in the caller's pt_status block; outputs are then truncated
 *    but valid.  The status block is only ever OR-ed / added into: clear it
 *    when you want a fresh reading.
 *  - Indices: hit indices are int32 positions in the hit arrays as passed.
 *    Cell, link and n-tuplet indices are positions in their output arrays.
 *  - Units: cm, GeV, tesla, radians.  kappa > 0 turns counter-clockwise seen
 *    from +z (a negative particle in a field along +z).
 *  - Order: doublets, links and n-tuplets are sets; they come out in an
 *    order that depends only on the inputs and the configuration (the same
 *    on every run), which is not part of this contract.  The fit writes
 *    track i for kept n-tuplet i.
 */
#ifndef PIXELTRACK_H
#define PIXELTRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pt_stream; /* same type as hipStream_t */

typedef enum {
  PT_OK = 0,
  PT_ERR_ARG = 1,         /* invalid argument; nothing was enqueued */
  PT_ERR_DEVICE = 2,      /* a HIP runtime call or kernel launch failed */
  PT_ERR_UNSUPPORTED = 3, /* valid request that the library does not implement */
  PT_ERR_WORKSPACE = 4,   /* workspace smaller than pt_workspace_size() */
  PT_ERR_TOO_LARGE = 5    /* request beyond the fixed scratch of pt_fit_broken_line_noalloc */
} pt_err;

enum { PT_F32 = 0, PT_F64 = 1 };

/* Fit precision.
 *  PT_FIT_F64           all arithmetic in double; params/chi2 are double.
 *  PT_FIT_F32           single-precision fit; params/chi2 are float.  Sums and
 *                       differences of absolute coordinates (hit + offset,
 *                       positions relative to the first hit, their local frame
 *                       coordinates) and the final perigee conversion are
 *                       formed in double, where single precision would cancel.
 *  PT_FIT_F32_F64SOLVE  as PT_FIT_F32, but a track is fitted again in double
 *                       when its conditioning estimate exceeds
 *                       pt_config.f64_solve_threshold or when its
 *                       single-precision solve breaks down. */
enum { PT_FIT_F64 = 0, PT_FIT_F32 = 1, PT_FIT_F32_F64SOLVE = 2 };

/* Doublet cuts of Table 1 (bits of pt_config.cut_mask). */
enum { PT_CUT_PHIW = 1, PT_CUT_ZW = 2, PT_CUT_ZIP = 4, PT_CUT_PT = 8 };

#define PT_MAX_PAIRS 32
#define PT_N_LAYERS 10
#define PT_MAX_HITS 8 /* longest n-tuplet; rows of pt_ntuplets.hits */

/* Status block: PT_STATUS_WORDS uint32 words of device memory. */
#define PT_STATUS_WORDS 16
enum {
  PT_ST_FLAGS = 0,          /* OR of PT_FLAG_* */
  PT_ST_BAD_HITS = 1,       /* hits skipped: non-finite coordinate or layer >= 10 */
  PT_ST_TRUNCATED = 2,      /* searches that reached max_hits with links left */
  PT_ST_FIT_BAD_ORDER = 3,  /* tracks whose hits are not ordered along the pre-fit */
  PT_ST_FIT_F64 = 4,        /* tracks whose solve was routed to double */
  PT_ST_FIT_FAILED = 5      /* tracks with a non-finite result */
};
enum {
  PT_FLAG_CELLS_OVERFLOW = 1u << 0,
  PT_FLAG_LINKS_OVERFLOW = 1u << 1,
  PT_FLAG_TUPLETS_OVERFLOW = 1u << 2,
  PT_FLAG_BAD_HITS = 1u << 3,
  PT_FLAG_TRUNCATED = 1u << 4,
  PT_FLAG_FIT_BAD_ORDER = 1u << 5,
  PT_FLAG_FIT_FAILED = 1u << 6,
  PT_FLAG_VERTICES_OVERFLOW = 1u << 7
};
/* Per-track fit status bits (pt_tracks.status). */
enum { PT_FIT_OK = 0, PT_FIT_ST_BAD_ORDER = 1, PT_FIT_ST_F64_SOLVE = 2, PT_FIT_ST_FAILED = 4 };

/* Reconstruction settings (host struct).  The library derives its cut
 * constants from these fields on the host with these expressions, evaluated
 * in double in this order:
 *   tan_dphi[p] = tan(pair_dphi[p])                 (C library tan)
 *   kappa_max   = (0.299792458 * bfield) / (100.0 * pt_min),  kappa_max2 = kappa_max * kappa_max
 *   theta2_*    = ca_theta_* * ca_theta_*
 * so that another implementation following the same expressions makes
 * bit-identical decisions. */
typedef struct {
  double bfield;                      /* T, along +z */
  int32_t n_pairs;                    /* 1..PT_MAX_PAIRS */
  uint8_t pair_inner[PT_MAX_PAIRS];   /* layer of the inner hit of pair p */
  uint8_t pair_outer[PT_MAX_PAIRS];   /* layer of the outer hit; inner != outer */
  double pair_dphi[PT_MAX_PAIRS];     /* PhiW window (rad), in (0, pi/2) */
  double pair_zlo[PT_MAX_PAIRS];      /* ZW window on the inner hit's z (cm) */
  double pair_zhi[PT_MAX_PAIRS];
  double pt_min;                      /* PT cut (GeV) > 0 */
  double z0_max;                      /* ZIP cut (cm) */
  uint32_t cut_mask;                  /* PT_CUT_* applied */
  double ca_theta_barrel;             /* triplet R-Z kink sine, outer hit on barrel */
  double ca_theta_endcap;             /* same, outer hit on a disk */
  double ca_rmax_bpix1;               /* circle-to-beam distance (cm), inner hit on layer 0 */
  double ca_rmax_other;               /* same, other inner layers */
  uint32_t root_always_mask;          /* layers whose doublets always start a search */
  uint32_t root_if_free_mask;         /* layers whose doublets start one without inner link */
  int32_t min_hits;                   /* shortest n-tuplet emitted, >= 3 */
  int32_t max_hits;                   /* longest, <= PT_MAX_HITS */
  uint8_t layer_barrel[PT_N_LAYERS];  /* 1 = barrel layer, 0 = disk */
  double x_over_x0;                   /* material per layer crossing (radiation lengths) */
  double highland_a;                  /* 0.0136 GeV */
  double highland_b;                  /* 0.038 */
  double sigma_rphi;                  /* transverse hit resolution (cm) */
  double sigma_z;                     /* barrel longitudinal resolution (cm) */
  double sigma_r;                     /* disk radial resolution (cm) */
  double p_cap;                       /* momentum cap of the scattering estimate (GeV) */
  int32_t n_modules;                  /* rows of the module offset / gradient tables */
  /* performance settings: never change a result */
  int32_t n_phi_bins;                 /* azimuth bins per layer for the pair search; 0 = 128 */
  int32_t block_doublets;             /* threads per block of the doublet count pass: 64, 128,
                                         256 or 512; other values mean 256 */
  int32_t block_links;                /* threads per block of the link sweep (one wavefront per
                                         middle hit): 64, 128 or 256; other values mean 64 */
  double f64_solve_threshold;         /* see PT_FIT_F32_F64SOLVE; <= 0 means 1024 */
  /* pixel vertices (section 3.6), see pt_find_vertices */
  int32_t vtx_min_hits;               /* fewest hits of a track that is used */
  int32_t vtx_kmeans_iter;            /* most rounds of the two-means split, >= 1 */
  double vtx_pt_min;                  /* smallest p_T of a track that is used (GeV) */
  double vtx_err_max;                 /* largest sigma(z0) of a track whose density is computed (cm) */
  double vtx_dz_cut;                  /* largest |dz0| of close-by tracks (cm), > 0 */
  double vtx_chi2_max;                /* largest (dz0)^2 / (var_i + var_j) of compatible tracks */
  double vtx_split_chi2_ndf;          /* chi2/ndf above which a vertex is split in two */
  double vtx_pt_cap;                  /* p_T cap in the sum of p_T^2 that orders the vertices (GeV) */
  /* Fishbone (section 3.3), see pt_build_doublets; 0 = off */
  double fishbone_theta;              /* largest sine of the angle between two aligned doublets */
  /* 1: no hit belongs to two of the n-tuplets given to pt_fit_broken_line_bwd
   * (nor twice to one), so the adjoint may add into grad_hits with plain loads
   * and stores instead of atomic additions (the same sums); results are
   * undefined when hits are shared.  0: atomic additions. */
  int32_t exclusive_hits;
} pt_config;

/* Hits of n_events events.  Event e owns hits [event_offsets[e], event_offsets[e+1]). */
typedef struct {
  int32_t n_hits;                 /* length of every hit array, >= 0 */
  int32_t n_events;               /* >= 0 */
  const int32_t* event_offsets;   /* device [n_events + 1], nondecreasing, within [0, n_hits] */
  int32_t dtype;                  /* PT_F32 or PT_F64: element type of x, y, z */
  const void* x;                  /* device [n_hits] */
  const void* y;
  const void* z;
  const uint8_t* layer;           /* device [n_hits], 0..9 (others are skipped and counted) */
  const int16_t* module;          /* device [n_hits], 0..n_modules-1; used by the fit when
                                     module offsets or their gradient are requested */
} pt_hits;

/* Caller-owned scratch memory (device), at least pt_workspace_size() bytes, 256-byte aligned. */
typedef struct {
  void* ptr;
  size_t bytes;
} pt_workspace;

/* Doublets ("cells").  count[0] receives the number found, which may exceed
 * cap; only min(count, cap) entries are written (PT_FLAG_CELLS_OVERFLOW set).
 * The cells whose inner hit is h are [inner_first[h], inner_first[h] +
 * inner_count[h]) (clipped to cap): pt_build_doublets writes them grouped by
 * inner hit, and pt_link_cells relies on this index. */
typedef struct {
  int32_t cap;
  int32_t* inner;       /* [cap] inner hit index */
  int32_t* outer;       /* [cap] outer hit index */
  uint8_t* pair;        /* [cap] layer-pair index */
  int32_t* count;       /* [1] */
  int32_t* inner_first; /* [n_hits] */
  int32_t* inner_count; /* [n_hits] */
} pt_cells;

/* Cell links c_in -> c_out: c_out starts on the outer hit of c_in.  The links
 * are ordered by inner cell, and those of one inner cell by outer cell: cell
 * c's outer links are out_cell[j] for j in [out_start[c], out_start[c] +
 * out_count[c]) (clipped to cap).  out_start is the exclusive prefix sum of
 * out_count, so a cell's run ends where the next cell's starts, and the last
 * cell's at count[0]; the n-tuplet search relies on this.  has_inner[c] = 1
 * when some link ends on c.
 * The per-cell arrays hold the cells' capacity; entries below count[0] of
 * the cells are written. */
typedef struct {
  int32_t cap;
  int32_t* in_cell;   /* [cap] */
  int32_t* out_cell;  /* [cap] */
  int32_t* count;     /* [1] links found (may exceed cap) */
  int32_t* out_start; /* [cells.cap] */
  int32_t* out_count; /* [cells.cap] */
  uint8_t* has_inner; /* [cells.cap] */
} pt_links;

/* n-tuplets.  Rows hold every maximal path found by the search; `kept` lists
 * the rows that survive duplicate removal. */
typedef struct {
  int32_t cap;
  int32_t* hits;       /* [cap][PT_MAX_HITS] hit indices inside -> out, -1 padded */
  int32_t* cells;      /* [cap][PT_MAX_HITS-1] cell indices, -1 padded */
  uint8_t* n;          /* [cap] number of hits */
  int32_t* count_raw;  /* [1] paths found (may exceed cap) */
  int32_t* kept;       /* [cap] rows kept by duplicate removal */
  int32_t* count;      /* [1] number of kept rows */
} pt_ntuplets;

/* Fitted tracks, one per kept n-tuplet (or per row, see pt_fit_broken_line). */
typedef struct {
  int32_t cap;
  void* params;       /* [cap][5] (kappa, phi0, cot(theta), d0, z0): double for
                         PT_FIT_F64, float otherwise */
  void* chi2;         /* [cap] same type */
  uint8_t* status;    /* [cap] PT_FIT_ST_* bits */
  void* cov;          /* [cap][15] or NULL (not computed): the covariance of the
                         five parameters, same type, upper triangle row by row
                         ((0,0) (0,1) .. (0,4) (1,1) .. (4,4)) */
} pt_tracks;

/* Version of this interface (the value of PT_ABI_VERSION). */
#define PT_ABI_VERSION 2
int32_t pt_abi_version(void);
const char* pt_err_string(pt_err e);
/* The HIP error behind the calling thread's last PT_ERR_DEVICE, as
 * "hipErrorName: description" (a thread-local buffer, valid until the thread's
 * next call of this function); "" when no call on this thread has failed so. */
const char* pt_last_device_error(void);

/* Bytes of workspace the calls below need for these sizes.  0 on invalid arguments. */
size_t pt_workspace_size(const pt_config* cfg, int32_t n_hits, int32_t n_events,
                         int32_t cells_cap, int32_t links_cap, int32_t tuplets_cap);

/* Doublet building (section 3.2, Table 1).
 * For every layer pair p, every hit o on its outer layer and every hit i on
 * its inner layer of the same event, the doublet (i, o, p) is emitted when:
 *   PhiW  D = Xi Xo + Yi Yo > 0 and |C| <= tan_dphi[p] D, C = Xi Yo - Yi Xo
 *   ZW    pair_zlo[p] <= Zi <= pair_zhi[p]
 *   ZIP   Ro - Ri > 0 and |Zi Ro - Zo Ri| <= z0_max (Ro - Ri)
 *   PT    (4 C) C <= (kappa_max2 (R2i R2o)) L2, L2 = |P_o - P_i|^2
 * for the cuts in cut_mask, with X, Y, Z the hit coordinates in double,
 * R2 = X X + Y Y and R = sqrt(R2), evaluated exactly as parenthesised
 * without contraction.  Candidate inner hits come from azimuth bins around
 * the outer hit (the binned window of Table 1), widened by one bin so that the
 * result equals the all-pairs definition.
 * With fishbone_theta > 0 the Fishbone of section 3.3 follows: of two
 * doublets c = (a, h) and c' = (b, h) sharing their outer hit, with
 * u = P_h - P_a, v = P_h - P_b in double, w = u x v = (uy vz - uz vy,
 * uz vx - ux vz, ux vy - uy vx), W2 = (wx wx + wy wy) + wz wz and
 * U2, V2 the squared lengths in the same order, c is dropped when
 * W2 <= fishbone_theta^2 (U2 V2) and V2 < U2 (a shorter aligned doublet
 * exists).  The remaining cells keep their order, grouped by inner hit; when
 * the cells overflowed their capacity the Fishbone is not applied.
 * Requires a workspace of pt_workspace_size(cfg, hits->n_hits, hits->n_events, ...). */
pt_err pt_build_doublets(const pt_hits* hits, const pt_config* cfg, pt_cells* cells,
                         uint32_t* status, pt_workspace ws, pt_stream stream);

/* Cell linking (section 3.2: doublets sharing a hit tested for a triplet).
 * For c' = (h0, h1) and c = (h1, h2), the link c' -> c is made when
 *   R-Z   A A <= theta2 ((ar ar + az az) (br br + bz bz)),
 *         ar = R1 - R0, az = Z1 - Z0, br = R2 - R1, bz = Z2 - Z1, A = ar bz - az br,
 *         theta2 from the barrel value when h2 is on a barrel layer, else the end-cap value;
 *   beam  with u = P1 - P0, v = P2 - P0 (x, y) and Dd = 2 (ux vy - uy vx):
 *         Dd == 0: (X0 vy - Y0 vx)^2 <= rmax^2 (vx^2 + vy^2);
 *         else cx = (U2 vy - V2 uy) / Dd, cy = (V2 ux - U2 vx) / Dd, U2 = |u|^2,
 *         V2 = |v|^2, rho2 = cx^2 + cy^2, c2 = (X0 + cx)^2 + (Y0 + cy)^2 and
 *         |sqrt(c2) - sqrt(rho2)| <= rmax,
 *         rmax the BPix1 value when h0 is on layer 0, else the other value;
 * in double, as parenthesised, without contraction.  cells must be the
 * output of pt_build_doublets for the same hits (only min(count, cap) used). */
pt_err pt_link_cells(const pt_hits* hits, const pt_config* cfg, const pt_cells* cells,
                     pt_links* links, uint32_t* status, pt_workspace ws, pt_stream stream);

/* n-tuplet search and duplicate removal (section 3.2, section 3.3).
 * Root cells: inner hit on a layer of root_always_mask, or of
 * root_if_free_mask with has_inner == 0 (the inner hit's layer is read as
 * the inner layer of the cell's pair).  From every root a depth-first
 * search follows outer links; a path is emitted when its last cell has no
 * outer link or it has max_hits hits (then PT_ST_TRUNCATED counts it), and
 * it has at least min_hits hits.  A row is kept unless one of its cells
 * belongs to a row with more hits.  The links must be laid out as
 * pt_link_cells writes them (runs in cell order, links->count[0] after the
 * last); links->count may not be NULL. */
pt_err pt_find_ntuplets(const pt_hits* hits, const pt_config* cfg, const pt_cells* cells,
                        const pt_links* links, pt_ntuplets* tuplets, uint32_t* status,
                        pt_workspace ws, pt_stream stream);

/* Broken-line fit (section 3.4), one GPU thread per track.
 * Tracks are the kept rows of `tuplets` (tuplets->kept != NULL: track i is row
 * kept[i], i < count[0]) or, with kept == NULL, rows 0..count[0]-1.  The
 * number of tracks is read on the device; at most min(tuplets->cap, tracks->cap)
 * are fitted.  Hit k of a track is P_k = hit + module_offsets[module] when
 * module_offsets (device float [n_modules][3]) is not NULL.
 * Steps: a circle through hits 0, n/2 and n-1 (pre-fit); arc lengths s_k and
 * left offsets u_k of every hit along it; slope t and momentum
 * p = min(p_T sqrt(1+t^2), p_cap); Highland scattering at the inner hits with
 * material x_over_x0 times the path length (1/sin(theta) barrel,
 * 1/|cos(theta)| disks), kink variances theta0^2 (1+t^2) transverse and
 * theta0^2 (1+t^2)^2 in S-Z; measurement variances sigma_rphi^2 and
 * sigma_z^2 (barrel) or (sigma_r t)^2 (disks); the circle broken-line solve
 * for offsets and the curvature correction, the S-Z broken-line solve; the
 * perigee (kappa, phi0, cot(theta), d0, z0) with respect to the origin and
 * chi2 = circle + line chi^2 at the optimum (2n - 5 degrees of freedom).
 * When tracks->cov is not NULL it also writes the covariance of the five
 * parameters (section 3.4: the circle and line fits give parameters with
 * covariances, combined at the end): with the kinks as zero-mean
 * pseudo-measurements the covariance of the circle unknowns (offsets,
 * curvature correction) is the inverse of its normal matrix and that of the
 * line unknowns the inverse of its own; propagated through the linearised
 * perigee conversion (pre-fit held fixed), C = Jc Ac^-1 Jc^T + Jl Al^-1 Jl^T.
 * Hits must be ordered along the track; tracks that are not get NaN
 * parameters (and covariance) and PT_FIT_ST_BAD_ORDER. */
pt_err pt_fit_broken_line(const pt_hits* hits, const pt_config* cfg, const pt_ntuplets* tuplets,
                          const float* module_offsets, int32_t precision, pt_tracks* tracks,
                          uint32_t* status, pt_workspace ws, pt_stream stream);

/* Adjoint of pt_fit_broken_line (same tracks, same precision).  With the
 * upstream gradients g_params (device [cap][5]) and g_chi2 (device [cap], may
 * be NULL), both double for PT_FIT_F64 and float otherwise, adds
 *   grad_hits[h]    += sum over tracks t containing h of J_t(h)^T (g_params[t], g_chi2[t])
 *   grad_offsets[m] += sum over hits h on module m of the same
 * where J_t(h) = d(kappa, phi0, cot, d0, z0, chi2)_t / d(x, y, z)_h of the
 * whole fit, including its dependence through the pre-fit and the scattering
 * weights.  The forward fit is recomputed, not stored.  grad_hits is device
 * [n_hits][3], double for PT_FIT_F64 and float otherwise (may be NULL);
 * grad_offsets is device double [n_modules][3] (may be NULL); both are
 * accumulated into (atomically: hits may be shared between tracks, so the
 * order of the additions is not fixed).  Tracks whose fit fails add nothing. */
pt_err pt_fit_broken_line_bwd(const pt_hits* hits, const pt_config* cfg,
                              const pt_ntuplets* tuplets, const float* module_offsets,
                              int32_t precision, const void* g_params, const void* g_chi2,
                              void* grad_hits, double* grad_offsets, uint32_t* status,
                              pt_workspace ws, pt_stream stream);

/* Ambiguity resolution (section 3.5) among the fitted tracks of
 * pt_fit_broken_line (same tuplets, precision and tracks; cells are the
 * n-tuplets' cells, whose indices must lie below cells->cap).
 *   1. Tracks sharing a hit doublet (a cell) are ambiguous: a track is
 *      dropped when a track sharing one of its cells has a smaller chi2.
 *   2. Among the 3-hit tracks that survive 1, tracks sharing a hit are
 *      ambiguous: a triplet is dropped when a triplet sharing one of its
 *      hits has a smaller |d0| (transverse impact parameter).
 * Equal values keep both; tracks with a non-finite chi2 take no part and are
 * dropped.  Values are compared in the fit's precision.  selected (device
 * int32 [min(tuplets->cap, tracks->cap)]) receives the indices of the tracks
 * that stay, in increasing order, and n_selected[0] their number. */
pt_err pt_resolve_ambiguities(const pt_hits* hits, const pt_config* cfg, const pt_cells* cells,
                              const pt_ntuplets* tuplets, int32_t precision, const pt_tracks* tracks,
                              int32_t* selected, int32_t* n_selected, uint32_t* status, pt_workspace ws,
                              pt_stream stream);

/* Pixel vertices of each event (section 3.6). */
typedef struct {
  int32_t cap;           /* vertex capacity */
  double* z;             /* [cap] weighted mean of the tracks' z0 (cm) */
  double* var;           /* [cap] its variance */
  double* chi2;          /* [cap] sum of (z0 - z)^2 / var_z0 over the tracks */
  int32_t* ndf;          /* [cap] tracks - 1 */
  int32_t* n_tracks;     /* [cap] */
  double* sum_pt2;       /* [cap] sum of min(p_T, vtx_pt_cap)^2 over the tracks */
  int32_t* event_first;  /* [n_events + 1]: event e's vertices are [event_first[e], event_first[e+1]) */
  int32_t* count;        /* [1] vertices found (may exceed cap) */
  int32_t* track_vertex; /* [min(tuplets->cap, tracks->cap)] vertex of each track, -1 for none */
} pt_vertices;

/* Pixel vertices (section 3.6) from the fitted tracks, which must carry
 * their covariance (tracks->cov).  Tracks take part when selected (the
 * output of pt_resolve_ambiguities; every track when selected is NULL), with
 * at least vtx_min_hits hits, p_T = 0.299792458 B / 100 / |kappa| above
 * vtx_pt_min and a finite z0 with a positive variance var = cov[14].  A
 * track belongs to the event of its first hit.  Per event:
 *   density of track i (0 unless sqrt(var_i) <= vtx_err_max): the number of
 *     other tracks j with |z_i - z_j| < vtx_dz_cut and
 *     (z_i - z_j)^2 < vtx_chi2_max (var_i + var_j);
 *   each track links to the nearest track of higher rank (density, then
 *     track index) with |z_i - z_j| < vtx_dz_cut and
 *     (z_i - z_j)^2 <= vtx_chi2_max (var_i + var_j) (equal distances: the
 *     smaller index); the links form trees;
 *   a tree whose root has density > 1 and with at least 2 tracks is a
 *     vertex: with members in (z0, track index) order, weights 1/var,
 *     z = sum w z0 / sum w, var = 1 / sum w, chi2 = sum (z0 - z)^2 / var_z0,
 *     ndf = members - 1;
 *   a vertex with chi2/ndf > vtx_split_chi2_ndf is split by 1-D two-means:
 *     centres at its smallest and largest z0, members to the nearer centre
 *     (the first on a tie), centres to the weighted means, until no member
 *     moves or vtx_kmeans_iter rounds; each part with at least 2 members is
 *     a vertex (fitted as above), the members of a part of one are dropped;
 *   vertices are ordered by sum_pt2, largest first (the primary vertex);
 *     equal sums keep the order of their first member.
 * All of it in double, sums in member order, without contraction.  Vertices
 * beyond out->cap are counted but not written (PT_FLAG_VERTICES_OVERFLOW). */
pt_err pt_find_vertices(const pt_hits* hits, const pt_config* cfg, const pt_ntuplets* tuplets, int32_t precision,
                        const pt_tracks* tracks, const int32_t* selected, const int32_t* n_selected,
                        pt_vertices* out, uint32_t* status, pt_workspace ws, pt_stream stream);

/* The forward fit of pt_fit_broken_line for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same arguments without a workspace.  Its
 * scratch (the tracks binned by hit count and the list of tracks refitted in
 * double) is a fixed device array inside the library, one per GPU, which it
 * keeps until the process ends; the call allocates and frees nothing.
 * Limit: min(tuplets->cap, tracks->cap) <= PT_NOALLOC_FIT_MAX_TRACKS, else
 * PT_ERR_TOO_LARGE and nothing is enqueued.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (on different streams, or
 * from different threads) race and must be serialised by the caller.  The
 * call clears what it needs at the start, so consecutive calls are
 * independent.  Results equal those of pt_fit_broken_line. */
#define PT_NOALLOC_FIT_MAX_TRACKS 262144
pt_err pt_fit_broken_line_noalloc(const pt_hits* hits, const pt_config* cfg, const pt_ntuplets* tuplets,
                                  const float* module_offsets, int32_t precision, pt_tracks* tracks,
                                  uint32_t* status, pt_stream stream);

/* ------------------------------------------------------------------------
 * Batched plans: one hipGraph per step.
 *
 * A plan runs the whole path -- pt_build_doublets, pt_link_cells,
 * pt_find_ntuplets, pt_fit_broken_line, then the optional stages chosen at
 * creation: PT_STAGE_ADJOINT (pt_fit_broken_line_bwd), PT_STAGE_AMBIGUITY
 * (pt_resolve_ambiguities), PT_STAGE_VERTICES (pt_find_vertices over the
 * tracks the ambiguity stage selects, or over every track without it) -- over
 * all events of a batch as one graph launch.
 * pt_plan_create allocates the plan's workspace (this and pt_plan_destroy are
 * the only calls that allocate or free device memory) and a private,
 * default-priority capture stream.  The first pt_plan_run, and every run whose
 * arguments (pointers, sizes, capacities) differ from the captured ones,
 * records the step into a graph; every run then launches the graph on
 * `stream`.  Arguments have the meaning of the individual calls; g_params is
 * required with PT_STAGE_ADJOINT, selected and n_selected with
 * PT_STAGE_AMBIGUITY, vertices and tracks->cov with PT_STAGE_VERTICES (the
 * fit writes the covariance whenever tracks->cov is set).  A plan is not
 * thread-safe.  Sizes above the ones given at creation return PT_ERR_ARG. */
enum { PT_STAGE_ADJOINT = 1, PT_STAGE_AMBIGUITY = 2, PT_STAGE_VERTICES = 4 };
typedef struct pt_plan_s* pt_plan;
pt_err pt_plan_create(const pt_config* cfg, int32_t n_hits_max, int32_t n_events_max, int32_t cells_cap,
                      int32_t links_cap, int32_t tuplets_cap, int32_t precision, int32_t stages,
                      pt_plan* plan);
pt_err pt_plan_run(pt_plan plan, const pt_hits* hits, pt_cells* cells, pt_links* links, pt_ntuplets* tuplets,
                   pt_tracks* tracks, const float* module_offsets, const void* g_params, const void* g_chi2,
                   void* grad_hits, double* grad_offsets, int32_t* selected, int32_t* n_selected,
                   pt_vertices* vertices, uint32_t* status, pt_stream stream);
void pt_plan_destroy(pt_plan plan);

/* Kernel timing (instrumentation).  While enabled, the individual calls (not
 * graph launches) record a pair of HIP events around their main kernels on
 * their stream, one kernel each unless noted: "doublets_count",
 * "doublets_write", "fishbone" (every kernel of the Fishbone, when it is
 * on), "cell_index" (the index of cells by outer hit), "link_segments"
 * (placing the index segments), "links" (the triplet sweep), "link_emit"
 * (placing the links), "root_count", "root_write", "dfs_count",
 * "dfs_write", "dedup" (several kernels), "fit_fwd" and "fit_bwd" (every
 * kernel of the fit and of its adjoint).  pt_timing_read waits for the
 * recorded events and returns the summed milliseconds and the number of
 * launches since the last reset (PT_ERR_ARG when the name has no record). */
void pt_timing_enable(int32_t on);
void pt_timing_reset(void);
int32_t pt_timing_read(const char* kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* PIXELTRACK_H */
