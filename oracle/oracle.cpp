// CPU oracle of the pixel-track hot path.  TEST INFRASTRUCTURE ONLY.
//
// Plain and slow: predicates in double precision (the GPU library must
// reproduce them bit for bit), the fit in extended precision.  It exists so
// that tests, the smoke check and the CPU baseline of the benchmark have
// something obviously correct to compare the GPU library with.  It shares no
// code with the GPU library and is never called by it.  Built with
// -ffp-contract=off so that every predicate below is evaluated exactly as
// parenthesised.
//
// What it computes (Bocci et al., "Heterogeneous reconstruction of tracks and
// primary vertices with the CMS pixel tracker"):
//   * doublets between hits of chosen layer pairs, all inner x outer hits
//     tested by brute force against the cuts of Table 1 (section 3.2);
//   * cell links: doublets sharing a hit, compatible in R-Z alignment and in
//     the distance of their circle from the beam spot (section 3.2);
//   * n-tuplets: depth-first search from the root doublets over the cell
//     graph, keeping maximal paths only (section 3.2);
//   * duplicate removal: among n-tuplets sharing a hit doublet only those with
//     the most hits survive (section 3.3, last paragraph);
//   * the broken-line fit of each n-tuplet: a three-point pre-fit giving the
//     momentum for multiple scattering, a line fit in S-Z and a circle fit in
//     the transverse plane, combined into perigee parameters (section 3.4,
//     after Blobel's broken lines);
//   * the gradient of that fit with respect to hit coordinates by forward-mode
//     dual numbers through the same templated code.
//
// Where the paper gives names but no formulas (cut definitions, material,
// resolutions, the exact pre-fit) the readings are documented at each
// function.  Parity pins for every function live in tests/test_oracle_*.py.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

namespace {

constexpr int kMaxPairs = 32;
constexpr int kMaxHits = 8;
constexpr int kLayers = 10;

enum { CUT_PHIW = 1, CUT_ZW = 2, CUT_ZIP = 4, CUT_PT = 8 };

}  // namespace

extern "C" {

// Configuration as the Python side fills it (mirrors synth.config keys).
struct oracle_config {
  double bfield;
  int32_t n_pairs;
  int32_t pair_inner[kMaxPairs];
  int32_t pair_outer[kMaxPairs];
  double pair_dphi[kMaxPairs];
  double pair_zlo[kMaxPairs];
  double pair_zhi[kMaxPairs];
  double pt_min;
  double z0_max;
  int32_t cut_mask;
  double ca_theta_barrel;
  double ca_theta_endcap;
  double ca_rmax_bpix1;
  double ca_rmax_other;
  int32_t root_always_mask;
  int32_t root_if_free_mask;
  int32_t min_hits;
  int32_t max_hits;
  int32_t layer_barrel[kLayers];
  double x_over_x0;
  double highland_a;
  double highland_b;
  double sigma_rphi;
  double sigma_z;
  double sigma_r;
  double p_cap;
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Doublet cuts (section 3.2, Table 1).  For inner hit i and outer hit o:
//   PhiW: the azimuth difference is below the pair's window dphi:
//         D = Xi Xo + Yi Yo > 0  and  |Xi Yo - Yi Xo| <= tan(dphi) D
//   ZW:   zlo <= Zi <= zhi (window on the inner hit's z)
//   ZIP:  the straight R-Z line through both hits meets r = 0 within z0_max:
//         Ro - Ri > 0 and |Zi Ro - Zo Ri| <= z0_max (Ro - Ri)
//   PT:   the circle through the origin and both hits has curvature
//         <= kappa_max = 0.299792458 B / (100 pt_min):
//         (4 C) C <= (kappa_max^2 (Ri^2 Ro^2)) L^2 with C the cross product
//         and L the distance between the hits
// PhiHist (the 128-bin histogram of Table 1) is a search structure, not a
// predicate; the brute force here needs none.
struct DoubletCuts {
  double tan_dphi[kMaxPairs];
  double zlo[kMaxPairs], zhi[kMaxPairs];
  double z0_max;
  double kappa_max2;
  int mask;
};

DoubletCuts doublet_cuts(const oracle_config& c) {
  DoubletCuts k{};
  for (int p = 0; p < c.n_pairs; ++p) {
    k.tan_dphi[p] = std::tan(c.pair_dphi[p]);
    k.zlo[p] = c.pair_zlo[p];
    k.zhi[p] = c.pair_zhi[p];
  }
  k.z0_max = c.z0_max;
  const double kappa_max = (0.299792458 * c.bfield) / (100.0 * c.pt_min);
  k.kappa_max2 = kappa_max * kappa_max;
  k.mask = c.cut_mask;
  return k;
}

bool doublet_passes(const DoubletCuts& k, int p, double Xi, double Yi, double Zi,
                    double Xo, double Yo, double Zo) {
  const double R2i = Xi * Xi + Yi * Yi;
  const double R2o = Xo * Xo + Yo * Yo;
  const double Ri = std::sqrt(R2i);
  const double Ro = std::sqrt(R2o);
  const double D = Xi * Xo + Yi * Yo;
  const double C = Xi * Yo - Yi * Xo;
  if (k.mask & CUT_PHIW) {
    if (!(D > 0.0 && std::fabs(C) <= k.tan_dphi[p] * D)) return false;
  }
  if (k.mask & CUT_ZW) {
    if (!(k.zlo[p] <= Zi && Zi <= k.zhi[p])) return false;
  }
  if (k.mask & CUT_ZIP) {
    const double dR = Ro - Ri;
    if (!(dR > 0.0 && std::fabs(Zi * Ro - Zo * Ri) <= k.z0_max * dR)) return false;
  }
  if (k.mask & CUT_PT) {
    const double dx = Xo - Xi;
    const double dy = Yo - Yi;
    const double L2 = dx * dx + dy * dy;
    if (!((4.0 * C) * C <= (k.kappa_max2 * (R2i * R2o)) * L2)) return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Triplet compatibility (section 3.2): two doublets (h0,h1) and (h1,h2)
//   R-Z alignment: the sine of the kink between the two R-Z segments is at
//     most theta:  A = a_r b_z - a_z b_r,
//     A A <= theta^2 ((a_r a_r + a_z a_z) (b_r b_r + b_z b_z));
//     theta is the barrel value when h2 is on a barrel layer, else the
//     end-cap value (barrel and end-caps get separate cuts, section 4.2).
//   Beam spot: the circle through the three hits passes within r_max of the
//     beam line (at the origin): | |centre| - radius | <= r_max, with the
//     straight-line distance when the three hits are collinear; r_max is the
//     BPix1 value when h0 is on BPix1, else the other value.
struct LinkCuts {
  double theta2_barrel, theta2_endcap;
  double rmax_bpix1, rmax_other;
  int barrel[kLayers];
};

LinkCuts link_cuts(const oracle_config& c) {
  LinkCuts k{};
  k.theta2_barrel = c.ca_theta_barrel * c.ca_theta_barrel;
  k.theta2_endcap = c.ca_theta_endcap * c.ca_theta_endcap;
  k.rmax_bpix1 = c.ca_rmax_bpix1;
  k.rmax_other = c.ca_rmax_other;
  for (int l = 0; l < kLayers; ++l) k.barrel[l] = c.layer_barrel[l];
  return k;
}

bool link_passes(const LinkCuts& k, int layer0, int layer2,
                 double X0, double Y0, double Z0,
                 double X1, double Y1, double Z1,
                 double X2, double Y2, double Z2) {
  const double R0 = std::sqrt(X0 * X0 + Y0 * Y0);
  const double R1 = std::sqrt(X1 * X1 + Y1 * Y1);
  const double R2 = std::sqrt(X2 * X2 + Y2 * Y2);
  const double ar = R1 - R0, az = Z1 - Z0;
  const double br = R2 - R1, bz = Z2 - Z1;
  const double A = ar * bz - az * br;
  const double theta2 = k.barrel[layer2] ? k.theta2_barrel : k.theta2_endcap;
  if (!(A * A <= theta2 * ((ar * ar + az * az) * (br * br + bz * bz)))) return false;

  const double rmax = (layer0 == 0) ? k.rmax_bpix1 : k.rmax_other;
  const double ux = X1 - X0, uy = Y1 - Y0;
  const double vx = X2 - X0, vy = Y2 - Y0;
  const double Dd = 2.0 * (ux * vy - uy * vx);
  if (Dd == 0.0) {
    const double cr = X0 * vy - Y0 * vx;
    return cr * cr <= (rmax * rmax) * (vx * vx + vy * vy);
  }
  const double U2 = ux * ux + uy * uy;
  const double V2 = vx * vx + vy * vy;
  const double cx = (U2 * vy - V2 * uy) / Dd;
  const double cy = (V2 * ux - U2 * vx) / Dd;
  const double rho2 = cx * cx + cy * cy;
  const double Cx = X0 + cx, Cy = Y0 + cy;
  const double c2 = Cx * Cx + Cy * Cy;
  return std::fabs(std::sqrt(c2) - std::sqrt(rho2)) <= rmax;
}

}  // namespace

extern "C" {

// All doublets of one event.  Hits are the arrays as given (indices 0..n-1).
// For every pair p, every outer hit o on the pair's outer layer and every
// inner hit i on its inner layer, in that order, the doublet (i, o, p) is
// emitted when it passes the cuts.  Returns the number found; only the first
// `cap` are written.
int64_t oracle_doublets(const oracle_config* cfg, int32_t n, const double* x, const double* y,
                        const double* z, const uint8_t* layer, int64_t cap, int32_t* inner,
                        int32_t* outer, uint8_t* pair) {
  const DoubletCuts k = doublet_cuts(*cfg);
  std::vector<std::vector<int32_t>> by_layer(kLayers);
  for (int32_t h = 0; h < n; ++h) by_layer[layer[h]].push_back(h);
  int64_t count = 0;
  for (int p = 0; p < cfg->n_pairs; ++p) {
    const auto& outs = by_layer[cfg->pair_outer[p]];
    const auto& ins = by_layer[cfg->pair_inner[p]];
    for (int32_t o : outs) {
      for (int32_t i : ins) {
        if (doublet_passes(k, p, x[i], y[i], z[i], x[o], y[o], z[o])) {
          if (count < cap) {
            inner[count] = i;
            outer[count] = o;
            pair[count] = static_cast<uint8_t>(p);
          }
          ++count;
        }
      }
    }
  }
  return count;
}

// The same doublets found faster: the hits of each layer binned in azimuth
// (n_bins bins of width w), and for each outer hit only the inner hits of
// the bins within ceil(dphi / w) + 1 of its own bin are tested -- a pair
// passing the PhiW cut differs in azimuth by less than dphi, and the extra
// bin absorbs the rounding of atan2 -- with the same predicate as above.
// Without the PhiW cut every bin is scanned.  The set equals the brute-force
// set (in another order).
int64_t oracle_doublets_binned(const oracle_config* cfg, int32_t n, const double* x, const double* y,
                               const double* z, const uint8_t* layer, int32_t n_bins, int64_t cap,
                               int32_t* inner, int32_t* outer, uint8_t* pair) {
  const DoubletCuts k = doublet_cuts(*cfg);
  if (n_bins < 1) n_bins = 1;
  const double w = 2.0 * M_PI / n_bins;
  auto bin_of = [&](int32_t h) {
    int b = static_cast<int>(std::floor((std::atan2(y[h], x[h]) + M_PI) / w));
    return std::min(std::max(b, 0), n_bins - 1);
  };
  std::vector<std::vector<std::vector<int32_t>>> bins(kLayers, std::vector<std::vector<int32_t>>(n_bins));
  for (int32_t h = 0; h < n; ++h) bins[layer[h]][bin_of(h)].push_back(h);
  int64_t count = 0;
  for (int p = 0; p < cfg->n_pairs; ++p) {
    int wb = n_bins;
    if (cfg->cut_mask & CUT_PHIW) wb = static_cast<int>(std::ceil(cfg->pair_dphi[p] / w)) + 1;
    const bool all = 2 * wb + 1 >= n_bins;
    for (int bo = 0; bo < n_bins; ++bo) {
      for (int32_t o : bins[cfg->pair_outer[p]][bo]) {
        const int first = all ? 0 : bo - wb, last = all ? n_bins - 1 : bo + wb;
        for (int bb = first; bb <= last; ++bb) {
          const int b = ((bb % n_bins) + n_bins) % n_bins;
          for (int32_t i : bins[cfg->pair_inner[p]][b]) {
            if (doublet_passes(k, p, x[i], y[i], z[i], x[o], y[o], z[o])) {
              if (count < cap) {
                inner[count] = i;
                outer[count] = o;
                pair[count] = static_cast<uint8_t>(p);
              }
              ++count;
            }
          }
        }
      }
    }
  }
  return count;
}

// Fishbone (section 3.3): among the doublets that share their outer hit, a
// doublet is dropped when another one is aligned with it and shorter.  For
// c = (a, h) and c' = (b, h), with u = P_h - P_a and v = P_h - P_b in double:
//   w = u x v = (uy vz - uz vy, uz vx - ux vz, ux vy - uy vx),
//   W2 = (wx wx + wy wy) + wz wz, U2 = (ux ux + uy uy) + uz uz, V2 likewise;
//   aligned iff W2 <= theta2 (U2 V2) (the sine of the angle between the two
//   doublets is at most theta), and c is dropped iff such a c' has V2 < U2.
// keep [n_cells] receives 1 for the doublets that stay.  Returns how many.
int64_t oracle_fishbone(double theta2, int32_t n, const double* x, const double* y, const double* z,
                        int32_t n_cells, const int32_t* cell_inner, const int32_t* cell_outer, uint8_t* keep) {
  std::vector<std::vector<int32_t>> ending_at(n);
  for (int32_t c = 0; c < n_cells; ++c) ending_at[cell_outer[c]].push_back(c);
  int64_t kept = 0;
  for (int32_t c = 0; c < n_cells; ++c) {
    const int32_t a = cell_inner[c], h = cell_outer[c];
    const double ux = x[h] - x[a], uy = y[h] - y[a], uz = z[h] - z[a];
    const double U2 = (ux * ux + uy * uy) + uz * uz;
    bool stay = true;
    for (int32_t d : ending_at[h]) {
      if (d == c) continue;
      const int32_t b = cell_inner[d];
      const double vx = x[h] - x[b], vy = y[h] - y[b], vz = z[h] - z[b];
      const double V2 = (vx * vx + vy * vy) + vz * vz;
      if (!(V2 < U2)) continue;
      const double wx = uy * vz - uz * vy, wy = uz * vx - ux * vz, wz = ux * vy - uy * vx;
      const double W2 = (wx * wx + wy * wy) + wz * wz;
      if (W2 <= theta2 * (U2 * V2)) {
        stay = false;
        break;
      }
    }
    keep[c] = stay ? 1 : 0;
    kept += stay;
  }
  return kept;
}

// Cell links of one event: for every cell c = (h1, h2) and every cell
// c' = (h0, h1) ending on its inner hit, the link (c' -> c) when the triplet
// passes the cuts.  Cells are given as (inner, outer) hit index arrays.
// Returns the number of links; only the first `cap` are written.
int64_t oracle_links(const oracle_config* cfg, int32_t n, const double* x, const double* y,
                     const double* z, const uint8_t* layer, int32_t n_cells,
                     const int32_t* cell_inner, const int32_t* cell_outer, int64_t cap,
                     int32_t* link_in, int32_t* link_out) {
  const LinkCuts k = link_cuts(*cfg);
  std::vector<std::vector<int32_t>> ending_at(n);
  for (int32_t c = 0; c < n_cells; ++c) ending_at[cell_outer[c]].push_back(c);
  int64_t count = 0;
  for (int32_t c = 0; c < n_cells; ++c) {
    const int32_t h1 = cell_inner[c], h2 = cell_outer[c];
    for (int32_t cp : ending_at[h1]) {
      const int32_t h0 = cell_inner[cp];
      if (link_passes(k, layer[h0], layer[h2], x[h0], y[h0], z[h0], x[h1], y[h1], z[h1], x[h2],
                      y[h2], z[h2])) {
        if (count < cap) {
          link_in[count] = cp;
          link_out[count] = c;
        }
        ++count;
      }
    }
  }
  return count;
}

// n-tuplets of one event (section 3.2, then the duplicate removal of section
// 3.3).  Root doublets: inner hit on a layer in root_always_mask, or on a
// layer in root_if_free_mask with no inner neighbour.  From every root a
// depth-first search follows outer links; a path is emitted when it cannot be
// extended (or has reached max_hits hits, which sets *truncated) and has at
// least min_hits hits.  With dedup != 0, an n-tuplet is then dropped when one
// of its cells belongs to an n-tuplet with more hits.
//
// Output: hits [cap][8] (-1 padded, inside -> out), cells [cap][7], nhits
// [cap].  Returns the number of n-tuplets (after dedup when requested);
// *n_raw receives the count before dedup.
int64_t oracle_ntuplets(const oracle_config* cfg, int32_t n, const uint8_t* layer, int32_t n_cells,
                        const int32_t* cell_inner, const int32_t* cell_outer, int32_t n_links,
                        const int32_t* link_in, const int32_t* link_out, int32_t dedup,
                        int64_t cap, int32_t* out_hits, int32_t* out_cells, uint8_t* out_n,
                        int64_t* n_raw, int32_t* truncated) {
  (void)n;
  std::vector<std::vector<int32_t>> outer_links(n_cells);
  std::vector<uint8_t> has_inner(n_cells, 0);
  for (int32_t l = 0; l < n_links; ++l) {
    outer_links[link_in[l]].push_back(link_out[l]);
    has_inner[link_out[l]] = 1;
  }
  const int max_hits = std::min<int>(cfg->max_hits, kMaxHits);
  std::vector<std::vector<int32_t>> paths;  // each: the cells of a path
  *truncated = 0;
  std::vector<int32_t> path;
  // Recursive depth-first search, written with an explicit lambda.
  struct Dfs {
    const std::vector<std::vector<int32_t>>& links;
    int max_hits, min_hits;
    std::vector<std::vector<int32_t>>& paths;
    int32_t* truncated;
    void go(std::vector<int32_t>& path) {
      const int32_t last = path.back();
      const int nh = static_cast<int>(path.size()) + 1;
      if (links[last].empty() || nh == max_hits) {
        if (!links[last].empty()) *truncated = 1;
        if (nh >= min_hits) paths.push_back(path);
        return;
      }
      for (int32_t next : links[last]) {
        path.push_back(next);
        go(path);
        path.pop_back();
      }
    }
  } dfs{outer_links, max_hits, cfg->min_hits, paths, truncated};
  for (int32_t c = 0; c < n_cells; ++c) {
    const int L = layer[cell_inner[c]];
    const bool root = ((cfg->root_always_mask >> L) & 1) ||
                      (((cfg->root_if_free_mask >> L) & 1) && !has_inner[c]);
    if (!root) continue;
    path.assign(1, c);
    dfs.go(path);
  }
  *n_raw = static_cast<int64_t>(paths.size());

  std::vector<uint8_t> keep(paths.size(), 1);
  if (dedup) {
    std::vector<int> max_n(n_cells, 0);
    for (const auto& p : paths)
      for (int32_t c : p) max_n[c] = std::max<int>(max_n[c], static_cast<int>(p.size()) + 1);
    for (size_t t = 0; t < paths.size(); ++t)
      for (int32_t c : paths[t])
        if (max_n[c] != static_cast<int>(paths[t].size()) + 1) keep[t] = 0;
  }
  int64_t count = 0;
  for (size_t t = 0; t < paths.size(); ++t) {
    if (!keep[t]) continue;
    if (count < cap) {
      const auto& p = paths[t];
      for (int k = 0; k < kMaxHits; ++k) out_hits[count * kMaxHits + k] = -1;
      for (int k = 0; k < kMaxHits - 1; ++k) out_cells[count * (kMaxHits - 1) + k] = -1;
      out_hits[count * kMaxHits + 0] = cell_inner[p[0]];
      for (size_t j = 0; j < p.size(); ++j) {
        out_hits[count * kMaxHits + j + 1] = cell_outer[p[j]];
        out_cells[count * (kMaxHits - 1) + j] = p[j];
      }
      out_n[count] = static_cast<uint8_t>(p.size() + 1);
    }
    ++count;
  }
  return count;
}

}  // extern "C"

// ===========================================================================
// Broken-line fit (section 3.4), templated on the scalar so that the same code
// runs in double and in forward-mode dual numbers.

namespace {

struct Dual {
  long double v;  // value
  long double d;  // derivative along the seeded direction
};
inline Dual mk(double v) { return {v, 0.0L}; }
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  const long double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
inline Dual sqrt(Dual a) {
  const long double r = std::sqrt(a.v);
  return {r, a.d / (2.0L * r)};
}
inline Dual asin(Dual a) { return {std::asin(a.v), a.d / std::sqrt(1.0L - a.v * a.v)}; }
inline Dual atan(Dual a) { return {std::atan(a.v), a.d / (1.0L + a.v * a.v)}; }
inline Dual atan2(Dual y, Dual x) {
  const long double r2 = x.v * x.v + y.v * y.v;
  return {std::atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2};
}
inline Dual log(Dual a) { return {std::log(a.v), a.d / a.v}; }
inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }
inline double val(Dual a) { return static_cast<double>(a.v); }
inline double val(double a) { return a; }
inline double val(long double a) { return static_cast<double>(a); }
template <class T> inline T cst(double v) { return T(v); }
template <> inline Dual cst<Dual>(double v) { return mk(v); }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }

using std::asin;
using std::atan;
using std::atan2;
using std::fabs;
using std::log;
using std::sqrt;

// The fit's values are evaluated in extended precision (x87 long double, 64-bit
// significand): its plain centre-based pre-fit and dense elimination lose up
// to ~2e-9 relative on the stiffest forward tracks in double, more than the
// double-precision GPU path it checks.  The dual numbers of the gradient carry
// extended-precision values and derivatives for the same reason.
using Real = long double;

struct FitSettings {
  double K;             // 0.299792458 B / 100: p_T [GeV] = K / |kappa| [1/cm]
  double x_over_x0, ha, hb;
  double VT;            // transverse measurement variance
  double VZ_barrel;     // sigma_z^2
  double VR_disk;       // sigma_r^2
  double p_cap;
  int barrel[kLayers];
};

FitSettings fit_settings(const oracle_config& c) {
  FitSettings f{};
  f.K = 0.299792458 * c.bfield / 100.0;
  f.x_over_x0 = c.x_over_x0;
  f.ha = c.highland_a;
  f.hb = c.highland_b;
  f.VT = c.sigma_rphi * c.sigma_rphi;
  f.VZ_barrel = c.sigma_z * c.sigma_z;
  f.VR_disk = c.sigma_r * c.sigma_r;
  f.p_cap = c.p_cap;
  for (int l = 0; l < kLayers; ++l) f.barrel[l] = c.layer_barrel[l];
  return f;
}

enum { FIT_OK = 0, FIT_BAD_ORDER = 1, FIT_SINGULAR = 4 };

// Solve A x = b (dense, m x m, row-major) by Gaussian elimination with
// partial pivoting.  Returns false when a pivot is exactly zero.
template <class T>
bool gauss_solve(int m, std::vector<T> A, std::vector<T> b, std::vector<T>& x) {
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(val(A[r * m + col])) > std::fabs(val(A[piv * m + col]))) piv = r;
    if (val(A[piv * m + col]) == 0.0) return false;
    if (piv != col) {
      for (int j = 0; j < m; ++j) std::swap(A[col * m + j], A[piv * m + j]);
      std::swap(b[col], b[piv]);
    }
    for (int r = col + 1; r < m; ++r) {
      const T f = A[r * m + col] / A[col * m + col];
      for (int j = col; j < m; ++j) A[r * m + j] = A[r * m + j] - f * A[col * m + j];
      b[r] = b[r] - f * b[col];
    }
  }
  x.assign(m, cst<T>(0.0));
  for (int r = m - 1; r >= 0; --r) {
    T s = b[r];
    for (int j = r + 1; j < m; ++j) s = s - A[r * m + j] * x[j];
    x[r] = s / A[r * m + r];
  }
  return true;
}

template <class T>
struct FitResult {
  T kappa, phi0, cot, d0, z0, chi2;
  int status;
  // intermediate quantities, exported for the tests' independent checks
  std::vector<T> s, um, delta, wT, wZ, VZ, ucirc, vline;
  T kappa_pre, t_pre, p;
  T tx, ty;  // direction of the pre-fit at P_0
  std::vector<T> A, b, N, q;
};

// 8. Perigee parameters from the fitted quantities at s = 0 (section 3.4:
// the circle fit gives d0, p_T and phi, the line fit cot(theta) and the z
// of the point of closest approach, combined here).
//   u0, u1, dk   circle solution: offsets at hits 0 and 1, curvature correction
//   v0, v1       line solution: z at hits 0 and 1
//   kappa_pre, D0 (= s_1 - s_0), P_0 = (X0, Y0) and the pre-fit direction
//   (tx, ty) at P_0 define the local frame.
// The fitted point is Q = P_0 + u0 n (n the left normal), its direction psi
// the pre-fit direction turned by atan(u'_0) with
// u'_0 = (u1 - u0) / D0 - dk D0 / 2; the circle of curvature
// kappa = kappa_pre + dk through Q with direction psi has the signed distance
// d0 to the origin (U = kappa |Q|^2 + 2 Q x (cos psi, sin psi),
// d0 = U / (1 + sqrt(1 + kappa U))) and the direction phi0 at its point of
// closest approach; cot(theta) = (v1 - v0) / D0, and z0 extrapolates v0 back
// along the arc ds from the point of closest approach to Q.
template <class T>
void perigee(T u0, T u1, T dk, T v0, T v1, T kappa_pre, T D0, T X0, T Y0, T tx, T ty, T out[5]) {
  const T one = cst<T>(1.0), two = cst<T>(2.0);
  const T nx = -ty, ny = tx;
  const T kappa = kappa_pre + dk;
  const T Qx = X0 + u0 * nx;
  const T Qy = Y0 + u0 * ny;
  const T du0 = (u1 - u0) / D0 - dk * D0 / two;
  // direction psi = psi_pre + atan(du0): (tx, ty) rotated by atan(du0)
  const T ca = one / sqrt(one + du0 * du0);
  const T sa = du0 * ca;
  const T cpsi = tx * ca - ty * sa;
  const T spsi = ty * ca + tx * sa;
  const T U = kappa * (Qx * Qx + Qy * Qy) + two * (-Qx * spsi + Qy * cpsi);
  const T d0 = U / (one + sqrt(one + kappa * U));
  // direction at the point of closest approach
  const T hx = cpsi + kappa * Qy, hy = spsi - kappa * Qx;
  const T phi0 = atan2(hy, hx);
  const T hn = sqrt(hx * hx + hy * hy);
  const T cph = hx / hn, sph = hy / hn;
  const T at = Qx * cph + Qy * sph;
  const T an = -Qx * sph + Qy * cph;
  T ds = at;
  if (val(kappa) != 0.0) ds = atan2(kappa * at, one + kappa * (d0 - an)) / kappa;
  const T cot = (v1 - v0) / D0;
  const T z0 = v0 - cot * ds;
  out[0] = kappa;
  out[1] = phi0;
  out[2] = cot;
  out[3] = d0;
  out[4] = z0;
}

// The fit of one n-tuplet, hits P_k = (X_k, Y_k, Z_k), k = 0..n-1, inside out.
//
// 1. Pre-fit: the circle through P_0, P_b (b = n/2 rounded down) and P_{n-1};
//    its curvature kappa_pre > 0 when the three points turn counter-clockwise.
//    The momentum estimate p_T = K / |kappa_pre| feeds multiple scattering.
// 2. Along that circle: s_k, the arc length from P_0 to the foot of P_k
//    (chord form), and u_k, the signed offset of P_k to the left of the
//    circle.  The s_k must increase.
// 3. Slope t = (Z_{n-1} - Z_0) / s_{n-1}; p = min(p_T sqrt(1 + t^2), p_cap).
// 4. Scattering at every inner hit k = 1..n-2 (Highland): with material
//    X = x/X0 * path length (1/sin(theta) in the barrel, 1/|cos(theta)| on
//    disks), theta0^2 = (a/p)^2 X (1 + b ln X)^2; projected kink variances
//    theta0^2 (1+t^2) in the transverse plane and theta0^2 (1+t^2)^2 in S-Z.
// 5. Measurement variances: sigma_rphi^2 transverse; sigma_z^2 on barrel
//    layers and (sigma_r t)^2 on disks longitudinally.
// 6. Circle fit: unknowns u_0..u_{n-1} and the curvature correction dk,
//    minimising sum (um_k - u_k)^2 / VT + sum beta_k^2 / thetaT_k^2 with the
//    kink beta_k = (u_{k+1}-u_k)/D_k - (u_k-u_{k-1})/D_{k-1} - dk (D_{k-1}+D_k)/2.
// 7. Line fit: unknowns v_0..v_{n-1}, minimising sum (Z_k - v_k)^2 / VZ_k +
//    sum gamma_k^2 / thetaZ_k^2, gamma_k the same second difference of v.
// 8. Perigee: kappa = kappa_pre + dk; the fitted point Q = P_0 + u_0 n_0 and
//    direction psi = psi_pre + atan(u'_0) at s = 0 give d0 and phi0 of the
//    circle of curvature kappa through Q; cot(theta) = (v_1 - v_0)/D_0 and z0
//    extrapolates v_0 back to the point of closest approach.
//    chi2 = chi2_circle + chi2_line at the optimum (2n - 5 degrees of freedom).
template <class T>
FitResult<T> fit_track(const FitSettings& F, int n, const T* X, const T* Y, const T* Z,
                       const int* lay) {
  FitResult<T> R;
  R.status = FIT_OK;
  const T zero = cst<T>(0.0), one = cst<T>(1.0), two = cst<T>(2.0);
  const int b = n / 2;

  // 1. pre-fit circle
  const T ux = X[b] - X[0], uy = Y[b] - Y[0];
  const T vx = X[n - 1] - X[0], vy = Y[n - 1] - Y[0];
  const T Dd = two * (ux * vy - uy * vx);
  const T wx = X[n - 1] - X[b], wy = Y[n - 1] - Y[b];
  const double sigma = (val(ux * wy - uy * wx) >= 0.0) ? 1.0 : -1.0;
  const bool straight = val(Dd) == 0.0;
  T cx = zero, cy = zero, rho = zero, kappa_pre = zero;
  if (!straight) {
    const T U2 = ux * ux + uy * uy, V2 = vx * vx + vy * vy;
    const T ccx = (U2 * vy - V2 * uy) / Dd;
    const T ccy = (V2 * ux - U2 * vx) / Dd;
    cx = X[0] + ccx;
    cy = Y[0] + ccy;
    rho = sqrt(ccx * ccx + ccy * ccy);
    kappa_pre = cst<T>(sigma) / rho;
  }
  R.kappa_pre = kappa_pre;

  // direction of motion and left normal of the pre-fit at P_0
  T tx, ty;
  if (!straight) {
    const T rx = X[0] - cx, ry = Y[0] - cy;
    tx = cst<T>(sigma) * (-ry) / rho;
    ty = cst<T>(sigma) * rx / rho;
  } else {
    const T lv = sqrt(vx * vx + vy * vy);
    tx = vx / lv;
    ty = vy / lv;
  }
  const T nx = -ty, ny = tx;
  R.tx = tx;
  R.ty = ty;

  // 2. arc lengths and offsets
  R.s.assign(n, zero);
  R.um.assign(n, zero);
  T f0x = X[0], f0y = Y[0];
  if (!straight) {
    const T dx0 = X[0] - cx, dy0 = Y[0] - cy;
    const T l0 = sqrt(dx0 * dx0 + dy0 * dy0);
    f0x = cx + rho * dx0 / l0;
    f0y = cy + rho * dy0 / l0;
  }
  // P_0 is on the pre-fit circle: s_0 = 0 and u_0 = 0 by definition.
  for (int k = 1; k < n; ++k) {
    if (straight) {
      const T rx = X[k] - X[0], ry = Y[k] - Y[0];
      R.s[k] = rx * tx + ry * ty;
      R.um[k] = rx * nx + ry * ny;
      continue;
    }
    const T dx = X[k] - cx, dy = Y[k] - cy;
    const T lk = sqrt(dx * dx + dy * dy);
    const T fx = cx + rho * dx / lk, fy = cy + rho * dy / lk;
    const T chx = fx - f0x, chy = fy - f0y;
    const T d = sqrt(chx * chx + chy * chy);
    T s = d;
    if (val(d) > 0.0) {
      const T half = fabs(kappa_pre) * d / two;
      s = d * asin(half) / half;
    }
    const double ahead = val(chx * tx + chy * ty);
    R.s[k] = (ahead >= 0.0) ? s : -s;
    R.um[k] = -cst<T>(sigma) * (lk - rho);
  }
  R.delta.assign(n - 1, zero);
  for (int k = 0; k + 1 < n; ++k) {
    R.delta[k] = R.s[k + 1] - R.s[k];
    if (!(val(R.delta[k]) > 0.0)) R.status = FIT_BAD_ORDER;
  }
  if (R.status != FIT_OK) return R;

  // 3. slope and momentum
  const T t = (Z[n - 1] - Z[0]) / R.s[n - 1];
  const T sec2 = one + t * t;  // 1 + cot^2 = 1 / sin^2(theta)
  T p = cst<T>(F.p_cap);
  if (val(kappa_pre) != 0.0) {
    const T pt = cst<T>(F.K) / fabs(kappa_pre);
    const T pp = pt * sqrt(sec2);
    if (val(pp) < F.p_cap) p = pp;
  }
  R.t_pre = t;
  R.p = p;

  // 4. scattering weights at the inner hits
  R.wT.assign(n, zero);
  R.wZ.assign(n, zero);
  for (int k = 1; k + 1 < n; ++k) {
    T path = sqrt(sec2);
    if (!F.barrel[lay[k]]) path = path / fabs(t);
    const T Xm = cst<T>(F.x_over_x0) * path;
    const T lg = one + cst<T>(F.hb) * log(Xm);
    const T th0 = (cst<T>(F.ha) / p);
    const T theta02 = th0 * th0 * Xm * lg * lg;
    R.wT[k] = one / (theta02 * sec2);
    R.wZ[k] = one / (theta02 * sec2 * sec2);
  }

  // 5. longitudinal measurement variances
  R.VZ.assign(n, zero);
  for (int k = 0; k < n; ++k)
    R.VZ[k] = F.barrel[lay[k]] ? cst<T>(F.VZ_barrel) : cst<T>(F.VR_disk) * t * t;

  // 6. circle fit, dense normal equations of size n + 1
  const int m = n + 1;
  std::vector<T> A(m * m, zero), rhs(m, zero), xsol;
  const T wmeas = one / cst<T>(F.VT);
  for (int k = 0; k < n; ++k) {
    A[k * m + k] = A[k * m + k] + wmeas;
    rhs[k] = R.um[k] * wmeas;
  }
  auto kink_row = [&](int k, std::vector<T>& g, bool with_kappa) {
    g.assign(m, zero);
    g[k - 1] = one / R.delta[k - 1];
    g[k] = -(one / R.delta[k - 1]) - one / R.delta[k];
    g[k + 1] = one / R.delta[k];
    if (with_kappa) g[n] = -(R.delta[k - 1] + R.delta[k]) / two;
  };
  std::vector<T> g;
  for (int k = 1; k + 1 < n; ++k) {
    kink_row(k, g, true);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) A[i * m + j] = A[i * m + j] + R.wT[k] * g[i] * g[j];
  }
  R.A = A;
  R.b = rhs;
  if (!gauss_solve(m, A, rhs, xsol)) {
    R.status = FIT_SINGULAR;
    return R;
  }
  R.ucirc = xsol;
  T chi2T = zero;
  for (int k = 0; k < n; ++k) {
    const T r = R.um[k] - xsol[k];
    chi2T = chi2T + r * r * wmeas;
  }
  for (int k = 1; k + 1 < n; ++k) {
    kink_row(k, g, true);
    T beta = zero;
    for (int i = 0; i < m; ++i) beta = beta + g[i] * xsol[i];
    chi2T = chi2T + beta * beta * R.wT[k];
  }

  // 7. line fit, n x n
  std::vector<T> N(n * n, zero), q(n, zero), vsol;
  for (int k = 0; k < n; ++k) {
    N[k * n + k] = N[k * n + k] + one / R.VZ[k];
    q[k] = Z[k] / R.VZ[k];
  }
  for (int k = 1; k + 1 < n; ++k) {
    kink_row(k, g, false);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) N[i * n + j] = N[i * n + j] + R.wZ[k] * g[i] * g[j];
  }
  R.N = N;
  R.q = q;
  if (!gauss_solve(n, N, q, vsol)) {
    R.status = FIT_SINGULAR;
    return R;
  }
  R.vline = vsol;
  T chi2Z = zero;
  for (int k = 0; k < n; ++k) {
    const T r = Z[k] - vsol[k];
    chi2Z = chi2Z + r * r / R.VZ[k];
  }
  for (int k = 1; k + 1 < n; ++k) {
    kink_row(k, g, false);
    T gam = zero;
    for (int i = 0; i < n; ++i) gam = gam + g[i] * vsol[i];
    chi2Z = chi2Z + gam * gam * R.wZ[k];
  }

  // 8. perigee parameters
  T par[5];
  perigee<T>(xsol[0], xsol[1], xsol[n], vsol[0], vsol[1], kappa_pre, R.delta[0], X[0], Y[0], tx, ty, par);
  R.kappa = par[0];
  R.phi0 = par[1];
  R.cot = par[2];
  R.d0 = par[3];
  R.z0 = par[4];
  R.chi2 = chi2T + chi2Z;
  return R;
}

void gather(int n, const int32_t* hit, const double* x, const double* y, const double* z,
            const uint8_t* layer, const int16_t* module, const double* offsets, double* X,
            double* Y, double* Z, int* lay) {
  for (int k = 0; k < n; ++k) {
    const int32_t h = hit[k];
    X[k] = x[h];
    Y[k] = y[h];
    Z[k] = z[h];
    if (offsets) {
      const int m = module[h];
      X[k] += offsets[3 * m + 0];
      Y[k] += offsets[3 * m + 1];
      Z[k] += offsets[3 * m + 2];
    }
    lay[k] = layer[h];
  }
}

// Covariance of the fitted (kappa, phi0, cot, d0, z0) (section 3.4: the
// circle fit and the line fit each give their parameters with a covariance,
// and the two are combined).  The broken-line solutions are linear in the
// measurements with the kinks as zero-mean pseudo-measurements, so the
// covariance of the circle unknowns (u_0..u_{n-1}, dk) is A^-1 and that of
// the line unknowns (v_0..v_{n-1}) is N^-1, the inverses of the two normal
// matrices; the two fits share no measurement and are independent.  Through
// the perigee map of step 8, linearised at the solution (pre-fit held fixed):
//   C = Jc A^-1 Jc^T + Jl N^-1 Jl^T,
// Jc = d(params)/d(circle unknowns), Jl = d(params)/d(line unknowns).  The
// map depends on the circle only through u_0, u_1 and dk and on the line only
// through v_0 and v_1; those columns of Jc and Jl come from dual numbers
// seeded on each, the others are zero.
// jc [5][n+1], jl [5][n] and cov [5][5] are row-major.
int fit_cov(const FitSettings& F, int n, const Real* X, const Real* Y, const Real* Z, const int* lay,
            Real* jc, Real* jl, Real* cov) {
  const FitResult<Real> R = fit_track<Real>(F, n, X, Y, Z, lay);
  if (R.status != FIT_OK) return R.status;
  const int m = n + 1;
  // inverses column by column
  std::vector<Real> Ainv(m * m), Ninv(n * n), e, col;
  for (int j = 0; j < m; ++j) {
    e.assign(m, 0.0L);
    e[j] = 1.0L;
    if (!gauss_solve(m, R.A, e, col)) return FIT_SINGULAR;
    for (int i = 0; i < m; ++i) Ainv[i * m + j] = col[i];
  }
  for (int j = 0; j < n; ++j) {
    e.assign(n, 0.0L);
    e[j] = 1.0L;
    if (!gauss_solve(n, R.N, e, col)) return FIT_SINGULAR;
    for (int i = 0; i < n; ++i) Ninv[i * n + j] = col[i];
  }
  // Jacobians: one dual pass per unknown the perigee map reads
  auto D = [](Real v, bool seed) { return Dual{v, seed ? 1.0L : 0.0L}; };
  for (int i = 0; i < 5 * m; ++i) jc[i] = 0.0L;
  for (int i = 0; i < 5 * n; ++i) jl[i] = 0.0L;
  const int ids[5] = {0, 1, n, 0, 1};  // circle u0, u1, dk; line v0, v1
  for (int q = 0; q < 5; ++q) {
    Dual out[5];
    perigee<Dual>(D(R.ucirc[0], q == 0), D(R.ucirc[1], q == 1), D(R.ucirc[n], q == 2), D(R.vline[0], q == 3),
                  D(R.vline[1], q == 4), D(R.kappa_pre, false), D(R.delta[0], false), D(X[0], false),
                  D(Y[0], false), D(R.tx, false), D(R.ty, false), out);
    for (int o = 0; o < 5; ++o) {
      if (q < 3) jc[o * m + ids[q]] = out[o].d;
      else jl[o * n + ids[q]] = out[o].d;
    }
  }
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b) {
      Real s = 0.0L;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) s += jc[a * m + i] * Ainv[i * m + j] * jc[b * m + j];
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) s += jl[a * n + i] * Ninv[i * n + j] * jl[b * n + j];
      cov[a * 5 + b] = s;
    }
  return FIT_OK;
}

}  // namespace

extern "C" {

// Fit every n-tuplet: tuplets [n_tracks][8] hit indices, nhits [n_tracks].
// P_k = hit + offsets[module] when offsets is not NULL.  Outputs params
// [n_tracks][5] = (kappa, phi0, cot(theta), d0, z0), chi2 [n_tracks], status
// [n_tracks] (0 ok, 1 hits not ordered along the pre-fit, 4 singular).
void oracle_fit(const oracle_config* cfg, int64_t n_tracks, const int32_t* tuplets,
                const uint8_t* nhits, const double* x, const double* y, const double* z,
                const uint8_t* layer, const int16_t* module, const double* offsets,
                double* params, double* chi2, uint8_t* status) {
  const FitSettings F = fit_settings(*cfg);
  double X[kMaxHits], Y[kMaxHits], Z[kMaxHits];
  int lay[kMaxHits];
  for (int64_t t = 0; t < n_tracks; ++t) {
    const int n = nhits[t];
    gather(n, tuplets + t * kMaxHits, x, y, z, layer, module, offsets, X, Y, Z, lay);
    long double XL[kMaxHits], YL[kMaxHits], ZL[kMaxHits];
    for (int k = 0; k < n; ++k) {
      XL[k] = X[k];
      YL[k] = Y[k];
      ZL[k] = Z[k];
    }
    const FitResult<Real> r = fit_track<Real>(F, n, XL, YL, ZL, lay);
    status[t] = static_cast<uint8_t>(r.status);
    double* o = params + 5 * t;
    if (r.status != FIT_OK) {
      for (int i = 0; i < 5; ++i) o[i] = NAN;
      chi2[t] = NAN;
      continue;
    }
    o[0] = static_cast<double>(r.kappa);
    o[1] = static_cast<double>(r.phi0);
    o[2] = static_cast<double>(r.cot);
    o[3] = static_cast<double>(r.d0);
    o[4] = static_cast<double>(r.z0);
    chi2[t] = static_cast<double>(r.chi2);
  }
}

// Intermediate quantities of one track, for the tests' independent checks.
// Arrays are sized for n = 8: s, um, delta, wT, wZ, VZ [8]; ucirc [9];
// vline [8]; A [9*9]; b [9]; N [8*8]; q [8]; scal = (kappa_pre, t_pre, p).
int32_t oracle_fit_debug(const oracle_config* cfg, int32_t n, const double* X, const double* Y,
                         const double* Z, const int32_t* layer_k, double* s, double* um,
                         double* delta, double* wT, double* wZ, double* VZ, double* ucirc,
                         double* vline, double* A, double* b, double* N, double* q,
                         double* scal, double* params) {
  const FitSettings F = fit_settings(*cfg);
  int lay[kMaxHits];
  for (int k = 0; k < n; ++k) lay[k] = layer_k[k];
  long double XL[kMaxHits], YL[kMaxHits], ZL[kMaxHits];
  for (int k = 0; k < n; ++k) {
    XL[k] = X[k];
    YL[k] = Y[k];
    ZL[k] = Z[k];
  }
  const FitResult<Real> r = fit_track<Real>(F, n, XL, YL, ZL, lay);
  auto cp = [](const std::vector<Real>& v, double* dst) {
    for (size_t i = 0; i < v.size(); ++i) dst[i] = static_cast<double>(v[i]);
  };
  cp(r.s, s);
  cp(r.um, um);
  cp(r.delta, delta);
  if (r.status == FIT_OK) {
    cp(r.wT, wT);
    cp(r.wZ, wZ);
    cp(r.VZ, VZ);
    cp(r.ucirc, ucirc);
    cp(r.vline, vline);
    cp(r.A, A);
    cp(r.b, b);
    cp(r.N, N);
    cp(r.q, q);
    scal[0] = static_cast<double>(r.kappa_pre);
    scal[1] = static_cast<double>(r.t_pre);
    scal[2] = static_cast<double>(r.p);
    params[0] = static_cast<double>(r.kappa);
    params[1] = static_cast<double>(r.phi0);
    params[2] = static_cast<double>(r.cot);
    params[3] = static_cast<double>(r.d0);
    params[4] = static_cast<double>(r.z0);
    params[5] = static_cast<double>(r.chi2);
  }
  return r.status;
}

// Jacobian of (kappa, phi0, cot, d0, z0, chi2) with respect to the 3n hit
// coordinates of one track (forward-mode dual numbers, one pass per input).
// jac is [6][3n], column 3k+c = d/d(coordinate c of hit k).
int32_t oracle_fit_jacobian(const oracle_config* cfg, int32_t n, const double* X, const double* Y,
                            const double* Z, const int32_t* layer_k, double* jac) {
  const FitSettings F = fit_settings(*cfg);
  int lay[kMaxHits];
  for (int k = 0; k < n; ++k) lay[k] = layer_k[k];
  Dual DX[kMaxHits], DY[kMaxHits], DZ[kMaxHits];
  int status = FIT_OK;
  for (int col = 0; col < 3 * n; ++col) {
    for (int k = 0; k < n; ++k) {
      DX[k] = {X[k], (col == 3 * k + 0) ? 1.0L : 0.0L};
      DY[k] = {Y[k], (col == 3 * k + 1) ? 1.0L : 0.0L};
      DZ[k] = {Z[k], (col == 3 * k + 2) ? 1.0L : 0.0L};
    }
    const FitResult<Dual> r = fit_track<Dual>(F, n, DX, DY, DZ, lay);
    status = r.status;
    if (status != FIT_OK) return status;
    const Dual outs[6] = {r.kappa, r.phi0, r.cot, r.d0, r.z0, r.chi2};
    for (int o = 0; o < 6; ++o) jac[o * 3 * n + col] = static_cast<double>(outs[o].d);
  }
  return status;
}

// Reference gradient of the fit (the adjoint's definition):
//   grad_hits[h]    += sum over tracks containing h of J^T (g_params, g_chi2)
//   grad_offsets[m] += the same, summed over the hits on module m
// Both outputs are accumulated into.  Tracks whose fit fails contribute nothing.
void oracle_fit_grad(const oracle_config* cfg, int64_t n_tracks, const int32_t* tuplets,
                     const uint8_t* nhits, const double* x, const double* y, const double* z,
                     const uint8_t* layer, const int16_t* module, const double* offsets,
                     const double* g_params, const double* g_chi2, double* grad_hits,
                     double* grad_offsets) {
  double X[kMaxHits], Y[kMaxHits], Z[kMaxHits];
  int lay[kMaxHits];
  int32_t layk[kMaxHits];
  double jac[6 * 3 * kMaxHits];
  for (int64_t t = 0; t < n_tracks; ++t) {
    const int n = nhits[t];
    const int32_t* hit = tuplets + t * kMaxHits;
    gather(n, hit, x, y, z, layer, module, offsets, X, Y, Z, lay);
    for (int k = 0; k < n; ++k) layk[k] = lay[k];
    if (oracle_fit_jacobian(cfg, n, X, Y, Z, layk, jac) != FIT_OK) continue;
    double g[6];
    for (int o = 0; o < 5; ++o) g[o] = g_params[5 * t + o];
    g[5] = g_chi2 ? g_chi2[t] : 0.0;
    for (int col = 0; col < 3 * n; ++col) {
      double acc = 0.0;
      for (int o = 0; o < 6; ++o) acc += jac[o * 3 * n + col] * g[o];
      const int k = col / 3, c = col % 3;
      grad_hits[3 * hit[k] + c] += acc;
      if (grad_offsets) grad_offsets[3 * module[hit[k]] + c] += acc;
    }
  }
}

// Covariance of every fit: cov [n_tracks][15], the upper triangle of the
// symmetric 5x5 covariance of (kappa, phi0, cot, d0, z0) row by row
// ((0,0) (0,1) .. (0,4) (1,1) .. (4,4)); NaN for tracks whose fit fails.
// Inputs as oracle_fit.  See fit_cov for the definition.
void oracle_fit_cov(const oracle_config* cfg, int64_t n_tracks, const int32_t* tuplets, const uint8_t* nhits,
                    const double* x, const double* y, const double* z, const uint8_t* layer,
                    const int16_t* module, const double* offsets, double* cov_out) {
  const FitSettings F = fit_settings(*cfg);
  double X[kMaxHits], Y[kMaxHits], Z[kMaxHits];
  int lay[kMaxHits];
  Real jc[5 * (kMaxHits + 1)], jl[5 * kMaxHits], cov[25];
  for (int64_t t = 0; t < n_tracks; ++t) {
    const int n = nhits[t];
    double* o = cov_out + 15 * t;
    gather(n, tuplets + t * kMaxHits, x, y, z, layer, module, offsets, X, Y, Z, lay);
    Real XL[kMaxHits], YL[kMaxHits], ZL[kMaxHits];
    for (int k = 0; k < n; ++k) {
      XL[k] = X[k];
      YL[k] = Y[k];
      ZL[k] = Z[k];
    }
    const int st = fit_cov(F, n, XL, YL, ZL, lay, jc, jl, cov);
    int q = 0;
    for (int a = 0; a < 5; ++a)
      for (int b = a; b < 5; ++b) o[q++] = st == FIT_OK ? static_cast<double>(cov[a * 5 + b]) : NAN;
  }
}

// The pieces of one track's covariance, for the tests: jc [5][n+1], jl
// [5][n], cov [5][5] (row-major).  Returns the fit status.
int32_t oracle_fit_cov_debug(const oracle_config* cfg, int32_t n, const double* X, const double* Y,
                             const double* Z, const int32_t* layer_k, double* jc, double* jl, double* cov) {
  const FitSettings F = fit_settings(*cfg);
  if (n < 3 || n > kMaxHits) return FIT_SINGULAR;
  int lay[kMaxHits] = {};
  Real XL[kMaxHits] = {}, YL[kMaxHits] = {}, ZL[kMaxHits] = {};
  for (int k = 0; k < n; ++k) {
    lay[k] = layer_k[k];
    XL[k] = X[k];
    YL[k] = Y[k];
    ZL[k] = Z[k];
  }
  Real a[5 * (kMaxHits + 1)], b[5 * kMaxHits], c[25];
  const int st = fit_cov(F, n, XL, YL, ZL, lay, a, b, c);
  if (st != FIT_OK) return st;
  for (int i = 0; i < 5 * (n + 1); ++i) jc[i] = static_cast<double>(a[i]);
  for (int i = 0; i < 5 * n; ++i) jl[i] = static_cast<double>(b[i]);
  for (int i = 0; i < 25; ++i) cov[i] = static_cast<double>(c[i]);
  return st;
}

// Ambiguity resolution among fitted tracks (section 3.5).
// Tracks: hit rows hits [n][8], cell rows cells [n][7] (the row's doublets,
// inside -> out), nhits [n]; chi2 [n] and tip [n] (the transverse impact
// parameter d0) of their fits.  A track takes part when its chi2 is finite.
//   1. Tracks sharing a hit doublet (a cell) are ambiguous: a track is
//      dropped when a track sharing one of its cells has a smaller chi2
//      (equal chi2: both stay).
//   2. Among the 3-hit tracks that survive step 1, tracks sharing a hit are
//      ambiguous: a triplet is dropped when a triplet sharing one of its hits
//      has a smaller |tip| (equal: both stay).
// keep [n] receives 1 for the tracks that stay, 0 otherwise.  Returns the
// number kept.
int64_t oracle_ambiguity(int64_t n_tracks, const int32_t* hits, const int32_t* cells, const uint8_t* nhits,
                         const double* chi2, const double* tip, uint8_t* keep) {
  std::vector<uint8_t> cand(n_tracks), keep1(n_tracks, 0);
  for (int64_t t = 0; t < n_tracks; ++t) cand[t] = std::isfinite(chi2[t]) ? 1 : 0;
  // step 1: the smallest chi2 among the candidates through each cell
  std::map<int32_t, double> best_cell;
  for (int64_t t = 0; t < n_tracks; ++t) {
    if (!cand[t]) continue;
    for (int k = 0; k + 1 < nhits[t]; ++k) {
      const int32_t c = cells[t * (kMaxHits - 1) + k];
      auto it = best_cell.find(c);
      if (it == best_cell.end() || chi2[t] < it->second) best_cell[c] = chi2[t];
    }
  }
  for (int64_t t = 0; t < n_tracks; ++t) {
    if (!cand[t]) continue;
    bool ok = true;
    for (int k = 0; k + 1 < nhits[t]; ++k)
      if (best_cell[cells[t * (kMaxHits - 1) + k]] < chi2[t]) ok = false;
    keep1[t] = ok ? 1 : 0;
  }
  // step 2: the smallest |tip| among the surviving triplets through each hit
  std::map<int32_t, double> best_hit;
  for (int64_t t = 0; t < n_tracks; ++t) {
    if (!keep1[t] || nhits[t] != 3) continue;
    for (int k = 0; k < 3; ++k) {
      const int32_t h = hits[t * kMaxHits + k];
      const double a = std::fabs(tip[t]);
      auto it = best_hit.find(h);
      if (it == best_hit.end() || a < it->second) best_hit[h] = a;
    }
  }
  int64_t kept = 0;
  for (int64_t t = 0; t < n_tracks; ++t) {
    bool ok = keep1[t] != 0;
    if (ok && nhits[t] == 3)
      for (int k = 0; k < 3; ++k)
        if (best_hit[hits[t * kMaxHits + k]] < std::fabs(tip[t])) ok = false;
    keep[t] = ok ? 1 : 0;
    kept += ok;
  }
  return kept;
}

// Pixel vertices of one event (section 3.6), from its fitted tracks.
// Per track: z0, var_z0 (its variance, the (z0, z0) element of the fit
// covariance), kappa, nhits and use (1 for tracks that survived ambiguity
// resolution).  Settings: min_hits, pt_min, err_max (largest sigma(z0) for
// which a density is computed), dz_cut, chi2_max, split_chi2_ndf, pt_cap,
// kmeans_iter, K (p_T = K / |kappa|).
//  1. Tracks take part when used, with at least min_hits hits, p_T > pt_min
//     and a finite z0 with a positive finite variance.
//  2. Density of track i (only when sigma(z0) <= err_max, else 0): the
//     number of other taking-part tracks j with |z_i - z_j| < dz_cut and
//     (z_i - z_j)^2 < chi2_max (var_i + var_j).
//  3. Tracks are ranked by (density, index).  Each track links to the
//     nearest (smallest |z_i - z_j|, then smallest j) higher-ranked track
//     with |z_i - z_j| < dz_cut and (z_i - z_j)^2 <= chi2_max (var_i + var_j);
//     links only climb in rank, so they form trees.
//  4. The tracks of a tree whose root has density > 1 (a seed) form a vertex
//     candidate; candidates with at least 2 tracks are vertices.
//  5. Each vertex: members in order of (z0, index); weights w = 1 / var;
//     z = sum w z0 / sum w, var = 1 / sum w, chi2 = sum w (z0 - z)^2,
//     ndf = members - 1, sums taken in member order.
//  6. A vertex with chi2 / ndf > split_chi2_ndf is split in two by 1-D
//     k-means: centres at its smallest and largest z0; each member goes to
//     the nearer centre (the first on a tie); centres move to the weighted
//     means of their members (member order); repeated until no member moves
//     or kmeans_iter rounds.  Each part with at least 2 members becomes a
//     vertex (step 5); members of a part of one track are left out.
//  7. Vertices are ordered by sum over members of min(p_T, pt_cap)^2,
//     largest first (the first is the primary vertex); equal sums keep the
//     order of their smallest-z member.
// Outputs (capacity cap): vz, vvar, vchi2, vndf, vn, vsum; track_vertex [n]
// (vertex position in that order, or -1).  Returns the number of vertices.
int64_t oracle_vertices(int64_t n, const double* z0, const double* var_z0, const double* kappa,
                        const uint8_t* nhits, const uint8_t* use, int32_t min_hits, double pt_min,
                        double err_max, double dz_cut, double chi2_max, double split_chi2_ndf, double pt_cap,
                        int32_t kmeans_iter, double K, int64_t cap, double* vz, double* vvar, double* vchi2,
                        int32_t* vndf, int32_t* vn, double* vsum, int32_t* track_vertex) {
  std::vector<double> pt(n);
  std::vector<uint8_t> part(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    pt[i] = K / std::fabs(kappa[i]);
    part[i] = use[i] && nhits[i] >= min_hits && pt[i] > pt_min && std::isfinite(z0[i]) &&
              std::isfinite(var_z0[i]) && var_z0[i] > 0.0;
    track_vertex[i] = -1;
  }
  // 2. densities
  std::vector<int64_t> rho(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (!part[i] || !(std::sqrt(var_z0[i]) <= err_max)) continue;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i || !part[j]) continue;
      const double d = z0[i] - z0[j];
      if (std::fabs(d) < dz_cut && d * d < chi2_max * (var_z0[i] + var_z0[j])) ++rho[i];
    }
  }
  // 3. links to the nearest higher-ranked compatible track
  auto higher = [&](int64_t j, int64_t i) { return rho[j] > rho[i] || (rho[j] == rho[i] && j > i); };
  std::vector<int64_t> parent(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    if (!part[i]) continue;
    double best = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (!part[j] || !higher(j, i)) continue;
      const double d = z0[i] - z0[j];
      if (!(std::fabs(d) < dz_cut && d * d <= chi2_max * (var_z0[i] + var_z0[j]))) continue;
      if (parent[i] < 0 || std::fabs(d) < best) {  // j ascending: ties keep the smaller j
        parent[i] = j;
        best = std::fabs(d);
      }
    }
  }
  // 4. trees, seeds, candidates
  std::map<int64_t, std::vector<int64_t>> trees;
  for (int64_t i = 0; i < n; ++i) {
    if (!part[i]) continue;
    int64_t r = i;
    while (parent[r] >= 0) r = parent[r];
    trees[r].push_back(i);
  }
  struct Vtx {
    std::vector<int64_t> m;  // members in (z0, index) order
    double z, var, chi2, sum;
    int ndf;
  };
  auto by_z = [&](int64_t a, int64_t b) { return z0[a] < z0[b] || (z0[a] == z0[b] && a < b); };
  auto fit = [&](Vtx& v) {
    double W = 0.0, S = 0.0;
    for (int64_t i : v.m) {
      const double w = 1.0 / var_z0[i];
      W = W + w;
      S = S + w * z0[i];
    }
    v.z = S / W;
    v.var = 1.0 / W;
    double c = 0.0, s2 = 0.0;
    for (int64_t i : v.m) {
      const double d = z0[i] - v.z;
      c = c + (d * d) / var_z0[i];
      const double p = std::min(pt[i], pt_cap);
      s2 = s2 + p * p;
    }
    v.chi2 = c;
    v.sum = s2;
    v.ndf = static_cast<int>(v.m.size()) - 1;
  };
  std::vector<Vtx> out;
  for (auto& kv : trees) {
    if (!(rho[kv.first] > 1) || kv.second.size() < 2) continue;
    Vtx v;
    v.m = kv.second;
    std::sort(v.m.begin(), v.m.end(), by_z);
    fit(v);
    if (!(v.chi2 / v.ndf > split_chi2_ndf)) {
      out.push_back(v);
      continue;
    }
    // 6. two-means split
    const size_t M = v.m.size();
    double c1 = z0[v.m.front()], c2 = z0[v.m.back()];
    std::vector<uint8_t> side(M, 0), prev(M, 2);
    bool empty = false;
    for (int it = 0; it < kmeans_iter; ++it) {
      for (size_t q = 0; q < M; ++q) side[q] = std::fabs(z0[v.m[q]] - c1) <= std::fabs(z0[v.m[q]] - c2) ? 0 : 1;
      if (side == prev) break;
      prev = side;
      double W1 = 0.0, S1 = 0.0, W2 = 0.0, S2 = 0.0;
      for (size_t q = 0; q < M; ++q) {
        const double w = 1.0 / var_z0[v.m[q]];
        if (side[q] == 0) {
          W1 = W1 + w;
          S1 = S1 + w * z0[v.m[q]];
        } else {
          W2 = W2 + w;
          S2 = S2 + w * z0[v.m[q]];
        }
      }
      if (W1 == 0.0 || W2 == 0.0) {
        empty = true;
        break;
      }
      c1 = S1 / W1;
      c2 = S2 / W2;
    }
    if (empty) {
      out.push_back(v);
      continue;
    }
    for (int p = 0; p < 2; ++p) {
      Vtx h;
      for (size_t q = 0; q < M; ++q)
        if (side[q] == p) h.m.push_back(v.m[q]);
      if (h.m.size() < 2) continue;
      fit(h);
      out.push_back(h);
    }
  }
  // 7. order by the sum of p_T^2; ties by the smallest z0 of the members
  std::stable_sort(out.begin(), out.end(), [&](const Vtx& a, const Vtx& b) { return by_z(a.m.front(), b.m.front()); });
  std::stable_sort(out.begin(), out.end(), [](const Vtx& a, const Vtx& b) { return a.sum > b.sum; });
  for (size_t k = 0; k < out.size(); ++k) {
    for (int64_t i : out[k].m) track_vertex[i] = static_cast<int32_t>(k);
    if (static_cast<int64_t>(k) >= cap) continue;
    vz[k] = out[k].z;
    vvar[k] = out[k].var;
    vchi2[k] = out[k].chi2;
    vndf[k] = out[k].ndf;
    vn[k] = static_cast<int32_t>(out[k].m.size());
    vsum[k] = out[k].sum;
  }
  return static_cast<int64_t>(out.size());
}

// ---------------------------------------------------------------------------
// Batches for timing the oracle as a CPU baseline (OpenMP over events or
// tracks; n_threads = 1 runs them in order on the calling thread).

// The whole chain of each event: binned doublets, links, n-tuplets with
// duplicate removal, the fit and the dual-number gradient of every track
// (unit cotangents, module offsets applied when given).  Events in parallel.
// Returns the number of tracks; tracks [n_events] receives each event's.
int64_t oracle_chain_batch(const oracle_config* cfg, int32_t n_events, const int32_t* event_offsets,
                           const double* x, const double* y, const double* z, const uint8_t* layer,
                           const int16_t* module, const double* offsets, int32_t n_bins, int32_t n_threads,
                           int64_t* tracks) {
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(+ : total)
  for (int32_t e = 0; e < n_events; ++e) {
    const int32_t a = event_offsets[e], n = event_offsets[e + 1] - a;
    std::vector<int32_t> ci, co;
    std::vector<uint8_t> cp;
    int64_t cap = 64 * static_cast<int64_t>(n) + 1024, nc = 0;
    for (;;) {
      ci.resize(cap);
      co.resize(cap);
      cp.resize(cap);
      nc = oracle_doublets_binned(cfg, n, x + a, y + a, z + a, layer + a, n_bins, cap, ci.data(), co.data(),
                                  cp.data());
      if (nc <= cap) break;
      cap = nc;
    }
    std::vector<int32_t> li, lo;
    int64_t lcap = 4 * nc + 1024, nl = 0;
    for (;;) {
      li.resize(lcap);
      lo.resize(lcap);
      nl = oracle_links(cfg, n, x + a, y + a, z + a, layer + a, static_cast<int32_t>(nc), ci.data(), co.data(),
                        lcap, li.data(), lo.data());
      if (nl <= lcap) break;
      lcap = nl;
    }
    int64_t tcap = nc + 256, nt = 0, n_raw = 0;
    int32_t trunc = 0;
    std::vector<int32_t> th, tc;
    std::vector<uint8_t> tn;
    for (;;) {
      th.resize(tcap * kMaxHits);
      tc.resize(tcap * (kMaxHits - 1));
      tn.resize(tcap);
      nt = oracle_ntuplets(cfg, n, layer + a, static_cast<int32_t>(nc), ci.data(), co.data(),
                           static_cast<int32_t>(nl), li.data(), lo.data(), 1, tcap, th.data(), tc.data(), tn.data(),
                           &n_raw, &trunc);
      if (nt <= tcap) break;
      tcap = nt;
    }
    std::vector<double> params(5 * nt + 5), chi2(nt + 1), gp(5 * nt + 5, 1.0), gc(nt + 1, 1.0), gh(3 * n + 3, 0.0);
    std::vector<uint8_t> st(nt + 1);
    oracle_fit(cfg, nt, th.data(), tn.data(), x + a, y + a, z + a, layer + a, module + a, offsets, params.data(),
               chi2.data(), st.data());
    oracle_fit_grad(cfg, nt, th.data(), tn.data(), x + a, y + a, z + a, layer + a, module + a, offsets, gp.data(),
                    gc.data(), gh.data(), nullptr);
    tracks[e] = nt;
    total += nt;
  }
  return total;
}

// The fit and the dual-number gradient of n_tracks given tracks, tracks in
// parallel: params [n][5], chi2 [n] and grad_hits [n_hits][3] (added into).
void oracle_fit_grad_batch(const oracle_config* cfg, int64_t n_tracks, const int32_t* tuplets,
                           const uint8_t* nhits, const double* x, const double* y, const double* z,
                           const uint8_t* layer, const int16_t* module, const double* offsets,
                           const double* g_params, const double* g_chi2, int32_t n_threads, double* params,
                           double* chi2, double* grad_hits) {
#pragma omp parallel for schedule(dynamic, 256) num_threads(n_threads)
  for (int64_t t = 0; t < n_tracks; ++t) {
    uint8_t st = 0;
    oracle_fit(cfg, 1, tuplets + t * kMaxHits, nhits + t, x, y, z, layer, module, offsets, params + 5 * t,
               chi2 + t, &st);
    const int n = nhits[t];
    double X[kMaxHits], Y[kMaxHits], Z[kMaxHits], jac[6 * 3 * kMaxHits];
    int lay[kMaxHits];
    int32_t layk[kMaxHits];
    gather(n, tuplets + t * kMaxHits, x, y, z, layer, module, offsets, X, Y, Z, lay);
    for (int k = 0; k < n; ++k) layk[k] = lay[k];
    if (oracle_fit_jacobian(cfg, n, X, Y, Z, layk, jac) != FIT_OK) continue;
    for (int col = 0; col < 3 * n; ++col) {
      double acc = 0.0;
      for (int o = 0; o < 5; ++o) acc += jac[o * 3 * n + col] * g_params[5 * t + o];
      acc += jac[5 * 3 * n + col] * (g_chi2 ? g_chi2[t] : 0.0);
      const int64_t at = 3 * static_cast<int64_t>(tuplets[t * kMaxHits + col / 3]) + col % 3;
#pragma omp atomic
      grad_hits[at] += acc;
    }
  }
}

int32_t oracle_abi_version(void) { return 1; }

}  // extern "C"
