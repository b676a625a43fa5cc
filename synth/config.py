"""Detector description and reconstruction settings, as plain data.

This module is input, not method: it holds the geometry of the pixel detector
(four barrel layers and three forward disks per side, paper section 3.1), the
list of layer pairs that may form doublets (section 3.2, Fig. 3), and the cut
and fit settings the paper names but does not give values for (section 3.2,
Table 1; section 3.4).  Both the CPU oracle and the GPU library receive the
dict returned by :func:`default_config` and derive whatever constants their
predicates need on their own side.

Units: cm, GeV, tesla, radians.

Layer ids: 0-3 barrel BPix1-4; 4-6 forward disks at +z (FPix+1..3);
7-9 forward disks at -z (FPix-1..3).
"""
from __future__ import annotations

import copy
import math

N_LAYERS = 10
BARREL_R = (2.9, 6.8, 10.9, 16.0)
BARREL_HALF_Z = 26.7
DISK_Z = (32.0, 39.0, 48.0)
DISK_RMIN = 4.5
DISK_RMAX = 16.0
N_MODULES = 1856

# Barrel segmentation: phi ladders per layer x 8 z slices.
BARREL_LADDERS = (12, 28, 44, 64)
BARREL_ZSLICES = 8
# Disk segmentation: inner ring (r < DISK_RING_SPLIT) and outer ring sectors.
DISK_RING_SPLIT = 10.25
DISK_INNER_SECTORS = 44
DISK_OUTER_SECTORS = 68

# Layer pairs (inner, outer) that may form doublets.  Adjacent pairs plus
# the pairs that skip one layer to recover from gaps and inefficiency
# (section 3.2; the figure that draws them is not available, this list is
# our reading of it).
PAIRS = (
    (0, 1), (1, 2), (2, 3),                 # barrel, adjacent
    (0, 2), (1, 3),                         # barrel, skip one
    (0, 4), (1, 4), (2, 4), (4, 5), (5, 6),  # forward +z, adjacent
    (0, 5), (1, 5), (4, 6),                 # forward +z, skip one
    (0, 7), (1, 7), (2, 7), (7, 8), (8, 9),  # forward -z, adjacent
    (0, 8), (1, 8), (7, 9),                 # forward -z, skip one
)

# Bits of ``cut_mask``: which doublet cuts of Table 1 are applied.
CUT_PHIW = 1
CUT_ZW = 2
CUT_ZIP = 4
CUT_PT = 8
CUT_ALL = CUT_PHIW | CUT_ZW | CUT_ZIP | CUT_PT

# A z window that never cuts (finite, so it travels through every format).
Z_OPEN = 1.0e9

K_CURV = 0.299792458 / 100.0  # GeV / (T cm): p_T = K_CURV * B / |kappa|


def is_barrel(layer: int) -> bool:
    return layer < 4


def disk_z(layer: int) -> float:
    """Signed z of a disk layer (4-6 at +z, 7-9 at -z)."""
    if 4 <= layer <= 6:
        return DISK_Z[layer - 4]
    if 7 <= layer <= 9:
        return -DISK_Z[layer - 7]
    raise ValueError(f"layer {layer} is not a disk")


def layer_r_range(layer: int) -> tuple[float, float]:
    if is_barrel(layer):
        r = BARREL_R[layer]
        return r, r
    return DISK_RMIN, DISK_RMAX


def _phi_window(inner: int, outer: int, pt_min: float, bfield: float, rmax_ca: float) -> float:
    """The tuned PhiW window of a layer pair (rad).

    The largest azimuth difference between the inner and the outer hit of a
    track with p_T >= pt_min and transverse impact parameter <= rmax_ca: the
    bending term at the extreme radii plus the impact-parameter term.  This is
    how this configuration chooses its windows; the method only applies them.
    """
    rho_min = pt_min / (K_CURV * bfield)
    ri_min = layer_r_range(inner)[0]
    ro_max = layer_r_range(outer)[1]
    bend = math.asin(min(1.0, ro_max / (2.0 * rho_min))) - math.asin(min(1.0, ri_min / (2.0 * rho_min)))
    return bend + rmax_ca * (1.0 / ri_min - 1.0 / ro_max)


def _z_window(inner: int, outer: int, z0_max: float) -> tuple[float, float]:
    """ZW: allowed z range of the inner hit of a pair (cm).

    Only barrel -> disk pairs are restricted: a track from |z0| <= z0_max that
    reaches a disk at z_d inside its outer radius must cross the barrel radius
    r1 above the line from (r=0, z=-z0_max) to (r=DISK_RMAX, z=z_d).  The -z
    side uses the exact negation of the +z constants.
    """
    if is_barrel(inner) and not is_barrel(outer):
        zd = abs(disk_z(outer))
        r1 = BARREL_R[inner]
        zlo = -z0_max + (zd + z0_max) * r1 / DISK_RMAX
        if disk_z(outer) > 0:
            return zlo, Z_OPEN
        return -Z_OPEN, -zlo
    return -Z_OPEN, Z_OPEN


def default_config(**overrides) -> dict:
    """The reconstruction configuration used by every workload.

    Keys (all plain numbers or lists):
      bfield            solenoid field along +z (T)
      pairs             [[inner, outer], ...] layer pairs
      pair_dphi         PhiW window per pair (rad)
      pair_zlo/zhi      ZW window on the inner hit's z per pair (cm)
      pt_min            PT cut: minimum p_T of a circle through the origin (GeV)
      z0_max            ZIP cut: |z at r=0| of the straight R-Z line (cm)
      cut_mask          CUT_* bits that are applied
      ca_theta_barrel   R-Z alignment of a triplet whose outer hit is on a
                        barrel layer: max sine of the kink angle
      ca_theta_endcap   same, outer hit on a disk
      ca_rmax_bpix1     circle-to-beamspot distance for triplets whose inner
                        hit is on BPix1 (cm)
      ca_rmax_other     same, any other inner layer (cm)
      root_always       layers whose doublets always start an n-tuplet
      root_if_free      layers whose doublets start one when they have no
                        inner neighbour (section 3.2)
      min_hits          shortest n-tuplet kept
      max_hits          longest n-tuplet the search follows
      layer_barrel      per layer: 1 for barrel, 0 for disk
      x_over_x0         material per layer crossing, in radiation lengths
      highland_a/b      multiple scattering constants (13.6 MeV, 0.038)
      sigma_rphi        transverse hit resolution (cm)
      sigma_z           barrel longitudinal resolution (cm)
      sigma_r           disk radial resolution (cm)
      p_cap             momentum cap in the scattering estimate (GeV)
      n_modules         number of detector modules (alignment offsets)
      vtx_min_hits      vertices: fewest hits of a track that is used (section 3.6)
      vtx_pt_min        vertices: smallest p_T of a track that is used (GeV)
      vtx_err_max       vertices: largest sigma(z0) of a track whose local density
                        is computed (cm)
      vtx_dz_cut        vertices: largest |dz0| of close-by tracks (cm)
      vtx_chi2_max      vertices: largest chi2 compatibility of two tracks' z0
      vtx_split_chi2_ndf vertices: chi2/ndf above which a vertex is split in two
      vtx_pt_cap        vertices: p_T cap in the sum of p_T^2 that orders them (GeV)
      vtx_kmeans_iter   vertices: most rounds of the two-means split
      fishbone_theta    Fishbone (section 3.3): largest sine of the angle between
                        two doublets sharing their outer hit for which the longer
                        one is dropped; 0 turns the Fishbone off
      exclusive_hits    1 when no hit belongs to two of the tracks given to the
                        adjoint (the fit workload), so that it may add into the
                        hit gradients without atomics; 0 otherwise
    """
    bfield = 3.8
    pt_min = 0.45
    z0_max = 15.0
    rmax_other = 0.25
    cfg = {
        "bfield": bfield,
        "pairs": [list(p) for p in PAIRS],
        "pair_dphi": [_phi_window(i, o, pt_min, bfield, rmax_other) for i, o in PAIRS],
        "pair_zlo": [_z_window(i, o, z0_max)[0] for i, o in PAIRS],
        "pair_zhi": [_z_window(i, o, z0_max)[1] for i, o in PAIRS],
        "pt_min": pt_min,
        "z0_max": z0_max,
        "cut_mask": CUT_ALL,
        "ca_theta_barrel": 0.010,
        "ca_theta_endcap": 0.015,
        "ca_rmax_bpix1": 0.15,
        "ca_rmax_other": rmax_other,
        "root_always": [0],
        "root_if_free": [1, 4, 7],
        "min_hits": 4,
        "max_hits": 8,
        "layer_barrel": [1 if is_barrel(l) else 0 for l in range(N_LAYERS)],
        "x_over_x0": 0.015,
        "highland_a": 0.0136,
        "highland_b": 0.038,
        "sigma_rphi": 10e-4,
        "sigma_z": 20e-4,
        "sigma_r": 20e-4,
        "p_cap": 1.0e4,
        "n_modules": N_MODULES,
        "vtx_min_hits": 4,
        "vtx_pt_min": 0.5,
        "vtx_err_max": 0.1,
        "vtx_dz_cut": 0.07,
        "vtx_chi2_max": 9.0,
        "vtx_split_chi2_ndf": 9.0,
        "vtx_pt_cap": 75.0,
        "vtx_kmeans_iter": 10,
        "fishbone_theta": 0.0,
        "exclusive_hits": 0,
    }
    for k, v in overrides.items():
        if k not in cfg:
            raise KeyError(f"unknown config key {k!r}")
        cfg[k] = copy.deepcopy(v)
    return cfg
