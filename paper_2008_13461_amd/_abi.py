"""ctypes mirror of include/pixeltrack.h and the loader of libpixeltrack.so.

Argument marshalling only: every step of the computation runs in the HIP
library.  Importing this module never falls back to anything else: if the
library is missing it raises.
"""
from __future__ import annotations

import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpixeltrack.so")

PT_MAX_PAIRS = 32
PT_N_LAYERS = 10
PT_MAX_HITS = 8
PT_STATUS_WORDS = 16
PT_ABI_VERSION = 2

PT_OK, PT_ERR_ARG, PT_ERR_DEVICE, PT_ERR_UNSUPPORTED, PT_ERR_WORKSPACE, PT_ERR_TOO_LARGE = range(6)
PT_NOALLOC_FIT_MAX_TRACKS = 262144
PT_F32, PT_F64 = 0, 1
PT_FIT_F64, PT_FIT_F32, PT_FIT_F32_F64SOLVE = 0, 1, 2
PT_CUT_PHIW, PT_CUT_ZW, PT_CUT_ZIP, PT_CUT_PT = 1, 2, 4, 8
(PT_ST_FLAGS, PT_ST_BAD_HITS, PT_ST_TRUNCATED, PT_ST_FIT_BAD_ORDER, PT_ST_FIT_F64,
 PT_ST_FIT_FAILED) = range(6)
PT_FLAG_CELLS_OVERFLOW = 1 << 0
PT_FLAG_LINKS_OVERFLOW = 1 << 1
PT_FLAG_TUPLETS_OVERFLOW = 1 << 2
PT_FLAG_BAD_HITS = 1 << 3
PT_FLAG_TRUNCATED = 1 << 4
PT_FLAG_FIT_BAD_ORDER = 1 << 5
PT_FLAG_FIT_FAILED = 1 << 6
PT_FLAG_VERTICES_OVERFLOW = 1 << 7
PT_FIT_OK, PT_FIT_ST_BAD_ORDER, PT_FIT_ST_F64_SOLVE, PT_FIT_ST_FAILED = 0, 1, 2, 4
PT_STAGE_ADJOINT, PT_STAGE_AMBIGUITY, PT_STAGE_VERTICES = 1, 2, 4

P = ct.c_void_p


class pt_config(ct.Structure):
    _fields_ = [
        ("bfield", ct.c_double),
        ("n_pairs", ct.c_int32),
        ("pair_inner", ct.c_uint8 * PT_MAX_PAIRS),
        ("pair_outer", ct.c_uint8 * PT_MAX_PAIRS),
        ("pair_dphi", ct.c_double * PT_MAX_PAIRS),
        ("pair_zlo", ct.c_double * PT_MAX_PAIRS),
        ("pair_zhi", ct.c_double * PT_MAX_PAIRS),
        ("pt_min", ct.c_double),
        ("z0_max", ct.c_double),
        ("cut_mask", ct.c_uint32),
        ("ca_theta_barrel", ct.c_double),
        ("ca_theta_endcap", ct.c_double),
        ("ca_rmax_bpix1", ct.c_double),
        ("ca_rmax_other", ct.c_double),
        ("root_always_mask", ct.c_uint32),
        ("root_if_free_mask", ct.c_uint32),
        ("min_hits", ct.c_int32),
        ("max_hits", ct.c_int32),
        ("layer_barrel", ct.c_uint8 * PT_N_LAYERS),
        ("x_over_x0", ct.c_double),
        ("highland_a", ct.c_double),
        ("highland_b", ct.c_double),
        ("sigma_rphi", ct.c_double),
        ("sigma_z", ct.c_double),
        ("sigma_r", ct.c_double),
        ("p_cap", ct.c_double),
        ("n_modules", ct.c_int32),
        ("n_phi_bins", ct.c_int32),
        ("block_doublets", ct.c_int32),
        ("block_links", ct.c_int32),
        ("f64_solve_threshold", ct.c_double),
        ("vtx_min_hits", ct.c_int32),
        ("vtx_kmeans_iter", ct.c_int32),
        ("vtx_pt_min", ct.c_double),
        ("vtx_err_max", ct.c_double),
        ("vtx_dz_cut", ct.c_double),
        ("vtx_chi2_max", ct.c_double),
        ("vtx_split_chi2_ndf", ct.c_double),
        ("vtx_pt_cap", ct.c_double),
        ("fishbone_theta", ct.c_double),
        ("exclusive_hits", ct.c_int32),
    ]


class pt_hits(ct.Structure):
    _fields_ = [
        ("n_hits", ct.c_int32),
        ("n_events", ct.c_int32),
        ("event_offsets", P),
        ("dtype", ct.c_int32),
        ("x", P),
        ("y", P),
        ("z", P),
        ("layer", P),
        ("module", P),
    ]


class pt_workspace(ct.Structure):
    _fields_ = [("ptr", P), ("bytes", ct.c_size_t)]


class pt_cells(ct.Structure):
    _fields_ = [
        ("cap", ct.c_int32),
        ("inner", P),
        ("outer", P),
        ("pair", P),
        ("count", P),
        ("inner_first", P),
        ("inner_count", P),
    ]


class pt_links(ct.Structure):
    _fields_ = [
        ("cap", ct.c_int32),
        ("in_cell", P),
        ("out_cell", P),
        ("count", P),
        ("out_start", P),
        ("out_count", P),
        ("has_inner", P),
    ]


class pt_ntuplets(ct.Structure):
    _fields_ = [
        ("cap", ct.c_int32),
        ("hits", P),
        ("cells", P),
        ("n", P),
        ("count_raw", P),
        ("kept", P),
        ("count", P),
    ]


class pt_tracks(ct.Structure):
    _fields_ = [
        ("cap", ct.c_int32),
        ("params", P),
        ("chi2", P),
        ("status", P),
        ("cov", P),
    ]


class pt_vertices(ct.Structure):
    _fields_ = [
        ("cap", ct.c_int32),
        ("z", P),
        ("var", P),
        ("chi2", P),
        ("ndf", P),
        ("n_tracks", P),
        ("sum_pt2", P),
        ("event_first", P),
        ("count", P),
        ("track_vertex", P),
    ]


# Every entry point of the header: name -> (restype, argtypes)
SIGNATURES = {
    "pt_abi_version": (ct.c_int32, []),
    "pt_err_string": (ct.c_char_p, [ct.c_int]),
    "pt_last_device_error": (ct.c_char_p, []),
    "pt_workspace_size": (ct.c_size_t, [ct.POINTER(pt_config), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32,
                                        ct.c_int32]),
    "pt_build_doublets": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_cells), P,
                                     pt_workspace, P]),
    "pt_link_cells": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_cells),
                                 ct.POINTER(pt_links), P, pt_workspace, P]),
    "pt_find_ntuplets": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_cells),
                                    ct.POINTER(pt_links), ct.POINTER(pt_ntuplets), P, pt_workspace, P]),
    "pt_fit_broken_line": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_ntuplets), P,
                                      ct.c_int32, ct.POINTER(pt_tracks), P, pt_workspace, P]),
    "pt_fit_broken_line_bwd": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_ntuplets),
                                          P, ct.c_int32, P, P, P, P, P, pt_workspace, P]),
    "pt_resolve_ambiguities": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_cells),
                                          ct.POINTER(pt_ntuplets), ct.c_int32, ct.POINTER(pt_tracks), P, P, P,
                                          pt_workspace, P]),
    "pt_find_vertices": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_ntuplets), ct.c_int32,
                                    ct.POINTER(pt_tracks), P, P, ct.POINTER(pt_vertices), P, pt_workspace, P]),
    "pt_fit_broken_line_noalloc": (ct.c_int, [ct.POINTER(pt_hits), ct.POINTER(pt_config), ct.POINTER(pt_ntuplets),
                                              P, ct.c_int32, ct.POINTER(pt_tracks), P, P]),
    "pt_plan_create": (ct.c_int, [ct.POINTER(pt_config), ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32,
                                  ct.c_int32, ct.c_int32, ct.POINTER(P)]),
    "pt_plan_run": (ct.c_int, [P, ct.POINTER(pt_hits), ct.POINTER(pt_cells), ct.POINTER(pt_links),
                               ct.POINTER(pt_ntuplets), ct.POINTER(pt_tracks), P, P, P, P, P, P, P,
                               ct.POINTER(pt_vertices), P, P]),
    "pt_plan_destroy": (None, [P]),
    "pt_timing_enable": (None, [ct.c_int32]),
    "pt_timing_reset": (None, []),
    "pt_timing_read": (ct.c_int32, [ct.c_char_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load libpixeltrack.so (built by paper_2008_13461_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # torch ships its own HIP runtime: load it before the library so that
        # the process holds one runtime (the library binds to the one loaded)
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} is not built: run `python -m paper_2008_13461_amd.build` "
                             "(or __graft_entry__.build())")
    L = ct.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.pt_abi_version() != PT_ABI_VERSION:
        raise LibraryMissing(f"{path} has ABI {L.pt_abi_version()}, expected {PT_ABI_VERSION}")
    _lib = L
    return L


def check(err: int, what: str) -> None:
    if err != PT_OK:
        msg = load().pt_err_string(err).decode()
        if err == PT_ERR_DEVICE:
            msg += f" [{load().pt_last_device_error().decode()}]"
        raise RuntimeError(f"{what} failed: {msg} (code {err})")


def make_config(cfg: dict, *, n_phi_bins: int = 0, block_doublets: int = 0, block_links: int = 0,
                f64_solve_threshold: float = 0.0) -> pt_config:
    """Fill a pt_config from the plain configuration dict (synth.config.default_config)."""
    c = pt_config()
    c.bfield = cfg["bfield"]
    pairs = cfg["pairs"]
    c.n_pairs = len(pairs)
    for p, (i, o) in enumerate(pairs):
        c.pair_inner[p] = i
        c.pair_outer[p] = o
        c.pair_dphi[p] = cfg["pair_dphi"][p]
        c.pair_zlo[p] = cfg["pair_zlo"][p]
        c.pair_zhi[p] = cfg["pair_zhi"][p]
    c.pt_min = cfg["pt_min"]
    c.z0_max = cfg["z0_max"]
    c.cut_mask = cfg["cut_mask"]
    c.ca_theta_barrel = cfg["ca_theta_barrel"]
    c.ca_theta_endcap = cfg["ca_theta_endcap"]
    c.ca_rmax_bpix1 = cfg["ca_rmax_bpix1"]
    c.ca_rmax_other = cfg["ca_rmax_other"]
    c.root_always_mask = sum(1 << l for l in cfg["root_always"])
    c.root_if_free_mask = sum(1 << l for l in cfg["root_if_free"])
    c.min_hits = cfg["min_hits"]
    c.max_hits = cfg["max_hits"]
    for l in range(PT_N_LAYERS):
        c.layer_barrel[l] = cfg["layer_barrel"][l]
    for k in ("x_over_x0", "highland_a", "highland_b", "sigma_rphi", "sigma_z", "sigma_r", "p_cap"):
        setattr(c, k, cfg[k])
    c.n_modules = cfg["n_modules"]
    c.n_phi_bins = n_phi_bins
    c.block_doublets = block_doublets
    c.block_links = block_links
    c.f64_solve_threshold = f64_solve_threshold
    for k in ("vtx_min_hits", "vtx_kmeans_iter", "vtx_pt_min", "vtx_err_max", "vtx_dz_cut", "vtx_chi2_max",
              "vtx_split_chi2_ndf", "vtx_pt_cap", "fishbone_theta", "exclusive_hits"):
        setattr(c, k, cfg[k])
    return c
