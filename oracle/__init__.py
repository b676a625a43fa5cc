"""CPU oracle of the pixel-track hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never calls it and shares no code with it.

Thin ctypes wrappers around oracle/oracle.cpp (built into liboracle.so).  All
arithmetic is double precision on the host; float32 hit arrays are promoted
exactly.  Functions work on one event at a time (hit indices 0..n-1 of the
arrays passed).

Parity status of each function (pins in tests/test_oracle_*.py):
  doublets      pinned: geometric meaning of each cut away from its boundary,
                exact symmetries, subset monotonicity, hand-built events
  links         pinned: angle / circle distance computed another way, exact
                symmetries, straight tracks from the origin
  ntuplets      pinned: brute-force path enumeration in Python, invariants,
                truth quadruplets of noise-free barrel events
  fit           pinned: exact recovery of generated helices, symmetries,
                no-scattering limit against textbook polynomial regression,
                dense solve against numpy, chi2 statistics
  fit gradient  pinned: central finite differences, translation identities
  fit covariance pinned: numpy inverses of the normal matrices, sample
                covariance of repeated simulations of one track, pulls of a
                population of tracks, symmetries
  ambiguity     pinned: brute force over all pairs of tracks in Python
  vertices      pinned: hand-built clusters with known answers (densities,
                links, splits, ordering), symmetries (z shift, order of the
                tracks), truth vertices of simulated events
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_MAX_PAIRS = 32
_MAX_HITS = 8


class OracleConfig(ct.Structure):
    _fields_ = [
        ("bfield", ct.c_double),
        ("n_pairs", ct.c_int32),
        ("pair_inner", ct.c_int32 * _MAX_PAIRS),
        ("pair_outer", ct.c_int32 * _MAX_PAIRS),
        ("pair_dphi", ct.c_double * _MAX_PAIRS),
        ("pair_zlo", ct.c_double * _MAX_PAIRS),
        ("pair_zhi", ct.c_double * _MAX_PAIRS),
        ("pt_min", ct.c_double),
        ("z0_max", ct.c_double),
        ("cut_mask", ct.c_int32),
        ("ca_theta_barrel", ct.c_double),
        ("ca_theta_endcap", ct.c_double),
        ("ca_rmax_bpix1", ct.c_double),
        ("ca_rmax_other", ct.c_double),
        ("root_always_mask", ct.c_int32),
        ("root_if_free_mask", ct.c_int32),
        ("min_hits", ct.c_int32),
        ("max_hits", ct.c_int32),
        ("layer_barrel", ct.c_int32 * 10),
        ("x_over_x0", ct.c_double),
        ("highland_a", ct.c_double),
        ("highland_b", ct.c_double),
        ("sigma_rphi", ct.c_double),
        ("sigma_z", ct.c_double),
        ("sigma_r", ct.c_double),
        ("p_cap", ct.c_double),
    ]


def _config(cfg: dict) -> OracleConfig:
    c = OracleConfig()
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
    for l in range(10):
        c.layer_barrel[l] = cfg["layer_barrel"][l]
    for k in ("x_over_x0", "highland_a", "highland_b", "sigma_rphi", "sigma_z", "sigma_r", "p_cap"):
        setattr(c, k, cfg[k])
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ct.CDLL(_LIB_PATH)
        P = ct.c_void_p
        L.oracle_doublets.restype = ct.c_int64
        L.oracle_doublets.argtypes = [P, ct.c_int32, P, P, P, P, ct.c_int64, P, P, P]
        L.oracle_fishbone.restype = ct.c_int64
        L.oracle_fishbone.argtypes = [ct.c_double, ct.c_int32, P, P, P, ct.c_int32, P, P, P]
        L.oracle_doublets_binned.restype = ct.c_int64
        L.oracle_doublets_binned.argtypes = [P, ct.c_int32, P, P, P, P, ct.c_int32, ct.c_int64, P, P, P]
        L.oracle_chain_batch.restype = ct.c_int64
        L.oracle_chain_batch.argtypes = [P, ct.c_int32, P, P, P, P, P, P, P, ct.c_int32, ct.c_int32, P]
        L.oracle_fit_grad_batch.restype = None
        L.oracle_fit_grad_batch.argtypes = [P, ct.c_int64, P, P, P, P, P, P, P, P, P, P, ct.c_int32, P, P, P]
        L.oracle_links.restype = ct.c_int64
        L.oracle_links.argtypes = [P, ct.c_int32, P, P, P, P, ct.c_int32, P, P, ct.c_int64, P, P]
        L.oracle_ntuplets.restype = ct.c_int64
        L.oracle_ntuplets.argtypes = [P, ct.c_int32, P, ct.c_int32, P, P, ct.c_int32, P, P, ct.c_int32,
                                      ct.c_int64, P, P, P, P, P]
        L.oracle_fit.restype = None
        L.oracle_fit.argtypes = [P, ct.c_int64, P, P, P, P, P, P, P, P, P, P, P]
        L.oracle_fit_debug.restype = ct.c_int32
        L.oracle_fit_debug.argtypes = [P, ct.c_int32] + [P] * 18
        L.oracle_fit_jacobian.restype = ct.c_int32
        L.oracle_fit_jacobian.argtypes = [P, ct.c_int32, P, P, P, P, P]
        L.oracle_fit_cov.restype = None
        L.oracle_fit_cov.argtypes = [P, ct.c_int64, P, P, P, P, P, P, P, P, P]
        L.oracle_fit_cov_debug.restype = ct.c_int32
        L.oracle_fit_cov_debug.argtypes = [P, ct.c_int32, P, P, P, P, P, P, P]
        L.oracle_ambiguity.restype = ct.c_int64
        L.oracle_ambiguity.argtypes = [ct.c_int64, P, P, P, P, P, P]
        L.oracle_vertices.restype = ct.c_int64
        L.oracle_vertices.argtypes = [ct.c_int64, P, P, P, P, P, ct.c_int32, ct.c_double, ct.c_double,
                                      ct.c_double, ct.c_double, ct.c_double, ct.c_double, ct.c_int32, ct.c_double,
                                      ct.c_int64, P, P, P, P, P, P, P]
        L.oracle_fit_grad.restype = None
        L.oracle_fit_grad.argtypes = [P, ct.c_int64, P, P, P, P, P, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def doublets(cfg, x, y, z, layer):
    """All doublets of one event: int32 arrays (inner, outer) and uint8 pair."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    n = x.shape[0]
    c = _config(cfg)
    cap = max(1024, 16 * n)
    while True:
        inner = np.empty(cap, np.int32)
        outer = np.empty(cap, np.int32)
        pair = np.empty(cap, np.uint8)
        cnt = lib().oracle_doublets(ct.byref(c), n, _p(x), _p(y), _p(z), _p(layer), cap,
                                    _p(inner), _p(outer), _p(pair))
        if cnt <= cap:
            return inner[:cnt], outer[:cnt], pair[:cnt]
        cap = int(cnt)


def doublets_binned(cfg, x, y, z, layer, n_bins=64):
    """The doublets of `doublets`, found through azimuth bins (same set, other order)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    n = x.shape[0]
    c = _config(cfg)
    cap = max(1024, 16 * n)
    while True:
        inner = np.empty(cap, np.int32)
        outer = np.empty(cap, np.int32)
        pair = np.empty(cap, np.uint8)
        cnt = lib().oracle_doublets_binned(ct.byref(c), n, _p(x), _p(y), _p(z), _p(layer), n_bins, cap,
                                           _p(inner), _p(outer), _p(pair))
        if cnt <= cap:
            return inner[:cnt], outer[:cnt], pair[:cnt]
        cap = int(cnt)


def chain_batch(cfg, event_offsets, x, y, z, layer, module, offsets, n_threads=1, n_bins=64):
    """Whole chain (binned doublets .. dual-number gradient) of every event,
    events over n_threads OpenMP threads; returns tracks per event."""
    off = np.ascontiguousarray(event_offsets, dtype=np.int32)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    mod = np.ascontiguousarray(module, dtype=np.int16)
    o = _f64(offsets).reshape(-1) if offsets is not None else None
    tr = np.zeros(off.shape[0] - 1, np.int64)
    lib().oracle_chain_batch(ct.byref(_config(cfg)), off.shape[0] - 1, _p(off), _p(x), _p(y), _p(z), _p(layer),
                             _p(mod), _p(o), n_bins, n_threads, _p(tr))
    return tr


def fit_grad_batch(cfg, tuplets, nhits, x, y, z, layer, module, offsets, g_params, g_chi2, n_threads=1):
    """Fit and dual-number gradient of given tracks over n_threads OpenMP
    threads: (params [N, 5], chi2 [N], grad_hits [n_hits, 3])."""
    tup = np.ascontiguousarray(tuplets, dtype=np.int32)
    nh = np.ascontiguousarray(nhits, dtype=np.uint8)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    mod = np.ascontiguousarray(module, dtype=np.int16)
    o = _f64(offsets).reshape(-1) if offsets is not None else None
    gp = _f64(g_params).reshape(-1)
    gc = _f64(g_chi2)
    n = tup.shape[0]
    params = np.empty((n, 5))
    chi2 = np.empty(n)
    gh = np.zeros((x.shape[0], 3))
    lib().oracle_fit_grad_batch(ct.byref(_config(cfg)), n, _p(tup), _p(nh), _p(x), _p(y), _p(z), _p(layer), _p(mod),
                                _p(o), _p(gp), _p(gc), n_threads, _p(params), _p(chi2), _p(gh))
    return params, chi2, gh


def fishbone(cfg, x, y, z, cell_inner, cell_outer):
    """Fishbone of section 3.3 (see oracle.cpp): bool keep [n_cells] of the
    doublets that stay; theta from cfg["fishbone_theta"]."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    ci = np.ascontiguousarray(cell_inner, dtype=np.int32)
    co = np.ascontiguousarray(cell_outer, dtype=np.int32)
    keep = np.empty(ci.shape[0], np.uint8)
    th = float(cfg["fishbone_theta"])
    lib().oracle_fishbone(th * th, x.shape[0], _p(x), _p(y), _p(z), ci.shape[0], _p(ci), _p(co), _p(keep))
    return keep.astype(bool)


def links(cfg, x, y, z, layer, cell_inner, cell_outer):
    """All cell links of one event: int32 arrays (in_cell, out_cell)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    ci = np.ascontiguousarray(cell_inner, dtype=np.int32)
    co = np.ascontiguousarray(cell_outer, dtype=np.int32)
    c = _config(cfg)
    cap = max(1024, 4 * ci.shape[0])
    while True:
        a = np.empty(cap, np.int32)
        b = np.empty(cap, np.int32)
        cnt = lib().oracle_links(ct.byref(c), x.shape[0], _p(x), _p(y), _p(z), _p(layer), ci.shape[0],
                                 _p(ci), _p(co), cap, _p(a), _p(b))
        if cnt <= cap:
            return a[:cnt], b[:cnt]
        cap = int(cnt)


def ntuplets(cfg, layer, cell_inner, cell_outer, link_in, link_out, dedup=True):
    """n-tuplets of one event.

    Returns dict with hits [N, 8] int32 (-1 padded), cells [N, 7], n [N] uint8,
    n_raw (count before duplicate removal), truncated (bool).
    """
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    ci = np.ascontiguousarray(cell_inner, dtype=np.int32)
    co = np.ascontiguousarray(cell_outer, dtype=np.int32)
    li = np.ascontiguousarray(link_in, dtype=np.int32)
    lo = np.ascontiguousarray(link_out, dtype=np.int32)
    c = _config(cfg)
    cap = max(256, ci.shape[0])
    while True:
        hits = np.empty((cap, _MAX_HITS), np.int32)
        cells = np.empty((cap, _MAX_HITS - 1), np.int32)
        nh = np.empty(cap, np.uint8)
        n_raw = ct.c_int64(0)
        trunc = ct.c_int32(0)
        cnt = lib().oracle_ntuplets(ct.byref(c), layer.shape[0], _p(layer), ci.shape[0], _p(ci), _p(co),
                                    li.shape[0], _p(li), _p(lo), int(bool(dedup)), cap, _p(hits),
                                    _p(cells), _p(nh), ct.byref(n_raw), ct.byref(trunc))
        if cnt <= cap:
            return {"hits": hits[:cnt], "cells": cells[:cnt], "n": nh[:cnt],
                    "n_raw": int(n_raw.value), "truncated": bool(trunc.value)}
        cap = int(cnt)


def fit(cfg, tuplets, nhits, x, y, z, layer, module=None, offsets=None):
    """Broken-line fit of every n-tuplet.

    Returns params [N, 5] = (kappa, phi0, cot_theta, d0, z0), chi2 [N],
    status [N] (0 ok, 1 not ordered, 4 singular).
    """
    tup = np.ascontiguousarray(tuplets, dtype=np.int32)
    nh = np.ascontiguousarray(nhits, dtype=np.uint8)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    mod = np.ascontiguousarray(module if module is not None else np.zeros(x.shape[0]), dtype=np.int16)
    off = _f64(offsets).reshape(-1) if offsets is not None else None
    n = tup.shape[0]
    params = np.empty((n, 5), np.float64)
    chi2 = np.empty(n, np.float64)
    st = np.empty(n, np.uint8)
    c = _config(cfg)
    lib().oracle_fit(ct.byref(c), n, _p(tup), _p(nh), _p(x), _p(y), _p(z), _p(layer), _p(mod), _p(off),
                     _p(params), _p(chi2), _p(st))
    return params, chi2, st


def fit_debug(cfg, X, Y, Z, layers):
    """Intermediate quantities of the fit of one track given its hit coordinates."""
    n = len(X)
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    lay = np.ascontiguousarray(layers, dtype=np.int32)
    out = {k: np.full(sz, np.nan) for k, sz in (
        ("s", 8), ("um", 8), ("delta", 8), ("wT", 8), ("wZ", 8), ("VZ", 8), ("ucirc", 9), ("vline", 8),
        ("A", 81), ("b", 9), ("N", 64), ("q", 8), ("scal", 3), ("params", 6))}
    c = _config(cfg)
    st = lib().oracle_fit_debug(ct.byref(c), n, _p(X), _p(Y), _p(Z), _p(lay),
                                *[_p(out[k]) for k in ("s", "um", "delta", "wT", "wZ", "VZ", "ucirc",
                                                        "vline", "A", "b", "N", "q", "scal", "params")])
    m = n + 1
    res = {
        "status": int(st), "s": out["s"][:n], "um": out["um"][:n], "delta": out["delta"][:n - 1],
        "wT": out["wT"][:n], "wZ": out["wZ"][:n], "VZ": out["VZ"][:n], "ucirc": out["ucirc"][:m],
        "vline": out["vline"][:n], "A": out["A"][:m * m].reshape(m, m), "b": out["b"][:m],
        "N": out["N"][:n * n].reshape(n, n), "q": out["q"][:n],
        "kappa_pre": out["scal"][0], "t_pre": out["scal"][1], "p": out["scal"][2],
        "params": out["params"][:5], "chi2": out["params"][5],
    }
    return res


def fit_jacobian(cfg, X, Y, Z, layers):
    """d(kappa, phi0, cot, d0, z0, chi2) / d(hit coords), shape [6, n, 3]."""
    n = len(X)
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    lay = np.ascontiguousarray(layers, dtype=np.int32)
    jac = np.empty(6 * 3 * n, np.float64)
    c = _config(cfg)
    st = lib().oracle_fit_jacobian(ct.byref(c), n, _p(X), _p(Y), _p(Z), _p(lay), _p(jac))
    if st != 0:
        raise ValueError(f"fit status {st}")
    return jac.reshape(6, n, 3)


COV_INDEX = [(a, b) for a in range(5) for b in range(a, 5)]


def cov_full(c15):
    """[..., 15] upper triangles -> [..., 5, 5] symmetric matrices."""
    c15 = np.asarray(c15)
    out = np.empty(c15.shape[:-1] + (5, 5))
    for q, (a, b) in enumerate(COV_INDEX):
        out[..., a, b] = c15[..., q]
        out[..., b, a] = c15[..., q]
    return out


def fit_cov(cfg, tuplets, nhits, x, y, z, layer, module=None, offsets=None):
    """Covariance of every fit: [N, 15], the upper triangle of the 5x5
    covariance of (kappa, phi0, cot_theta, d0, z0) row by row; NaN rows for
    failed fits."""
    tup = np.ascontiguousarray(tuplets, dtype=np.int32)
    nh = np.ascontiguousarray(nhits, dtype=np.uint8)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    mod = np.ascontiguousarray(module if module is not None else np.zeros(x.shape[0]), dtype=np.int16)
    off = _f64(offsets).reshape(-1) if offsets is not None else None
    cov = np.empty((tup.shape[0], 15), np.float64)
    lib().oracle_fit_cov(ct.byref(_config(cfg)), tup.shape[0], _p(tup), _p(nh), _p(x), _p(y), _p(z), _p(layer),
                         _p(mod), _p(off), _p(cov))
    return cov


def fit_cov_debug(cfg, X, Y, Z, layers):
    """(jc [5, n+1], jl [5, n], cov [5, 5]) of one track given its hit coordinates."""
    n = len(X)
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    lay = np.ascontiguousarray(layers, dtype=np.int32)
    jc = np.empty(5 * (n + 1))
    jl = np.empty(5 * n)
    cov = np.empty(25)
    st = lib().oracle_fit_cov_debug(ct.byref(_config(cfg)), n, _p(X), _p(Y), _p(Z), _p(lay), _p(jc), _p(jl),
                                    _p(cov))
    if st != 0:
        raise ValueError(f"fit status {st}")
    return jc.reshape(5, n + 1), jl.reshape(5, n), cov.reshape(5, 5)


def ambiguity(hits, cells, nhits, chi2, tip):
    """Ambiguity resolution of section 3.5: bool keep [N] (see oracle.cpp)."""
    h = np.ascontiguousarray(hits, dtype=np.int32)
    c = np.ascontiguousarray(cells, dtype=np.int32)
    nh = np.ascontiguousarray(nhits, dtype=np.uint8)
    c2 = _f64(chi2)
    tp = _f64(tip)
    keep = np.empty(h.shape[0], np.uint8)
    lib().oracle_ambiguity(h.shape[0], _p(h), _p(c), _p(nh), _p(c2), _p(tp), _p(keep))
    return keep.astype(bool)


def vertices(cfg, z0, var_z0, kappa, nhits, use=None):
    """Pixel vertices of one event (section 3.6; see oracle.cpp).

    Returns dict: z, var, chi2, ndf, n_tracks, sum_pt2 per vertex (largest
    sum_pt2 first) and track_vertex [N] (vertex index or -1)."""
    z0, var = _f64(z0), _f64(var_z0)
    kap = _f64(kappa)
    nh = np.ascontiguousarray(nhits, dtype=np.uint8)
    n = z0.shape[0]
    u = np.ascontiguousarray(np.ones(n, bool) if use is None else use, dtype=np.uint8)
    K = 0.299792458 * cfg["bfield"] / 100.0
    cap = max(16, n)
    out = {k: np.empty(cap, np.float64) for k in ("z", "var", "chi2", "sum_pt2")}
    ndf = np.empty(cap, np.int32)
    nt = np.empty(cap, np.int32)
    tv = np.empty(n, np.int32)
    nv = lib().oracle_vertices(n, _p(z0), _p(var), _p(kap), _p(nh), _p(u), cfg["vtx_min_hits"], cfg["vtx_pt_min"],
                               cfg["vtx_err_max"], cfg["vtx_dz_cut"], cfg["vtx_chi2_max"], cfg["vtx_split_chi2_ndf"],
                               cfg["vtx_pt_cap"], cfg["vtx_kmeans_iter"], K, cap, _p(out["z"]), _p(out["var"]),
                               _p(out["chi2"]), _p(ndf), _p(nt), _p(out["sum_pt2"]), _p(tv))
    res = {k: v[:nv] for k, v in out.items()}
    res.update(ndf=ndf[:nv], n_tracks=nt[:nv], track_vertex=tv)
    return res


def fit_grad(cfg, tuplets, nhits, x, y, z, layer, module, offsets, g_params, g_chi2, n_modules=1856):
    """Reference gradient: (grad_hits [n_hits, 3], grad_offsets [n_modules, 3])."""
    tup = np.ascontiguousarray(tuplets, dtype=np.int32)
    nh = np.ascontiguousarray(nhits, dtype=np.uint8)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(layer, dtype=np.uint8)
    mod = np.ascontiguousarray(module, dtype=np.int16)
    off = _f64(offsets).reshape(-1) if offsets is not None else None
    gp = _f64(g_params).reshape(-1)
    gc = _f64(g_chi2) if g_chi2 is not None else None
    gh = np.zeros((x.shape[0], 3), np.float64)
    go = np.zeros((n_modules, 3), np.float64)
    c = _config(cfg)
    lib().oracle_fit_grad(ct.byref(c), tup.shape[0], _p(tup), _p(nh), _p(x), _p(y), _p(z), _p(layer),
                          _p(mod), _p(off), _p(gp), _p(gc), _p(gh), _p(go))
    return gh, go


def reconstruct_event(cfg, x, y, z, layer, dedup=True):
    """Doublets (then the Fishbone when cfg["fishbone_theta"] > 0) -> links ->
    n-tuplets of one event (dict of every product)."""
    ci, co, cp = doublets(cfg, x, y, z, layer)
    if cfg.get("fishbone_theta", 0.0) > 0.0:
        keep = fishbone(cfg, x, y, z, ci, co)
        ci, co, cp = ci[keep], co[keep], cp[keep]
    li, lo = links(cfg, x, y, z, layer, ci, co)
    nt = ntuplets(cfg, layer, ci, co, li, lo, dedup=dedup)
    return {"cell_inner": ci, "cell_outer": co, "cell_pair": cp, "link_in": li, "link_out": lo, **nt}
