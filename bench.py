#!/usr/bin/env python3
"""Benchmark of the pixel-track hot path on one MI355X.

Step: one pass of the whole path over a batch of 64 synthetic events at
pileup 200 -- doublets, cell links, n-tuplets with duplicate removal, the
broken-line fit (single precision with the double-precision refit of stiff
tracks) and its adjoint -- launched as one hipGraph (pt_plan_run).  Inputs
are resident in device memory before timing starts.

Also reported: the same 64 events processed one event per call sequence
(the per-event form), the fit forward + adjoint throughput on 10^6 tracks
against the HBM roofline, per-kernel durations from HIP events, and the
CPU oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s at PU200, batched vs per-event; fit fwd+bwd tracks/s vs HBM roofline"
# fp64 VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (T ops/s)
FP64_VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# timing regions (one kernel each, see pixeltrack.h) in step order
TIMED = ("doublets_count", "doublets_write", "cell_index", "link_segments", "links", "link_emit", "root_count",
         "root_write", "dfs_count", "dfs_write", "dedup", "fit_fwd", "fit_bwd")
# source file of each timed kernel (for the traffic record)
KERNEL_SOURCE = {"doublets_count": "doublets.hip", "doublets_write": "doublets.hip", "cell_index": "links.hip",
                 "link_segments": "links.hip", "links": "links.hip", "link_emit": "links.hip",
                 "root_count": "ntuplets.hip", "root_write": "ntuplets.hip", "dfs_count": "ntuplets.hip",
                 "dfs_write": "ntuplets.hip", "fit_fwd": "fit.hip", "fit_bwd": "fit.hip"}
KERNEL_SYMBOL = {"doublets_count": "k_doublets<false>", "doublets_write": "k_doublets<true>",
                 "cell_index": "k_cell_index", "link_segments": "k_seg_scatter", "links": "k_link_hits",
                 "link_emit": "k_link_place", "root_count": "k_root_count", "root_write": "k_mask_write",
                 "dfs_count": "k_dfs<true>", "dfs_write": "k_dfs<false>", "fit_fwd": "k_fit<4,6>",
                 "fit_bwd": "k_grad<4,6>"}
# Algorithmic work per unit, for the roofline of whichever kernel dominates:
#  links: 12 B per candidate pair the search examines (the two segments'
#    dr, dz as the test needs them, less what the wavefront shares) and 8 B
#    per link; the R-Z test of an examined pair is 7 fp64 VALU operations
#    (A = ar bz - az br: 2 mul + 1 sub; A A; La Lb; theta2 (La Lb); compare)
#  cell_index: per cell read inner, outer (8 B), write the 8-byte index
#    entry, and clear out_count and has_inner (5 B)
#  doublets_write: per cell write inner, outer and pair (9 B)
LINK_OPS_PER_CANDIDATE = 7.0
LINK_BYTES_PER_CANDIDATE = 12.0
LINK_BYTES_PER_LINK = 8.0
LINK_BUCKETS_MAX = 128  # direction buckets of the windowed link search, at most
LINK_WIN_CAP = 224      # out-cells of a hit it stages (copies included)
CELL_INDEX_BYTES_PER_CELL = 21.0
DOUBLET_BYTES_PER_CELL = 9.0
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def caps(n_hits, n_events):
    cells = 128 * n_hits
    return dict(n_hits=n_hits, n_events=n_events, cells_cap=cells, links_cap=cells // 4, tuplets_cap=n_hits)


def chain_workload(args):
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    cfg_d = C.default_config()
    t0 = time.time()
    h = E.config5(n_events=args.events)
    off_np = E.module_offsets()
    log(f"generated {h.n_events} events, {h.n_hits} hits in {time.time() - t0:.1f}s")
    cp = caps(h.n_hits, h.n_events)
    hits = api.Hits.from_host(h)
    perf = settings(args, cfg_d, hits, cp)
    cfg = A.make_config(cfg_d, **perf)
    offsets = torch.from_numpy(off_np).cuda()
    cells = api.Cells.empty(cp["cells_cap"], h.n_hits)
    links = api.Links.empty(cp["links_cap"], cp["cells_cap"])
    tup = api.Tuplets.empty(cp["tuplets_cap"])
    tracks = api.Tracks.empty(cp["tuplets_cap"], A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    gp_np, gc_np = E.cotangents(5, cp["tuplets_cap"])
    g_params = torch.from_numpy(gp_np).cuda()
    g_chi2 = torch.from_numpy(gc_np).cuda()
    grad_hits = torch.zeros((h.n_hits, 3), dtype=torch.float32, device="cuda")
    grad_off = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")
    plan = api.Plan(cfg, precision=A.PT_FIT_F32_F64SOLVE, with_adjoint=True, **cp)

    def step():
        plan.run(hits, cells, links, tup, tracks, status, offsets=offsets, g_params=g_params, g_chi2=g_chi2,
                 grad_hits=grad_hits, grad_offsets=grad_off)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    flags = int(status[A.PT_ST_FLAGS].item()) & 0xFFFFFFFF
    if flags & (A.PT_FLAG_CELLS_OVERFLOW | A.PT_FLAG_LINKS_OVERFLOW | A.PT_FLAG_TUPLETS_OVERFLOW):
        raise RuntimeError(f"capacity overflow (flags {flags:#x}); raise the capacities")
    n_cells = int(cells.count.item())
    n_links = int(links.count.item())
    n_raw = int(tup.count_raw.item())
    n_trk = int(tup.count.item())
    log(f"per batch: {n_cells} doublets, {n_links} links, {n_raw} n-tuplets, {n_trk} tracks")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    log(f"batched (graph): {t_batched * 1e3:.3f} ms per step")
    # the graph must keep producing the eager results
    if int(cells.count.item()) != n_cells or int(tup.count.item()) != n_trk:
        raise RuntimeError("graph replay changed the products")

    # the same step with the hits copied from pinned host memory first
    host = [t.cpu().pin_memory() for t in (hits.x, hits.y, hits.z, hits.layer, hits.module, hits.event_offsets)]
    dev = (hits.x, hits.y, hits.z, hits.layer, hits.module, hits.event_offsets)

    def step_h2d():
        for d, hsrc in zip(dev, host):
            d.copy_(hsrc, non_blocking=True)
        step()

    step_h2d()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_h2d()
    torch.cuda.synchronize()
    t_h2d = (time.perf_counter() - t0) / args.steps
    log(f"batched with the host-to-device copy of the hits: {t_h2d * 1e3:.3f} ms per step")

    # per-event form: the same calls event by event, no graph
    ev_hits = []
    for e in range(h.n_events):
        a, b = int(h.event_offsets[e]), int(h.event_offsets[e + 1])
        ev_hits.append(api.Hits(hits.x[a:b], hits.y[a:b], hits.z[a:b], hits.layer[a:b], hits.module[a:b],
                                torch.tensor([0, b - a], dtype=torch.int32, device="cuda")))
    max_ev = max(x.n_hits for x in ev_hits)
    cpe = caps(max_ev, 1)
    pipe = api.Pipeline(cfg_d, precision=A.PT_FIT_F32_F64SOLVE, **perf, **cpe)
    gh_e = torch.zeros((max_ev, 3), dtype=torch.float32, device="cuda")

    def per_event_pass():
        for eh in ev_hits:
            pipe.reconstruct(eh, offsets=offsets)
            pipe.backward(eh, g_params[: pipe.tuplets.cap], g_chi2[: pipe.tuplets.cap], gh_e[: eh.n_hits], grad_off,
                          offsets=offsets)

    per_event_pass()
    torch.cuda.synchronize()
    pe_steps = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(pe_steps):
        per_event_pass()
    torch.cuda.synchronize()
    t_per_event = (time.perf_counter() - t0) / pe_steps
    log(f"per-event: {t_per_event * 1e3:.3f} ms per pass")

    # kernel durations (HIP events on the call stream), eager calls of the same step
    api.timing_reset()
    api.timing_enable(True)
    pipe_b = api.Pipeline(cfg_d, precision=A.PT_FIT_F32_F64SOLVE, **perf, **cp)
    kt_steps = max(3, args.steps // 2)
    for _ in range(kt_steps):
        pipe_b.reconstruct(hits, offsets=offsets)
        pipe_b.backward(hits, g_params, g_chi2, grad_hits, grad_off, offsets=offsets)
    torch.cuda.synchronize()
    api.timing_enable(False)
    kern = {}
    for name in TIMED:
        ms, n = api.timing_read(name)
        if n:
            kern[name] = ms / n
    api.timing_reset()
    # cell pairs sharing a hit, and those the link search examines (for the
    # link kernel's work accounting)
    n_pairs, n_examined = link_pair_counts(pipe_b.cells, h, cfg_d)
    counts = dict(hits=h.n_hits, doublets=n_cells, links=n_links, ntuplets=n_raw, tracks=n_trk,
                  link_candidates=n_pairs, link_examined=n_examined)
    table2 = table2_counters(pipe_b, cfg_d, h.n_events)
    del pipe_b, pipe, plan
    torch.cuda.empty_cache()
    workflows = {name: full_chain(args, cfg, perf, h, hits, name) for name, cfg in
                 (("quadruplets", cfg_d), ("triplets", C.default_config(min_hits=3)))}
    mixed = mixed_pileup(args, cfg_d) if args.mixed_events else None
    fishbone = fishbone_workload(args, perf)
    return dict(t_batched=t_batched, t_per_event=t_per_event, t_h2d=t_h2d, kernels_ms=kern, counts=counts,
                n_events=h.n_events, hits_np=h, cfg_d=cfg_d, perf=perf, mixed=mixed, table2=table2,
                workflows=workflows, fishbone=fishbone)


def fishbone_workload(args, perf):
    """The overlap geometry (a quarter of the layer crossings leave a second
    hit on an overlapping module) at pileup 200: the forward path (doublets ..
    fit) as one graph per step with the Fishbone off and on, and the
    Fishbone's own kernels timed eagerly."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    h = E.overlap_batch(n_events=args.events, pileup=200)
    hits = api.Hits.from_host(h)
    cp = caps(h.n_hits, h.n_events)
    out = {"events": h.n_events, "hits": h.n_hits,
           "workload": f"{h.n_events} events at pileup 200 in the overlap geometry (second hits on overlapping "
                       "ladders and blades for a quarter of the layer crossings), forward path doublets .. fit, "
                       "one hipGraph per step"}
    for name, theta in (("off", 0.0), ("on", 0.01)):
        cfg = A.make_config(C.default_config(fishbone_theta=theta), **perf)
        cells = api.Cells.empty(cp["cells_cap"], h.n_hits)
        links = api.Links.empty(cp["links_cap"], cp["cells_cap"])
        tup = api.Tuplets.empty(cp["tuplets_cap"])
        tracks = api.Tracks.empty(cp["tuplets_cap"], A.PT_FIT_F32_F64SOLVE)
        status = api.new_status()
        plan = api.Plan(cfg, precision=A.PT_FIT_F32_F64SOLVE, **cp)
        for _ in range(max(args.warmup, 1)):
            plan.run(hits, cells, links, tup, tracks, status)
        torch.cuda.synchronize()
        flags = int(status[A.PT_ST_FLAGS].item()) & 0xFFFFFFFF
        if flags & (A.PT_FLAG_CELLS_OVERFLOW | A.PT_FLAG_LINKS_OVERFLOW | A.PT_FLAG_TUPLETS_OVERFLOW):
            raise RuntimeError(f"capacity overflow in the overlap batch (flags {flags:#x})")
        steps = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.run(hits, cells, links, tup, tracks, status)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        rec = dict(events_per_s=h.n_events / t, ms_per_step=t * 1e3, doublets=int(cells.count.item()),
                   links=int(links.count.item()), tracks=int(tup.count.item()))
        del plan
        if theta > 0.0:
            ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, h.n_events, cp["cells_cap"], cp["links_cap"],
                                                      cp["tuplets_cap"]))
            api.timing_reset()
            api.timing_enable(True)
            for _ in range(steps):
                api.build_doublets(hits, cfg, cells, status, ws)
            torch.cuda.synchronize()
            api.timing_enable(False)
            ms, n = api.timing_read("fishbone")
            api.timing_reset()
            rec["fishbone_ms"] = ms / max(n, 1)
            del ws
        out[name] = rec
        log(f"overlap batch, Fishbone {name}: {t * 1e3:.3f} ms per step, {rec['doublets']} doublets, "
            f"{rec['tracks']} tracks")
        del cells, links, tup, tracks
        torch.cuda.empty_cache()
    return out


def table2_counters(pipe, cfg_d, n_events):
    """Per-event counters in the shape of the paper's Table 2 (doublets,
    n-tuplets and tracks per event, the fraction of doublets without any
    link), plus roots, n-tuplets by hit count and the fit's fallback and
    failure counts, from the products of one eager pass."""
    import torch

    from paper_2008_13461_amd import _abi as A
    n_cells = min(int(pipe.cells.count.item()), pipe.cells.cap)
    out_count = pipe.links.out_count[:n_cells]
    has_inner = pipe.links.has_inner[:n_cells]
    unconn = ((out_count == 0) & (has_inner == 0)).sum().item()
    inner_layer = torch.tensor([p[0] for p in cfg_d["pairs"]], device="cuda")[pipe.cells.pair[:n_cells].long()]
    always = torch.zeros(10, dtype=torch.bool, device="cuda")
    always[cfg_d["root_always"]] = True
    if_free = torch.zeros(10, dtype=torch.bool, device="cuda")
    if_free[cfg_d["root_if_free"]] = True
    roots = (always[inner_layer] | (if_free[inner_layer] & (has_inner == 0))).sum().item()
    raw_n = pipe.tuplets.raw()[1].long().cpu().numpy()
    kept_n = pipe.tuplets.kept_rows()[1].long().cpu().numpy()
    st = pipe.status.cpu().numpy()
    return dict(doublets_per_event=n_cells / n_events, unconn_fraction=unconn / max(n_cells, 1),
                roots_per_event=roots / n_events, ntuplets_per_event=len(raw_n) / n_events,
                tracks_per_event=len(kept_n) / n_events,
                ntuplets_by_hits={int(k): int(v) for k, v in zip(*np.unique(raw_n, return_counts=True))},
                tracks_by_hits={int(k): int(v) for k, v in zip(*np.unique(kept_n, return_counts=True))},
                fit_f64_refits=int(st[A.PT_ST_FIT_F64]), fit_failed=int(st[A.PT_ST_FIT_FAILED]),
                truncated_searches=int(st[A.PT_ST_TRUNCATED]))


def full_chain(args, cfg_d, perf, h, hits, name):
    """The whole workflow of the paper's throughput measurement minus local
    reconstruction, as one graph per step: doublets .. fit with covariance,
    ambiguity resolution and pixel vertices (no adjoint), on the same batch;
    plus the eager time of the ambiguity and vertex stages alone."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api

    cp = caps(h.n_hits, h.n_events)
    if cfg_d["min_hits"] == 3:   # triplets: about 18 rows per hit at pileup 200
        cp["tuplets_cap"] = 24 * h.n_hits
    cfg = A.make_config(cfg_d, **perf)
    cells = api.Cells.empty(cp["cells_cap"], h.n_hits)
    links = api.Links.empty(cp["links_cap"], cp["cells_cap"])
    tup = api.Tuplets.empty(cp["tuplets_cap"])
    tracks = api.Tracks.empty(cp["tuplets_cap"], A.PT_FIT_F32_F64SOLVE, with_cov=True)
    status = api.new_status()
    sel = torch.empty(cp["tuplets_cap"], dtype=torch.int32, device="cuda")
    nsel = torch.zeros(1, dtype=torch.int32, device="cuda")
    vtx = api.Vertices.empty(cp["tuplets_cap"], h.n_events, cp["tuplets_cap"])
    plan = api.Plan(cfg, precision=A.PT_FIT_F32_F64SOLVE, stages=A.PT_STAGE_AMBIGUITY | A.PT_STAGE_VERTICES, **cp)

    def step():
        plan.run(hits, cells, links, tup, tracks, status, selected=sel, n_selected=nsel, vertices=vtx)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    flags = int(status[A.PT_ST_FLAGS].item()) & 0xFFFFFFFF
    if flags & (A.PT_FLAG_CELLS_OVERFLOW | A.PT_FLAG_LINKS_OVERFLOW | A.PT_FLAG_TUPLETS_OVERFLOW |
                A.PT_FLAG_VERTICES_OVERFLOW):
        raise RuntimeError(f"capacity overflow in the {name} workflow (flags {flags:#x})")
    steps = max(3, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    # the two stages alone, eagerly, timed with events on the current stream
    ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, h.n_events, cp["cells_cap"], cp["links_cap"],
                                              cp["tuplets_cap"]))
    stage_ms = {}
    for stage in ("ambiguity", "vertices"):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            if stage == "ambiguity":
                api.resolve_ambiguities(hits, cfg, cells, tup, A.PT_FIT_F32_F64SOLVE, tracks, status, ws)
            else:
                api.find_vertices(hits, cfg, tup, A.PT_FIT_F32_F64SOLVE, tracks, sel, nsel, vtx, status, ws)
        b.record()
        b.synchronize()
        stage_ms[stage] = a.elapsed_time(b) / steps
    nv = int(vtx.count.item())
    out = dict(events_per_s=h.n_events / t, ms_per_step=t * 1e3, min_hits=cfg_d["min_hits"],
               tracks=int(tup.count.item()), selected_tracks=int(nsel.item()), vertices=nv,
               vertices_per_event=nv / h.n_events, stage_ms=stage_ms,
               workload=f"{h.n_events} events at pileup 200: doublets, links, n-tuplets (min {cfg_d['min_hits']} "
                        "hits), dedup, fit with covariance, ambiguity resolution, pixel vertices; one hipGraph")
    log(f"{name} workflow: {t * 1e3:.3f} ms per step, {nv} vertices, stages {stage_ms}")
    del plan, cells, links, tup, tracks, vtx, ws
    torch.cuda.empty_cache()
    return out


def link_pair_counts(cells, h, cfg_d):
    """(pairs, examined): the in-cell/out-cell pairs that share a middle hit,
    and how many of them the link search tests.  The search bins a hit's
    out-cells by the direction key of their R-Z segment (B buckets) and tests
    each in-cell against its own and the neighbouring buckets; a hit whose
    out-cells (with the copies of the two end buckets) exceed WIN_CAP, or one
    with a keyless out-cell, has every pair tested.  Recomputed here from the
    hits (h.x, h.y, h.z) with the same operations, for reporting only."""
    import math

    import numpy as np
    import torch

    ci, co, _ = cells.valid()
    ci, co = ci.long(), co.long()
    n = ci.numel()
    n_hits = h.n_hits
    nb = torch.zeros(n_hits, dtype=torch.int64, device=ci.device)
    nb.index_add_(0, ci, torch.ones_like(ci))
    pairs = int(nb[co].sum().item())
    th = max(abs(cfg_d["ca_theta_barrel"]), abs(cfg_d["ca_theta_endcap"]))
    B = 0
    if th < 0.5:
        b = math.floor(2.0 / (math.asin(th) + 1e-4))
        B = min(b, LINK_BUCKETS_MAX) if b >= 4 else 0
    if B == 0 or n == 0:
        return pairs, pairs
    x, y = (np.asarray(a, np.float64) for a in (h.x, h.y))
    r = torch.from_numpy(np.sqrt(x * x + y * y)).to(ci.device)
    z = torch.from_numpy(np.asarray(h.z, np.float64)).to(ci.device)
    dr, dz = r[co] - r[ci], z[co] - z[ci]
    flip = dr < 0
    r = torch.where(flip, -dr, dr).float()
    z = torch.where(flip, -dz, dz).float()
    key = z / (r + z.abs())
    ok = key == key
    bk = ((key + 1.0) * (0.5 * B)).nan_to_num(0.0).to(torch.int64).clamp(0, B - 1)
    hist = torch.zeros(n_hits * B, dtype=torch.int64, device=ci.device)
    hist.index_add_(0, ci * B + bk, ok.long())
    hist = hist.view(n_hits, B)
    bad = torch.zeros(n_hits, dtype=torch.int64, device=ci.device)
    bad.index_add_(0, ci, (~ok).long())
    win = (nb + hist[:, 0] + hist[:, B - 1] <= LINK_WIN_CAP) & (bad == 0)
    h = co
    w = hist[h, (bk - 1) % B] + hist[h, bk] + hist[h, (bk + 1) % B]
    w = torch.where(ok, w, nb[h])
    examined = torch.where(win[h], w, nb[h])
    return pairs, int(examined.sum().item())


def mixed_pileup(args, cfg_d):
    """256 events with pileup uniform in 20..200: the batched form (one graph
    per step, settings tuned for this batch) and the per-event form (the same
    calls event by event on one stream, no graph), forward path."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import events as E

    h = E.config3(n_events=args.mixed_events)
    cp = caps(h.n_hits, h.n_events)
    hits = api.Hits.from_host(h)
    perf = settings(args, cfg_d, hits, cp)
    cells = api.Cells.empty(cp["cells_cap"], h.n_hits)
    links = api.Links.empty(cp["links_cap"], cp["cells_cap"])
    tup = api.Tuplets.empty(cp["tuplets_cap"])
    tracks = api.Tracks.empty(cp["tuplets_cap"], A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    plan = api.Plan(A.make_config(cfg_d, **perf), precision=A.PT_FIT_F32_F64SOLVE, **cp)

    def step():
        plan.run(hits, cells, links, tup, tracks, status)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    flags = int(status[A.PT_ST_FLAGS].item()) & 0xFFFFFFFF
    if flags & (A.PT_FLAG_CELLS_OVERFLOW | A.PT_FLAG_LINKS_OVERFLOW | A.PT_FLAG_TUPLETS_OVERFLOW):
        raise RuntimeError(f"capacity overflow in the mixed-pileup batch (flags {flags:#x})")
    steps = max(3, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    n_trk = int(tup.count.item())
    n_dbl = int(cells.count.item())
    del plan, cells, links, tup, tracks
    torch.cuda.empty_cache()
    # kernel times of the eager batched calls: per doublet, against the
    # uniform PU200 batch, they show whether uneven events leave the flat
    # all-event kernels idle in a tail
    pipe_b = api.Pipeline(cfg_d, precision=A.PT_FIT_F32_F64SOLVE, **perf, **cp)
    pipe_b.reconstruct(hits)
    torch.cuda.synchronize()
    api.timing_reset()
    api.timing_enable(True)
    for _ in range(steps):
        pipe_b.reconstruct(hits)
    torch.cuda.synchronize()
    api.timing_enable(False)
    kern = {}
    for name in TIMED:
        ms, n = api.timing_read(name)
        if n:
            kern[name] = ms / n
    api.timing_reset()
    del pipe_b
    torch.cuda.empty_cache()
    # per-event form
    ev_hits = []
    for e in range(h.n_events):
        a, b = int(h.event_offsets[e]), int(h.event_offsets[e + 1])
        ev_hits.append(api.Hits(hits.x[a:b], hits.y[a:b], hits.z[a:b], hits.layer[a:b], hits.module[a:b],
                                torch.tensor([0, b - a], dtype=torch.int32, device="cuda")))
    pipe = api.Pipeline(cfg_d, precision=A.PT_FIT_F32_F64SOLVE, **perf, **caps(max(x.n_hits for x in ev_hits), 1))

    def per_event_pass():
        for eh in ev_hits:
            pipe.reconstruct(eh)

    per_event_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, steps // 2)):
        per_event_pass()
    torch.cuda.synchronize()
    t_pe = (time.perf_counter() - t0) / max(1, steps // 2)
    out = dict(events=h.n_events, hits=h.n_hits, doublets=n_dbl, tracks=n_trk, tuned=perf,
               kernel_ms=kern, kernel_ns_per_doublet={k: v * 1e6 / n_dbl for k, v in kern.items()},
               ms_per_step=t * 1e3, events_per_s=h.n_events / t, per_event_ms=t_pe * 1e3,
               per_event_events_per_s=h.n_events / t_pe, batched_over_per_event=t_pe / t,
               workload=f"{h.n_events} events, pileup uniform in 20..200, forward path (no adjoint); batched: one "
                        "hipGraph per step; per-event: the same calls event by event, no graph")
    log(f"mixed pileup: {h.n_events} events, {h.n_hits} hits, {t * 1e3:.3f} ms batched, {t_pe * 1e3:.3f} ms "
        "per-event")
    del pipe, hits, ev_hits
    torch.cuda.empty_cache()
    return out


def fit_workload(args):
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    t0 = time.time()
    ts = E.config4(n_tracks=args.fit_tracks)
    log(f"generated {len(ts.nhits)} tracks in {time.time() - t0:.1f}s")
    cfg = A.make_config(C.default_config(exclusive_hits=1))
    hits = api.Hits.from_host(ts.hits)
    n = len(ts.nhits)
    tup = api.Tuplets.from_rows(torch.from_numpy(ts.tuplets).cuda(), torch.from_numpy(ts.nhits).cuda())
    tracks = api.Tracks.empty(n, A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, ts.hits.n_hits, 1, 0, 0, n))
    off = torch.from_numpy(E.module_offsets()).cuda()
    gp, gc = (torch.from_numpy(a).cuda() for a in E.cotangents(4, n))
    gh = torch.zeros((ts.hits.n_hits, 3), dtype=torch.float32, device="cuda")
    go = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")

    def step():
        api.fit_broken_line(hits, cfg, tup, off, A.PT_FIT_F32_F64SOLVE, tracks, status, ws)
        api.fit_broken_line_bwd(hits, cfg, tup, off, A.PT_FIT_F32_F64SOLVE, gp, gc, gh, go, status, ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(args.steps, 5)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    api.timing_reset()
    api.timing_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    api.timing_enable(False)
    fwd_ms, nf = api.timing_read("fit_fwd")
    bwd_ms, nb = api.timing_read("fit_bwd")
    api.timing_reset()
    # forward + adjoint captured as one graph (torch's capture of the library's
    # kernels on the capture stream), replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / steps
    del graph
    nh = ts.nhits.astype(np.int64)
    out = dict(t_step=t_step, t_graph=t_graph, fwd_ms=fwd_ms / max(nf, 1), bwd_ms=bwd_ms / max(nb, 1), n_tracks=n,
               n_hits_total=int(nh.sum()), mean_n=float(nh.mean()), nhits=nh)
    del tup, tracks, ws, gh, hits
    torch.cuda.empty_cache()
    if args.fit_tiles > 1:
        out["asymptote"] = fit_asymptote(args, ts)
    return out


def fit_asymptote(args, ts):
    """Forward + adjoint on fit_tiles copies of the fit workload side by side
    (each copy's rows point at its own copy of the hits), eagerly."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    k = args.fit_tiles
    h = ts.hits
    n_h = h.n_hits
    big = E.Hits(np.tile(h.x, k), np.tile(h.y, k), np.tile(h.z, k), np.tile(h.layer, k), np.tile(h.module, k),
                 np.zeros(0, np.int32), np.array([0, k * n_h], np.int32))
    rows = np.concatenate([np.where(ts.tuplets >= 0, ts.tuplets + c * n_h, -1) for c in range(k)]).astype(np.int32)
    nhits = np.tile(ts.nhits, k)
    n = rows.shape[0]
    cfg = A.make_config(C.default_config(exclusive_hits=1))
    hits = api.Hits.from_host(big)
    tup = api.Tuplets.from_rows(torch.from_numpy(rows).cuda(), torch.from_numpy(nhits).cuda())
    tracks = api.Tracks.empty(n, A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, big.n_hits, 1, 0, 0, n))
    off = torch.from_numpy(E.module_offsets()).cuda()
    gp, gc = (torch.from_numpy(a).cuda() for a in E.cotangents(4, n))
    gh = torch.zeros((big.n_hits, 3), dtype=torch.float32, device="cuda")
    go = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")

    def step():
        api.fit_broken_line(hits, cfg, tup, off, A.PT_FIT_F32_F64SOLVE, tracks, status, ws)
        api.fit_broken_line_bwd(hits, cfg, tup, off, A.PT_FIT_F32_F64SOLVE, gp, gc, gh, go, status, ws)

    step()
    torch.cuda.synchronize()
    steps = max(3, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    nh = nhits.astype(np.int64)
    nbytes = float((19 * nh + 26).sum() + (31 * nh + 25).sum())
    out = dict(tracks=n, ms_fwd_bwd_step=t * 1e3, tracks_per_s=n / t, achieved_gbs=nbytes / t / 1e9,
               frac=nbytes / t / 1e9 / HBM_PEAK_GBS,
               workload=f"{k} copies of the fit workload side by side ({n} tracks), forward + adjoint, eager calls")
    log(f"fit asymptote: {n} tracks, {t * 1e3:.3f} ms per forward + adjoint")
    del tup, tracks, ws, gh, hits
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, chain):
    """The oracle as it stands, timed on this host's cores on bounded samples
    of the same workloads: the whole chain of pileup-200 events (binned
    doublet search, links, n-tuplets, dedup, fit, dual-number gradient with
    unit cotangents), events over OpenMP threads, on one core and on every
    core this process may use; and the fit forward + dual-number gradient of
    fit-workload tracks on one core and on all."""
    import oracle as O
    from synth import config as C
    from synth import events as E

    h = chain["hits_np"]
    cfg_d = chain["cfg_d"]
    off = E.module_offsets()
    cores = len(os.sched_getaffinity(0))

    def chain_rate(n_events, threads):
        sub_off = h.event_offsets[: n_events + 1]
        last = int(sub_off[-1])
        t0 = time.perf_counter()
        tr = O.chain_batch(cfg_d, sub_off, h.x[:last], h.y[:last], h.z[:last], h.layer[:last], h.module[:last], off,
                           n_threads=threads)
        dt = time.perf_counter() - t0
        return n_events / dt, dt, int(tr.sum())

    budget = args.cpu_seconds
    # one core: events one after the other until about half the budget is spent
    r1, dt1, tr1 = chain_rate(1, 1)
    n1 = max(1, min(h.n_events, int(0.5 * budget / max(dt1, 1e-3))))
    if n1 > 1:
        r1, dt1, tr1 = chain_rate(n1, 1)
    # every core: enough events for every thread
    nall = min(h.n_events, max(cores, int(0.5 * budget * cores / max(dt1 / n1, 1e-3))))
    rall, dtall, trall = chain_rate(nall, cores)
    # the fit workload: forward + dual-number gradient
    ts = E.config4(n_tracks=60_000)
    gp, gc = E.cotangents(4, len(ts.nhits))
    fit_rates = {}
    for threads, n in ((1, 10_000), (cores, 60_000)):
        t0 = time.perf_counter()
        O.fit_grad_batch(C.default_config(), ts.tuplets[:n], ts.nhits[:n], ts.hits.x, ts.hits.y, ts.hits.z,
                         ts.hits.layer, ts.hits.module, off, gp[:n], gc[:n], n_threads=threads)
        fit_rates[threads] = n / (time.perf_counter() - t0)
    return dict(value=rall, unit="events/s", cores=cores, kind="oracle",
                sample=f"{nall} of the {h.n_events} pileup-200 events, whole path (binned doublet search, links, "
                       f"n-tuplets, dedup, fit, dual-number gradient of {trall} tracks) over {cores} OpenMP threads "
                       f"in {dtall:.1f} s",
                cpu_model=cpu_model(), single_core_events_per_s=r1,
                single_core_sample=f"{n1} events ({tr1} tracks) on 1 thread in {dt1:.1f} s",
                fit_tracks_per_s=fit_rates[cores], fit_single_core_tracks_per_s=fit_rates[1],
                fit_sample="fit-workload tracks (50/30/20% 4/5/6 hits), forward fit + dual-number gradient "
                           f"(a reference, not an optimised CPU adjoint): 10000 tracks on 1 thread, 60000 on {cores}")


def source_sha(*files):
    """SHA-256 of kernel sources (under paper_2008_13461_amd/csrc) together
    with the internal header every kernel includes."""
    import hashlib

    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2008_13461_amd", "csrc")
    return hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                   for f in files + ("pt_internal.h",))).hexdigest()


def traffic_record(name):
    """(HBM bytes per launch, VALU issue fraction or None) of a kernel from
    the committed counter summary (profiles/pu200_step_counters.txt), or None
    when its sources have changed since the counters were taken."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "pu200_step_counters.txt")
    src = KERNEL_SOURCE.get(name)
    if src is None or not os.path.exists(path):
        return None
    sha = source_sha(src)
    for line in open(path):
        if not line.startswith("traffic "):
            continue
        f = dict(kv.split("=", 1) for kv in line.split()[1:])
        if f.get("kernel") == name and f.get("sha256") == sha:
            issue = float(f["valu_issue_frac"]) if "valu_issue_frac" in f else None
            return float(f["fetch_bytes"]) + float(f["write_bytes"]), issue
    return None


def fit_counter_record():
    """Counters of the fit workload's kernels from profiles/fit_config4_counters.txt
    (its 'fit_counters' line), or None when the fit sources changed since."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "fit_config4_counters.txt")
    if not os.path.exists(path):
        return None
    sha = source_sha("fit.hip", "fit_core.h")
    for line in open(path):
        if line.startswith("fit_counters "):
            f = dict(kv.split("=", 1) for kv in line.split()[1:])
            if f.get("sha256") == sha:
                return {"traffic_bytes": float(f["traffic_bytes"]), "valu_issue_frac": float(f["valu_issue_frac"])}
    return None


def roofline(kern, cnt):
    """Roofline object of the dominant timed kernel of the step."""
    if not kern:
        return None
    name = max(kern, key=kern.get)
    sec = kern[name] * 1e-3
    roof = {"kernel": KERNEL_SYMBOL.get(name, name), "timing_region": name}
    if name == "links":
        nbytes = LINK_BYTES_PER_CANDIDATE * cnt["link_examined"] + LINK_BYTES_PER_LINK * cnt["links"]
        achieved = nbytes / sec / 1e9
        alu = LINK_OPS_PER_CANDIDATE * cnt["link_examined"] / sec / 1e12
        roof.update(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    algorithmic_bytes=nbytes,
                    alu={"achieved": alu, "peak": FP64_VALU_PEAK_TOPS, "unit": "TOP/s",
                         "frac": alu / FP64_VALU_PEAK_TOPS},
                    all_pairs_rate_tops=LINK_OPS_PER_CANDIDATE * cnt["link_candidates"] / sec / 1e12,
                    note="12 B per examined candidate pair + 8 B per link, over the kernel time; alu: 7 fp64 VALU "
                         "ops per examined pair against 256 CU x 4 SIMD x 16 lanes x 2.4 GHz (no FMA: contraction "
                         "is off); all_pairs_rate_tops counts every pair sharing a hit, most of which the direction "
                         "buckets skip.  Neither bound is reached: the kernel is limited by VALU instruction "
                         "issue (valu_issue_frac, from the committed SQ counters), the fixed work of each "
                         "hit's windowed search (staging, keys, scans, dealing pairs to lanes, beam-spot "
                         "batches) rather than its R-Z tests.")
    else:
        per_cell = {"cell_index": CELL_INDEX_BYTES_PER_CELL, "doublets_write": DOUBLET_BYTES_PER_CELL}.get(name)
        achieved = per_cell * cnt["doublets"] / sec / 1e9 if per_cell else None
        roof.update(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS if achieved else None)
    t = traffic_record(name)
    roof["traffic"] = t[0] if t else None
    if t and t[1] is not None:
        roof["valu_issue_frac"] = t[1]
    roof["traffic_unit"] = "bytes per launch (FETCH_SIZE and WRITE_SIZE, copy-calibrated)"
    return roof


def settings(args, cfg_d, hits, cp):
    """Bin count and block sizes: the ones given, else autotuned for this
    batch shape (they never change a result)."""
    if args.bins or args.block_doublets or args.block_links:
        from paper_2008_13461_amd import autotune

        perf = dict(autotune.DEFAULT)
        for name, v in (("n_phi_bins", args.bins), ("block_doublets", args.block_doublets),
                        ("block_links", args.block_links)):
            if v:
                perf[name] = v
        return perf
    from paper_2008_13461_amd import autotune

    t0 = time.time()
    perf = autotune.tune(cfg_d, hits, cp, cache=None)
    log(f"autotuned {perf} in {time.time() - t0:.1f}s")
    return perf


def profile_fit_run(args):
    """Two eager forward + adjoint passes over the fit workload, then two
    copies of 1 GiB (the calibration of the traffic counters)."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    ts = E.config4(n_tracks=args.fit_tracks)
    cfg = A.make_config(C.default_config(exclusive_hits=1))
    hits = api.Hits.from_host(ts.hits)
    n = len(ts.nhits)
    tup = api.Tuplets.from_rows(torch.from_numpy(ts.tuplets).cuda(), torch.from_numpy(ts.nhits).cuda())
    tracks = api.Tracks.empty(n, A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, ts.hits.n_hits, 1, 0, 0, n))
    off = torch.from_numpy(E.module_offsets()).cuda()
    gp, gc = (torch.from_numpy(a).cuda() for a in E.cotangents(4, n))
    gh = torch.zeros((ts.hits.n_hits, 3), dtype=torch.float32, device="cuda")
    go = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")
    for rep in range(2):
        api.fit_broken_line(hits, cfg, tup, off, A.PT_FIT_F32_F64SOLVE, tracks, status, ws)
        api.fit_broken_line_bwd(hits, cfg, tup, off, A.PT_FIT_F32_F64SOLVE, gp, gc, gh, go, status, ws)
        torch.cuda.synchronize()
        log(f"fit profile pass {rep}")
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("profile copies done (2^30 bytes read and written each)")


def profile_fishbone_run(args):
    """Two eager doublet passes with the Fishbone on the PU200 batch of the
    overlap geometry, for kernel traces of the Fishbone."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    h = E.overlap_batch(n_events=args.events, pileup=200)
    hits = api.Hits.from_host(h)
    cp = caps(h.n_hits, h.n_events)
    cfg = A.make_config(C.default_config(fishbone_theta=0.01), n_phi_bins=args.bins or 512,
                        block_doublets=args.block_doublets or 64, block_links=args.block_links or 64)
    cells = api.Cells.empty(cp["cells_cap"], h.n_hits)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, h.n_events, cp["cells_cap"], cp["links_cap"],
                                              cp["tuplets_cap"]))
    for rep in range(2):
        api.build_doublets(hits, cfg, cells, status, ws)
        torch.cuda.synchronize()
        log(f"Fishbone pass {rep}: {int(cells.count.item())} doublets kept, flags {int(status[0].item())}")


def profile_workflows_run(args):
    """Two eager passes of each workflow on the PU200 batch (reconstruction,
    fit with covariance, ambiguity resolution, vertices), with the bench's
    fixed settings, for kernel traces of the stages after the fit."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    h = E.config5(n_events=args.events)
    hits = api.Hits.from_host(h)
    perf = dict(n_phi_bins=args.bins or 512, block_doublets=args.block_doublets or 64,
                block_links=args.block_links or 64)
    for min_hits in (4, 3):
        cfg_d = C.default_config(min_hits=min_hits)
        cp = caps(h.n_hits, h.n_events)
        if min_hits == 3:
            cp["tuplets_cap"] = 24 * h.n_hits
        pipe = api.Pipeline(cfg_d, precision=A.PT_FIT_F32_F64SOLVE, **perf, **cp)
        pipe.tracks = api.Tracks.empty(cp["tuplets_cap"], pipe.precision, with_cov=True)
        sel = torch.empty(cp["tuplets_cap"], dtype=torch.int32, device="cuda")
        vtx = api.Vertices.empty(cp["tuplets_cap"], h.n_events, cp["tuplets_cap"])
        for rep in range(2):
            pipe.reconstruct(hits)
            sel, nsel = api.resolve_ambiguities(hits, pipe.cfg, pipe.cells, pipe.tuplets, pipe.precision,
                                                pipe.tracks, pipe.status, pipe.ws)
            api.find_vertices(hits, pipe.cfg, pipe.tuplets, pipe.precision, pipe.tracks, sel, nsel, vtx,
                              pipe.status, pipe.ws)
            torch.cuda.synchronize()
            log(f"workflow min_hits={min_hits} pass {rep}: flags {pipe.flags()}, {int(vtx.count.item())} vertices")
        del pipe, vtx, sel
        torch.cuda.empty_cache()


def profile_run(args):
    """Two eager passes of the batched step (with the settings the bench
    tunes), then two copies of 1 GiB: the copy
    kernel's FETCH_SIZE / WRITE_SIZE against its known 2^30 bytes read and
    written calibrate the traffic counters."""
    import torch

    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from synth import config as C
    from synth import events as E

    h = E.config5(n_events=args.events)
    cp = caps(h.n_hits, h.n_events)
    hits = api.Hits.from_host(h)
    perf = settings(args, C.default_config(), hits, cp)
    pipe = api.Pipeline(C.default_config(), precision=A.PT_FIT_F32_F64SOLVE, **perf, **cp)
    offsets = torch.from_numpy(E.module_offsets()).cuda()
    gp_np, gc_np = E.cotangents(5, cp["tuplets_cap"])
    g_params = torch.from_numpy(gp_np).cuda()
    g_chi2 = torch.from_numpy(gc_np).cuda()
    grad_hits = torch.zeros((h.n_hits, 3), dtype=torch.float32, device="cuda")
    for rep in range(2):
        pipe.reconstruct(hits, offsets=offsets)
        pipe.backward(hits, g_params, g_chi2, grad_hits, None, offsets=offsets)
        torch.cuda.synchronize()
        log(f"profile pass {rep}: flags {pipe.flags()}")
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("profile copies done (2^30 bytes read and written each)")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=64)
    ap.add_argument("--fit-tracks", type=int, default=1_000_000)
    ap.add_argument("--fit-tiles", type=int, default=8,
                    help="copies of the fit workload for the large-batch figure (1: skip)")
    ap.add_argument("--bins", type=int, default=0, help="azimuth bins per layer (0: autotuned)")
    ap.add_argument("--block-doublets", type=int, default=0, help="doublet kernel block size (0: autotuned)")
    ap.add_argument("--block-links", type=int, default=0, help="link sweep block size (0: autotuned)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-events", type=int, default=256,
                    help="events of the mixed-pileup batch also reported (0: skip)")
    ap.add_argument("--profile-fit", action="store_true",
                    help="only two eager passes of the fit workload (forward + adjoint) and two 1 GiB copies, for "
                         "profiler counter runs; prints no JSON")
    ap.add_argument("--profile-fishbone", action="store_true",
                    help="only two eager doublet passes with the Fishbone on the overlap-geometry PU200 batch, for "
                         "kernel traces; prints no JSON")
    ap.add_argument("--profile-workflows", action="store_true",
                    help="only two eager passes of each workflow (quadruplets, triplets) with ambiguity resolution "
                         "and vertices, for kernel traces; prints no JSON")
    ap.add_argument("--profile", action="store_true",
                    help="only two eager passes of the batched step (reconstruction + adjoint) and two 1 GiB "
                         "copies, for profiler counter runs; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); events shard across GPUs with no "
              "communication, so run one process per GPU.", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2008_13461_amd import _abi as A

    A.load()
    if args.profile:
        profile_run(args)
        return
    if args.profile_fit:
        profile_fit_run(args)
        return
    if args.profile_workflows:
        profile_workflows_run(args)
        return
    if args.profile_fishbone:
        profile_fishbone_run(args)
        return
    chain = chain_workload(args)
    fit = fit_workload(args)

    n_ev = chain["n_events"]
    value = n_ev / chain["t_batched"]
    per_event = n_ev / chain["t_per_event"]
    kern = chain["kernels_ms"]
    cnt = chain["counts"]
    dominant = max(kern, key=kern.get) if kern else None

    # fit roofline: algorithmic bytes per track (float hits): forward 19n+26, adjoint 31n+25
    nh = fit["nhits"]
    fwd_bytes = float((19 * nh + 26).sum())
    bwd_bytes = float((31 * nh + 25).sum())
    fit_ms = fit["fwd_ms"] + fit["bwd_ms"]
    fit_gbs = (fwd_bytes + bwd_bytes) / (fit_ms * 1e-3) / 1e9
    fit_counters = fit_counter_record()
    fit_obj = {
        "workload": f"{fit['n_tracks']} tracks (50% 4-hit, 30% 5-hit, 20% 6-hit), module offsets, f32 with f64 refit",
        "tracks_per_s": fit["n_tracks"] / fit["t_graph"],
        "ms_fwd_bwd_step": fit["t_graph"] * 1e3,
        "ms_fwd_bwd_step_eager": fit["t_step"] * 1e3,
        "region_ms": {"fit_fwd": fit["fwd_ms"], "fit_bwd": fit["bwd_ms"]},
        "roofline": {"bound": "hbm", "achieved": fit_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": fit_gbs / HBM_PEAK_GBS,
                     "traffic": fit_counters.get("traffic_bytes") if fit_counters else None,
                     "valu_issue_frac": fit_counters.get("valu_issue_frac") if fit_counters else None,
                     "bytes_per_track": (fwd_bytes + bwd_bytes) / fit["n_tracks"],
                     "note": "algorithmic bytes (19n+26 forward, 31n+25 adjoint per track of n float hits) over "
                             "the timing regions of every fit and adjoint kernel; traffic and the VALU issue "
                             "fraction from the committed rocprofv3 counters of the same kernels, when they "
                             "match the current sources"},
        "asymptote": fit.get("asymptote"),
    }

    roof = roofline(kern, cnt)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chain["t_batched"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 predicates, f32 fit (f64 refit of stiff tracks)",
        "data": "synthetic",
        "config": {"workload": f"{n_ev} events at pileup 200 (200 vertices x Poisson(35) tracks, 15% noise), "
                               "full path with fit adjoint, one hipGraph per step",
                   "events": n_ev, "hits": cnt["hits"], "parallelism": "single GPU"},
        "per_event_events_per_s": per_event,
        "events_per_s_with_h2d": n_ev / chain["t_h2d"],
        "tuned": chain["perf"],
        "mixed_pileup": chain["mixed"],
        "batched_over_per_event": value / per_event,
        "tracks_per_s": cnt["tracks"] / chain["t_batched"],
        "counts_per_batch": cnt,
        "kernel_ms": kern,
        "kernel_ns_per_doublet": {k: v * 1e6 / cnt["doublets"] for k, v in kern.items()},
        "roofline": roof,
        "fit": fit_obj,
        "workflows": chain["workflows"],
        "fishbone": chain["fishbone"],
        "table2_per_event": chain["table2"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, chain)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
