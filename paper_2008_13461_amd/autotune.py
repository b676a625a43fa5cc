"""Autotuner of the performance settings of the reconstruction.

The settings tuned here never change a result: the number of azimuth bins
per layer of the doublet search (the search is widened by one bin, so any
count gives the same doublets) and the block sizes of the doublet and link
kernels.  For a given batch the tuner times doublets + links + n-tuplets for
each candidate with HIP events on the current stream and keeps the fastest;
results are cached in a JSON file keyed by device, HIP version, configuration
and batch size class.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import _abi as A
from . import api

CANDIDATES = {
    "n_phi_bins": (64, 128, 256, 512),
    "block_doublets": (64, 128, 256, 512),
    "block_links": (64, 128, 256),
}
DEFAULT = {"n_phi_bins": 128, "block_doublets": 256, "block_links": 64}
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pixeltrack_autotune.json")


def _key(cfg_dict: dict, n_hits: int, n_events: int) -> str:
    dev = torch.cuda.get_device_name()
    cfg_hash = hashlib.sha1(json.dumps(cfg_dict, sort_keys=True).encode()).hexdigest()[:12]
    size_class = f"{1 << max(0, (n_hits - 1).bit_length())}h/{n_events}e"
    return f"{dev}|hip{torch.version.hip}|{cfg_hash}|{size_class}"


def _time_chain(cfg_dict, hits, caps, settings, repeats):
    pipe = api.Pipeline(cfg_dict, **caps, **settings)
    # warm-up (also checks capacities)
    api.build_doublets(hits, pipe.cfg, pipe.cells, pipe.status, pipe.ws)
    api.link_cells(hits, pipe.cfg, pipe.cells, pipe.links, pipe.status, pipe.ws)
    api.find_ntuplets(hits, pipe.cfg, pipe.cells, pipe.links, pipe.tuplets, pipe.status, pipe.ws)
    torch.cuda.synchronize()
    if pipe.flags() & (A.PT_FLAG_CELLS_OVERFLOW | A.PT_FLAG_LINKS_OVERFLOW | A.PT_FLAG_TUPLETS_OVERFLOW):
        raise RuntimeError("capacity overflow while tuning")
    times = []
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        api.build_doublets(hits, pipe.cfg, pipe.cells, pipe.status, pipe.ws)
        api.link_cells(hits, pipe.cfg, pipe.cells, pipe.links, pipe.status, pipe.ws)
        api.find_ntuplets(hits, pipe.cfg, pipe.cells, pipe.links, pipe.tuplets, pipe.status, pipe.ws)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    del pipe
    torch.cuda.empty_cache()
    times.sort()
    return times[len(times) // 2]


def tune(cfg_dict: dict, hits: "api.Hits", caps: dict, *, repeats: int = 3, cache: str | None = CACHE,
         verbose: bool = False) -> dict:
    """Best settings for this batch; coordinate descent over CANDIDATES."""
    key = _key(cfg_dict, hits.n_hits, hits.n_events)
    table = {}
    if cache and os.path.exists(cache):
        try:
            table = json.load(open(cache))
        except (OSError, ValueError):
            table = {}
        if key in table:
            return dict(table[key]["settings"])
    best = dict(DEFAULT)
    best_ms = _time_chain(cfg_dict, hits, caps, best, repeats)
    trials = [(dict(best), best_ms)]
    for name, values in CANDIDATES.items():
        for v in values:
            if v == best[name]:
                continue
            trial = dict(best, **{name: v})
            ms = _time_chain(cfg_dict, hits, caps, trial, repeats)
            trials.append((trial, ms))
            if verbose:
                print(f"[autotune] {trial} {ms:.3f} ms", flush=True)
            if ms < best_ms:
                best, best_ms = trial, ms
    if cache:
        table[key] = {"settings": best, "ms": best_ms, "trials": [{"settings": s, "ms": m} for s, m in trials]}
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1)
        os.replace(tmp, cache)
    return best
