"""Helpers of the GPU parity tests: run the HIP library on synthetic events and
bring the products back as numpy arrays."""
import numpy as np
import torch

from paper_2008_13461_amd import _abi as A
from paper_2008_13461_amd import api


def caps_for(n_hits, n_events, cells_per_hit=160, links_frac=0.25):
    cells = max(1024, cells_per_hit * n_hits)
    return dict(n_hits=n_hits, n_events=max(n_events, 1), cells_cap=cells,
                links_cap=max(1024, int(links_frac * cells)), tuplets_cap=max(1024, n_hits))


def run_chain(h, cfg, precision=A.PT_FIT_F32_F64SOLVE, offsets=None, caps=None, **perf):
    """Doublets -> links -> n-tuplets -> fit on the GPU; returns (pipeline, hits)."""
    caps = caps or caps_for(h.n_hits, h.n_events)
    pipe = api.Pipeline(cfg, precision=precision, **caps, **perf)
    hits = api.Hits.from_host(h)
    off = torch.from_numpy(offsets).cuda() if offsets is not None else None
    pipe.reconstruct(hits, offsets=off)
    torch.cuda.synchronize()
    return pipe, hits


def products(pipe):
    """numpy copies of every product of the chain."""
    ci, co, cp = (t.cpu().numpy() for t in pipe.cells.valid())
    li, lo = (t.cpu().numpy() for t in pipe.links.valid())
    rh, rn = (t.cpu().numpy() for t in pipe.tuplets.raw())
    kh, kn = (t.cpu().numpy() for t in pipe.tuplets.kept_rows())
    nk = kn.shape[0]
    params = pipe.tracks.params[:nk].cpu().numpy().astype(np.float64)
    chi2 = pipe.tracks.chi2[:nk].cpu().numpy().astype(np.float64)
    st = pipe.tracks.status[:nk].cpu().numpy()
    return dict(cell_inner=ci, cell_outer=co, cell_pair=cp, link_in=li, link_out=lo, raw_hits=rh, raw_n=rn,
                kept_hits=kh, kept_n=kn, params=params, chi2=chi2, fit_status=st)


def event_slice(h, e):
    a, b = int(h.event_offsets[e]), int(h.event_offsets[e + 1])
    return a, b
