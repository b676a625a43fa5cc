"""GPU parity of the two workflows of the paper's throughput measurements
(quadruplets, and triplets with the "outer triplets" of section 3.2) run
end to end -- n-tuplets, fit with covariance, ambiguity resolution (section
3.5) and pixel vertices (section 3.6) -- eagerly and as one batched plan."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import param_rel_err, tuplet_set

pytestmark = pytest.mark.gpu

CFG = C.default_config()
TRIPLETS = C.default_config(min_hits=3)


def _caps(h, cfg_d):
    """Capacities: the triplet workflow has many more rows (about 1.2 per hit
    at pileup 50, 18 at pileup 200)."""
    from tests.gpu_helpers import caps_for
    caps = caps_for(h.n_hits, h.n_events)
    if cfg_d["min_hits"] == 3:
        caps["tuplets_cap"] = 24 * max(h.n_hits, 64)
    return caps


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_triplet_workflow_equals_the_oracle():
    """min_hits = 3 on a PU50 event: raw and kept n-tuplets (3-hit paths from
    BPix1 roots and from BPix2 / FPix1 roots without an inner link) as sets,
    every fit (3-hit ones included) within 1e-4, and the selection of the
    ambiguity resolution (chi2 rule, then the |d0| rule among triplets)."""
    _need_gpu()
    from paper_2008_13461_amd import api
    from tests.gpu_helpers import products, run_chain  # noqa: F401
    h = E.config2()
    pipe, hits = run_chain(h, TRIPLETS, caps=_caps(h, TRIPLETS))
    assert pipe.flags() == 0
    prod = products(pipe)
    raw = O.reconstruct_event(TRIPLETS, h.x, h.y, h.z, h.layer, dedup=False)
    ded = O.ntuplets(TRIPLETS, h.layer, raw["cell_inner"], raw["cell_outer"], raw["link_in"], raw["link_out"])
    assert tuplet_set(prod["raw_hits"], prod["raw_n"]) == tuplet_set(raw["hits"], raw["n"])
    assert tuplet_set(prod["kept_hits"], prod["kept_n"]) == tuplet_set(ded["hits"], ded["n"])
    n3 = prod["kept_n"] == 3
    assert n3.sum() > 500
    # outer triplets: 3-hit rows whose first hit is not on BPix1
    assert np.any(h.layer[prod["kept_hits"][n3, 0]] != 0)
    params, chi2, st = O.fit(TRIPLETS, prod["kept_hits"], prod["kept_n"], h.x, h.y, h.z, h.layer)
    assert np.all(st == 0) and np.all(prod["fit_status"] & 5 == 0)
    assert param_rel_err(prod["params"], params).max() <= 1e-4
    sel, nsel = api.resolve_ambiguities(hits, pipe.cfg, pipe.cells, pipe.tuplets, pipe.precision, pipe.tracks,
                                        pipe.status, pipe.ws)
    torch.cuda.synchronize()
    nk = len(prod["kept_n"])
    rows = pipe.tuplets.kept[:nk].long()
    keep = O.ambiguity(prod["kept_hits"], pipe.tuplets.cells[rows].cpu().numpy(), prod["kept_n"], prod["chi2"],
                       prod["params"][:, 3])
    assert np.array_equal(sel[: int(nsel.item())].cpu().numpy(), np.nonzero(keep)[0])


def _plan_products(h, cfg_d, stages, reps=1, between=None):
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    caps = _caps(h, cfg_d)
    cfg = A.make_config(cfg_d)
    hits = api.Hits.from_host(h)
    cells = api.Cells.empty(caps["cells_cap"], h.n_hits)
    links = api.Links.empty(caps["links_cap"], caps["cells_cap"])
    tup = api.Tuplets.empty(caps["tuplets_cap"])
    tracks = api.Tracks.empty(caps["tuplets_cap"], A.PT_FIT_F32_F64SOLVE, with_cov=True)
    status = api.new_status()
    sel = torch.empty(caps["tuplets_cap"], dtype=torch.int32, device="cuda")
    nsel = torch.zeros(1, dtype=torch.int32, device="cuda")
    vtx = api.Vertices.empty(caps["tuplets_cap"], h.n_events, caps["tuplets_cap"])
    plan = api.Plan(cfg, precision=A.PT_FIT_F32_F64SOLVE, stages=stages, **caps)
    outs = []
    for _ in range(reps):
        plan.run(hits, cells, links, tup, tracks, status, selected=sel, n_selected=nsel, vertices=vtx)
        torch.cuda.synchronize()
        nv = int(vtx.count.item())
        outs.append(dict(
            kept=tup.kept_rows()[0].cpu().numpy(), params=tracks.params[: int(tup.count.item())].cpu().numpy(),
            cov=tracks.cov[: int(tup.count.item())].cpu().numpy(), sel=sel[: int(nsel.item())].cpu().numpy(),
            vz=vtx.z[:nv].cpu().numpy(), vn=vtx.n_tracks[:nv].cpu().numpy(), vfirst=vtx.event_first.cpu().numpy(),
            tv=vtx.track_vertex[: int(tup.count.item())].cpu().numpy(), flags=int(status[0].item())))
        if between is not None:      # eager work between the replays
            between()
            torch.cuda.synchronize()
    del plan
    return outs


@pytest.mark.parametrize("cfg_name", ["quadruplets", "triplets"])
def test_full_chain_plan_replays_equal_the_eager_calls(cfg_name):
    """The plan with the ambiguity and vertex stages, replayed three times
    with eager work in between: every replay gives the eager results bit for
    bit (selection, covariance, vertices and their members)."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    cfg_d = CFG if cfg_name == "quadruplets" else TRIPLETS
    h = E.config3(n_events=4)
    caps = _caps(h, cfg_d)
    pipe = api.Pipeline(cfg_d, **caps)
    pipe.tracks = api.Tracks.empty(caps["tuplets_cap"], pipe.precision, with_cov=True)
    hits = api.Hits.from_host(h)
    pipe.reconstruct(hits)
    sel, nsel = api.resolve_ambiguities(hits, pipe.cfg, pipe.cells, pipe.tuplets, pipe.precision, pipe.tracks,
                                        pipe.status, pipe.ws)
    vtx = api.Vertices.empty(caps["tuplets_cap"], h.n_events, caps["tuplets_cap"])
    api.find_vertices(hits, pipe.cfg, pipe.tuplets, pipe.precision, pipe.tracks, sel, nsel, vtx, pipe.status, pipe.ws)
    torch.cuda.synchronize()
    nk = int(pipe.tuplets.count.item())
    nv = int(vtx.count.item())
    ref = dict(kept=pipe.tuplets.kept_rows()[0].cpu().numpy(), params=pipe.tracks.params[:nk].cpu().numpy(),
               cov=pipe.tracks.cov[:nk].cpu().numpy(), sel=sel[: int(nsel.item())].cpu().numpy(),
               vz=vtx.z[:nv].cpu().numpy(), vn=vtx.n_tracks[:nv].cpu().numpy(), vfirst=vtx.event_first.cpu().numpy(),
               tv=vtx.track_vertex[:nk].cpu().numpy())
    assert nv > 10 and len(ref["sel"]) > 100
    outs = _plan_products(h, cfg_d, A.PT_STAGE_AMBIGUITY | A.PT_STAGE_VERTICES, reps=3,
                          between=lambda: pipe.reconstruct(hits))
    for rep, got in enumerate(outs):
        assert got["flags"] == 0
        for k in ref:
            assert np.array_equal(got[k], ref[k], equal_nan=True), (rep, k)
