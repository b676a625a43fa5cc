"""GPU edge cases: empty inputs, empty events, invalid hits, capacity
overflow, input permutation, and graph replays of the batched plan."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import doublet_set, tuplet_set

pytestmark = pytest.mark.gpu

CFG = C.default_config()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(h, caps=None, **kw):
    from tests.gpu_helpers import products, run_chain
    pipe, hits = run_chain(h, CFG, caps=caps, **kw)
    return pipe, products(pipe)


def test_empty_input():
    _need_gpu()
    e = np.zeros(0, np.float32)
    h = E.Hits(e, e, e, np.zeros(0, np.uint8), np.zeros(0, np.int16), np.zeros(0, np.int32),
               np.array([0], np.int32))
    from tests.gpu_helpers import caps_for
    pipe, prod = _run(h, caps=caps_for(0, 0))
    assert len(prod["cell_inner"]) == 0 and len(prod["kept_n"]) == 0 and pipe.flags() == 0


def test_empty_events_between_events():
    _need_gpu()
    ev = E.config3(n_events=2)
    a = int(ev.event_offsets[1])
    off = np.array([0, 0, a, a, ev.n_hits, ev.n_hits], np.int32)
    h = E.Hits(ev.x, ev.y, ev.z, ev.layer, ev.module, ev.track, off)
    _, got = _run(h)
    _, ref = _run(ev)
    assert doublet_set(got["cell_inner"], got["cell_outer"]) == doublet_set(ref["cell_inner"], ref["cell_outer"])
    assert tuplet_set(got["kept_hits"], got["kept_n"]) == tuplet_set(ref["kept_hits"], ref["kept_n"])


def test_invalid_hits_are_skipped_and_counted():
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    h = E.config2()
    x, y, z, layer = h.x.copy(), h.y.copy(), h.z.copy(), h.layer.copy()
    rng = np.random.default_rng(5)
    bad_nan = rng.choice(h.n_hits, 30, replace=False)
    x[bad_nan[:10]] = np.nan
    z[bad_nan[10:20]] = np.inf
    layer[bad_nan[20:]] = 12
    hb = E.Hits(x, y, z, layer, h.module, h.track, h.event_offsets)
    pipe, got = _run(hb)
    assert pipe.flags() & A.PT_FLAG_BAD_HITS
    assert int(pipe.status[A.PT_ST_BAD_HITS].item()) == 30
    good = np.setdiff1d(np.arange(h.n_hits), bad_nan)
    ref = O.reconstruct_event(CFG, h.x[good], h.y[good], h.z[good], h.layer[good])
    want = doublet_set(good[ref["cell_inner"]], good[ref["cell_outer"]])
    assert doublet_set(got["cell_inner"], got["cell_outer"]) == want
    want_t = {tuple(good[list(t)].tolist()) for t in tuplet_set(ref["hits"], ref["n"])}
    assert tuplet_set(got["kept_hits"], got["kept_n"]) == want_t


@pytest.mark.parametrize("which", ["cells", "links", "tuplets"])
def test_capacity_overflow_is_flagged(which):
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from tests.gpu_helpers import caps_for
    h = E.config2()
    full_pipe, full = _run(h)
    n_cells = len(full["cell_inner"])
    n_links = len(full["link_in"])
    n_raw = len(full["raw_n"])
    caps = caps_for(h.n_hits, 1)
    if which == "cells":
        caps["cells_cap"] = n_cells // 2
        flag = A.PT_FLAG_CELLS_OVERFLOW
    elif which == "links":
        caps["links_cap"] = n_links // 2
        flag = A.PT_FLAG_LINKS_OVERFLOW
    else:
        caps["tuplets_cap"] = n_raw // 2
        flag = A.PT_FLAG_TUPLETS_OVERFLOW
    pipe, got = _run(h, caps=caps)
    assert pipe.flags() & flag
    if which == "cells":
        assert int(pipe.cells.count.item()) == n_cells      # the size needed is reported
    if which == "links":
        assert int(pipe.links.count.item()) == n_links
    if which == "tuplets":
        assert int(pipe.tuplets.count_raw.item()) == n_raw
        # rows come out in root order: the rows that fit are the first rows
        # of the full run (the root whose rows straddle the capacity included)
        cap = caps["tuplets_cap"]
        assert np.array_equal(got["raw_hits"], full["raw_hits"][:cap])
        assert np.array_equal(got["raw_n"], full["raw_n"][:cap])


def test_permuted_hits_give_the_same_sets():
    _need_gpu()
    h = E.config2()
    perm = np.random.default_rng(11).permutation(h.n_hits)
    hp = E.Hits(h.x[perm], h.y[perm], h.z[perm], h.layer[perm], h.module[perm], h.track[perm], h.event_offsets)
    _, a = _run(h)
    _, b = _run(hp)
    # map permuted indices back to the original ones
    d_b = {(int(perm[i]), int(perm[o])) for i, o in zip(b["cell_inner"], b["cell_outer"])}
    assert d_b == doublet_set(a["cell_inner"], a["cell_outer"])
    t_b = {tuple(perm[list(t)].tolist()) for t in tuplet_set(b["kept_hits"], b["kept_n"])}
    assert t_b == tuplet_set(a["kept_hits"], a["kept_n"])


def test_plan_graph_replays_match_eager():
    """Several replays of the captured step (module offsets, the adjoint with
    hit and module gradients), with eager work in between, each checked
    against the eager calls: the same rows in the same order, the same
    parameters bit for bit, gradients equal up to the order of the atomic
    additions."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from tests.gpu_helpers import caps_for
    h = E.config3(n_events=4)
    caps = caps_for(h.n_hits, h.n_events)
    cfg = A.make_config(CFG)
    hits = api.Hits.from_host(h)
    off = torch.from_numpy(E.module_offsets()).cuda()
    # rows come out in the same order on every run, so each row has its own
    # cotangent
    g_np, c_np = E.cotangents(3, caps["tuplets_cap"])
    gp = torch.from_numpy(g_np).cuda()
    gc = torch.from_numpy(c_np).cuda()
    # eager reference
    pipe = api.Pipeline(CFG, **caps)
    pipe.reconstruct(hits, offsets=off)
    gh_ref = torch.zeros((h.n_hits, 3), dtype=torch.float32, device="cuda")
    go_ref = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")
    pipe.backward(hits, gp, gc, gh_ref, go_ref, offsets=off)
    torch.cuda.synchronize()
    nk = int(pipe.tuplets.count.item())
    ref_rows, ref_n = (t.cpu().numpy() for t in pipe.tuplets.kept_rows())
    ref_p = pipe.tracks.params[:nk].cpu().numpy()
    ref_c = pipe.tracks.chi2[:nk].cpu().numpy()
    plan = api.Plan(cfg, precision=A.PT_FIT_F32_F64SOLVE, with_adjoint=True, **caps)
    cells = api.Cells.empty(caps["cells_cap"], h.n_hits)
    links = api.Links.empty(caps["links_cap"], caps["cells_cap"])
    tup = api.Tuplets.empty(caps["tuplets_cap"])
    tracks = api.Tracks.empty(caps["tuplets_cap"], A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    gh = torch.zeros((h.n_hits, 3), dtype=torch.float32, device="cuda")
    go = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")
    for rep in range(4):
        gh.zero_()
        go.zero_()
        plan.run(hits, cells, links, tup, tracks, status, offsets=off, g_params=gp, g_chi2=gc, grad_hits=gh,
                 grad_offsets=go)
        torch.cuda.synchronize()
        got_rows, got_n = (t.cpu().numpy() for t in tup.kept_rows())
        assert np.array_equal(got_rows, ref_rows) and np.array_equal(got_n, ref_n), rep
        assert np.array_equal(tracks.params[:nk].cpu().numpy(), ref_p, equal_nan=True), rep
        assert np.array_equal(tracks.chi2[:nk].cpu().numpy(), ref_c, equal_nan=True), rep
        # hit gradients: float sums in another order
        assert (torch.linalg.norm(gh - gh_ref) / torch.linalg.norm(gh_ref)).item() <= 1e-5, rep
        # module gradients: double sums in another order
        assert (torch.abs(go - go_ref).max() / torch.abs(go_ref).max()).item() <= 1e-12, rep
        # eager work between replays
        pipe.reconstruct(hits, offsets=off)
        torch.cuda.synchronize()


def _link_layout_ok(pipe):
    """Every cell's links are one run [out_start, out_start + out_count) whose
    entries start on that cell, sorted by out-cell, and the runs follow the
    cell order; has_inner marks exactly the cells some link ends on."""
    li, lo = (t.cpu().numpy() for t in pipe.links.valid())
    n_cells = min(int(pipe.cells.count.item()), pipe.cells.cap)
    start = pipe.links.out_start[:n_cells].cpu().numpy()
    cnt = pipe.links.out_count[:n_cells].cpu().numpy()
    has = pipe.links.has_inner[:n_cells].cpu().numpy()
    assert int(cnt.sum()) == len(li)
    assert np.all(np.diff(li) >= 0)
    assert np.array_equal(start[1:], (start + cnt)[:-1])
    for c in np.nonzero(cnt)[0]:
        run = slice(start[c], start[c] + cnt[c])
        assert np.all(li[run] == c)
        assert np.all(np.diff(lo[run]) > 0)
    want = np.zeros(n_cells, bool)
    want[lo] = True
    assert np.array_equal(has.astype(bool), want)


@pytest.mark.parametrize("block", [64, 128, 256])
def test_link_block_sizes_and_layout(block):
    """The link sweep with 1, 2 and 4 wavefronts per block: same links as the
    oracle, one sorted run per in-cell."""
    _need_gpu()
    from tests.gpu_helpers import products
    h = E.config2()
    pipe, got = _run(h, block_links=block)
    ref = O.reconstruct_event(CFG, h.x, h.y, h.z, h.layer)
    from tests.helpers import link_set
    assert link_set(got["cell_inner"], got["cell_outer"], got["link_in"], got["link_out"]) == \
        link_set(ref["cell_inner"], ref["cell_outer"], ref["link_in"], ref["link_out"])
    _link_layout_ok(pipe)


def _fan_event(n_out=20):
    """One cell (BPix1 -> BPix2) followed by n_out compatible cells on BPix3:
    hits on a nearly straight radial line, spread by a few micrometres in
    azimuth, so that the in-cell has more links than the sweep keeps in LDS."""
    R = np.array([C.BARREL_R[0], C.BARREL_R[1]] + [C.BARREL_R[2]] * n_out)
    phi = np.array([0.3, 0.3] + [0.3 + 2e-5 * (k - n_out / 2) for k in range(n_out)])
    cot = 0.2
    z = np.array([R[0] * cot, R[1] * cot] + [R[2] * cot + 1e-4 * k for k in range(n_out)])
    x = (R * np.cos(phi)).astype(np.float32)
    y = (R * np.sin(phi)).astype(np.float32)
    layer = np.array([0, 1] + [2] * n_out, np.uint8)
    n = len(x)
    return E.Hits(x, y, z.astype(np.float32), layer, np.zeros(n, np.int16), np.arange(n, dtype=np.int32),
                  np.array([0, n], np.int32))


def test_inner_cell_with_many_links_takes_the_overflow_path():
    _need_gpu()
    from tests.helpers import link_set
    h = _fan_event(20)
    ref = O.reconstruct_event(CFG, h.x, h.y, h.z, h.layer)
    rl = link_set(ref["cell_inner"], ref["cell_outer"], ref["link_in"], ref["link_out"])
    fan = [l for l in rl if l[0] == 0 and l[1] == 1]
    assert len(fan) == 20      # the oracle links the first cell to every outer cell
    pipe, got = _run(h)
    assert link_set(got["cell_inner"], got["cell_outer"], got["link_in"], got["link_out"]) == rl
    _link_layout_ok(pipe)
    assert tuplet_set(got["kept_hits"], got["kept_n"]) == tuplet_set(ref["hits"], ref["n"])


def test_autotuned_settings_give_the_same_products():
    """The autotuner only picks performance settings: the tuned run produces
    the same doublets, links and kept n-tuplets as the defaults."""
    _need_gpu()
    from paper_2008_13461_amd import api, autotune
    from tests.gpu_helpers import caps_for
    from tests.helpers import link_set
    h = E.config2()
    caps = caps_for(h.n_hits, h.n_events)
    hits = api.Hits.from_host(h)
    perf = autotune.tune(CFG, hits, caps, repeats=1, cache=None)
    assert set(perf) == set(autotune.CANDIDATES)
    for name, v in perf.items():
        assert v in autotune.CANDIDATES[name]
    _, a = _run(h)
    _, b = _run(h, **perf)
    assert doublet_set(a["cell_inner"], a["cell_outer"]) == doublet_set(b["cell_inner"], b["cell_outer"])
    assert link_set(a["cell_inner"], a["cell_outer"], a["link_in"], a["link_out"]) == \
        link_set(b["cell_inner"], b["cell_outer"], b["link_in"], b["link_out"])
    assert tuplet_set(a["kept_hits"], a["kept_n"]) == tuplet_set(b["kept_hits"], b["kept_n"])


def _cone_event(n0=200, n1=5000, n2=5, seed=9):
    """A narrow cone with n0 hits on BPix1, n1 on BPix2 and n2 on BPix3:
    every BPix1-BPix2 pair is a doublet (~n0 n1 cells), so each block of
    4096 consecutive cells holds the cells of about one BPix1 hit and every
    BPix2 hit collects its n0 in-cells from about n0 different blocks -- more
    index segments than the sweep handles in one window."""
    rng = np.random.default_rng(seed)
    cot = 0.5
    rows = []
    for lay, n, dphi, dz in ((0, n0, 0.002, 0.05), (1, n1, 0.003, 0.1), (2, n2, 0.003, 0.1)):
        R = C.BARREL_R[lay]
        phi = 0.3 + rng.uniform(-dphi, dphi, n)
        z = R * cot + rng.uniform(-dz, dz, n)
        rows.append((R * np.cos(phi), R * np.sin(phi), z, np.full(n, lay, np.uint8)))
    x, y, z, layer = (np.concatenate(v) for v in zip(*rows))
    perm = rng.permutation(len(x))
    n = len(x)
    return E.Hits(x[perm].astype(np.float32), y[perm].astype(np.float32), z[perm].astype(np.float32), layer[perm],
                  np.zeros(n, np.int16), np.arange(n, dtype=np.int32), np.array([0, n], np.int32))


def test_hits_with_in_cells_from_many_blocks():
    _need_gpu()
    from tests.helpers import link_set
    h = _cone_event()
    ref = O.reconstruct_event(CFG, h.x, h.y, h.z, h.layer)
    assert len(ref["cell_inner"]) > 900_000 and len(ref["link_in"]) > 0
    caps = dict(n_hits=h.n_hits, n_events=1, cells_cap=1_200_000, links_cap=2_000_000, tuplets_cap=4096)
    pipe, got = _run(h, caps=caps)
    assert pipe.flags() == 0
    assert doublet_set(got["cell_inner"], got["cell_outer"]) == doublet_set(ref["cell_inner"], ref["cell_outer"])
    assert link_set(got["cell_inner"], got["cell_outer"], got["link_in"], got["link_out"]) == \
        link_set(ref["cell_inner"], ref["cell_outer"], ref["link_in"], ref["link_out"])
    _link_layout_ok(pipe)


def _doublets_and_links(h, cfg_d, cells_cap, links_cap):
    """pt_build_doublets and pt_link_cells alone; (cells inner, outer, links in, out) on the host."""
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    cfg = A.make_config(cfg_d)
    hits = api.Hits.from_host(h)
    cells = api.Cells.empty(cells_cap, h.n_hits)
    links = api.Links.empty(links_cap, cells_cap)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, h.n_events, cells_cap, links_cap, 1024))
    api.build_doublets(hits, cfg, cells, status, ws)
    api.link_cells(hits, cfg, cells, links, status, ws)
    torch.cuda.synchronize()
    assert int(status[0].item()) == 0  # no overflow
    ci, co, _ = (t.cpu().numpy() for t in cells.valid())
    li, lo = (t.cpu().numpy() for t in links.valid())
    return ci, co, li, lo


def _star_event(n_in, n_out, seed=3):
    """One BPix2 hit with n_in inner hits on BPix1 and n_out outer hits on
    BPix3, all at one azimuth (every triplet passes the beam-spot test), the
    R-Z directions of the segments spread over the whole half turn, with many
    close to the beam axis, where the direction keys wrap round."""
    rng = np.random.default_rng(seed)
    half = np.pi / 2
    a_in = np.concatenate([rng.uniform(-half + 2e-3, half - 2e-3, n_in - 8),
                           half - rng.uniform(1e-4, 3e-2, 4), -half + rng.uniform(1e-4, 3e-2, 4)])
    a_out = np.concatenate([rng.uniform(-half + 2e-3, half - 2e-3, n_out - 8),
                            half - rng.uniform(1e-4, 3e-2, 4), -half + rng.uniform(1e-4, 3e-2, 4)])
    R0, R1, R2 = C.BARREL_R[:3]
    R = np.concatenate([np.full(n_in, R0), [R1], np.full(n_out, R2)])
    z = np.concatenate([-(R1 - R0) * np.tan(a_in), [0.0], (R2 - R1) * np.tan(a_out)])
    phi = 0.3 + rng.uniform(-1e-7, 1e-7, len(R))
    layer = np.concatenate([np.zeros(n_in), [1], np.full(n_out, 2)]).astype(np.uint8)
    n = len(R)
    return E.Hits((R * np.cos(phi)).astype(np.float32), (R * np.sin(phi)).astype(np.float32), z.astype(np.float32),
                  layer, np.zeros(n, np.int16), np.arange(n, dtype=np.int32), np.array([0, n], np.int32))


@pytest.mark.parametrize("n_out", [120, 300])
def test_links_of_segments_in_every_direction(n_out):
    """The link search bins a hit's out-cells by R-Z direction and tests each
    in-cell against its own and the neighbouring bins only (up to 256
    out-cells; beyond, every pair): with directions over the whole half turn,
    near-vertical ones included, the links equal the oracle's."""
    _need_gpu()
    from tests.helpers import link_set
    cfg_d = C.default_config(cut_mask=C.CUT_PHIW)
    h = _star_event(150, n_out)
    ci, co, li, lo = _doublets_and_links(h, cfg_d, 1 << 16, 1 << 16)
    rci, rco, _ = O.doublets(cfg_d, h.x, h.y, h.z, h.layer)
    rli, rlo = O.links(cfg_d, h.x, h.y, h.z, h.layer, rci, rco)
    assert doublet_set(ci, co) == doublet_set(rci, rco)
    ref = link_set(rci, rco, rli, rlo)
    assert len(ref) > 100
    assert link_set(ci, co, li, lo) == ref


@pytest.mark.parametrize("theta", [0.05, 0.3, 0.6])
def test_links_with_wide_theta_cuts(theta):
    """Wider R-Z cuts make fewer, wider direction bins (none from 0.5 on,
    where every pair is tested): the links equal the oracle's."""
    _need_gpu()
    from tests.helpers import link_set
    cfg_d = C.default_config(ca_theta_barrel=theta, ca_theta_endcap=theta)
    h = E.config2()
    rci, rco, _ = O.doublets(cfg_d, h.x, h.y, h.z, h.layer)
    rli, rlo = O.links(cfg_d, h.x, h.y, h.z, h.layer, rci, rco)
    ci, co, li, lo = _doublets_and_links(h, cfg_d, 2 * len(rci) + 1024, 2 * len(rli) + 1024)
    assert link_set(ci, co, li, lo) == link_set(rci, rco, rli, rlo)
