"""GPU parity of the Fishbone (paper section 3.3) on the overlap geometry:
the doublets left after it, and everything built on them (links, n-tuplets,
fits), equal the oracle's doublets -> Fishbone -> links -> n-tuplets chain.
Integer products as sets, fits within 1e-4 as in the other parity tests."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import doublet_set

pytestmark = pytest.mark.gpu

FB = C.default_config(fishbone_theta=0.01)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inner_index_ok(pipe, n_hits):
    """The compacted cells stay grouped by inner hit, and (inner_first,
    inner_count) index exactly those groups."""
    ci = pipe.cells.valid()[0].cpu().numpy()
    first = pipe.cells.inner_first[:n_hits].cpu().numpy()
    cnt = pipe.cells.inner_count[:n_hits].cpu().numpy()
    assert int(cnt.sum()) == len(ci)
    for h in np.nonzero(cnt)[0]:
        assert np.all(ci[first[h]:first[h] + cnt[h]] == h)


def test_fishbone_on_an_overlap_event_equals_the_oracle():
    _need_gpu()
    from tests.gpu_helpers import products, run_chain
    from tests.test_gpu_parity import _compare_event
    h = E.overlap_event()
    pipe, _ = run_chain(h, FB)
    assert pipe.flags() == 0
    prod = products(pipe)
    nd, nl, nk = _compare_event(prod, h, 0, cfg=FB, fit_tol=1e-4)
    _inner_index_ok(pipe, h.n_hits)
    # the Fishbone removed something: fewer doublets than without it
    off, _ = run_chain(h, C.default_config())
    n_off = int(off.cells.count.item())
    assert nd < n_off
    print(f"overlap event: {n_off} doublets -> {nd} after the Fishbone, {nl} links, {nk} n-tuplets")


def test_fishbone_on_an_overlap_batch_equals_the_oracle():
    """Eight PU50 events in one launch, each compared with the oracle."""
    _need_gpu()
    from tests.gpu_helpers import products, run_chain
    from tests.test_gpu_parity import _compare_event
    h = E.overlap_batch(n_events=8)
    pipe, _ = run_chain(h, FB)
    assert pipe.flags() == 0
    prod = products(pipe)
    for e in range(h.n_events):
        _compare_event(prod, h, e, cfg=FB, fit_tol=1e-4)
    _inner_index_ok(pipe, h.n_hits)


@pytest.mark.parametrize("theta", [0.002, 0.05])
def test_fishbone_angles_equal_the_oracle(theta):
    """Other angles: the kept doublets as a set."""
    _need_gpu()
    from tests.gpu_helpers import run_chain
    cfg = C.default_config(fishbone_theta=theta)
    h = E.overlap_event(seed=16, n_vertices=20)
    pipe, _ = run_chain(h, cfg)
    ci, co, _ = (t.cpu().numpy() for t in pipe.cells.valid())
    ri, ro, _ = O.doublets(cfg, h.x, h.y, h.z, h.layer)
    keep = O.fishbone(cfg, h.x, h.y, h.z, ri, ro)
    assert 0 < (~keep).sum() < len(keep)
    assert doublet_set(ci, co) == doublet_set(ri[keep], ro[keep])


def test_fishbone_skipped_when_the_cells_overflow():
    """With too small a cell capacity the overflow flag is set and the stored
    cells are left as the doublet search wrote them (no Fishbone)."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    h = E.overlap_event(seed=16, n_vertices=20)
    hits = api.Hits.from_host(h)
    out = {}
    for name, cfg_d in (("on", FB), ("off", C.default_config())):
        cfg = A.make_config(cfg_d)
        cells = api.Cells.empty(4096, h.n_hits)
        status = api.new_status()
        ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, h.n_events, 4096, 0, 0))
        api.build_doublets(hits, cfg, cells, status, ws)
        torch.cuda.synchronize()
        assert int(status[0].item()) & A.PT_FLAG_CELLS_OVERFLOW
        out[name] = (int(cells.count.item()), cells.inner.cpu().numpy(), cells.outer.cpu().numpy())
    assert out["on"][0] == out["off"][0] > 4096
    assert np.array_equal(out["on"][1], out["off"][1]) and np.array_equal(out["on"][2], out["off"][2])


def test_fishbone_in_a_plan_replays_equal_the_eager_chain():
    """The Fishbone inside a captured plan: three replays give the eager
    cells and kept n-tuplets."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    from tests.gpu_helpers import caps_for, run_chain
    h = E.overlap_batch(n_events=4)
    ref, _ = run_chain(h, FB)
    ref_cells = [t.cpu().numpy() for t in ref.cells.valid()]
    ref_kept = [t.cpu().numpy() for t in ref.tuplets.kept_rows()]
    caps = caps_for(h.n_hits, h.n_events)
    cfg = A.make_config(FB)
    hits = api.Hits.from_host(h)
    cells = api.Cells.empty(caps["cells_cap"], h.n_hits)
    links = api.Links.empty(caps["links_cap"], caps["cells_cap"])
    tup = api.Tuplets.empty(caps["tuplets_cap"])
    tracks = api.Tracks.empty(caps["tuplets_cap"], A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    plan = api.Plan(cfg, precision=A.PT_FIT_F32_F64SOLVE, **caps)
    for rep in range(3):
        plan.run(hits, cells, links, tup, tracks, status)
        torch.cuda.synchronize()
        assert int(status[0].item()) == 0
        got_cells = [t.cpu().numpy() for t in cells.valid()]
        got_kept = [t.cpu().numpy() for t in tup.kept_rows()]
        for a, b in zip(got_cells + got_kept, ref_cells + ref_kept):
            assert np.array_equal(a, b), rep
        ref.reconstruct(hits)           # eager work between the replays
        torch.cuda.synchronize()
    del plan


def test_fishbone_of_outer_hits_with_many_cells():
    """BPix2 hits reached from 3600, 600 and 200 BPix1 hits (pairs 1 µm apart
    in z, and neighbours within the cut angle): more cells than a work-group
    stages (all pairs from global memory), more than a wavefront stages (one
    work-group for the hit) and fewer (one wavefront); against the oracle."""
    _need_gpu()
    from tests.gpu_helpers import run_chain
    rng = np.random.default_rng(7)
    xs, ys, zs, ls = [], [], [], []
    for phi_o, npair in ((0.0, 300), (1.0, 100), (2.0, 1800)):
        xs.append(6.8 * np.cos(phi_o))
        ys.append(6.8 * np.sin(phi_o))
        zs.append(0.3)
        ls.append(1)
        for _ in range(npair):
            z, dphi = rng.uniform(-4, 4), rng.uniform(-0.005, 0.005)
            for dz in (0.0, 1e-4):
                xs.append(2.9 * np.cos(phi_o + dphi))
                ys.append(2.9 * np.sin(phi_o + dphi))
                zs.append(z + dz)
                ls.append(0)
    n = len(xs)
    h = E.Hits(np.array(xs, np.float32), np.array(ys, np.float32), np.array(zs, np.float32),
               np.array(ls, np.uint8), np.zeros(n, np.int16), np.full(n, -1, np.int32),
               np.array([0, n], np.int32))
    ri, ro, _ = O.doublets(FB, h.x, h.y, h.z, h.layer)
    per_hit = np.bincount(ro)
    assert per_hit.max() > 3072 and np.any((per_hit > 512) & (per_hit <= 3072))
    keep = O.fishbone(FB, h.x, h.y, h.z, ri, ro)
    assert 0 < keep.sum() < len(keep) // 2
    pipe, _ = run_chain(h, FB)
    ci, co, _ = (t.cpu().numpy() for t in pipe.cells.valid())
    assert doublet_set(ci, co) == doublet_set(ri[keep], ro[keep])
    _inner_index_ok(pipe, h.n_hits)
