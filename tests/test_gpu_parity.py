"""GPU parity: the HIP library against the CPU oracle.

Integer products (doublets, links, n-tuplets before and after duplicate
removal) must be identical as sets; fits must agree within 1e-9 relative in
double precision and 1e-4 relative in single precision (with the floors of
tests/helpers.py for quantities that cross zero), chi2 within 1e-9 (double)
and 1e-3 (single) of max(chi2, 1).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import doublet_set, link_set, param_rel_err, tuplet_set

pytestmark = pytest.mark.gpu

CFG = C.default_config()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _compare_event(prod, h, e, cfg=CFG, fit_tol=None, precision_f64=False):
    """Compare the GPU products of event e with the oracle on that event."""
    from tests.gpu_helpers import event_slice
    a, b = event_slice(h, e)
    sub = h.event(e)
    ref = O.reconstruct_event(cfg, sub.x, sub.y, sub.z, sub.layer, dedup=False)
    ded = O.ntuplets(cfg, sub.layer, ref["cell_inner"], ref["cell_outer"], ref["link_in"], ref["link_out"])
    ci, co = prod["cell_inner"], prod["cell_outer"]
    sel = (ci >= a) & (ci < b)
    got_d = doublet_set(ci[sel] - a, co[sel] - a)
    assert got_d == doublet_set(ref["cell_inner"], ref["cell_outer"]), f"doublets differ in event {e}"
    li, lo = prod["link_in"], prod["link_out"]
    lsel = (ci[li] >= a) & (ci[li] < b)
    got_l = link_set(ci - a, co - a, li[lsel], lo[lsel])
    assert got_l == link_set(ref["cell_inner"], ref["cell_outer"], ref["link_in"], ref["link_out"]), \
        f"links differ in event {e}"
    rh, rn = prod["raw_hits"], prod["raw_n"]
    rsel = (rh[:, 0] >= a) & (rh[:, 0] < b)
    rows = rh[rsel].copy()
    rows[rows >= 0] -= a
    assert tuplet_set(rows, rn[rsel]) == tuplet_set(ref["hits"], ref["n"]), f"raw n-tuplets differ in event {e}"
    kh, kn = prod["kept_hits"], prod["kept_n"]
    ksel = (kh[:, 0] >= a) & (kh[:, 0] < b)
    krows = kh[ksel].copy()
    krows[krows >= 0] -= a
    assert tuplet_set(krows, kn[ksel]) == tuplet_set(ded["hits"], ded["n"]), f"kept n-tuplets differ in event {e}"
    if fit_tol is not None:
        params, chi2, st = O.fit(cfg, kh[ksel], kn[ksel], h.x, h.y, h.z, h.layer, h.module)
        assert np.all(st == 0)
        assert np.all(prod["fit_status"][ksel] & 5 == 0)
        err = param_rel_err(prod["params"][ksel], params)
        assert err.max() <= fit_tol, (err.max(axis=0), e)
        cerr = np.abs(prod["chi2"][ksel] - chi2) / np.maximum(np.abs(chi2), 1.0)
        # chi2 of the single-precision fit: within 1e-3 of max(chi2, 1)
        assert cerr.max() <= (fit_tol if precision_f64 else 1e-3)
    return len(got_d), len(got_l), int(ksel.sum())


def test_library_loads_and_abi():
    from paper_2008_13461_amd import _abi as A
    L = A.load()
    assert L.pt_abi_version() == A.PT_ABI_VERSION


def test_config1_f64_chain():
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from tests.gpu_helpers import products, run_chain
    h = E.config1()
    pipe, _ = run_chain(h, CFG, precision=A.PT_FIT_F64)
    prod = products(pipe)
    nd, nl, nk = _compare_event(prod, h, 0, fit_tol=1e-9, precision_f64=True)
    assert nk >= 10 and pipe.flags() == 0


def test_config2_f32_chain():
    _need_gpu()
    from tests.gpu_helpers import products, run_chain
    h = E.config2()
    pipe, _ = run_chain(h, CFG)
    prod = products(pipe)
    nd, nl, nk = _compare_event(prod, h, 0, fit_tol=1e-4)
    assert nd > 100000 and nk > 500
    assert pipe.flags() == 0


def test_config2_f64_fit():
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from tests.gpu_helpers import products, run_chain
    h = E.config2()
    pipe, _ = run_chain(h, CFG, precision=A.PT_FIT_F64)
    prod = products(pipe)
    _compare_event(prod, h, 0, fit_tol=1e-9, precision_f64=True)


@pytest.mark.parametrize("bins", [16, 512])
def test_bin_count_does_not_change_results(bins):
    _need_gpu()
    from tests.gpu_helpers import products, run_chain
    h = E.config2()
    base = products(run_chain(h, CFG)[0])
    other = products(run_chain(h, CFG, n_phi_bins=bins)[0])
    assert doublet_set(base["cell_inner"], base["cell_outer"]) == doublet_set(other["cell_inner"], other["cell_outer"])
    assert tuplet_set(base["kept_hits"], base["kept_n"]) == tuplet_set(other["kept_hits"], other["kept_n"])


def test_batched_pu200_sampled_events():
    """64 events at pileup 200 in one batch; two sampled events against the oracle."""
    _need_gpu()
    from tests.gpu_helpers import products, run_chain
    h = E.config5()
    pipe, _ = run_chain(h, CFG)
    assert pipe.flags() == 0
    prod = products(pipe)
    for e in (0, 37):
        _compare_event(prod, h, e, fit_tol=1e-4)


def test_batched_equals_per_event():
    _need_gpu()
    from tests.gpu_helpers import products, run_chain
    h = E.config3(n_events=6)
    full = products(run_chain(h, CFG)[0])
    for e in range(h.n_events):
        a, b = int(h.event_offsets[e]), int(h.event_offsets[e + 1])
        one = products(run_chain(h.event(e), CFG)[0])
        sel = (full["kept_hits"][:, 0] >= a) & (full["kept_hits"][:, 0] < b)
        rows = full["kept_hits"][sel].copy()
        rows[rows >= 0] -= a
        assert tuplet_set(rows, full["kept_n"][sel]) == tuplet_set(one["kept_hits"], one["kept_n"])
        ci = full["cell_inner"]
        s2 = (ci >= a) & (ci < b)
        assert doublet_set(ci[s2] - a, full["cell_outer"][s2] - a) == doublet_set(one["cell_inner"], one["cell_outer"])


def test_cut_set_without_zip():
    """Doublet cuts without ZIP (as in the loose cut sets of Table 2): cells may
    then run inwards (dr <= 0), which the link sweep must handle without its
    angle windows.  Same sets as the oracle."""
    _need_gpu()
    from tests.gpu_helpers import caps_for, products, run_chain
    cfg = C.default_config(cut_mask=C.CUT_PHIW | C.CUT_ZW | C.CUT_PT)
    h = E.config2()
    pipe, _ = run_chain(h, cfg, caps=caps_for(h.n_hits, 1, cells_per_hit=400, links_frac=0.5))
    assert pipe.flags() == 0
    prod = products(pipe)
    ci, co = prod["cell_inner"], prod["cell_outer"]
    ref = O.reconstruct_event(cfg, h.x, h.y, h.z, h.layer)
    assert doublet_set(ci, co) == doublet_set(ref["cell_inner"], ref["cell_outer"])
    assert link_set(ci, co, prod["link_in"], prod["link_out"]) == \
        link_set(ref["cell_inner"], ref["cell_outer"], ref["link_in"], ref["link_out"])
    assert tuplet_set(prod["kept_hits"], prod["kept_n"]) == tuplet_set(ref["hits"], ref["n"])


def test_cell_pairs_match_their_hits():
    """Each cell's layer pair has the layers of its two hits: the link step
    takes the barrel or end-cap class of an out-cell's outer hit, which
    selects its theta cut, from the pair's outer layer."""
    _need_gpu()
    from tests.gpu_helpers import run_chain
    h = E.config2()
    pipe, _ = run_chain(h, CFG)
    ci, co, cp = (t.cpu().numpy().astype(np.int64) for t in pipe.cells.valid())
    assert len(ci) > 0
    pairs = np.asarray(CFG["pairs"])
    assert np.array_equal(pairs[cp, 0], h.layer[ci])
    assert np.array_equal(pairs[cp, 1], h.layer[co])
    barrel = np.asarray(CFG["layer_barrel"], bool)
    assert barrel[h.layer[co]].any() and (~barrel[h.layer[co]]).any()  # both classes of outer hit
