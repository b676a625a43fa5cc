"""GPU parity of the fit paths the pileup workloads rarely reach: tracks of
3, 7 and 8 hits (their own kernel instantiations), the single-precision fit
without the double refit, and the search truncated at max_hits."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import param_rel_err, tuplet_set

pytestmark = pytest.mark.gpu

CFG = C.default_config()
RADII = [2.9, 4.4, 6.8, 8.6, 10.9, 13.2, 16.0, 18.2]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _fit(ts, precision, offsets=None, g=None):
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    cfg = A.make_config(CFG)
    h = ts.hits
    hits = api.Hits.from_host(h)
    n = ts.nhits.shape[0]
    tup = api.Tuplets.from_rows(torch.from_numpy(ts.tuplets).cuda(), torch.from_numpy(ts.nhits).cuda())
    tracks = api.Tracks.empty(n, precision)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, 1, 0, 0, n))
    off = torch.from_numpy(offsets).cuda() if offsets is not None else None
    api.fit_broken_line(hits, cfg, tup, off, precision, tracks, status, ws)
    out = dict(params=tracks.params.cpu().numpy().astype(np.float64),
               chi2=tracks.chi2.cpu().numpy().astype(np.float64), status=tracks.status.cpu().numpy())
    if g is not None:
        gdt = torch.float64 if precision == A.PT_FIT_F64 else torch.float32
        gh = torch.zeros((h.n_hits, 3), dtype=gdt, device="cuda")
        go = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")
        api.fit_broken_line_bwd(hits, cfg, tup, off, precision, torch.from_numpy(g[0]).cuda().to(gdt),
                                torch.from_numpy(g[1]).cuda().to(gdt), gh, go, status, ws)
        out["grad_hits"] = gh.cpu().numpy().astype(np.float64)
        out["grad_offsets"] = go.cpu().numpy()
    torch.cuda.synchronize()
    out["flags"] = status.cpu().numpy()
    return out


@pytest.mark.parametrize("n", [3, 7, 8])
@pytest.mark.parametrize("precision_name,tol,gtol", [("PT_FIT_F64", 1e-9, 1e-8),
                                                     ("PT_FIT_F32_F64SOLVE", 1e-4, 1e-3)])
def test_fit_and_adjoint_of_n_hit_tracks(n, precision_name, tol, gtol):
    """k_fit<3,3>, k_fit<7,8>, k_grad<3,3>, k_grad<7,8> against the oracle
    on tracks through n cylinders (module offsets on)."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    precision = getattr(A, precision_name)
    dtype = np.float64 if precision == A.PT_FIT_F64 else np.float32
    ts = E.cylinder_tracks(9 + n, 3000, RADII[:n], dtype=dtype)
    off = E.module_offsets()
    g = E.cotangents(n, len(ts.nhits))
    h = ts.hits
    ref, chi2, st = O.fit(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off)
    assert np.all(st == 0)
    got = _fit(ts, precision, off, g)
    assert np.all(got["status"] & 5 == 0)
    err = param_rel_err(got["params"], ref)
    assert err.max() <= tol, err.max(axis=0)
    cerr = np.abs(got["chi2"] - chi2) / np.maximum(np.abs(chi2), 1.0)
    assert cerr.max() <= (tol if precision == A.PT_FIT_F64 else 1e-3), cerr.max()
    gh_ref, go_ref = O.fit_grad(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off, g[0], g[1])
    rows = ts.tuplets[:, :n]
    num = np.linalg.norm(got["grad_hits"][rows] - gh_ref[rows], axis=(1, 2))
    den = np.linalg.norm(gh_ref[rows], axis=(1, 2))
    assert np.all(num <= gtol * den), (num / den).max()
    assert np.abs(got["grad_offsets"] - go_ref).max() <= gtol * np.abs(go_ref).max()


def test_f32_fit_without_the_double_refit():
    """PT_FIT_F32: no track goes to the double refit; every track the mixed
    mode leaves in single precision gets bit-identical parameters in both
    modes and agrees with the oracle within 1e-4; the tracks the mixed mode
    refits (the stiff ones) are fitted in float here."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    ts = E.config4(n_tracks=200_000)
    off = E.module_offsets()
    h = ts.hits
    ref, _, st = O.fit(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off)
    assert np.all(st == 0)
    mixed = _fit(ts, A.PT_FIT_F32_F64SOLVE, off)
    plain = _fit(ts, A.PT_FIT_F32, off)
    assert plain["flags"][A.PT_ST_FIT_F64] == 0
    assert np.all(plain["status"] & A.PT_FIT_ST_F64_SOLVE == 0)
    stiff = (mixed["status"] & A.PT_FIT_ST_F64_SOLVE) != 0
    assert 0 < stiff.sum() < 0.01 * len(stiff)
    assert np.array_equal(plain["params"][~stiff], mixed["params"][~stiff])
    assert np.array_equal(plain["chi2"][~stiff], mixed["chi2"][~stiff])
    err = param_rel_err(plain["params"][~stiff], ref[~stiff])
    assert err.max() <= 1e-4, err.max(axis=0)
    ok = (plain["status"][stiff] & 5) == 0
    stiff_err = param_rel_err(plain["params"][stiff][ok], ref[stiff][ok])
    print(f"stiff tracks fitted in float: {int(stiff.sum())}, failed {int((~ok).sum())}, "
          f"max rel err per parameter {stiff_err.max(axis=0)}")
    assert np.all(np.isfinite(plain["params"][stiff][ok]))


def test_search_truncated_at_max_hits():
    """A five-hit forward helix searched with max_hits = 4: 4-hit rows, the
    truncation counted and flagged, the same rows as the oracle."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from tests.gpu_helpers import caps_for, products, run_chain
    from tests.test_oracle_ntuplets import _forward_helix_hits
    x, y, z, layer = _forward_helix_hits()
    cfg = C.default_config(max_hits=4)
    h = E.Hits(x, y, z, layer, E.module_id(layer, x, y, z), np.zeros(5, np.int32), np.array([0, 5], np.int32))
    pipe, _ = run_chain(h, cfg, precision=A.PT_FIT_F64, caps=caps_for(5, 1))
    prod = products(pipe)
    ci, co, _ = O.doublets(cfg, x, y, z, layer)
    li, lo = O.links(cfg, x, y, z, layer, ci, co)
    raw = O.ntuplets(cfg, layer, ci, co, li, lo, dedup=False)
    assert raw["truncated"]
    assert tuplet_set(prod["raw_hits"], prod["raw_n"]) == tuplet_set(raw["hits"], raw["n"])
    assert set(prod["raw_n"].tolist()) == {4}
    assert pipe.flags() & A.PT_FLAG_TRUNCATED
    assert int(pipe.status[A.PT_ST_TRUNCATED].item()) >= 1
    kept = O.ntuplets(cfg, layer, ci, co, li, lo, dedup=True)
    assert tuplet_set(prod["kept_hits"], prod["kept_n"]) == tuplet_set(kept["hits"], kept["n"])
