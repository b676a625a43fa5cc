"""GPU parity of the broken-line fit and its adjoint on fit-only workloads
(hits stored in track order, 4/5/6-hit tracks, module offsets)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import param_rel_err

pytestmark = pytest.mark.gpu

CFG = C.default_config()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run_fit(ts, precision, offsets, with_grad=False, g=None, cfg_d=CFG):
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    cfg = A.make_config(cfg_d)
    h = ts.hits
    hits = api.Hits.from_host(h)
    n = ts.nhits.shape[0]
    tup = api.Tuplets.from_rows(torch.from_numpy(ts.tuplets).cuda(), torch.from_numpy(ts.nhits).cuda())
    tracks = api.Tracks.empty(n, precision)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, 1, 0, 0, n))
    off = torch.from_numpy(offsets).cuda() if offsets is not None else None
    api.fit_broken_line(hits, cfg, tup, off, precision, tracks, status, ws)
    out = dict(params=tracks.params.cpu().numpy().astype(np.float64), chi2=tracks.chi2.cpu().numpy().astype(np.float64),
               status=tracks.status.cpu().numpy(), flags=status.cpu().numpy())
    if with_grad:
        gdt = torch.float64 if precision == A.PT_FIT_F64 else torch.float32
        gp = torch.from_numpy(g[0]).cuda().to(gdt)
        gc = torch.from_numpy(g[1]).cuda().to(gdt)
        gh = torch.zeros((h.n_hits, 3), dtype=gdt, device="cuda")
        go = torch.zeros((C.N_MODULES, 3), dtype=torch.float64, device="cuda")
        api.fit_broken_line_bwd(hits, cfg, tup, off, precision, gp, gc, gh, go, status, ws)
        out["grad_hits"] = gh.cpu().numpy().astype(np.float64)
        out["grad_offsets"] = go.cpu().numpy()
    torch.cuda.synchronize()
    return out


@pytest.fixture(scope="module")
def tracks200k():
    return E.config4(n_tracks=200_000), E.module_offsets()


def test_fit_f32_with_f64_fallback(tracks200k):
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    ts, off = tracks200k
    h = ts.hits
    ref, chi2, st = O.fit(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off)
    assert np.all(st == 0)
    got = _run_fit(ts, A.PT_FIT_F32_F64SOLVE, off)
    assert np.all(got["status"] & 5 == 0)
    err = param_rel_err(got["params"], ref)
    assert err.max() <= 1e-4, err.max(axis=0)
    n_f64 = int(np.sum(got["status"] & 2 != 0))
    assert 0 < n_f64 < 0.01 * len(ts.nhits)
    assert got["flags"][A.PT_ST_FIT_F64] == n_f64


def test_fit_f64(tracks200k):
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    ts, off = tracks200k
    h = ts.hits
    sub = slice(0, 50_000)
    ref, chi2, st = O.fit(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off)
    got = _run_fit(ts, A.PT_FIT_F64, off)
    err = param_rel_err(got["params"][sub], ref[sub])
    assert err.max() <= 1e-9, err.max(axis=0)
    cerr = np.abs(got["chi2"][sub] - chi2[sub]) / np.maximum(np.abs(chi2[sub]), 1.0)
    assert cerr.max() <= 1e-9


@pytest.mark.parametrize("precision_name,tol", [("PT_FIT_F64", 1e-8), ("PT_FIT_F32_F64SOLVE", 1e-3)])
def test_adjoint_against_dual_numbers(precision_name, tol):
    """Hit and module gradients against the oracle's forward-mode gradient."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    precision = getattr(A, precision_name)
    ts = E.config4(n_tracks=3000)
    off = E.module_offsets()
    g = E.cotangents(4, len(ts.nhits))
    h = ts.hits
    got = _run_fit(ts, precision, off, with_grad=True, g=g)
    gh_ref, go_ref = O.fit_grad(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off, g[0], g[1])
    # per track, norm-wise over its hits (hits are not shared between tracks here)
    worst = 0.0
    for t in range(len(ts.nhits)):
        hs = ts.tuplets[t, : ts.nhits[t]]
        r = gh_ref[hs]
        e = np.linalg.norm(got["grad_hits"][hs] - r) / max(np.linalg.norm(r), 1e-30)
        worst = max(worst, e)
    assert worst <= tol
    scale = np.abs(go_ref).max()
    assert np.abs(got["grad_offsets"] - go_ref).max() <= tol * scale


@pytest.mark.parametrize("precision_name", ["PT_FIT_F64", "PT_FIT_F32_F64SOLVE"])
def test_adjoint_with_exclusive_hits_equals_the_atomic_one(tracks200k, precision_name):
    """exclusive_hits = 1 (plain additions into grad_hits, for tracks that
    share no hit, as here) gives the atomic additions' gradients bit for bit."""
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    precision = getattr(A, precision_name)
    ts, off = tracks200k
    g = E.cotangents(4, len(ts.nhits))
    a = _run_fit(ts, precision, off, with_grad=True, g=g)
    b = _run_fit(ts, precision, off, with_grad=True, g=g, cfg_d=C.default_config(exclusive_hits=1))
    assert np.array_equal(a["grad_hits"], b["grad_hits"])
    assert np.array_equal(a["params"], b["params"])
    assert np.allclose(a["grad_offsets"], b["grad_offsets"], rtol=1e-12, atol=1e-12 * np.abs(a["grad_offsets"]).max())


def test_bad_and_short_tracks():
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    ts = E.config4(n_tracks=200)
    tup = ts.tuplets.copy()
    nh = ts.nhits.copy()
    tup[0, [1, 2]] = tup[0, [2, 1]]   # out of order
    nh[1] = 2                         # too short to fit
    ts2 = E.TrackSet(ts.hits, tup, nh, ts.params)
    got = _run_fit(ts2, A.PT_FIT_F32_F64SOLVE, None)
    assert got["status"][0] & A.PT_FIT_ST_BAD_ORDER
    assert got["status"][1] & A.PT_FIT_ST_FAILED
    assert np.all(np.isnan(got["params"][:2]))
    assert np.all(got["status"][2:] & 5 == 0)
    assert got["flags"][A.PT_ST_FIT_BAD_ORDER] == 1 and got["flags"][A.PT_ST_FIT_FAILED] == 1
