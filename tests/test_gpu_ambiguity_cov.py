"""GPU parity of the fit covariance and of the ambiguity resolution (paper
sections 3.4 and 3.5) against the oracle.

Covariance: every element within 1e-9 (double fit) or 1e-3 (single) of the
oracle's, relative to sqrt(C_ii C_jj).  Ambiguity resolution: the oracle is
given the GPU's own chi2 and d0 values (the decision is taken in the fit's
precision on both sides), and the selected tracks must be identical.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from synth import config as C
from synth import events as E

pytestmark = pytest.mark.gpu

CFG = C.default_config()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cov_err(got15, ref15):
    g, r = O.cov_full(got15), O.cov_full(ref15)
    d = np.sqrt(np.abs(np.einsum("...ii->...i", r)))
    return np.abs(g - r) / (d[..., :, None] * d[..., None, :])


@pytest.mark.parametrize("precision_name,tol", [("PT_FIT_F64", 1e-9), ("PT_FIT_F32_F64SOLVE", 1e-3)])
def test_covariance_equals_the_oracle(precision_name, tol):
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    precision = getattr(A, precision_name)
    dtype = np.float64 if precision == A.PT_FIT_F64 else np.float32
    ts = E.config4(n_tracks=100_000, dtype=dtype)
    off_np = E.module_offsets()
    h = ts.hits
    cfg = A.make_config(CFG)
    hits = api.Hits.from_host(h)
    n = len(ts.nhits)
    tup = api.Tuplets.from_rows(torch.from_numpy(ts.tuplets).cuda(), torch.from_numpy(ts.nhits).cuda())
    tracks = api.Tracks.empty(n, precision, with_cov=True)
    status = api.new_status()
    ws = api.new_workspace(api.workspace_size(cfg, h.n_hits, 1, 0, 0, n))
    off = torch.from_numpy(off_np).cuda()
    api.fit_broken_line(hits, cfg, tup, off, precision, tracks, status, ws)
    plain = api.Tracks.empty(n, precision)
    api.fit_broken_line(hits, cfg, tup, off, precision, plain, status, ws)
    torch.cuda.synchronize()
    got = tracks.cov.cpu().numpy().astype(np.float64)
    ref = O.fit_cov(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off_np)
    assert np.all(np.isfinite(ref))
    err = _cov_err(got, ref)
    print(f"{precision_name}: covariance error / sqrt(Cii Cjj): worst {err.max():.2e}")
    assert err.max() <= tol
    # the covariance output does not change the parameters
    assert np.array_equal(tracks.params.cpu().numpy(), plain.params.cpu().numpy())


def _chain(h, cfg_d, min_hits=4):
    from tests.gpu_helpers import caps_for, run_chain
    cfg = dict(cfg_d, min_hits=min_hits)
    caps = caps_for(h.n_hits, h.n_events)
    if min_hits == 3:      # the triplet workflow has more rows than hits
        caps["tuplets_cap"] = 4 * max(h.n_hits, 256)
    pipe, hits = run_chain(h, cfg, caps=caps)
    assert pipe.flags() == 0
    return pipe, hits, cfg


def _resolve(pipe, hits):
    from paper_2008_13461_amd import api
    sel, n_sel = api.resolve_ambiguities(hits, pipe.cfg, pipe.cells, pipe.tuplets, pipe.precision, pipe.tracks,
                                         pipe.status, pipe.ws)
    torch.cuda.synchronize()
    return sel[: int(n_sel.item())].cpu().numpy()


def _oracle_keep(pipe):
    nk = int(pipe.tuplets.count.item())
    rows = pipe.tuplets.kept[:nk].long()
    hits = pipe.tuplets.hits[rows].cpu().numpy()
    cells = pipe.tuplets.cells[rows].cpu().numpy()
    n = pipe.tuplets.n[rows].cpu().numpy()
    chi2 = pipe.tracks.chi2[:nk].cpu().numpy().astype(np.float64)
    d0 = pipe.tracks.params[:nk, 3].cpu().numpy().astype(np.float64)
    return O.ambiguity(hits, cells, n, chi2, d0), n


@pytest.mark.parametrize("min_hits", [4, 3])
def test_ambiguity_resolution_equals_the_oracle(min_hits):
    """Quadruplet and triplet workflows on a PU50 event."""
    _need_gpu()
    pipe, hits, _ = _chain(E.config2(), CFG, min_hits=min_hits)
    got = _resolve(pipe, hits)
    keep, n = _oracle_keep(pipe)
    assert np.array_equal(got, np.nonzero(keep)[0])
    assert np.all(np.diff(got) > 0)               # listed in track order
    assert 0 < len(got) < len(keep)
    if min_hits == 3:
        assert (n[got] == 3).sum() > 100


def test_ambiguity_resolution_on_the_pileup_200_batch():
    _need_gpu()
    pipe, hits, _ = _chain(E.config5(n_events=8), CFG)
    got = _resolve(pipe, hits)
    keep, _ = _oracle_keep(pipe)
    assert np.array_equal(got, np.nonzero(keep)[0])


def test_ambiguity_resolution_of_an_empty_input():
    _need_gpu()
    from tests.gpu_helpers import caps_for, run_chain
    e = np.zeros(0, np.float32)
    h = E.Hits(e, e, e, np.zeros(0, np.uint8), np.zeros(0, np.int16), np.zeros(0, np.int32), np.array([0], np.int32))
    pipe, hits = run_chain(h, CFG, caps=caps_for(0, 0))
    assert len(_resolve(pipe, hits)) == 0
