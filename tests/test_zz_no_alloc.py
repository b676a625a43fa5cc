"""The allocation-free forward fit (pt_fit_broken_line_noalloc) against the
workspace entry point pt_fit_broken_line, through the C ABI: two calls in a
row, the second with fewer tracks, in both precisions; sizes beyond the
fixed scratch are refused on the host."""
import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import config as C
from synth import events as E

pytestmark = pytest.mark.gpu

CFG = C.default_config()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(ts, n):
    from paper_2008_13461_amd import api
    hits = api.Hits.from_host(ts.hits)
    tup = api.Tuplets.from_rows(torch.from_numpy(ts.tuplets[:n].copy()).cuda(),
                                torch.from_numpy(ts.nhits[:n].copy()).cuda())
    return hits, tup


def _outputs(tracks, status):
    torch.cuda.synchronize()
    return (tracks.params.cpu().numpy(), tracks.chi2.cpu().numpy(), tracks.status.cpu().numpy(),
            status.cpu().numpy())


@pytest.mark.parametrize("precision_name", ["PT_FIT_F32_F64SOLVE", "PT_FIT_F64"])
def test_noalloc_fit_equals_the_workspace_fit(precision_name):
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    precision = getattr(A, precision_name)
    dtype = np.float64 if precision == A.PT_FIT_F64 else np.float32
    ts = E.config4(n_tracks=150_000, dtype=dtype)
    off = torch.from_numpy(E.module_offsets()).cuda()
    cfg = A.make_config(CFG)
    for n in (150_000, 40_000):      # the second call with a smaller input
        hits, tup = _inputs(ts, n)
        ref_t = api.Tracks.empty(n, precision)
        ref_s = api.new_status()
        ws = api.new_workspace(api.workspace_size(cfg, hits.n_hits, 1, 0, 0, n))
        api.fit_broken_line(hits, cfg, tup, off, precision, ref_t, ref_s, ws)
        ref = _outputs(ref_t, ref_s)
        got_t = api.Tracks.empty(n, precision)
        got_s = api.new_status()
        api.fit_broken_line_noalloc(hits, cfg, tup, off, precision, got_t, got_s)
        got = _outputs(got_t, got_s)
        assert np.array_equal(got[0], ref[0], equal_nan=True), n
        assert np.array_equal(got[1], ref[1], equal_nan=True), n
        assert np.array_equal(got[2], ref[2]), n
        assert np.array_equal(got[3], ref[3]), n
        if precision != A.PT_FIT_F64:
            assert got[3][A.PT_ST_FIT_F64] > 0          # the refit list in the scratch was used


def test_noalloc_fit_refuses_more_tracks_than_its_scratch():
    _need_gpu()
    from paper_2008_13461_amd import _abi as A
    from paper_2008_13461_amd import api
    ts = E.config4(n_tracks=2000)
    hits = api.Hits.from_host(ts.hits)
    n = A.PT_NOALLOC_FIT_MAX_TRACKS + 1
    rows = torch.full((n, 8), -1, dtype=torch.int32, device="cuda")
    tup = api.Tuplets.from_rows(rows, torch.zeros(n, dtype=torch.uint8, device="cuda"))
    tracks = api.Tracks.empty(n, A.PT_FIT_F32_F64SOLVE)
    status = api.new_status()
    cfg = A.make_config(CFG)
    err = A.load().pt_fit_broken_line_noalloc(ct.byref(hits.abi()), ct.byref(cfg), ct.byref(tup.abi()), None,
                                              A.PT_FIT_F32_F64SOLVE, ct.byref(tracks.abi()), api._p(status),
                                              api._stream())
    assert err == A.PT_ERR_TOO_LARGE
