"""Pins of the oracle's fit covariance (paper section 3.4: parameters and
covariance matrices from the circle and line fits, combined).

* the covariance is the Jacobian sandwich of the two normal matrices'
  inverses, recomputed with numpy;
* pulls (fitted - generated) / sigma of a population of tracks simulated
  with scattering are standard normal;
* the sample covariance of many simulations of one track equals the
  predicted covariance;
* exact symmetries (rotation about z, z and y mirrors) act on it as on the
  parameters.
"""
from collections import Counter

import numpy as np
import pytest

import oracle as O
from synth import config as C
from synth import events as E

CFG = C.default_config()
DIAG = [0, 5, 9, 12, 14]


def _ms_tracks(seed, trk_or_n, pt="loguniform", eta_max=2.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    trk = E.draw_tracks(rng, trk_or_n, pt=pt, eta_max=eta_max) if np.isscalar(trk_or_n) else trk_or_n
    n = trk["kappa"].shape[0]
    ti, li, x, y, z = E.track_hits_ms(rng, trk, scatter_first=False)
    nh = np.bincount(ti, minlength=n)
    starts = np.concatenate([[0], np.cumsum(nh)])
    sel = np.nonzero(nh >= 4)[0]
    tup = np.full((len(sel), 8), -1, np.int32)
    for j, t in enumerate(sel):
        tup[j, : nh[t]] = np.arange(starts[t], starts[t] + nh[t])
    truth = np.stack([trk[k][sel] for k in ("kappa", "phi0", "cot", "d0", "z0")], 1)
    return tup, nh[sel].astype(np.uint8), x, y, z, li, truth


def _corr_err(a, b):
    """|a - b| relative to sqrt(b_ii b_jj), for [.., 5, 5] matrices."""
    d = np.sqrt(np.abs(np.einsum("...ii->...i", b)))
    return np.abs(a - b) / (d[..., :, None] * d[..., None, :])


def test_covariance_is_the_jacobian_sandwich_of_the_inverses():
    tup, n, x, y, z, li, _ = _ms_tracks(41, 200)
    worst = 0.0
    for t in range(0, len(n), 5):
        hs = tup[t, : n[t]]
        d = O.fit_debug(CFG, x[hs], y[hs], z[hs], li[hs])
        jc, jl, cov = O.fit_cov_debug(CFG, x[hs], y[hs], z[hs], li[hs])
        want = jc @ np.linalg.inv(d["A"]) @ jc.T + jl @ np.linalg.inv(d["N"]) @ jl.T
        worst = max(worst, _corr_err(cov, want).max())
        assert np.allclose(cov, cov.T, rtol=0, atol=0)
        assert np.all(np.linalg.eigvalsh(cov) > 0)
    assert worst < 1e-6, worst


@pytest.mark.parametrize("pt", ["loguniform", "power"])
def test_pulls_are_standard_normal(pt):
    tup, n, x, y, z, li, truth = _ms_tracks(42 if pt == "power" else 43, 12000, pt=pt)
    p, _, st = O.fit(CFG, tup, n, x, y, z, li)
    cov = O.fit_cov(CFG, tup, n, x, y, z, li)
    assert np.all(st == 0) and np.all(np.isfinite(cov))
    d = p - truth
    d[:, 1] = (d[:, 1] + np.pi) % (2 * np.pi) - np.pi
    pull = d / np.sqrt(cov[:, DIAG])
    assert np.all(np.abs(pull.mean(axis=0)) < 0.04), pull.mean(axis=0)
    assert np.all(np.abs(pull.std(axis=0) - 1.0) < 0.07), pull.std(axis=0)


@pytest.mark.parametrize("pt,eta", [(1.0, 0.3), (3.0, 1.9), (0.6, -1.2)])
def test_sample_covariance_of_one_track(pt, eta):
    """4000 simulations of one track (same perigee, independent scattering
    and smearing): the covariance of the fitted parameters equals the
    predicted one (diagonal within 10%, correlations within 0.06)."""
    rng = np.random.Generator(np.random.PCG64(44))
    one = E.draw_tracks(rng, 1, pt="loguniform")
    q = 1.0
    kappa = -q * C.K_CURV * 3.8 / pt
    phi_v, vz = 0.4, 1.0
    cot = np.sinh(eta)
    phi0, d0, z0, s_v = E.perigee_from_vertex(np.zeros(1), np.zeros(1), np.full(1, vz), np.full(1, phi_v),
                                              np.full(1, kappa), np.full(1, cot))
    trk = dict(one, kappa=np.full(1, kappa), cot=np.full(1, cot), phi0=phi0, d0=d0, z0=z0, s_v=s_v,
               pt=np.full(1, pt), vx=np.zeros(1), vy=np.zeros(1), vz=np.full(1, vz))
    reps = {k: np.repeat(v, 4000) for k, v in trk.items()}
    tup, n, x, y, z, li, truth = _ms_tracks(45, reps)
    # keep the realisations with the most common layer sequence
    seqs = [tuple(li[tup[t, : n[t]]].tolist()) for t in range(len(n))]
    common = Counter(seqs).most_common(1)[0][0]
    keep = np.array([s == common for s in seqs])
    assert keep.sum() > 3000
    p, _, st = O.fit(CFG, tup[keep], n[keep], x, y, z, li)
    cov = O.fit_cov(CFG, tup[keep], n[keep], x, y, z, li)
    d = p - truth[keep]
    d[:, 1] = (d[:, 1] + np.pi) % (2 * np.pi) - np.pi
    sample = np.cov(d.T)
    pred = O.cov_full(cov).mean(axis=0)
    ratio = np.diag(sample) / np.diag(pred)
    assert np.all(np.abs(ratio - 1.0) < 0.1), ratio
    cs = sample / np.sqrt(np.outer(np.diag(sample), np.diag(sample)))
    cp = pred / np.sqrt(np.outer(np.diag(pred), np.diag(pred)))
    assert np.abs(cs - cp).max() < 0.06, (cs, cp)


def test_covariance_symmetries():
    tup, n, x, y, z, li, _ = _ms_tracks(46, 300)
    base = O.cov_full(O.fit_cov(CFG, tup, n, x, y, z, li))
    a = 0.731
    ca, sa = np.cos(a), np.sin(a)
    rot = O.cov_full(O.fit_cov(CFG, tup, n, ca * x - sa * y, sa * x + ca * y, z, li))
    assert _corr_err(rot, base).max() < 1e-9
    # z mirror (disk layers swap sides): cot and z0 change sign
    swap = np.array([0, 1, 2, 3, 7, 8, 9, 4, 5, 6], np.uint8)
    zm = O.cov_full(O.fit_cov(CFG, tup, n, x, y, -z, swap[li]))
    s = np.array([1, 1, -1, 1, -1])
    assert _corr_err(zm, base * np.outer(s, s)).max() < 1e-9
    # y mirror: kappa, phi0 and d0 change sign
    ym = O.cov_full(O.fit_cov(CFG, tup, n, x, -y, z, li))
    s = np.array([-1, -1, 1, -1, 1])
    assert _corr_err(ym, base * np.outer(s, s)).max() < 1e-9
