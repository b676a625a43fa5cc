"""Pins of the oracle's pixel vertices (paper section 3.6): hand-built sets of
tracks whose densities, links, trees, vertex fits, splits and ordering are
worked out here from the definition, a shift of every z0, and the truth
vertices of a simulated event."""
import numpy as np

import oracle as O
from synth import config as C
from synth import events as E

CFG = C.default_config()
K = 0.299792458 * CFG["bfield"] / 100.0


def _kappa(pt):
    return np.full(len(pt), K) / np.asarray(pt, float)


def _run(z, sig, pt=None, n=None, use=None, **over):
    cfg = dict(CFG, **over)
    z = np.asarray(z, float)
    pt = np.full(len(z), 2.0) if pt is None else np.asarray(pt, float)
    n = np.full(len(z), 4) if n is None else np.asarray(n)
    return O.vertices(cfg, z, np.asarray(sig, float) ** 2 * np.ones(len(z)), _kappa(pt), n, use)


def _fit(z, var):
    w = 1.0 / var
    zv = np.sum(w * z) / np.sum(w)
    return zv, 1.0 / np.sum(w), np.sum((z - zv) ** 2 / var)


def test_two_clusters_and_the_isolated_tracks():
    z = np.array([1.000, 1.004, 0.998, 1.002, 1.001,     # cluster A (5 tracks)
                  -2.000, -2.003, -1.998,                  # cluster B (3 tracks)
                  5.0,                                     # isolated
                  3.00, 3.004])                            # a pair: densities 1, no seed
    sig = np.full(len(z), 0.004)
    pt = np.array([1, 1, 1, 1, 1, 5, 5, 5, 9, 9, 9], float)
    v = _run(z, sig, pt)
    assert len(v["z"]) == 2
    # B has the larger sum of p_T^2: 3 x 25 > 5 x 1
    assert np.array_equal(v["n_tracks"], [3, 5])
    for k, sel in ((0, slice(5, 8)), (1, slice(0, 5))):
        zv, var, chi2 = _fit(z[sel], sig[sel] ** 2)
        assert abs(v["z"][k] - zv) < 1e-12 and abs(v["var"][k] - var) < 1e-18
        assert abs(v["chi2"][k] - chi2) < 1e-9 and v["ndf"][k] == (sel.stop - sel.start) - 1
    assert np.isclose(v["sum_pt2"], [75.0, 5.0]).all()
    assert np.array_equal(v["track_vertex"], [1, 1, 1, 1, 1, 0, 0, 0, -1, -1, -1])


def test_selection_of_the_tracks():
    z = np.array([0.0, 0.001, 0.002, 0.003, 0.004])
    sig = np.full(5, 0.004)
    # a 3-hit track, a soft track, an unused track and a non-finite z0 take no part
    v = _run(z, sig, pt=[2, 2, 0.4, 2, 2], n=[4, 3, 4, 4, 4], use=[1, 1, 1, 1, 0])
    assert len(v["z"]) == 0      # two tracks left: densities 1, no seed
    v = _run(z, sig, pt=[2, 2, 2, 2, 2], n=[4, 4, 4, 4, 4], use=[1, 1, 1, 1, 0])
    assert np.array_equal(v["track_vertex"], [0, 0, 0, 0, -1])
    z2 = z.copy()
    z2[0] = np.nan
    v = _run(z2, sig)
    assert v["track_vertex"][0] == -1 and v["n_tracks"][0] == 4


def test_density_needs_chi2_compatibility_and_small_errors():
    # 4 tracks within dz_cut but pairwise incompatible in chi2: no links, no seed
    z = np.array([0.0, 0.05, 0.10, 0.15]) * 0.4
    v = _run(z, np.full(4, 0.002))
    assert len(v["z"]) == 0
    # the same positions with large errors: compatible, but a density is
    # computed only for sigma(z0) <= err_max, so no seed either
    v = _run(z, np.full(4, 0.2))
    assert len(v["z"]) == 0
    # with err_max raised the four form one vertex
    v = _run(z, np.full(4, 0.2), vtx_err_max=1.0)
    assert np.array_equal(v["track_vertex"], [0, 0, 0, 0])


def test_links_follow_the_nearest_higher_density_track():
    # a dense core and a chain of tracks hanging off it, each within reach
    # of the next only: the chain joins the core's vertex through its links
    core = [0.0, 0.001, -0.001, 0.0005]
    chain = [0.012, 0.024, 0.036]
    z = np.array(core + chain)
    v = _run(z, np.full(len(z), 0.005))
    assert np.array_equal(v["track_vertex"], [0] * 7)


def test_vertex_with_large_chi2_is_split_by_two_means():
    # two groups 0.03 apart bridged by two tracks: one tree, chi2/ndf > 9
    g1 = [0.000, 0.0004, -0.0004, 0.0002]
    g2 = [0.030, 0.0304, 0.0296, 0.0302]
    bridge = [0.010, 0.020]
    z = np.array(g1 + bridge + g2)
    sig = np.full(len(z), 0.004)
    v_unsplit = _run(z, sig, vtx_split_chi2_ndf=1e9)
    assert len(v_unsplit["z"]) == 1
    assert v_unsplit["chi2"][0] / v_unsplit["ndf"][0] > 9
    v = _run(z, sig)
    assert len(v["z"]) == 2
    # two-means from the extreme members, written out
    zs = np.sort(z)
    c1, c2 = zs[0], zs[-1]
    for _ in range(10):
        side = np.abs(zs - c1) > np.abs(zs - c2)
        c1, c2 = zs[~side].mean(), zs[side].mean()
    assert sorted(v["n_tracks"].tolist()) == sorted([int((~side).sum()), int(side.sum())])
    assert np.allclose(np.sort(v["z"]), [c1, c2], atol=1e-12)
    tv = v["track_vertex"]
    assert len(set(tv[:4])) == 1 and len(set(tv[6:])) == 1 and tv[0] != tv[6]


def test_a_shift_of_every_z0_shifts_the_vertices():
    rng = np.random.Generator(np.random.PCG64(61))
    vz = rng.normal(0, 1.0, 30)
    z = np.repeat(vz, 8) + rng.normal(0, 0.004, 240)
    sig = rng.uniform(0.003, 0.006, 240)
    pt = rng.uniform(0.6, 5, 240)
    a = _run(z, sig, pt)
    b = _run(z + 0.5, sig, pt)
    assert np.array_equal(a["track_vertex"], b["track_vertex"])
    assert np.allclose(b["z"] - a["z"], 0.5, atol=1e-12)
    assert np.allclose(a["chi2"], b["chi2"], rtol=1e-9, atol=1e-9)


def test_truth_vertices_of_a_simulated_event():
    """Genuine tracks of a PU50 event, fitted: most truth vertices with at
    least 6 used tracks have a vertex within 3 sigma (a sanity check of the
    reading, not parity)."""
    h = E.config2()
    r = O.reconstruct_event(CFG, h.x, h.y, h.z, h.layer)
    p, c2, st = O.fit(CFG, r["hits"], r["n"], h.x, h.y, h.z, h.layer)
    cov = O.fit_cov(CFG, r["hits"], r["n"], h.x, h.y, h.z, h.layer)
    tid = h.track[r["hits"][:, :4]]
    genuine = np.all(tid == tid[:, :1], axis=1) & (tid[:, 0] >= 0)
    v = O.vertices(CFG, p[:, 4], cov[:, 14], p[:, 0], r["n"], genuine)
    vz_true = h.truth[0]["vz"]
    used = genuine & (K / np.abs(p[:, 0]) > CFG["vtx_pt_min"])
    counts = {}
    for t in np.nonzero(used)[0]:
        counts[vz_true[tid[t, 0]]] = counts.get(vz_true[tid[t, 0]], 0) + 1
    big = [z for z, c in counts.items() if c >= 6]
    assert len(big) >= 20
    found = [np.any(np.abs(v["z"] - z) < 3 * np.sqrt(v["var"]) + 0.003) for z in big]
    assert np.mean(found) > 0.8, np.mean(found)
    # the primary vertex is the one with the largest sum of p_T^2
    assert np.all(np.diff(v["sum_pt2"]) <= 0)
