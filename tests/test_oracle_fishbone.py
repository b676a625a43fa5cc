"""Pins of the oracle's Fishbone (paper section 3.3): among the doublets that
share their outer hit, the longer of two aligned ones is dropped.  A hand
built track through overlapping modules, a brute force written with numpy
from the definition, and its effect on an event of the overlap geometry
(duplicates removed, genuine tracks kept)."""
import numpy as np

import oracle as O
from synth import config as C
from synth import events as E

FB = C.default_config(fishbone_theta=0.01)


def test_hand_built_track_through_overlapping_modules():
    # a straight line from the origin: P0 (BPix1), P1a and P1b (BPix2 and its
    # overlapping ladder), P2 (BPix3), and a hit P3 off the line on BPix3
    d = np.array([0.6, 0.8, 0.3])
    r = np.array([2.9, 6.8, 7.15, 10.9])
    P = np.stack([d * (ri / 1.0) for ri in r])
    P3 = P[3] + np.array([0.5, -0.4, 0.0])
    x, y, z = (np.append(P[:, i], P3[i]) for i in range(3))
    #            (P0,P1a) (P0,P1b) (P1a,P2) (P1b,P2) (P0,P2) (P1b,P3)
    ci = np.array([0, 0, 1, 2, 0, 2])
    co = np.array([1, 2, 3, 3, 3, 4])
    keep = O.fishbone(FB, x, y, z, ci, co)
    # sharing P2: (P1a,P2), (P1b,P2), (P0,P2) are aligned; only the shortest stays
    assert keep.tolist() == [True, True, False, True, False, True]
    # a non-aligned pair sharing an outer hit keeps both
    assert O.fishbone(FB, x, y, z, np.array([0, 2]), np.array([4, 4])).tolist() == [True, True]


def _brute(theta, x, y, z, ci, co):
    keep = np.ones(len(ci), bool)
    for h in np.unique(co):
        cs = np.nonzero(co == h)[0]
        u = np.stack([x[h] - x[ci[cs]], y[h] - y[ci[cs]], z[h] - z[ci[cs]]], 1)
        L2 = (u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2]
        for a in range(len(cs)):
            w = np.cross(u[a], u)
            W2 = (w[:, 0] * w[:, 0] + w[:, 1] * w[:, 1]) + w[:, 2] * w[:, 2]
            hit = (L2 < L2[a]) & (W2 <= (theta * theta) * (L2[a] * L2))
            hit[a] = False
            keep[cs[a]] = not hit.any()
    return keep


def test_fishbone_equals_its_definition_by_brute_force():
    h = E.overlap_event(n_vertices=8)
    ci, co, _ = O.doublets(FB, h.x, h.y, h.z, h.layer)
    x, y, z = (np.asarray(v, np.float64) for v in (h.x, h.y, h.z))
    for theta in (0.002, 0.01, 0.05):
        cfg = C.default_config(fishbone_theta=theta)
        got = O.fishbone(cfg, x, y, z, ci, co)
        want = _brute(theta, x, y, z, ci, co)
        assert 0 < (~want).sum() < len(want)
        # np.cross evaluates the same three differences of products
        assert np.array_equal(got, want), theta


def test_fishbone_removes_duplicates_of_the_overlap_geometry():
    h = E.overlap_event()
    stats = {}
    for name, cfg in (("off", C.default_config()), ("on", FB)):
        r = O.reconstruct_event(cfg, h.x, h.y, h.z, h.layer)
        tid = h.track[r["hits"][:, :4]]
        gen = np.all(tid == tid[:, :1], axis=1) & (tid[:, 0] >= 0)
        ids, cnt = np.unique(tid[gen, 0], return_counts=True)
        stats[name] = dict(found=len(ids), duplicates=int((cnt - 1).sum()), fakes=int((~gen).sum()))
    assert stats["on"]["duplicates"] < 0.25 * stats["off"]["duplicates"]
    assert stats["on"]["found"] > 0.9 * stats["off"]["found"]
    assert stats["on"]["fakes"] < stats["off"]["fakes"]


def test_fishbone_off_changes_nothing():
    h = E.config2()
    a = O.reconstruct_event(C.default_config(), h.x, h.y, h.z, h.layer)
    b = O.reconstruct_event(C.default_config(fishbone_theta=0.0), h.x, h.y, h.z, h.layer)
    assert np.array_equal(a["hits"], b["hits"])
