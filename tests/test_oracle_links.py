"""Pins of the oracle's cell linking (paper section 3.2: triplet compatibility).

Each link's two conditions are recomputed another way: the R-Z kink angle
from atan2 of both segments, and the circle through the three hits from the
algebraic circle equation x^2 + y^2 + D x + E y + F = 0 solved with numpy.
Links whose values sit within a hair of a boundary are not judged.
"""
import numpy as np

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import link_set

CFG = C.default_config()


def _candidates(ci, co):
    """All (c', c) with outer(c') == inner(c)."""
    order = np.argsort(co, kind="stable")
    co_sorted = co[order]
    out = []
    for c in range(len(ci)):
        h1 = ci[c]
        lo, hi = np.searchsorted(co_sorted, h1), np.searchsorted(co_sorted, h1, side="right")
        for cp in order[lo:hi]:
            out.append((cp, c))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def _geometric_classes(cfg, x, y, z, layer, ci, co, margin=1e-7):
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    cand = _candidates(ci, co)
    cp, c = cand[:, 0], cand[:, 1]
    h0, h1, h2 = ci[cp], co[cp], co[c]
    r = np.hypot(x, y)
    a1 = np.arctan2(z[h1] - z[h0], r[h1] - r[h0])
    a2 = np.arctan2(z[h2] - z[h1], r[h2] - r[h1])
    sin_kink = np.abs(np.sin(a2 - a1))
    barrel = np.array(cfg["layer_barrel"])[layer[h2]] == 1
    theta = np.where(barrel, cfg["ca_theta_barrel"], cfg["ca_theta_endcap"])
    ok = sin_kink < theta * (1 - margin)
    bad = sin_kink > theta * (1 + margin)
    # algebraic circle through the three hits
    P = np.stack([np.stack([x[h], y[h]], -1) for h in (h0, h1, h2)], 1)  # [N,3,2]
    M = np.concatenate([P, np.ones(P.shape[:2] + (1,))], -1)              # rows (x, y, 1)
    rhs = -(P ** 2).sum(-1)
    det = np.linalg.det(M)
    well = np.abs(det) > 1e-6
    sol = np.zeros((len(cp), 3))
    sol[well] = np.linalg.solve(M[well], rhs[well][..., None])[..., 0]
    cx, cy = -sol[:, 0] / 2, -sol[:, 1] / 2
    rad = np.sqrt(np.maximum(cx ** 2 + cy ** 2 - sol[:, 2], 0))
    dist = np.abs(np.hypot(cx, cy) - rad)
    rmax = np.where(layer[h0] == 0, cfg["ca_rmax_bpix1"], cfg["ca_rmax_other"])
    ok &= well & (dist < rmax * (1 - 1e-6))
    bad |= well & (dist > rmax * (1 + 1e-6))
    key = lambda sel: set(zip(h0[sel].tolist(), h1[sel].tolist(), h2[sel].tolist()))
    return key(ok), key(bad), len(cand)


def _event_and_cells(h):
    ci, co, _ = O.doublets(CFG, h.x, h.y, h.z, h.layer)
    return ci, co


def test_links_match_geometry_config2():
    h = E.config2()
    ci, co = _event_and_cells(h)
    li, lo = O.links(CFG, h.x, h.y, h.z, h.layer, ci, co)
    got = link_set(ci, co, li, lo)
    sure, never, ncand = _geometric_classes(CFG, h.x, h.y, h.z, h.layer, ci, co)
    assert len(sure) > 1000
    assert sure <= got
    assert not (got & never)
    assert len(got) < ncand


def test_links_config1_truth():
    """Every true consecutive triplet of a noise-free barrel track is linked."""
    h = E.config1()
    ci, co = _event_and_cells(h)
    li, lo = O.links(CFG, h.x, h.y, h.z, h.layer, ci, co)
    got = link_set(ci, co, li, lo)
    for t in range(20):
        hs = np.nonzero(h.track == t)[0]
        hs = hs[np.argsort(h.layer[hs])]
        for a, b, c in zip(hs[:-2], hs[1:-1], hs[2:]):
            assert (a, b, c) in got


def test_link_symmetries_exact():
    h = E.config2()
    x, y, z = (np.asarray(a, np.float64) for a in (h.x, h.y, h.z))
    L = h.layer

    def links_of(x, y, z, L):
        ci, co, _ = O.doublets(CFG, x, y, z, L)
        li, lo = O.links(CFG, x, y, z, L, ci, co)
        return link_set(ci, co, li, lo)

    base = links_of(x, y, z, L)
    assert links_of(-y, x, z, L) == base
    assert links_of(-x, y, z, L) == base
    swap = np.array([0, 1, 2, 3, 7, 8, 9, 4, 5, 6], np.uint8)
    assert links_of(x, y, -z, swap[L]) == base


def test_straight_line_from_origin_links():
    """Three hits on a line through the origin are aligned and point at the beam."""
    phi, cot = -1.1, 0.8
    r = np.array(C.BARREL_R[:3])
    x, y, z = r * np.cos(phi), r * np.sin(phi), r * cot
    layer = np.array([0, 1, 2], np.uint8)
    ci, co = np.array([0, 1], np.int32), np.array([1, 2], np.int32)
    li, lo = O.links(CFG, x, y, z, layer, ci, co)
    assert list(zip(li.tolist(), lo.tolist())) == [(0, 1)]
    # a 1 cm offset of the middle hit in z breaks the R-Z alignment
    z2 = z.copy(); z2[1] += 1.0
    assert len(O.links(CFG, x, y, z2, layer, ci, co)[0]) == 0
    # a displaced circle (sagitta away from the beam) fails the beam-spot cut
    x3, y3 = x.copy(), y.copy()
    x3[1] += 0.5 * -np.sin(phi); y3[1] += 0.5 * np.cos(phi)
    assert len(O.links(CFG, x3, y3, z, layer, ci, co)[0]) == 0
