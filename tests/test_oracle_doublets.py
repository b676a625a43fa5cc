"""Pins of the oracle's doublet search (paper section 3.2, Table 1).

The oracle evaluates each cut in an algebraic, division-free form.  These
tests check it against what each cut means geometrically, computed another
way (angles with atan2, the line's z at r = 0, the circle's radius from a
linear solve), on every pair whose geometric value is not within a hair of
the cut boundary; against exact symmetries of the predicates; against the
subset structure of the cut sets of Table 2; and against hand-built events.
"""
import numpy as np
import pytest

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import doublet_set

CFG = C.default_config()
K = C.K_CURV


def _geometric_classes(cfg, x, y, z, layer, margin=1e-7):
    """(clear pass, clear fail) doublet sets from the cuts' geometric meaning."""
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    rho_min = cfg["pt_min"] / (K * cfg["bfield"])
    sure, never = set(), set()
    for p, (li, lo) in enumerate(cfg["pairs"]):
        I = np.nonzero(layer == li)[0]
        Oh = np.nonzero(layer == lo)[0]
        if len(I) == 0 or len(Oh) == 0:
            continue
        ii, oo = np.meshgrid(I, Oh, indexing="ij")
        ii, oo = ii.ravel(), oo.ravel()
        ok = np.ones(ii.shape, bool)
        bad = np.zeros(ii.shape, bool)
        m = cfg["cut_mask"]
        if m & C.CUT_PHIW:
            dphi = np.abs((phi[oo] - phi[ii] + np.pi) % (2 * np.pi) - np.pi)
            lim = cfg["pair_dphi"][p]
            ok &= dphi < lim - margin
            bad |= dphi > lim + margin
        if m & C.CUT_ZW:
            zi = z[ii]
            ok &= (zi > cfg["pair_zlo"][p] + margin) & (zi < cfg["pair_zhi"][p] - margin)
            bad |= (zi < cfg["pair_zlo"][p] - margin) | (zi > cfg["pair_zhi"][p] + margin)
        if m & C.CUT_ZIP:
            dr = r[oo] - r[ii]
            with np.errstate(divide="ignore", invalid="ignore"):
                z0 = z[ii] - r[ii] * (z[oo] - z[ii]) / dr
            fwd = dr > margin
            ok &= fwd & (np.abs(z0) < cfg["z0_max"] * (1 - margin))
            bad |= (dr < -margin) | (fwd & (np.abs(z0) > cfg["z0_max"] * (1 + margin)))
        if m & C.CUT_PT:
            # circle through the origin and both hits: 2 c.P = |P|^2 for P = Pi, Po
            M = np.stack([np.stack([x[ii], y[ii]], -1), np.stack([x[oo], y[oo]], -1)], -2) * 2.0
            rhs = np.stack([r[ii] ** 2, r[oo] ** 2], -1)
            det = M[:, 0, 0] * M[:, 1, 1] - M[:, 0, 1] * M[:, 1, 0]
            well = np.abs(det) > 1e-12
            cen = np.full((len(ii), 2), np.inf)
            cen[well] = np.linalg.solve(M[well], rhs[well][..., None])[..., 0]
            R = np.hypot(cen[:, 0], cen[:, 1])
            ok &= R > rho_min * (1 + margin)
            bad |= R < rho_min * (1 - margin)
        sure |= set(zip(ii[ok].tolist(), oo[ok].tolist()))
        never |= set(zip(ii[bad].tolist(), oo[bad].tolist()))
    return sure, never


def _subsample(h, per_layer, seed):
    rng = np.random.default_rng(seed)
    keep = []
    for l in range(10):
        idx = np.nonzero(h.layer == l)[0]
        keep.append(rng.permutation(idx)[:per_layer])
    keep = np.sort(np.concatenate(keep))
    return h.x[keep], h.y[keep], h.z[keep], h.layer[keep]


@pytest.mark.parametrize("mask", [C.CUT_ALL, C.CUT_PHIW, C.CUT_PHIW | C.CUT_ZW, C.CUT_PHIW | C.CUT_ZW | C.CUT_ZIP,
                                  C.CUT_PT | C.CUT_ZIP])
def test_cuts_match_geometry(mask):
    cfg = C.default_config(cut_mask=mask)
    x, y, z, layer = _subsample(E.config2(), 250, seed=mask)
    inner, outer, _ = O.doublets(cfg, x, y, z, layer)
    got = doublet_set(inner, outer)
    sure, never = _geometric_classes(cfg, x, y, z, layer)
    assert len(sure) > 100
    assert sure <= got, f"{len(sure - got)} clearly passing pairs missing"
    assert not (got & never), f"{len(got & never)} clearly failing pairs emitted"


def test_config1_geometry_full():
    h = E.config1()
    inner, outer, _ = O.doublets(CFG, h.x, h.y, h.z, h.layer)
    got = doublet_set(inner, outer)
    sure, never = _geometric_classes(CFG, h.x, h.y, h.z, h.layer)
    assert sure <= got and not (got & never)
    # every true consecutive pair of a track is a doublet
    for t in range(20):
        hs = np.nonzero(h.track == t)[0]
        hs = hs[np.argsort(h.layer[hs])]
        for a, b in zip(hs[:-1], hs[1:]):
            assert (a, b) in got


def _pair_index(cfg):
    return {tuple(p): i for i, p in enumerate(cfg["pairs"])}


def test_symmetries_exact():
    """Rotation by 90 degrees, x mirror and z mirror leave every predicate bit-identical."""
    h = E.config2()
    x, y, z = (np.asarray(a, np.float64) for a in (h.x, h.y, h.z))
    layer = h.layer
    base = doublet_set(*O.doublets(CFG, x, y, z, layer)[:2])
    assert len(base) > 10000
    assert doublet_set(*O.doublets(CFG, -y, x, z, layer)[:2]) == base
    assert doublet_set(*O.doublets(CFG, -x, y, z, layer)[:2]) == base
    swap = np.array([0, 1, 2, 3, 7, 8, 9, 4, 5, 6], np.uint8)
    assert doublet_set(*O.doublets(CFG, x, y, -z, swap[layer])[:2]) == base


def test_pair_labels():
    h = E.config2()
    inner, outer, pair = O.doublets(CFG, h.x, h.y, h.z, h.layer)
    pairs = np.array(CFG["pairs"])
    assert np.array_equal(h.layer[inner], pairs[pair, 0])
    assert np.array_equal(h.layer[outer], pairs[pair, 1])


def test_adding_a_cut_only_removes_doublets():
    """Table 2's cut sets are conjunctions: each added cut can only shrink the set."""
    h = E.config2()
    chain = [C.CUT_PHIW, C.CUT_PHIW | C.CUT_ZW, C.CUT_PHIW | C.CUT_ZW | C.CUT_ZIP, C.CUT_ALL]
    prev = None
    counts = []
    for m in chain:
        s = doublet_set(*O.doublets(C.default_config(cut_mask=m), h.x, h.y, h.z, h.layer)[:2])
        counts.append(len(s))
        if prev is not None:
            assert s <= prev
        prev = s
    assert counts[0] > counts[-1]


def _radial_line(phi, cot, layers):
    xs, ys, zs, ls = [], [], [], []
    for l in layers:
        if l < 4:
            r = C.BARREL_R[l]
            zz = r * cot
        else:
            zz = C.disk_z(l)
            r = zz / cot
        xs.append(r * np.cos(phi)); ys.append(r * np.sin(phi)); zs.append(zz); ls.append(l)
    return np.array(xs), np.array(ys), np.array(zs), np.array(ls, np.uint8)


def test_hand_event_radial_lines():
    """Hits on straight lines through the origin: every listed pair they span is a doublet.

    Barrel line (cot 0.5) crosses BPix1-4; forward line (cot 3) crosses BPix1,
    BPix2 and the three +z disks (r = 10.67, 13, 16).
    """
    xb, yb, zb, lb = _radial_line(0.3, 0.5, [0, 1, 2, 3])
    xf, yf, zf, lf = _radial_line(2.0, 3.0, [0, 1, 4, 5, 6])
    x, y, z = np.concatenate([xb, xf]), np.concatenate([yb, yf]), np.concatenate([zb, zf])
    layer = np.concatenate([lb, lf])
    got = doublet_set(*O.doublets(CFG, x, y, z, layer)[:2])
    barrel = {(0, 1), (1, 2), (2, 3), (0, 2), (1, 3)}
    fwd_layers = [0, 1, 4, 5, 6]
    fwd = {(fwd_layers.index(a) + 4, fwd_layers.index(b) + 4)
           for a, b in [(0, 1), (0, 4), (1, 4), (4, 5), (5, 6), (0, 5), (1, 5), (4, 6)]}
    assert got == barrel | fwd


def test_empty_and_single_layer():
    x = np.array([3.0, 2.9]); y = np.array([0.1, 0.0]); z = np.array([0.0, 1.0])
    assert len(O.doublets(CFG, x, y, z, np.array([0, 0], np.uint8))[0]) == 0
    e = np.zeros(0)
    assert len(O.doublets(CFG, e, e, e, np.zeros(0, np.uint8))[0]) == 0


def test_binned_search_equals_the_brute_force():
    """The oracle's azimuth-binned doublet search (used to time the oracle on
    whole pileup-200 events) finds exactly the brute-force set: configs 1
    and 2 with several bin counts, and 4 pileup-200 events."""
    import concurrent.futures as cf

    from tests.helpers import sorted_keys

    def same(h, n_bins=64, cfg=CFG):
        a = O.doublets(cfg, h.x, h.y, h.z, h.layer)
        b = O.doublets_binned(cfg, h.x, h.y, h.z, h.layer, n_bins)
        return len(a[0]) > 0 and np.array_equal(sorted_keys(a[0], a[1]), sorted_keys(b[0], b[1]))

    for bins in (1, 7, 64, 512):
        assert same(E.config1(), bins)
        assert same(E.config2(), bins)
    assert same(E.config2(), 64, C.default_config(cut_mask=C.CUT_ZW | C.CUT_ZIP | C.CUT_PT))
    h = E.config5(n_events=4)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        assert all(ex.map(lambda e: same(h.event(e)), range(4)))
