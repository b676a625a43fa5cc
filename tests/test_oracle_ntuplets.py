"""Pins of the oracle's n-tuplet search and duplicate removal.

Against an independent breadth-first enumeration of every root path written
here, the duplicate-removal rule applied by brute force over pairs of
n-tuplets, the structural invariants of the paper's description (section 3.2:
roots, maximal paths, disjoint buckets; section 3.3: no hit doublet shared by
n-tuplets of different length), and the truth quadruplets of noise-free
barrel events.
"""
import numpy as np

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import tuplet_set

CFG = C.default_config()


def _bfs_paths(cfg, layer, ci, co, li, lo):
    """Every maximal path from a root with >= min_hits hits, by breadth-first growth."""
    n_cells = len(ci)
    outs = [[] for _ in range(n_cells)]
    has_in = np.zeros(n_cells, bool)
    for a, b in zip(li.tolist(), lo.tolist()):
        outs[a].append(b)
        has_in[b] = True
    roots = [c for c in range(n_cells)
             if layer[ci[c]] in cfg["root_always"]
             or (layer[ci[c]] in cfg["root_if_free"] and not has_in[c])]
    done = []
    frontier = [[c] for c in roots]
    while frontier:
        nxt = []
        for p in frontier:
            if not outs[p[-1]] or len(p) + 1 == cfg["max_hits"]:
                done.append(p)
            else:
                nxt.extend(p + [o] for o in outs[p[-1]])
        frontier = nxt
    done = [p for p in done if len(p) + 1 >= cfg["min_hits"]]
    return done, outs, has_in, set(roots)


def _hits_of(path, ci, co):
    return tuple([int(ci[path[0]])] + [int(co[c]) for c in path])


def _reco(h, cfg=CFG):
    ci, co, _ = O.doublets(cfg, h.x, h.y, h.z, h.layer)
    li, lo = O.links(cfg, h.x, h.y, h.z, h.layer, ci, co)
    return ci, co, li, lo


def test_dfs_equals_bfs_enumeration():
    h = E.config2()
    ci, co, li, lo = _reco(h)
    raw = O.ntuplets(CFG, h.layer, ci, co, li, lo, dedup=False)
    paths, _, _, _ = _bfs_paths(CFG, h.layer, ci, co, li, lo)
    want = {_hits_of(p, ci, co) for p in paths}
    got = tuplet_set(raw["hits"], raw["n"])
    assert len(want) > 500
    assert got == want
    assert len(got) == len(raw["n"]) == raw["n_raw"]  # no exact duplicates


def test_dedup_rule_bruteforce():
    h = E.config2()
    ci, co, li, lo = _reco(h)
    raw = O.ntuplets(CFG, h.layer, ci, co, li, lo, dedup=False)
    kept = O.ntuplets(CFG, h.layer, ci, co, li, lo, dedup=True)
    cells = [set(r[r >= 0].tolist()) for r in raw["cells"]]
    n = raw["n"].astype(int)
    drop = set()
    for a in range(len(cells)):
        for b in range(len(cells)):
            if n[b] > n[a] and cells[a] & cells[b]:
                drop.add(a)
                break
    want = {tuple(raw["hits"][i, : n[i]].tolist()) for i in range(len(n)) if i not in drop}
    got = tuplet_set(kept["hits"], kept["n"])
    assert got == want
    assert 0 < len(got) < len(n)
    assert kept["n_raw"] == raw["n_raw"]


def test_invariants():
    h = E.config2()
    ci, co, li, lo = _reco(h)
    res = O.ntuplets(CFG, h.layer, ci, co, li, lo, dedup=True)
    cell_of = {(int(a), int(b)): c for c, (a, b) in enumerate(zip(ci, co))}
    linked = set(zip(li.tolist(), lo.tolist()))
    has_out = set(li.tolist())
    has_in = set(lo.tolist())
    pairs = {tuple(p) for p in CFG["pairs"]}
    per_cell_n = {}
    for row, cells, n in zip(res["hits"], res["cells"], res["n"]):
        hs = row[:n].tolist()
        assert n >= 4 and all(v == -1 for v in row[n:])
        cs = [cell_of[(a, b)] for a, b in zip(hs[:-1], hs[1:])]   # consecutive hits are doublets
        assert cs == cells[: n - 1].tolist()
        assert all((a, b) in linked for a, b in zip(cs[:-1], cs[1:]))   # consecutive cells linked
        assert all((h.layer[a], h.layer[b]) in pairs for a, b in zip(hs[:-1], hs[1:]))
        L0 = h.layer[hs[0]]
        assert L0 in CFG["root_always"] or (L0 in CFG["root_if_free"] and cs[0] not in has_in)
        assert cs[-1] not in has_out                                      # maximal
        for c in cs:
            per_cell_n.setdefault(c, set()).add(int(n))
    assert all(len(v) == 1 for v in per_cell_n.values())   # section 3.3 rule after dedup


def test_config1_truth_quadruplets():
    h = E.config1()
    ci, co, li, lo = _reco(h)
    res = O.ntuplets(CFG, h.layer, ci, co, li, lo)
    got = tuplet_set(res["hits"], res["n"])
    n_found = 0
    for t in range(20):
        hs = np.nonzero(h.track == t)[0]
        if len(hs) == 4:
            hs = hs[np.argsort(h.layer[hs])]
            assert tuple(hs.tolist()) in got
            n_found += 1
    assert n_found >= 10


def _forward_helix_hits():
    """Noise-free hits of a 5 GeV helix from the origin crossing BPix1, BPix2 and FPix+1..3."""
    kappa, phi0, cot = -C.K_CURV * 3.8 / 5.0, 0.7, 3.0
    zero = np.zeros(1)
    s = [E._barrel_s(np.array([kappa]), zero, C.BARREL_R[l])[0] for l in (0, 1)]
    s += [C.disk_z(l) / cot for l in (4, 5, 6)]
    s = np.array(s)
    x, y = E.helix_xy(kappa, phi0, 0.0, s)
    return x, y, s * cot, np.array([0, 1, 4, 5, 6], np.uint8)


def test_truncation_at_max_hits():
    """A five-hit forward track with max_hits = 4 yields 4-hit paths and the flag."""
    x, y, z, layer = _forward_helix_hits()
    cfg = C.default_config(max_hits=4)
    ci, co, _ = O.doublets(cfg, x, y, z, layer)
    li, lo = O.links(cfg, x, y, z, layer, ci, co)
    res = O.ntuplets(cfg, layer, ci, co, li, lo, dedup=False)
    assert res["truncated"]
    assert set(res["n"].tolist()) == {4}
    full = O.ntuplets(CFG, layer, ci, co, li, lo, dedup=False)
    assert not full["truncated"]
    assert (0, 1, 2, 3, 4) in tuplet_set(full["hits"], full["n"])
    # after duplicate removal only the five-hit path survives
    kept = O.ntuplets(CFG, layer, ci, co, li, lo, dedup=True)
    assert tuplet_set(kept["hits"], kept["n"]) == {(0, 1, 2, 3, 4)}


def test_no_cells():
    e = np.zeros(0, np.int32)
    res = O.ntuplets(CFG, np.zeros(3, np.uint8), e, e, e, e)
    assert len(res["n"]) == 0 and res["n_raw"] == 0
