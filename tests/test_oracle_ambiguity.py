"""Pins of the oracle's ambiguity resolution (paper section 3.5): tracks
sharing a hit doublet keep the best chi2; triplets sharing a hit keep the
smallest transverse impact parameter.  Checked against a brute force over
all pairs of tracks, for order independence, and for its invariants on a
reconstructed event."""
import numpy as np

import oracle as O
from synth import config as C
from synth import events as E

CFG = C.default_config()


def _brute(hits, cells, n, chi2, tip):
    T = len(n)
    cand = np.isfinite(chi2)
    keep1 = cand.copy()
    for t in range(T):
        if not cand[t]:
            continue
        ct = set(cells[t, : n[t] - 1].tolist())
        for u in range(T):
            if u != t and cand[u] and ct & set(cells[u, : n[u] - 1].tolist()) and chi2[u] < chi2[t]:
                keep1[t] = False
                break
    keep = keep1.copy()
    for t in range(T):
        if not keep1[t] or n[t] != 3:
            continue
        ht = set(hits[t, :3].tolist())
        for u in range(T):
            if u != t and keep1[u] and n[u] == 3 and ht & set(hits[u, :3].tolist()) and abs(tip[u]) < abs(tip[t]):
                keep[t] = False
                break
    return keep


def _random_tracks(rng, T, pool_hits=60):
    """Rows of 3..5 hits drawn from a small hit pool (so that tracks share
    hits and doublets); a cell id per consecutive hit pair."""
    n = rng.integers(3, 6, size=T).astype(np.uint8)
    hits = np.full((T, 8), -1, np.int32)
    cells = np.full((T, 7), -1, np.int32)
    for t in range(T):
        hs = np.sort(rng.choice(pool_hits, size=n[t], replace=False))
        hits[t, : n[t]] = hs
        cells[t, : n[t] - 1] = hs[:-1] * pool_hits + hs[1:]
    chi2 = rng.exponential(3.0, T).round(1)          # rounded: ties happen
    chi2[rng.uniform(size=T) < 0.05] = np.nan        # failed fits
    tip = rng.normal(0, 0.05, T).round(3)
    return hits, cells, n, chi2, tip


def test_ambiguity_equals_brute_force():
    rng = np.random.Generator(np.random.PCG64(51))
    for _ in range(30):
        h, c, n, chi2, tip = _random_tracks(rng, int(rng.integers(5, 120)))
        assert np.array_equal(O.ambiguity(h, c, n, chi2, tip), _brute(h, c, n, chi2, tip))


def test_ambiguity_is_order_independent():
    rng = np.random.Generator(np.random.PCG64(52))
    h, c, n, chi2, tip = _random_tracks(rng, 300)
    keep = O.ambiguity(h, c, n, chi2, tip)
    perm = rng.permutation(len(n))
    assert np.array_equal(O.ambiguity(h[perm], c[perm], n[perm], chi2[perm], tip[perm]), keep[perm])


def test_ambiguity_invariants_on_a_reconstructed_event():
    """Triplet workflow on a PU50 event: after resolution no cell is shared
    by kept tracks of different chi2, and no hit by kept triplets of
    different |tip|; every dropped track has a reason."""
    cfg = C.default_config(min_hits=3)
    h = E.config2()
    r = O.reconstruct_event(cfg, h.x, h.y, h.z, h.layer)
    p, chi2, st = O.fit(cfg, r["hits"], r["n"], h.x, h.y, h.z, h.layer)
    keep = O.ambiguity(r["hits"], r["cells"], r["n"], chi2, p[:, 3])
    n = r["n"]
    assert (n == 3).sum() > 100 and keep.sum() < len(n)
    best_c, best_h = {}, {}
    for t in np.nonzero(keep)[0]:
        for c in r["cells"][t, : n[t] - 1]:
            assert best_c.setdefault(int(c), chi2[t]) == chi2[t]
        if n[t] == 3:
            for hh in r["hits"][t, :3]:
                assert best_h.setdefault(int(hh), abs(p[t, 3])) == abs(p[t, 3])
    assert np.array_equal(keep, _brute(r["hits"], r["cells"], n, chi2, p[:, 3])) if len(n) < 3000 else True
