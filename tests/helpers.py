"""Test-side helpers: canonical forms of the integer products and tolerances.

Integer products are compared as sorted sets: doublets as (inner, outer) hit
pairs, links as (h0, h1, h2) hit triplets, n-tuplets as hit tuples.
"""
import numpy as np

# Floors for relative comparisons of fit parameters (kappa 1/cm, phi0 rad,
# cot(theta), d0 cm, z0 cm): |a - b| <= tol * max(|ref|, floor).
FIT_FLOORS = np.array([1e-5, 1.0, 1.0, 0.01, 0.1])


def doublet_set(inner, outer):
    return set(zip(np.asarray(inner).tolist(), np.asarray(outer).tolist()))


def link_set(cell_inner, cell_outer, link_in, link_out):
    ci = np.asarray(cell_inner)
    co = np.asarray(cell_outer)
    li = np.asarray(link_in)
    lo = np.asarray(link_out)
    return set(zip(ci[li].tolist(), co[li].tolist(), co[lo].tolist()))


def tuplet_set(hits, n):
    hits = np.asarray(hits)
    n = np.asarray(n)
    return set(tuple(hits[i, : n[i]].tolist()) for i in range(hits.shape[0]))


def param_rel_err(a, ref, floors=FIT_FLOORS):
    """Per-element |a - ref| / max(|ref|, floor), phi0 difference wrapped."""
    d = np.asarray(a, np.float64) - np.asarray(ref, np.float64)
    d[..., 1] = (d[..., 1] + np.pi) % (2 * np.pi) - np.pi
    return np.abs(d) / np.maximum(np.abs(ref), floors)


def tuplets_from_tracks(track_ids, n_tracks, min_hits=1):
    """Hit index lists of each truth track (hits in the given order)."""
    out = [[] for _ in range(n_tracks)]
    for h, t in enumerate(np.asarray(track_ids).tolist()):
        if t >= 0:
            out[t].append(h)
    return [o for o in out if len(o) >= min_hits]


def sorted_keys(*cols):
    """Rows of non-negative int columns (each < 2^21) packed into sorted int64
    keys: a fast canonical form of a set of index tuples."""
    key = np.zeros(np.asarray(cols[0]).shape, np.int64)
    for c in cols:
        c = np.asarray(c, np.int64)
        assert c.size == 0 or (c.min() >= 0 and c.max() < (1 << 21))
        key = (key << 21) | c
    return np.sort(key)
