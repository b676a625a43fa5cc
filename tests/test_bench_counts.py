"""The link-pair accounting that bench.py reports beside the link kernel's time.

The windowed link search examines, for every in-cell, the out-cells of its own and
the neighbouring direction buckets. Checked here on the host, from the oracle's
cells of one pileup-50 event:
* `link_pair_counts` counts every pair sharing a middle hit;
* it examines no more pairs than that;
* the examined pairs include every pair that passes the R-Z cut, counted by brute force.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import bench
import oracle as O
from synth import config as C
from synth import events as E


class _Cells:
    """The member of the library's cell container that the count reads."""

    def __init__(self, ci, co):
        self._ci, self._co = torch.from_numpy(ci), torch.from_numpy(co)

    def valid(self):
        return self._ci, self._co, None


@pytest.mark.parametrize("theta", [None, 0.2])
def test_examined_pairs_cover_every_passing_pair(theta):
    cfg = C.default_config() if theta is None else C.default_config(ca_theta_barrel=theta, ca_theta_endcap=theta)
    h = E.config2()
    ci, co, _ = O.doublets(cfg, h.x, h.y, h.z, h.layer)
    x, y, z = (np.asarray(a, np.float64) for a in (h.x, h.y, h.z))
    r = np.sqrt(x * x + y * y)
    dr, dz = r[co] - r[ci], z[co] - z[ci]
    pairs, examined = bench.link_pair_counts(_Cells(ci, co), h, cfg)
    # every (in-cell, out-cell) pair meeting on a hit, and those passing the R-Z cut
    order = np.argsort(ci, kind="stable")
    first = np.searchsorted(ci[order], np.arange(h.n_hits + 1))
    th2 = max(cfg["ca_theta_barrel"], cfg["ca_theta_endcap"]) ** 2
    want_pairs = passing = 0
    for c in range(len(ci)):
        outs = order[first[co[c]]:first[co[c] + 1]]
        want_pairs += len(outs)
        a = dr[c] * dz[outs] - dz[c] * dr[outs]
        passing += int(np.count_nonzero(a * a <= th2 * ((dr[c] * dr[c] + dz[c] * dz[c]) *
                                                       (dr[outs] * dr[outs] + dz[outs] * dz[outs]))))
    assert pairs == want_pairs
    assert passing <= examined <= pairs
    assert passing > 0
