"""Pins of the oracle's broken-line fit and its gradient (paper section 3.4).

* exact recovery of generated helix parameters from noise-free hits (pins the
  pre-fit, arc lengths, offsets and the perigee conversion);
* exact symmetries (rotation about z, mirrors);
* arc lengths and offsets recomputed independently (circle from its algebraic
  equation, arc length as radius x angle);
* the normal equations solved by numpy, and the optimum checked against the
  chi^2 written from its definition;
* the no-scattering limit against textbook weighted polynomial regression;
* chi^2 / ndof ~ 1 on tracks simulated with the same scattering model;
* the dual-number Jacobian against central finite differences, and the
  translation identities it must satisfy.
"""
import numpy as np
import pytest

import oracle as O
from synth import config as C
from synth import events as E
from tests.helpers import FIT_FLOORS, param_rel_err

CFG = C.default_config()


def _tracks(seed, n, *, smear=True, ms=False, pt="power", eta_max=2.5, disks=True, min_hits=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    trk = E.draw_tracks(rng, n, pt=pt, eta_max=eta_max)
    if ms:
        ti, li, x, y, z = E.track_hits_ms(rng, trk, disks=disks, smear=smear)
    else:
        ti, li, x, y, z, _ = E.track_hits(rng, trk, disks=disks, eff=1.0, smear=smear)
    nh = np.bincount(ti, minlength=n)
    starts = np.concatenate([[0], np.cumsum(nh)])
    sel = np.nonzero(nh >= min_hits)[0]
    tup = np.full((len(sel), 8), -1, np.int32)
    for j, t in enumerate(sel):
        tup[j, : nh[t]] = np.arange(starts[t], starts[t] + nh[t])
    truth = np.stack([trk[k][sel] for k in ("kappa", "phi0", "cot", "d0", "z0")], 1)
    return tup, nh[sel].astype(np.uint8), x, y, z, li, truth, {k: v[sel] for k, v in trk.items()}


def test_exact_recovery_noise_free():
    tup, n, x, y, z, li, truth, _ = _tracks(21, 4000, smear=False)
    p, chi2, st = O.fit(CFG, tup, n, x, y, z, li)
    assert np.all(st == 0)
    assert len(n) > 3000 and set(np.unique(n)) >= {4, 5}
    err = param_rel_err(p, truth)
    assert err.max() < 1e-9, err.max(axis=0)
    assert np.abs(chi2).max() < 1e-12


def test_symmetries():
    tup, n, x, y, z, li, truth, _ = _tracks(22, 500)
    base, c0, _ = O.fit(CFG, tup, n, x, y, z, li)
    a = 0.731
    ca, sa = np.cos(a), np.sin(a)
    rot, c1, _ = O.fit(CFG, tup, n, ca * x - sa * y, sa * x + ca * y, z, li)
    exp = base.copy(); exp[:, 1] = exp[:, 1] + a
    assert param_rel_err(rot, exp).max() < 1e-10
    assert np.allclose(c1, c0, rtol=1e-8, atol=1e-12)
    mir, c2, _ = O.fit(CFG, tup, n, x, -y, z, li)
    exp = base * np.array([-1, -1, 1, -1, 1])
    assert param_rel_err(mir, exp).max() < 1e-10
    assert np.allclose(c2, c0, rtol=1e-8, atol=1e-12)
    swap = np.array([0, 1, 2, 3, 7, 8, 9, 4, 5, 6], np.uint8)
    zm, c3, _ = O.fit(CFG, tup, n, x, y, -z, swap[li])
    exp = base * np.array([1, 1, -1, 1, -1])
    assert param_rel_err(zm, exp).max() < 1e-10
    assert np.allclose(c3, c0, rtol=1e-8, atol=1e-12)


def _circle3(P):
    """Centre and radius of the circle through three points (algebraic form)."""
    M = np.concatenate([P, np.ones((3, 1))], 1)
    D, Ee, F = np.linalg.solve(M, -(P ** 2).sum(1))
    c = np.array([-D / 2, -Ee / 2])
    return c, np.sqrt(c @ c - F)


def test_arc_lengths_and_offsets_independent():
    tup, n, x, y, z, li, _, _ = _tracks(23, 300)
    for t in range(0, len(n), 7):
        hs = tup[t, : n[t]]
        X, Y, Z = x[hs].astype(float), y[hs].astype(float), z[hs].astype(float)
        d = O.fit_debug(CFG, X, Y, Z, li[hs])
        P = np.stack([X, Y], 1)
        b = n[t] // 2
        c, R = _circle3(P[[0, b, n[t] - 1]])
        ang = np.arctan2(P[:, 1] - c[1], P[:, 0] - c[0])
        u, w = P[b] - P[0], P[-1] - P[b]
        turn = np.sign(u[0] * w[1] - u[1] * w[0])
        s = R * turn * ((ang - ang[0] + np.pi) % (2 * np.pi) - np.pi)
        u = -turn * (np.hypot(*(P - c).T) - R)
        assert np.allclose(d["s"], s, rtol=1e-9, atol=1e-9)
        assert np.allclose(d["um"], u, rtol=1e-7, atol=1e-10)
        assert np.isclose(d["kappa_pre"], turn / R, rtol=1e-9)


def _chi2_from_definition(d, x_c, v_l, VT):
    delta, n = d["delta"], len(d["s"])
    chi = np.sum((d["um"] - x_c[:n]) ** 2) / VT + np.sum((d["q"] * d["VZ"] - v_l) ** 2 / d["VZ"])
    for k in range(1, n - 1):
        beta = (x_c[k + 1] - x_c[k]) / delta[k] - (x_c[k] - x_c[k - 1]) / delta[k - 1] \
            - x_c[n] * (delta[k - 1] + delta[k]) / 2
        gam = (v_l[k + 1] - v_l[k]) / delta[k] - (v_l[k] - v_l[k - 1]) / delta[k - 1]
        chi += beta ** 2 * d["wT"][k] + gam ** 2 * d["wZ"][k]
    return chi


def test_normal_equations_and_optimum():
    tup, n, x, y, z, li, _, _ = _tracks(24, 300)
    VT = CFG["sigma_rphi"] ** 2
    for t in range(0, len(n), 5):
        hs = tup[t, : n[t]]
        d = O.fit_debug(CFG, x[hs], y[hs], z[hs], li[hs])
        assert d["status"] == 0
        xc = np.linalg.solve(d["A"], d["b"])
        vl = np.linalg.solve(d["N"], d["q"])
        assert np.allclose(xc, d["ucirc"], rtol=1e-7, atol=1e-13)
        assert np.allclose(vl, d["vline"], rtol=1e-10, atol=1e-12)
        chi = _chi2_from_definition(d, d["ucirc"], d["vline"], VT)
        assert np.isclose(chi, d["chi2"], rtol=1e-8, atol=1e-12)
        # stationarity: moving any unknown raises chi^2 quadratically, not linearly
        for i in range(len(xc)):
            step = np.zeros_like(xc); step[i] = 1e-4 * (1e-3 if i < n[t] else 1e-6)
            up = _chi2_from_definition(d, d["ucirc"] + step, d["vline"], VT)
            dn = _chi2_from_definition(d, d["ucirc"] - step, d["vline"], VT)
            assert abs(up - dn) <= 1e-6 * max(up + dn - 2 * chi, 1e-12) + 1e-9


def test_no_scattering_limit_is_polynomial_regression():
    """With vanishing material the kinks are forced to zero: the circle fit
    becomes a least-squares parabola u(s) = a + b s + (dk/2) s^2 and the S-Z
    fit a weighted straight line z(s) = c + cot s."""
    cfg = C.default_config(x_over_x0=1e-10)
    tup, n, x, y, z, li, _, _ = _tracks(25, 400)
    VT = cfg["sigma_rphi"] ** 2
    checked = 0
    for t in range(len(n)):
        if n[t] < 5:
            continue
        hs = tup[t, : n[t]]
        d = O.fit_debug(cfg, x[hs], y[hs], z[hs], li[hs])
        s, um = d["s"], d["um"]
        c2, c1, c0 = np.polyfit(s, um, 2)
        kappa = d["kappa_pre"] + 2 * c2
        w = 1.0 / np.sqrt(d["VZ"])
        zz = z[hs].astype(float)
        slope, icpt = np.polyfit(s, zz, 1, w=w)
        chi = np.sum((um - np.polyval([c2, c1, c0], s)) ** 2) / VT \
            + np.sum(((zz - (icpt + slope * s)) * w) ** 2)
        assert abs(d["params"][0] - kappa) <= 1e-6 * max(abs(kappa), 1e-5)
        assert abs(d["params"][2] - slope) <= 1e-6 * max(abs(slope), 1.0)
        assert np.isclose(d["chi2"], chi, rtol=1e-4, atol=1e-8)
        checked += 1
    assert checked > 20


def test_chi2_statistics_with_scattering():
    """Tracks simulated with the fit's own scattering model: chi^2/ndof ~ 1."""
    tup, n, x, y, z, li, _, _ = _tracks(26, 12000, ms=True, pt="loguniform")
    p, chi2, st = O.fit(CFG, tup, n, x, y, z, li)
    assert np.all(st == 0)
    ndof = 2 * n.astype(int) - 5
    for nn in (4, 5):
        m = n == nn
        assert m.sum() > 500
        mean = np.mean(chi2[m] / ndof[m])
        assert 0.95 < mean < 1.05, (nn, mean)
    # the tail: fraction above the 99% point of chi^2(3) for quadruplets
    m4 = n == 4
    frac = np.mean(chi2[m4] > 11.345)
    assert frac < 0.02


def test_bad_order_and_straight_line():
    tup, n, x, y, z, li, truth, _ = _tracks(27, 50)
    # hits out of order along the track (swap the 2nd and 3rd)
    bad = tup.copy()
    bad[:, [1, 2]] = tup[:, [2, 1]]
    p, chi2, st = O.fit(CFG, bad, n, x, y, z, li)
    assert np.all(st == 1) and np.all(np.isnan(p))
    # reversed order is the same helix traversed inwards: a valid fit
    rev = tup.copy()
    for t in range(len(n)):
        rev[t, : n[t]] = tup[t, : n[t]][::-1]
    p, chi2, st = O.fit(CFG, rev, n, x, y, z, li)
    assert np.all(st == 0)
    # an exactly straight track (y constant, so the pre-fit cross product is
    # exactly zero): kappa = 0, phi0 = 0, d0 = y, and the S-Z line
    cot, z0, d0 = 0.9, 1.5, 0.02
    X = np.array(C.BARREL_R)
    Y = np.full(4, d0)
    Z = z0 + cot * X
    d = O.fit_debug(CFG, X, Y, Z, np.arange(4))
    assert d["status"] == 0
    assert d["params"][0] == 0.0
    assert param_rel_err(d["params"][None], np.array([[0.0, 0.0, cot, d0, z0]])).max() < 1e-8


def _fd_jacobian(cfg, X, Y, Z, lay, h):
    n = len(X)
    J = np.zeros((6, n, 3))
    arrs = [X.copy(), Y.copy(), Z.copy()]
    for k in range(n):
        for c in range(3):
            a0 = arrs[c][k]
            arrs[c][k] = a0 + h
            r1 = O.fit_debug(cfg, *arrs, lay)
            arrs[c][k] = a0 - h
            r2 = O.fit_debug(cfg, *arrs, lay)
            arrs[c][k] = a0
            dv = np.append(r1["params"], r1["chi2"]) - np.append(r2["params"], r2["chi2"])
            dv[1] = (dv[1] + np.pi) % (2 * np.pi) - np.pi
            J[:, k, c] = dv / (2 * h)
    return J


def test_dual_jacobian_against_finite_differences():
    tup, n, x, y, z, li, _, _ = _tracks(28, 60)
    worst = 0.0
    for t in range(0, len(n), 3):
        hs = tup[t, : n[t]]
        X, Y, Z = (np.asarray(a[hs], np.float64) for a in (x, y, z))
        J = O.fit_jacobian(CFG, X, Y, Z, li[hs])
        h = 1e-4
        Jh = _fd_jacobian(CFG, X, Y, Z, li[hs], h)
        Jh2 = _fd_jacobian(CFG, X, Y, Z, li[hs], h / 2)
        Jr = (4 * Jh2 - Jh) / 3      # Richardson: removes the h^2 term
        for o in range(5):
            worst = max(worst, np.linalg.norm(J[o] - Jh[o]) / np.linalg.norm(J[o]))
        assert np.linalg.norm(J[5] - Jr[5]) / np.linalg.norm(J[5]) < 1e-5
    assert worst < 1e-5


def test_gradient_translation_identities():
    tup, n, x, y, z, li, _, _ = _tracks(29, 80)
    for t in range(0, len(n), 4):
        hs = tup[t, : n[t]]
        X, Y, Z = (np.asarray(a[hs], np.float64) for a in (x, y, z))
        J = O.fit_jacobian(CFG, X, Y, Z, li[hs])      # [6, n, 3]
        tot = J.sum(axis=1)                            # d/d(common translation)
        scale = np.abs(J).max(axis=(1, 2))
        d = O.fit_debug(CFG, X, Y, Z, li[hs])
        phi0 = d["params"][1]
        assert np.all(np.abs(tot[0]) < 1e-7 * scale[0])            # kappa
        assert np.all(np.abs(tot[2]) < 1e-7 * scale[2])            # cot(theta)
        assert np.abs(tot[5]).max() < 1e-6 * scale[5] + 1e-9       # chi^2
        assert np.allclose(tot[3, :2], [-np.sin(phi0), np.cos(phi0)], atol=1e-6)  # d0 moves along n(phi0)
        assert abs(tot[3, 2]) < 1e-9
        assert abs(tot[4, 2] - 1.0) < 1e-7                         # z0 moves with z
        # moving the circle along its tangent moves the point of closest approach:
        # d phi0 = -kappa / (1 + kappa d0) * (delta . t(phi0))
        kap, d0 = d["params"][0], d["params"][3]
        want = -kap / (1 + kap * d0) * np.array([np.cos(phi0), np.sin(phi0)])
        assert np.allclose(tot[1, :2], want, rtol=1e-5, atol=1e-9)
        assert abs(tot[1, 2]) < 1e-12


def test_module_gradient_is_sum_of_hit_gradients():
    ts = E.config4(n_tracks=300)
    off = E.module_offsets()
    gp, gc = E.cotangents(4, 300)
    h = ts.hits
    gh, go = O.fit_grad(CFG, ts.tuplets, ts.nhits, h.x, h.y, h.z, h.layer, h.module, off, gp, gc)
    want = np.zeros_like(go)
    np.add.at(want, h.module.astype(int), gh)
    assert np.allclose(go, want, rtol=1e-12, atol=1e-12)
    assert np.abs(gh).sum() > 0
