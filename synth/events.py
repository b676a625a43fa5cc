"""Seeded synthetic events: charged helices through the pixel geometry.

This is the only code that serves both the CPU oracle and the GPU library,
and it holds none of the reconstruction's arithmetic: it simulates tracks
(helix propagation, layer crossings, smearing, inefficiency, noise) and
returns hit arrays plus the generating truth.  The workloads stand in for the
paper's simulated t-tbar pileup samples (section 4.1), which are not
available: vertices spread along the beam, a p_T spectrum falling as p_T^-3,
uniform pseudorapidity, one hit per layer crossing.

Helix convention (perigee with respect to the origin): curvature kappa > 0
turns counter-clockwise seen from +z, phi0 is the direction at the point of
closest approach (PCA), d0 the signed distance of the PCA along the left
normal n(phi0) = (-sin phi0, cos phi0), cot(theta) = dz/ds with s the
transverse arc length, z0 the z of the PCA.  A particle of charge q has
kappa = -q * 0.299792458 * B / (100 p_T) in 1/cm.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import config as C


# ----------------------------------------------------------------------------
# containers

@dataclass
class Hits:
    """SoA hit arrays of one or more events (event_offsets delimits them)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    layer: np.ndarray          # uint8
    module: np.ndarray         # int16
    track: np.ndarray          # int32 truth track id within its event, -1 = noise
    event_offsets: np.ndarray  # int32 [n_events + 1]
    truth: list = field(default_factory=list)  # per event: dict of track arrays

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_events(self) -> int:
        return int(self.event_offsets.shape[0] - 1)

    @property
    def dtype(self):
        return self.x.dtype

    def event(self, e: int) -> "Hits":
        a, b = int(self.event_offsets[e]), int(self.event_offsets[e + 1])
        return Hits(self.x[a:b], self.y[a:b], self.z[a:b], self.layer[a:b],
                    self.module[a:b], self.track[a:b],
                    np.array([0, b - a], dtype=np.int32),
                    [self.truth[e]] if self.truth else [])


@dataclass
class TrackSet:
    """Hits stored in track order, for fitting without pattern recognition."""
    hits: Hits
    tuplets: np.ndarray        # int32 [n_tracks, 8], -1 padded
    nhits: np.ndarray          # uint8 [n_tracks]
    params: np.ndarray         # float64 [n_tracks, 5] generating (kappa, phi0, cot, d0, z0)


# ----------------------------------------------------------------------------
# helix geometry (simulation side)

def _wrap(a):
    return (a + np.pi) % (2.0 * np.pi) - np.pi


def perigee_from_vertex(vx, vy, vz, phi_v, kappa, cot):
    """Perigee parameters of the helix leaving (vx, vy, vz) in direction phi_v.

    Through the circle centre c = v + n(phi_v)/kappa: the PCA is the point of
    the circle on the line from c to the origin.
    """
    cx = vx - np.sin(phi_v) / kappa
    cy = vy + np.cos(phi_v) / kappa
    cn = np.hypot(cx, cy)
    shrink = 1.0 - 1.0 / (np.abs(kappa) * cn)
    px, py = cx * shrink, cy * shrink
    nx = np.sign(kappa) * cx / cn
    ny = np.sign(kappa) * cy / cn
    phi0 = np.arctan2(-nx, ny)
    d0 = px * nx + py * ny
    s_v = _wrap(phi_v - phi0) / kappa
    z0 = vz - cot * s_v
    return phi0, d0, z0, s_v


def helix_xy(kappa, phi0, d0, s):
    """Transverse position at arc length s (stable as kappa -> 0)."""
    half = 0.5 * kappa * s
    chord = s * np.sinc(half / np.pi)     # 2 sin(kappa s / 2) / kappa
    x = -d0 * np.sin(phi0) + chord * np.cos(phi0 + half)
    y = d0 * np.cos(phi0) + chord * np.sin(phi0 + half)
    return x, y


def _barrel_s(kappa, d0, radius):
    """First arc length at which the helix reaches the given radius (nan if never)."""
    h2 = (radius * radius - d0 * d0) / (1.0 + kappa * d0)
    h = np.sqrt(np.where(h2 > 0, h2, np.nan))
    a = 0.5 * np.abs(kappa) * h
    a_ok = np.where(a <= 1.0, a, np.nan)
    ratio = np.where(a_ok > 1e-8, np.arcsin(np.where(a_ok > 1e-8, a_ok, 0.5)) / np.where(a_ok > 1e-8, a_ok, 0.5), 1.0)
    return h * ratio


def module_id(layer, x, y, z):
    """Module index following the barrel ladder / disk ring segmentation."""
    layer = np.asarray(layer)
    phi = np.arctan2(y, x)
    u = (phi + np.pi) / (2.0 * np.pi)
    out = np.zeros(layer.shape, dtype=np.int64)
    base = 0
    for l in range(4):
        nl = C.BARREL_LADDERS[l]
        sel = layer == l
        lad = np.clip((u[sel] * nl).astype(np.int64), 0, nl - 1)
        zs = np.clip(((z[sel] + C.BARREL_HALF_Z) / (2 * C.BARREL_HALF_Z / C.BARREL_ZSLICES)).astype(np.int64),
                     0, C.BARREL_ZSLICES - 1)
        out[sel] = base + lad * C.BARREL_ZSLICES + zs
        base += nl * C.BARREL_ZSLICES
    per_disk = C.DISK_INNER_SECTORS + C.DISK_OUTER_SECTORS
    r = np.hypot(x, y)
    for l in range(4, 10):
        sel = layer == l
        inner = r[sel] < C.DISK_RING_SPLIT
        ns = np.where(inner, C.DISK_INNER_SECTORS, C.DISK_OUTER_SECTORS)
        sec = np.minimum((u[sel] * ns).astype(np.int64), ns - 1)
        out[sel] = base + np.where(inner, sec, C.DISK_INNER_SECTORS + sec)
        base += per_disk
    assert base == C.N_MODULES
    return out.astype(np.int16)


def _crossings(kappa, phi0, d0, cot, z0, s_v, disks):
    """Arc lengths of every layer crossing, shape [T, 10] (nan = no crossing)."""
    T = kappa.shape[0]
    S = np.full((T, C.N_LAYERS), np.nan)
    for l in range(4):
        s = _barrel_s(kappa, d0, C.BARREL_R[l])
        z = z0 + s * cot
        ok = (s > s_v) & (np.abs(z) <= C.BARREL_HALF_Z)
        S[:, l] = np.where(ok, s, np.nan)
    if disks:
        with np.errstate(divide="ignore", invalid="ignore"):
            for l in range(4, 10):
                zd = C.disk_z(l)
                s = (zd - z0) / cot
                ok = np.isfinite(s) & (s > s_v) & (np.abs(kappa) * s < np.pi)
                x, y = helix_xy(kappa, phi0, d0, np.where(ok, s, 0.0))
                r = np.hypot(x, y)
                ok &= (r >= C.DISK_RMIN) & (r <= C.DISK_RMAX)
                S[:, l] = np.where(ok, s, np.nan)
    return S


def _smear(rng, layer, x, y, z, sig):
    """Gaussian measurement error: barrel along phi and z, disks along phi and r."""
    r = np.hypot(x, y)
    phi = np.arctan2(y, x)
    barrel = layer < 4
    phi = phi + rng.normal(0.0, sig["sigma_rphi"], size=r.shape) / r
    dr = rng.normal(0.0, sig["sigma_r"], size=r.shape)
    dz = rng.normal(0.0, sig["sigma_z"], size=r.shape)
    r = np.where(barrel, r, r + dr)
    z = np.where(barrel, z + dz, z)
    return r * np.cos(phi), r * np.sin(phi), z


_SIGMAS = {"sigma_rphi": 10e-4, "sigma_z": 20e-4, "sigma_r": 20e-4}


def _noise(rng, n, disks):
    """Uniform noise hits: layer chosen in proportion to its area."""
    areas = [2 * np.pi * C.BARREL_R[l] * 2 * C.BARREL_HALF_Z for l in range(4)]
    if disks:
        areas += [np.pi * (C.DISK_RMAX ** 2 - C.DISK_RMIN ** 2)] * 6
    areas = np.array(areas)
    layer = rng.choice(len(areas), size=n, p=areas / areas.sum())
    phi = rng.uniform(-np.pi, np.pi, size=n)
    u = rng.uniform(0.0, 1.0, size=n)
    r = np.empty(n)
    z = np.empty(n)
    b = layer < 4
    r[b] = np.array(C.BARREL_R)[layer[b]]
    z[b] = (2 * u[b] - 1) * C.BARREL_HALF_Z
    d = ~b
    r[d] = np.sqrt(C.DISK_RMIN ** 2 + u[d] * (C.DISK_RMAX ** 2 - C.DISK_RMIN ** 2))
    z[d] = np.array([C.disk_z(l) for l in range(4, 10)])[layer[d] - 4]
    return layer.astype(np.uint8), r * np.cos(phi), r * np.sin(phi), z


# ----------------------------------------------------------------------------
# tracks

def draw_tracks(rng, n, *, pt="power", eta_max=2.5, z_sigma=3.5, xy_sigma=1.5e-3,
                vertex_z=None, bfield=3.8):
    """Kinematics of n charged particles and their perigee parameters."""
    if pt == "power":           # dN/dpT ~ pT^-3 above 0.3 GeV
        u = rng.uniform(0.0, 1.0, size=n)
        pts = 0.3 / np.sqrt(1.0 - u)
    elif pt == "loguniform":    # 0.5 - 10 GeV
        pts = np.exp(rng.uniform(np.log(0.5), np.log(10.0), size=n))
    else:
        raise ValueError(pt)
    eta = rng.uniform(-eta_max, eta_max, size=n)
    phi_v = rng.uniform(-np.pi, np.pi, size=n)
    q = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    if vertex_z is None:
        vz = rng.normal(0.0, z_sigma, size=n)
    else:
        vz = np.asarray(vertex_z, dtype=np.float64)
    vx = rng.normal(0.0, xy_sigma, size=n) if xy_sigma > 0 else np.zeros(n)
    vy = rng.normal(0.0, xy_sigma, size=n) if xy_sigma > 0 else np.zeros(n)
    kappa = -q * C.K_CURV * bfield / pts
    cot = np.sinh(eta)
    phi0, d0, z0, s_v = perigee_from_vertex(vx, vy, vz, phi_v, kappa, cot)
    return {"kappa": kappa, "phi0": phi0, "cot": cot, "d0": d0, "z0": z0, "s_v": s_v,
            "pt": pts, "eta": eta, "q": q, "vx": vx, "vy": vy, "vz": vz}


OVERLAP_DR = 0.35   # barrel: radial offset of an overlapping ladder (cm)
OVERLAP_DZ = 0.5    # disks: offset in |z| of an overlapping blade (cm)


def track_hits(rng, trk, *, disks=True, eff=1.0, smear=True, overlap=0.0):
    """Layer crossings of each track, ordered by arc length.

    overlap: probability that a crossing also leaves a second hit on the same
    layer, as where modules overlap (section 3.1 and the Fishbone of section
    3.3): a barrel ladder OVERLAP_DR further out, a disk blade OVERLAP_DZ
    further from z = 0.
    Returns (track index, layer, x, y, z, s) arrays over all kept crossings.
    """
    S = _crossings(trk["kappa"], trk["phi0"], trk["d0"], trk["cot"], trk["z0"], trk["s_v"], disks)
    if eff < 1.0:
        S = np.where(rng.uniform(size=S.shape) < eff, S, np.nan)
    ti, li = np.nonzero(np.isfinite(S))
    s = S[ti, li]
    r_nom = np.array(C.BARREL_R + (0,) * 6)[li]
    if overlap > 0.0:
        pick = rng.uniform(size=ti.shape[0]) < overlap
        t2, l2 = ti[pick], li[pick]
        bar2 = l2 < 4
        s2 = np.full(t2.shape[0], np.nan)
        rb = np.array(C.BARREL_R + (0,) * 6)[l2] + OVERLAP_DR
        sb = _barrel_s(trk["kappa"][t2], trk["d0"][t2], np.where(bar2, rb, 1.0))
        zb = trk["z0"][t2] + sb * trk["cot"][t2]
        s2 = np.where(bar2 & (np.abs(zb) <= C.BARREL_HALF_Z), sb, s2)
        with np.errstate(divide="ignore", invalid="ignore"):
            zd = np.array([0.0] * 4 + [C.disk_z(l) for l in range(4, 10)])[l2]
            sd = (zd + OVERLAP_DZ * np.sign(zd) - trk["z0"][t2]) / trk["cot"][t2]
            xd, yd = helix_xy(trk["kappa"][t2], trk["phi0"][t2], trk["d0"][t2], np.where(np.isfinite(sd), sd, 0.0))
            rd = np.hypot(xd, yd)
            okd = ~bar2 & np.isfinite(sd) & (sd > s[pick]) & (rd >= C.DISK_RMIN) & (rd <= C.DISK_RMAX)
        s2 = np.where(okd, sd, s2)
        keep2 = np.isfinite(s2)
        ti = np.concatenate([ti, t2[keep2]])
        li = np.concatenate([li, l2[keep2]])
        s = np.concatenate([s, s2[keep2]])
        r_nom = np.concatenate([r_nom, np.where(bar2, rb, 0.0)[keep2]])
    order = np.lexsort((s, ti))
    ti, li, s, r_nom = ti[order], li[order], s[order], r_nom[order]
    x, y = helix_xy(trk["kappa"][ti], trk["phi0"][ti], trk["d0"][ti], s)
    z = trk["z0"][ti] + s * trk["cot"][ti]
    bar = li < 4
    # put barrel hits exactly on their cylinder before smearing
    rr = np.hypot(x, y)
    x = np.where(bar, x * r_nom / np.where(bar, rr, 1.0), x)
    y = np.where(bar, y * r_nom / np.where(bar, rr, 1.0), y)
    if smear:
        x, y, z = _smear(rng, li, x, y, z, _SIGMAS)
    return ti, li.astype(np.uint8), x, y, z, s


def _truth_dict(trk):
    return {k: trk[k] for k in ("kappa", "phi0", "cot", "d0", "z0", "pt", "eta", "q", "vz")}


def make_event(rng, *, n_vertices=50, tracks_per_vertex=30.0, pt="power", eta_max=2.5,
               disks=True, eff=0.99, noise_frac=0.10, dtype=np.float32, fixed_tracks=None,
               xy_sigma=1.5e-3, shuffle=True, overlap=0.0):
    """One event: n_vertices vertices with Poisson(tracks_per_vertex) tracks each."""
    if fixed_tracks is not None:
        counts = np.array([fixed_tracks] * n_vertices)
    else:
        counts = rng.poisson(tracks_per_vertex, size=n_vertices)
    vz_each = rng.normal(0.0, 3.5, size=n_vertices)
    vz = np.repeat(vz_each, counts)
    n = int(counts.sum())
    trk = draw_tracks(rng, n, pt=pt, eta_max=eta_max, vertex_z=vz, xy_sigma=xy_sigma)
    ti, li, x, y, z, _ = track_hits(rng, trk, disks=disks, eff=eff, overlap=overlap)
    n_noise = int(round(noise_frac * ti.shape[0]))
    if n_noise:
        nl, nx, ny, nz = _noise(rng, n_noise, disks)
        li = np.concatenate([li, nl])
        x, y, z = np.concatenate([x, nx]), np.concatenate([y, ny]), np.concatenate([z, nz])
        ti = np.concatenate([ti, np.full(n_noise, -1)])
    if shuffle:
        perm = rng.permutation(li.shape[0])
        li, x, y, z, ti = li[perm], x[perm], y[perm], z[perm], ti[perm]
    x, y, z = x.astype(dtype), y.astype(dtype), z.astype(dtype)
    mod = module_id(li, x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))
    return Hits(x, y, z, li, mod, ti.astype(np.int32),
                np.array([0, li.shape[0]], dtype=np.int32), [_truth_dict(trk)])


def concat(events: list[Hits]) -> Hits:
    off = np.zeros(len(events) + 1, dtype=np.int32)
    off[1:] = np.cumsum([e.n_hits for e in events])
    cat = lambda a: np.concatenate([getattr(e, a) for e in events])
    return Hits(cat("x"), cat("y"), cat("z"), cat("layer"), cat("module"), cat("track"), off,
                [t for e in events for t in e.truth])


def make_batch(seed, n_events, *, pileup, **kw):
    """Independent events from SeedSequence(seed).spawn(n_events).

    pileup: an int (vertices per event) or a (lo, hi) pair for a per-event
    uniform integer choice.
    """
    children = np.random.SeedSequence(seed).spawn(n_events)
    events = []
    for ss in children:
        rng = np.random.Generator(np.random.PCG64(ss))
        if isinstance(pileup, tuple):
            nv = int(rng.integers(pileup[0], pileup[1] + 1))
        else:
            nv = int(pileup)
        events.append(make_event(rng, n_vertices=nv, **kw))
    return concat(events)


# ----------------------------------------------------------------------------
# the five workloads

def config1(seed=1):
    """Barrel only, one vertex, 20 tracks, FP64 hits, no noise, full efficiency."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_event(rng, n_vertices=1, fixed_tracks=20, pt="loguniform", eta_max=1.5,
                      disks=False, eff=1.0, noise_frac=0.0, dtype=np.float64, xy_sigma=0.0)


def config2(seed=2):
    """PU-50-like event, full geometry, FP32 hits."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_event(rng, n_vertices=50, tracks_per_vertex=30.0, eff=0.99, noise_frac=0.10)


def config3(seed=3, n_events=256):
    """Uneven batch: pileup uniform in [20, 200] per event."""
    return make_batch(seed, n_events, pileup=(20, 200), tracks_per_vertex=30.0, eff=0.99,
                      noise_frac=0.10)


def overlap_event(seed=6, n_vertices=50, overlap=0.25):
    """A PU50-like event in the overlap-geometry variant: a quarter of the
    layer crossings leave a second hit on the same layer (overlapping
    modules), the situation the Fishbone of section 3.3 resolves."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return make_event(rng, n_vertices=n_vertices, tracks_per_vertex=30.0, eff=0.99, noise_frac=0.10,
                      overlap=overlap)


def overlap_batch(seed=6, n_events=64, pileup=50, overlap=0.25):
    """Events of the overlap-geometry variant, batched."""
    return make_batch(seed, n_events, pileup=pileup, tracks_per_vertex=30.0, eff=0.99, noise_frac=0.10,
                      overlap=overlap)


def config5(seed=5, n_events=64):
    """HL-LHC scale: PU 200, Poisson(35) tracks per vertex, 15% noise."""
    return make_batch(seed, n_events, pileup=200, tracks_per_vertex=35.0, eff=0.99,
                      noise_frac=0.15)


def config4(seed=4, n_tracks=1_000_000, frac=(0.5, 0.3, 0.2), dtype=np.float32):
    """Tracks for the fit: hits in track order, 4/5/6-hit classes.

    The barrel+disk geometry gives no natural 6-hit tracks at useful rates, so
    the 6-hit class is a 5-hit track plus a second hit on its first disk
    0.5 cm further out in |z| (a blade overlap, paper section 3.1), on the
    neighbouring module.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    want = [int(round(f * n_tracks)) for f in frac]
    want[0] = n_tracks - want[1] - want[2]
    got = {4: [], 5: [], 6: []}
    have = {4: 0, 5: 0, 6: 0}
    target = {4: want[0], 5: want[1], 6: want[2]}
    while any(have[k] < target[k] for k in got):
        chunk = 400_000
        trk = draw_tracks(rng, chunk, pt="power", eta_max=2.5)
        S = _crossings(trk["kappa"], trk["phi0"], trk["d0"], trk["cot"], trk["z0"], trk["s_v"], True)
        S = np.where(rng.uniform(size=S.shape) < 0.99, S, np.nan)
        nh = np.isfinite(S).sum(axis=1)
        for cls, src in ((4, 4), (5, 5), (6, 5)):
            need = target[cls] - have[cls]
            if need <= 0:
                continue
            idx = np.nonzero(nh == src)[0]
            if cls == 5:
                idx = idx[: len(idx) // 2]     # leave some 5-hit tracks for the 6-hit class
            elif cls == 6:
                idx = idx[len(idx) // 2:]
            idx = idx[:need]
            got[cls].append((trk, S, idx))
            have[cls] += len(idx)
            nh[idx] = -1
    xs, ys, zs, ls, ts, tup_n, params = [], [], [], [], [], [], []
    base = 0
    for cls in (4, 5, 6):
        for trk, S, idx in got[cls]:
            if len(idx) == 0:
                continue
            sub = {k: v[idx] for k, v in trk.items()}
            Ssub = S[idx]
            if cls == 6:
                # overlap hit on the first disk crossed, 0.5 cm further from z=0
                first_disk = np.argmax(np.isfinite(Ssub[:, 4:]), axis=1) + 4
                zd = np.array([C.disk_z(l) for l in range(4, 10)])[first_disk - 4]
                zo = zd + 0.5 * np.sign(zd)
                so = (zo - sub["z0"]) / sub["cot"]
                extra = np.full((len(idx), 1), np.nan)
                extra[:, 0] = so
                Sfull = np.concatenate([Ssub, extra], axis=1)
                lay = np.concatenate([np.tile(np.arange(10), (len(idx), 1)), first_disk[:, None]], axis=1)
            else:
                Sfull = Ssub
                lay = np.tile(np.arange(10), (len(idx), 1))
            ti, col = np.nonzero(np.isfinite(Sfull))
            s = Sfull[ti, col]
            order = np.lexsort((s, ti))
            ti, col, s = ti[order], col[order], s[order]
            li = lay[ti, col]
            x, y = helix_xy(sub["kappa"][ti], sub["phi0"][ti], sub["d0"][ti], s)
            z = sub["z0"][ti] + s * sub["cot"][ti]
            bar = li < 4
            r_nom = np.array(C.BARREL_R + (0,) * 6)[li]
            rr = np.hypot(x, y)
            x = np.where(bar, x * r_nom / np.where(bar, rr, 1.0), x)
            y = np.where(bar, y * r_nom / np.where(bar, rr, 1.0), y)
            x, y, z = _smear(rng, li, x, y, z, _SIGMAS)
            counts = np.bincount(ti, minlength=len(idx))
            assert np.all(counts == cls), (cls, np.unique(counts))
            xs.append(x); ys.append(y); zs.append(z); ls.append(li)
            ts.append(ti + base)
            tup_n.append(np.full(len(idx), cls))
            params.append(np.stack([sub["kappa"], sub["phi0"], sub["cot"], sub["d0"], sub["z0"]], axis=1))
            base += len(idx)
    x = np.concatenate(xs).astype(dtype)
    y = np.concatenate(ys).astype(dtype)
    z = np.concatenate(zs).astype(dtype)
    li = np.concatenate(ls).astype(np.uint8)
    nh = np.concatenate(tup_n).astype(np.uint8)
    mod = module_id(li, x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))
    # overlap hits sit on the neighbouring module of the same disk ring
    is_dup = np.zeros(li.shape[0], dtype=bool)
    starts = np.zeros(nh.shape[0] + 1, dtype=np.int64)
    starts[1:] = np.cumsum(nh)
    six = np.nonzero(nh == 6)[0]
    if six.size:
        # within a 6-hit track the overlap hit is the one whose layer repeats the previous hit's
        cand = starts[six][:, None] + np.arange(6)[None, :]
        lay6 = li[cand]
        rep = np.zeros_like(lay6, dtype=bool)
        rep[:, 1:] = lay6[:, 1:] == lay6[:, :-1]
        is_dup[cand[rep]] = True
    per_disk = C.DISK_INNER_SECTORS + C.DISK_OUTER_SECTORS
    m = mod.astype(np.int64)
    dup = np.nonzero(is_dup)[0]
    disk_base = 1184 + (li[dup].astype(np.int64) - 4) * per_disk
    local = m[dup] - disk_base
    inner = local < C.DISK_INNER_SECTORS
    nsec = np.where(inner, C.DISK_INNER_SECTORS, C.DISK_OUTER_SECTORS)
    sec = np.where(inner, local, local - C.DISK_INNER_SECTORS)
    sec = (sec + 1) % nsec
    m[dup] = disk_base + np.where(inner, sec, C.DISK_INNER_SECTORS + sec)
    mod = m.astype(np.int16)
    n_tracks_total = nh.shape[0]
    tuplets = np.full((n_tracks_total, 8), -1, dtype=np.int32)
    for k in range(6):
        sel = nh > k
        tuplets[sel, k] = (starts[:-1][sel] + k).astype(np.int32)
    hits = Hits(x, y, z, li, mod, np.repeat(np.arange(n_tracks_total, dtype=np.int32), nh),
                np.array([0, x.shape[0]], dtype=np.int32), [])
    return TrackSet(hits, tuplets, nh, np.concatenate(params))


def module_offsets(seed=4, sigma=10e-4, n_modules=C.N_MODULES):
    """Per-module alignment translations ~ N(0, 10 um), float32 [n_modules, 3]."""
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    return rng.normal(0.0, sigma, size=(n_modules, 3)).astype(np.float32)


def cotangents(seed, n_tracks):
    """Upstream gradients for the fit adjoint: g_params [n, 5], g_chi2 [n] ~ N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64([seed, 2]))
    return (rng.normal(size=(n_tracks, 5)).astype(np.float32),
            rng.normal(size=n_tracks).astype(np.float32))


def track_hits_ms(rng, trk, *, x_over_x0=0.015, highland=(0.0136, 0.038), disks=True,
                  smear=True, bfield=3.8, scatter_first=True):
    """Layer crossings of tracks that scatter in the material of every layer.

    Piecewise helices: at each crossing the 3D direction is deflected by two
    independent Gaussian angles of width theta0 (Highland, with the material
    x/X0 times the path length through the layer: 1/sin(theta) for a barrel
    cylinder, 1/|cos(theta)| for a disk) and the next crossing is found from
    the deflected helix.  The momentum is unchanged (no energy loss).  With
    scatter_first=False the first crossing of each track deflects nothing, so
    that the generating perigee parameters describe the track up to its
    second hit.
    Returns (track index, layer, x, y, z) of all crossings ordered per track.
    """
    T = trk["kappa"].shape[0]
    q = -np.sign(trk["kappa"])
    p = trk["pt"] * np.sqrt(1.0 + trk["cot"] ** 2)
    # current state: point, transverse direction, cot(theta), curvature
    px, py, pz = trk["vx"].copy(), trk["vy"].copy(), trk["vz"].copy()
    kappa, cot = trk["kappa"].copy(), trk["cot"].copy()
    phi0, d0, z0, s_cur = trk["phi0"].copy(), trk["d0"].copy(), trk["z0"].copy(), trk["s_v"].copy()
    crossed = np.zeros((T, C.N_LAYERS), bool)
    active = np.ones(T, bool)
    n_crossed = np.zeros(T, np.int64)
    out_t, out_l, out_x, out_y, out_z = [], [], [], [], []
    for _ in range(C.N_LAYERS):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        S = _crossings(kappa[idx], phi0[idx], d0[idx], cot[idx], z0[idx], s_cur[idx] + 1e-7, disks)
        S[crossed[idx]] = np.nan
        has = np.isfinite(S).any(axis=1)
        active[idx[~has]] = False
        idx, S = idx[has], S[has]
        if idx.size == 0:
            break
        lay = np.nanargmin(S, axis=1)
        s = S[np.arange(idx.size), lay]
        x, y = helix_xy(kappa[idx], phi0[idx], d0[idx], s)
        z = z0[idx] + s * cot[idx]
        crossed[idx, lay] = True
        out_t.append(idx); out_l.append(lay); out_x.append(x); out_y.append(y); out_z.append(z)
        # direction at the crossing, then the deflection
        phi = phi0[idx] + kappa[idx] * s
        sin_t = 1.0 / np.sqrt(1.0 + cot[idx] ** 2)
        cos_t = cot[idx] * sin_t
        barrel = lay < 4
        path = np.where(barrel, 1.0 / sin_t, 1.0 / np.maximum(np.abs(cos_t), 1e-6))
        X = x_over_x0 * path
        th0 = highland[0] / p[idx] * np.sqrt(X) * (1.0 + highland[1] * np.log(X))
        if not scatter_first:
            th0 = np.where(n_crossed[idx] == 0, 0.0, th0)
        n_crossed[idx] += 1
        a1 = rng.normal(size=idx.size) * th0
        a2 = rng.normal(size=idx.size) * th0
        d = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], 1)
        e1 = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], 1)
        e2 = np.stack([cos_t * np.cos(phi), cos_t * np.sin(phi), -sin_t], 1)
        dn = d + a1[:, None] * e1 + a2[:, None] * e2
        dn /= np.linalg.norm(dn, axis=1, keepdims=True)
        phi_new = np.arctan2(dn[:, 1], dn[:, 0])
        cot_new = dn[:, 2] / np.hypot(dn[:, 0], dn[:, 1])
        pt_new = p[idx] / np.sqrt(1.0 + cot_new ** 2)
        kap_new = -q[idx] * C.K_CURV * bfield / pt_new
        f0, dd, zz, sv = perigee_from_vertex(x, y, z, phi_new, kap_new, cot_new)
        kappa[idx], cot[idx], phi0[idx], d0[idx], z0[idx], s_cur[idx] = kap_new, cot_new, f0, dd, zz, sv
    ti = np.concatenate(out_t) if out_t else np.zeros(0, np.int64)
    li = np.concatenate(out_l).astype(np.uint8) if out_l else np.zeros(0, np.uint8)
    x = np.concatenate(out_x) if out_x else np.zeros(0)
    y = np.concatenate(out_y) if out_y else np.zeros(0)
    z = np.concatenate(out_z) if out_z else np.zeros(0)
    order = np.argsort(ti, kind="stable")
    ti, li, x, y, z = ti[order], li[order], x[order], y[order], z[order]
    bar = li < 4
    r_nom = np.array(C.BARREL_R + (0,) * 6)[li]
    rr = np.hypot(x, y)
    x = np.where(bar, x * r_nom / np.where(bar, rr, 1.0), x)
    y = np.where(bar, y * r_nom / np.where(bar, rr, 1.0), y)
    if smear:
        x, y, z = _smear(rng, li, x, y, z, _SIGMAS)
    return ti, li, x, y, z


def cylinder_tracks(seed, n_tracks, radii, dtype=np.float32, eta_max=1.0):
    """Tracks crossing concentric cylinders at the given radii, hits in track
    order: fit rows with any number of hits (3 to 8), all on barrel-like
    surfaces (layer ids 0..3, the later cylinders labelled 3), smeared like
    barrel hits.  Tracks that do not reach the last radius are dropped."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    radii = np.asarray(radii, np.float64)
    n = len(radii)
    out = []
    have = 0
    while have < n_tracks:
        trk = draw_tracks(rng, 2 * n_tracks, pt="power", eta_max=eta_max)
        S = np.stack([_barrel_s(trk["kappa"], trk["d0"], R) for R in radii], axis=1)
        ok = np.all(np.isfinite(S), axis=1) & np.all(np.diff(S, axis=1) > 0, axis=1)
        idx = np.nonzero(ok)[0][: n_tracks - have]
        out.append(({k: v[idx] for k, v in trk.items()}, S[idx]))
        have += len(idx)
    sub = {k: np.concatenate([o[0][k] for o in out]) for k in out[0][0]}
    S = np.concatenate([o[1] for o in out])
    ti = np.repeat(np.arange(n_tracks), n)
    s = S.reshape(-1)
    li = np.tile(np.minimum(np.arange(n), 3), n_tracks).astype(np.uint8)
    x, y = helix_xy(sub["kappa"][ti], sub["phi0"][ti], sub["d0"][ti], s)
    z = sub["z0"][ti] + s * sub["cot"][ti]
    r_nom = np.tile(radii, n_tracks)
    rr = np.hypot(x, y)
    x, y = x * r_nom / rr, y * r_nom / rr
    x, y, z = _smear(rng, li, x, y, z, _SIGMAS)
    x, y, z = x.astype(dtype), y.astype(dtype), z.astype(dtype)
    mod = module_id(li, x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))
    tuplets = np.full((n_tracks, 8), -1, dtype=np.int32)
    tuplets[:, :n] = np.arange(n_tracks * n, dtype=np.int32).reshape(n_tracks, n)
    hits = Hits(x, y, z, li, mod, ti.astype(np.int32), np.array([0, x.shape[0]], dtype=np.int32), [])
    params = np.stack([sub["kappa"], sub["phi0"], sub["cot"], sub["d0"], sub["z0"]], axis=1)
    return TrackSet(hits, tuplets, np.full(n_tracks, n, np.uint8), params)
