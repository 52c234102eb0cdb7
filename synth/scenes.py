"""Scene generators (geometry only).

Units are micrometres throughout.  Seeds follow ``20251010 + 1000*config + k``.

Reading of the offset: the activation distance of a same-material pair is the
full thickness h (two half-thickness offsets, Sec. 3), and the biphasic split
a = eta + dhat of Sec. 3.3 then gives eta = h - dhat.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

BASE_SEED = 20251010


@dataclass
class Scene:
    """One mesh (possibly several connected components) and its deformed pose.

    kind   'rod' (polylines; contact pairs are edge-edge only) or 'shell'
           (triangle mesh; point-triangle and edge-edge pairs).
    x      float64 [V,3] deformed positions.
    edges  int32 [E,2].
    tris   int32 [F,3] (empty for rods).
    ref    rest-space parameters: rods float64 [V] arc length along the
           polyline; shells float64 [V,2] rest 2D coordinates.
    h      thickness (activation distance of unfiltered pairs).
    eta    biphasic offset (core thickness) of unfiltered pairs.
    """
    name: str
    kind: str
    x: np.ndarray
    edges: np.ndarray
    tris: np.ndarray
    ref: np.ndarray
    h: float
    eta: float
    kappa: float = 1.0
    seed: int = 0
    meta: dict = field(default_factory=dict)
    # reference distance: 0 in rest-space parameters (ref), 1 Euclidean at
    # the rest pose xrest [V,3] (the literal reading of Eq. 1 on the rest
    # configuration)
    refdist: int = 0
    xrest: np.ndarray | None = None

    @property
    def n_verts(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_prims(self) -> int:
        """Primitive count: edges for rods; points + edges + triangles for shells."""
        if self.kind == "rod":
            return self.n_edges
        return self.n_verts + self.n_edges + self.n_tris

    def with_positions(self, x: np.ndarray) -> "Scene":
        s = Scene(self.name, self.kind, np.ascontiguousarray(x, dtype=np.float64),
                  self.edges, self.tris, self.ref, self.h, self.eta, self.kappa,
                  self.seed, dict(self.meta), self.refdist, self.xrest)
        return s

    def with_euclid_rest(self, xrest: np.ndarray | None = None) -> "Scene":
        """The same scene under the Euclidean reading of the reference
        distance, with rest pose xrest (default: the scene's own positions)."""
        xr = np.ascontiguousarray(self.x if xrest is None else xrest, dtype=np.float64).copy()
        return Scene(self.name + "_euclid", self.kind, self.x, self.edges, self.tris, self.ref, self.h, self.eta,
                     self.kappa, self.seed, dict(self.meta), 1, xr)


def _smoothstep(t):
    t = np.clip(t, 0.0, 1.0)
    return t * t * (3.0 - 2.0 * t)


def _truncnormal(rng, sigma, clip, shape):
    """Normal(0, sigma) truncated to |v| <= clip*sigma by redrawing."""
    v = rng.normal(0.0, sigma, size=shape)
    bad = np.abs(v) > clip * sigma
    while bad.any():
        v[bad] = rng.normal(0.0, sigma, size=int(bad.sum()))
        bad = np.abs(v) > clip * sigma
    return v


# ----------------------------------------------------------------------------
# Config 0: a single open rod that winds as a helix and then loops back around
# itself (the paper's loop test has the same structure: one yarn, segments
# shorter than the thickness).
# ----------------------------------------------------------------------------

def _resample_by_chord(curve, t0, n_pts, ell, dt_max):
    """Walk along ``curve(t)`` placing points whose successive chords equal ell.

    Each new parameter is found by bisection on [t, t + dt_max] (the chord is
    monotone there for the gentle curves used here), to |chord - ell| < 1e-9.
    """
    pts = [curve(t0)]
    t = t0
    for _ in range(n_pts - 1):
        p = pts[-1]
        lo, hi = t, t + dt_max
        if np.linalg.norm(curve(hi) - p) <= ell:
            raise RuntimeError("chord bracket too small")
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            c = np.linalg.norm(curve(mid) - p)
            if abs(c - ell) < 1e-10:
                lo = hi = mid
                break
            if c < ell:
                lo = mid
            else:
                hi = mid
        t = 0.5 * (lo + hi)
        q = curve(t)
        if abs(np.linalg.norm(q - p) - ell) >= 1e-9:
            raise RuntimeError("chord bisection did not converge")
        pts.append(q)
    return np.array(pts, dtype=np.float64)


def helix_loop_rod(seed: int = BASE_SEED + 0, n_verts: int = 200, ell: float = 50.0,
                   radius: float = 500.0, pitch: float = 195.0, outer_gap: float = 197.0,
                   outer_pitch: float = 600.0, inner_turns: float = 1.5,
                   h: float = 200.0, dhat: float = 10.0) -> Scene:
    """Open polyline: ``inner_turns`` of an ascending helix (radius 500, pitch 195,
    so successive turns sit inside the active band (h - dhat, h)), a half-turn
    spiral out to radius 500 + 197 that turns the climb into a descent, then a
    descending outer helix that passes over the inner turns at radial gap 197.

    Chords are resampled to exactly ell (bisection); rest arc length s_k = ell*k.
    The seed draws the initial phase only, so distances do not depend on it.
    """
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    th1 = 2.0 * math.pi * inner_turns
    a = pitch / (2.0 * math.pi)
    b = -outer_pitch / (2.0 * math.pi)
    z1 = a * th1
    zh = z1 + a * math.pi * 0.5
    z2 = zh + a * math.pi * 0.5 + (b - a) * math.pi * 0.25

    def curve(th):
        # inner helix; then half a turn of spiral: the radius grows to
        # radius + outer_gap over the first quarter turn while still climbing,
        # and the climb blends into a descent over the second quarter turn;
        # then the descending outer helix.
        if th <= th1:
            r, z = radius, a * th
        elif th <= th1 + math.pi:
            t = (th - th1) / math.pi
            r = radius + outer_gap * float(_smoothstep(2.0 * t))
            if t <= 0.5:
                z = z1 + a * math.pi * t
            else:
                u = 2.0 * t - 1.0
                z = zh + a * math.pi * (t - 0.5) + (b - a) * math.pi * 0.5 * (u ** 3 - 0.5 * u ** 4)
        else:
            r, z = radius + outer_gap, z2 + b * (th - th1 - math.pi)
        ang = phi0 + th
        return np.array([r * math.cos(ang), r * math.sin(ang), z])

    x = _resample_by_chord(curve, 0.0, n_verts, ell, dt_max=2.0 * ell / radius)
    edges = np.stack([np.arange(n_verts - 1), np.arange(1, n_verts)], 1).astype(np.int32)
    s = ell * np.arange(n_verts, dtype=np.float64)
    return Scene("helix_loop_rod", "rod", x, edges, np.zeros((0, 3), np.int32), s,
                 h=float(h), eta=float(h - dhat), seed=seed,
                 meta=dict(ell=ell, radius=radius, pitch=pitch, outer_gap=outer_gap))


# ----------------------------------------------------------------------------
# Config 1: woven yarn patch (warp along x, weft along y), graded segments.
# ----------------------------------------------------------------------------

def graded_period(lmin: int = 20, lmax: int = 300, n: int = 16) -> np.ndarray:
    """Symmetric integer geometric ramp lmin -> lmax -> lmin over n edges."""
    half = n // 2
    q = (lmax / lmin) ** (1.0 / (half - 1))
    up = [int(round(lmin * q ** k)) for k in range(half)]
    up[-1] = lmax
    return np.array(up + up[::-1], dtype=np.int64)


def woven_patch(seed: int = BASE_SEED + 1000, n_warp: int = 32, n_weft: int = 32,
                verts_per_rod: int = 512, lmin: int = 20, lmax: int = 300,
                separation: float = 294.0, jitter: float = 5.0, jitter_clip: float = 2.0,
                h: float = 300.0, dhat: float = 30.0) -> Scene:
    """Plain weave: warp rod j runs along x at y = j*S, weft rod i along y at x = i*S,
    with sinusoidal over/under heights z = +-A cos(pi s / S + pi k) so that every
    crossing has centreline separation 2A = ``separation``.  S is one grading
    period (16 segments, 20 -> 300 -> 20 um), so the shortest segments sit at the
    crossings.  Rest arc length s is an exact integer sum of segment lengths;
    the 3D pose follows x = s along the rod plus the height wave, then every
    coordinate gets truncated-normal jitter N(0, 5 um) (|v| <= 2 sigma).
    """
    rng = np.random.default_rng(seed)
    per = graded_period(lmin, lmax)
    S = float(per.sum())
    A = 0.5 * separation
    nseg = verts_per_rod - 1
    seg = np.resize(per, nseg).astype(np.float64)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    xs, refs, edges = [], [], []
    base = 0
    for j in range(n_warp):
        p = np.stack([s, np.full_like(s, j * S), A * np.cos(math.pi * s / S + math.pi * j)], 1)
        xs.append(p)
        refs.append(s.copy())
        edges.append(np.stack([np.arange(nseg), np.arange(1, nseg + 1)], 1) + base)
        base += verts_per_rod
    for i in range(n_weft):
        p = np.stack([np.full_like(s, i * S), s, -A * np.cos(math.pi * s / S + math.pi * i)], 1)
        xs.append(p)
        refs.append(s.copy())
        edges.append(np.stack([np.arange(nseg), np.arange(1, nseg + 1)], 1) + base)
        base += verts_per_rod
    x = np.concatenate(xs, 0)
    x = x + _truncnormal(rng, jitter, jitter_clip, x.shape)
    return Scene("woven_patch", "rod", np.ascontiguousarray(x),
                 np.concatenate(edges, 0).astype(np.int32), np.zeros((0, 3), np.int32),
                 np.concatenate(refs, 0), h=float(h), eta=float(h - dhat), seed=seed,
                 meta=dict(period=S, lmin=lmin, lmax=lmax, separation=separation,
                           n_warp=n_warp, n_weft=n_weft, verts_per_rod=verts_per_rod))


# ----------------------------------------------------------------------------
# Config 2: thick shell cloth -- regular grid, sinusoid height field, and
# pleats (Z-folds) that bring layers to a gap inside the active band.
# ----------------------------------------------------------------------------

class _Turtle:
    """Unit-speed planar profile (X, Z) made of straight and circular pieces."""

    def __init__(self):
        self.pieces = []   # (s0, length, kind, data)
        self.pos = np.zeros(2)
        self.heading = 0.0
        self.s = 0.0

    def line(self, length):
        self.pieces.append((self.s, length, "line", (self.pos.copy(), self.heading)))
        d = np.array([math.cos(self.heading), math.sin(self.heading)])
        self.pos = self.pos + length * d
        self.s += length

    def arc(self, radius, turn):
        """Turn by ``turn`` radians (positive = counter-clockwise) on a circle."""
        sgn = 1.0 if turn > 0 else -1.0
        nrm = self.heading + sgn * 0.5 * math.pi
        center = self.pos + radius * np.array([math.cos(nrm), math.sin(nrm)])
        length = radius * abs(turn)
        self.pieces.append((self.s, length, "arc", (center, radius, self.heading, sgn)))
        self.heading += turn
        ang = self.heading - sgn * 0.5 * math.pi
        self.pos = center + radius * np.array([math.cos(ang), math.sin(ang)])
        self.s += length

    def eval(self, s):
        s = np.asarray(s, dtype=np.float64)
        out = np.zeros(s.shape + (2,))
        starts = np.array([p[0] for p in self.pieces])
        idx = np.clip(np.searchsorted(starts, s, side="right") - 1, 0, len(self.pieces) - 1)
        for k, (s0, length, kind, data) in enumerate(self.pieces):
            m = idx == k
            if not m.any():
                continue
            t = s[m] - s0
            if kind == "line":
                p0, hd = data
                out[m, 0] = p0[0] + t * math.cos(hd)
                out[m, 1] = p0[1] + t * math.sin(hd)
            else:
                c, r, hd0, sgn = data
                ang = hd0 - sgn * 0.5 * math.pi + sgn * t / r
                out[m, 0] = c[0] + r * np.cos(ang)
                out[m, 1] = c[1] + r * np.sin(ang)
        return out


def _solve_converge_angle(radius, l_conv, gap):
    """Angle theta with radius*(1 + cos theta) - l_conv*tan theta = gap."""
    lo, hi = 0.0, 1.2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = radius * (1.0 + math.cos(mid)) - l_conv * math.tan(mid) - gap
        if f > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def fold_profile(total_len, gaps, radius=750.0, l_mid=6000.0, l_conv=2500.0,
                 margin=1500.0, lead=None):
    """Profile (X(u1), Z(u1)) of a sheet with one Z-fold per entry of ``gaps``.

    Each fold: the lower layer runs flat, dips while it approaches the first
    apex, turns up through a semicircle-like apex of radius 750 (wide enough
    that points 1 mm apart along the sheet stay > 0.9 mm apart in space), runs
    back as a flat middle layer at height +gap, turns up through the second
    apex and returns at +2*gap after a converging leg.  Returns the turtle and
    the list of (u1_start, u1_end) bands where the sheet must stay flat.
    """
    tu = _Turtle()
    bands = []
    seg_lens = []
    for g in gaps:
        th = _solve_converge_angle(radius, l_conv, g)
        rs = radius * math.sin(th)
        bottom = l_mid - l_conv - rs + radius + margin
        top = (l_mid - rs) + radius + margin - l_conv
        seg_lens.append((th, bottom, top))
    fold_len = [b + l_conv / math.cos(th) + 2 * radius * (math.pi + th) + l_mid +
                l_conv / math.cos(th) + t for (th, b, t) in seg_lens]
    free = total_len - sum(fold_len)
    if free < 0:
        raise ValueError("sheet too short for the requested folds")
    gap_len = free / (len(gaps) + 1) if lead is None else None
    for k, g in enumerate(gaps):
        th, bottom, top = seg_lens[k]
        tu.line(gap_len if lead is None else (lead if k == 0 else (free - lead) / len(gaps)))
        u0 = tu.s
        tu.line(bottom)
        tu.heading = -th
        tu.line(l_conv / math.cos(th))
        tu.arc(radius, math.pi + th)
        tu.line(l_mid)
        tu.arc(radius, -(math.pi + th))
        tu.line(l_conv / math.cos(th))
        tu.heading = 0.0
        tu.line(top)
        bands.append((u0, tu.s))
        tu.heading = 0.0
    tu.line(max(total_len - tu.s, 0.0) + 1.0)
    return tu, bands


def folded_cloth(seed: int = BASE_SEED + 2000, n: int = 256, ell: float = 500.0,
                 gaps=(940.0, 960.0, 980.0), n_sines: int = 8, amp=(200.0, 1500.0),
                 wavelength=(15000.0, 60000.0), ramp: float = 4000.0,
                 shear: float = 150.0, shear_len: float = 23000.0,
                 h: float = 1000.0, dhat: float = 100.0, **fold_kw) -> Scene:
    """n x n vertex grid with rest coordinates u = ell*(i, j) (exact integers) and
    one diagonal pattern: 2(n-1)^2 triangles, 3(n-1)^2 + 2(n-1) edges.

    Pose: u1 -> (X, Z) follows the Z-fold profile (gaps inside (h - dhat, h)
    bring layers into the active band), u2 -> Y = u2, and a seeded sum of
    ``n_sines`` plane sinusoids (amplitude U(amp), wavelength log-U(wavelength),
    random direction and phase) is added to Z outside the fold bands with a
    smoothstep ramp of length ``ramp``.  An in-plane shear
    Y = u2 + shear * sin(2 pi u1 / shear_len) keeps the stacked layers of a
    fold from lining up vertex-for-vertex.
    """
    rng = np.random.default_rng(seed)
    total = (n - 1) * ell
    tu, bands = fold_profile(total, list(gaps), **fold_kw)
    i = np.arange(n)
    u1 = ell * i.astype(np.float64)
    prof = tu.eval(u1)
    # weight of the height field: 0 inside fold bands, smoothstep ramp outside
    dist = np.full(n, np.inf)
    for (a, b) in bands:
        d = np.where(u1 < a, a - u1, np.where(u1 > b, u1 - b, 0.0))
        dist = np.minimum(dist, d)
    w = _smoothstep(dist / ramp) if len(bands) else np.ones(n)
    A = rng.uniform(amp[0], amp[1], n_sines)
    lam = np.exp(rng.uniform(math.log(wavelength[0]), math.log(wavelength[1]), n_sines))
    alpha = rng.uniform(0.0, 2.0 * math.pi, n_sines)
    phase = rng.uniform(0.0, 2.0 * math.pi, n_sines)
    U1, U2 = np.meshgrid(u1, ell * np.arange(n, dtype=np.float64), indexing="ij")
    H = np.zeros_like(U1)
    for k in range(n_sines):
        H += A[k] * np.sin(2.0 * math.pi * (math.cos(alpha[k]) * U1 + math.sin(alpha[k]) * U2)
                           / lam[k] + phase[k])
    X = np.broadcast_to(prof[:, 0:1], U1.shape)
    Z = prof[:, 1:2] + w[:, None] * H
    Y = U2 + shear * np.sin(2.0 * math.pi * U1 / shear_len)
    x = np.stack([X, Y, Z], -1).reshape(-1, 3)
    ref = np.stack([U1, U2], -1).reshape(-1, 2)
    # topology: v = i*n + j
    ii, jj = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    v00 = (ii * n + jj).ravel()
    v10 = v00 + n
    v01 = v00 + 1
    v11 = v00 + n + 1
    tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)], 0)
    a_i, a_j = np.meshgrid(np.arange(n - 1), np.arange(n), indexing="ij")
    e_u1 = np.stack([(a_i * n + a_j).ravel(), ((a_i + 1) * n + a_j).ravel()], 1)
    b_i, b_j = np.meshgrid(np.arange(n), np.arange(n - 1), indexing="ij")
    e_u2 = np.stack([(b_i * n + b_j).ravel(), (b_i * n + b_j + 1).ravel()], 1)
    e_d = np.stack([v00, v11], 1)
    edges = np.concatenate([e_u1, e_u2, e_d], 0)
    return Scene("folded_cloth", "shell", np.ascontiguousarray(x, dtype=np.float64),
                 edges.astype(np.int32), tris.astype(np.int32), np.ascontiguousarray(ref),
                 h=float(h), eta=float(h - dhat), seed=seed,
                 meta=dict(n=n, ell=ell, gaps=list(gaps), bands=bands))


# ----------------------------------------------------------------------------
# Configs 3 and 4: many independent scenes of uneven size.
# ----------------------------------------------------------------------------

def _scene_of_size(kind, prims, seed):
    if kind == "rod":
        k = max(1, int(round(math.sqrt(prims / 32.0))))
        vpr = max(32, int(round(prims / (2 * k))) + 1)
        return woven_patch(seed=seed, n_warp=k, n_weft=k, verts_per_rod=vpr)
    n = max(8, 1 + int(round(math.sqrt(prims / 6.0))))
    n_folds = 0 if n < 72 else (1 if n < 128 else (2 if n < 192 else 3))
    gaps = [940.0, 960.0, 980.0][:n_folds]
    return folded_cloth(seed=seed, n=n, gaps=gaps)


def batch_scenes(seed: int = BASE_SEED + 3000, n_scenes: int = 64, lo: float = 1e3,
                 hi: float = 6.4e4):
    """Independent yarn / cloth patches, kind ~ Bernoulli(1/2), primitive count
    log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_scenes):
        kind = "rod" if rng.random() < 0.5 else "shell"
        prims = float(np.exp(rng.uniform(math.log(lo), math.log(hi))))
        out.append(_scene_of_size(kind, prims, seed + 1 + k))
    return out


def serving_scenes(seed: int = BASE_SEED + 4000, n_scenes: int = 256, median: float = 1.6e4,
                   sigma: float = 1.0, lo: float = 1e3, hi: float = 5e5):
    """Resident scenes for the serving loop: rod:shell 1:1, primitive counts
    lognormal(median, sigma) truncated to [lo, hi]."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_scenes):
        kind = "rod" if k % 2 == 0 else "shell"
        while True:
            prims = float(median * math.exp(rng.normal(0.0, sigma)))
            if lo <= prims <= hi:
                break
        out.append(_scene_of_size(kind, prims, seed + 1 + k))
    return out


def crossing_rods(z: float = 250.0, n: int = 14, ell: float = 100.0, h: float = 300.0,
                  eta: float = 270.0) -> Scene:
    """Two straight rods crossing at right angles, centrelines z apart
    (z < eta: the crossing starts inside the core).  n vertices per rod,
    segments of length ell centred on the crossing."""
    xs = (np.arange(n) - (n - 1) / 2.0) * ell
    a = np.stack([xs, np.zeros(n), np.zeros(n)], 1)
    b = np.stack([np.zeros(n), xs, np.full(n, float(z))], 1)
    e = np.stack([np.arange(n - 1), np.arange(1, n)], 1)
    s = xs - xs[0]
    return Scene("crossing_rods", "rod", np.concatenate([a, b]), np.concatenate([e, e + n]).astype(np.int32),
                 np.zeros((0, 3), np.int32), np.concatenate([s, s]), h=float(h), eta=float(eta), seed=0)


def straight_rod(ell: float, length: float = 50000.0, h: float = 300.0) -> Scene:
    """A straight rod at rest (the contact-locking toy of the paper: a 5 cm
    yarn) with uniform segments of length ell.  The offset follows the
    paper's comparison setting eta = 0.9 min(h, dbar_min), with
    dbar_min = ell (the rest gap of edges two apart) when ell < h."""
    n = int(round(length / ell)) + 1
    xs = np.arange(n) * float(ell)
    x = np.stack([xs, np.zeros(n), np.zeros(n)], 1)
    e = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)
    eta = 0.9 * min(h, float(ell))
    return Scene(f"straight_rod_l{ell:g}", "rod", x, e, np.zeros((0, 3), np.int32), xs.copy(), h=float(h),
                 eta=eta, seed=0)


def flat_sheet(ell: float, side: float = 20000.0, h: float = 1000.0) -> Scene:
    """A flat square sheet at rest, regular grid of spacing ell with one
    diagonal per cell (rest coordinates = positions).  eta = 0.9 min(h,
    dbar_min) with dbar_min = ell / sqrt(2) (a vertex to the diagonal of the
    next cell)."""
    n = int(round(side / ell)) + 1
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = np.stack([ii.ravel() * float(ell), jj.ravel() * float(ell)], 1)
    x = np.concatenate([u, np.zeros((n * n, 1))], 1)
    vid = lambda i, j: i * n + j
    tris = []
    for i in range(n - 1):
        for j in range(n - 1):
            tris.append((vid(i, j), vid(i + 1, j), vid(i + 1, j + 1)))
            tris.append((vid(i, j), vid(i + 1, j + 1), vid(i, j + 1)))
    tris = np.array(tris, np.int32)
    ed = set()
    for t in tris:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            ed.add((min(a, b), max(a, b)))
    edges = np.array(sorted(ed), np.int32)
    eta = 0.9 * min(h, float(ell) / np.sqrt(2.0))
    return Scene(f"flat_sheet_l{ell:g}", "shell", x, edges, tris, u, h=float(h), eta=eta, seed=0)


def search_direction(scene: Scene, seed: int = BASE_SEED + 5000) -> np.ndarray:
    """Seeded displacement field for line-search workloads: a squeeze of the
    scene toward its mid-plane in z (3 activation bands at the extremes) plus
    per-vertex Gaussian noise of 1.5 bands, so that many pairs close their
    gaps within the step."""
    rng = np.random.default_rng(seed)
    x = scene.x
    band = scene.h - scene.eta
    zc = 0.5 * (x[:, 2].max() + x[:, 2].min())
    p = np.zeros_like(x)
    p[:, 2] = -(x[:, 2] - zc) / max(1.0, np.abs(x[:, 2] - zc).max()) * 3.0 * band
    p += rng.normal(scale=1.5 * band, size=x.shape)
    return p


WORKLOADS = {
    "helix_loop_rod": lambda: helix_loop_rod(),
    "woven_patch": lambda: woven_patch(),
    "folded_cloth": lambda: folded_cloth(),
}


def workload(name: str) -> Scene:
    return WORKLOADS[name]()
