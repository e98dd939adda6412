"""Seeded synthetic inputs: fan-beam geometries, ellipse phantoms, analytic sinograms, Poisson counts.

This module produces test and benchmark data only.  It holds none of the
reconstruction arithmetic (no Joseph projector, no likelihood, no TV, no step
rule); the GPU library and the CPU oracle both consume what it produces.

The paper reconstructs measured TomoTherapy MVCT data of the Gammex and Cheese
phantoms and of patients (section 3.A): 512x512 slices from an 800-view
rotation (section 3.D).  Those data are not available, so seeded ellipse
phantoms with the same image size, view count and MV-like photon noise stand
in for them.  Line integrals are computed analytically from the ellipses (chord
length of a line through a rotated ellipse), so the counts do not come from the
discrete projector that reconstructs them.

Geometry convention (shared by every consumer, each re-implementing it):
  * pixel (i, j) centre: x = (i - (N-1)/2) * pixel, y = (j - (N-1)/2) * pixel,
    stored at index j * N + i;
  * view v: source angle beta = start + arc*v / n_views (arc = 2*pi for a full
    turn, less for limited-angle data), source at SAD * (cos beta, sin beta);
  * channel k on an arc centred on the source: fan angle
    gamma = (k - (n_ch-1)/2) * dgamma with dgamma = 2 * gamma_max / n_ch and
    gamma_max = asin(R / SAD) (R = N * pixel / 2), unless given;
  * ray direction (cos(beta + pi + gamma), sin(beta + pi + gamma)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MU_WATER_PER_MM = 0.0049
MU_BONE_PER_MM = 0.009


@dataclasses.dataclass(frozen=True)
class Geometry:
    """2D fan-beam geometry; lengths in mm, angles in radians."""

    n: int
    pixel_mm: float
    n_views: int
    n_channels: int
    sad_mm: float = 850.0
    sdd_mm: float = 1450.0
    fan_half_angle_rad: float = 0.0  # 0 means asin(R / SAD): the fan just covers the FOV circle
    start_angle_rad: float = 0.0
    scan_arc_rad: float = 0.0  # angular range of the views; 0 means a full turn (2 pi)

    @property
    def arc_rad(self) -> float:
        return self.scan_arc_rad if self.scan_arc_rad > 0 else 2 * math.pi

    @property
    def fov_radius_mm(self) -> float:
        return 0.5 * self.n * self.pixel_mm

    @property
    def gamma_max(self) -> float:
        if self.fan_half_angle_rad > 0:
            return self.fan_half_angle_rad
        return math.asin(self.fov_radius_mm / self.sad_mm)

    def as_tuple(self):
        return (self.n, self.pixel_mm, self.n_views, self.n_channels, self.sad_mm, self.sdd_mm,
                self.fan_half_angle_rad, self.start_angle_rad, self.scan_arc_rad)


@dataclasses.dataclass(frozen=True)
class Ellipse:
    cx: float
    cy: float
    a: float  # semi-axis along the ellipse's own x axis (mm)
    b: float
    phi: float  # rotation (rad)
    value: float  # additive attenuation (1/mm)


# ---------------------------------------------------------------------------
# Configurations (sizes of the paper's workload: 512^2 slice, 800-view rotation)
# ---------------------------------------------------------------------------

def config0_geometry() -> Geometry:
    """Tiny case: 128^2 at 3.125 mm, 180 views, 192 arc channels."""
    return Geometry(n=128, pixel_mm=3.125, n_views=180, n_channels=192)


def config1_geometry() -> Geometry:
    """Clinical-scale slice: 512^2 at 0.78125 mm (400 mm FOV), 800 views, 738 channels."""
    return Geometry(n=512, pixel_mm=400.0 / 512, n_views=800, n_channels=738)


# ---------------------------------------------------------------------------
# Phantoms
# ---------------------------------------------------------------------------

def _inside_ellipse(e: Ellipse, x, y):
    c, s = math.cos(e.phi), math.sin(e.phi)
    dx, dy = x - e.cx, y - e.cy
    xr = c * dx + s * dy
    yr = -s * dx + c * dy
    return (xr / e.a) ** 2 + (yr / e.b) ** 2 <= 1.0


def random_phantom(seed: int, *, low_contrast: bool = False, scale: float = 1.0) -> list[Ellipse]:
    """Seeded ellipse phantom: a water body plus 4-9 non-overlapping inserts.

    Body: semi-axes U(140,180) x U(100,150) mm, centre offset U(-10,10) mm, angle U(0,pi).
    Inserts: semi-axes U(8,40) mm, inside the body, pairwise disjoint.
      default: soft tissue water*(1+U(-3%,3%)), or bone 0.009/mm with p=0.2;
      low_contrast: water*(1 +- U(1%,3%)).
    `scale` shrinks every length (for small fields of view); values are unchanged.
    """
    rng = np.random.default_rng(seed)
    body = Ellipse(cx=rng.uniform(-10, 10) * scale, cy=rng.uniform(-10, 10) * scale,
                   a=rng.uniform(140, 180) * scale, b=rng.uniform(100, 150) * scale,
                   phi=rng.uniform(0, math.pi), value=MU_WATER_PER_MM)
    n_total = int(rng.integers(5, 11))
    inserts: list[tuple[float, float, float]] = []  # (cx, cy, bounding radius)
    out = [body]
    tries = 0
    while len(out) < n_total and tries < 2000:
        tries += 1
        a = rng.uniform(8, 40) * scale
        b = rng.uniform(8, 40) * scale
        phi = rng.uniform(0, math.pi)
        r = max(a, b)
        cx = body.cx + rng.uniform(-body.a, body.a)
        cy = body.cy + rng.uniform(-body.a, body.a)
        # bounding circle (plus a 2 mm margin) must sit inside a slightly shrunk body
        shrunk = dataclasses.replace(body, a=body.a - 2 * scale, b=body.b - 2 * scale)
        ang = np.linspace(0, 2 * math.pi, 96, endpoint=False)
        px = cx + (r + 2 * scale) * np.cos(ang)
        py = cy + (r + 2 * scale) * np.sin(ang)
        if not np.all(_inside_ellipse(shrunk, px, py)):
            continue
        if any(math.hypot(cx - qx, cy - qy) < r + qr + 2 * scale for qx, qy, qr in inserts):
            continue
        if low_contrast:
            sign = 1.0 if rng.uniform() < 0.5 else -1.0
            val = MU_WATER_PER_MM * (1 + sign * rng.uniform(0.01, 0.03))
        elif rng.uniform() < 0.2:
            val = MU_BONE_PER_MM
        else:
            val = MU_WATER_PER_MM * (1 + rng.uniform(-0.03, 0.03))
        inserts.append((cx, cy, r))
        out.append(Ellipse(cx, cy, a, b, phi, val - MU_WATER_PER_MM))
    return out


def rasterize(ellipses: list[Ellipse], n: int, pixel_mm: float, supersample: int = 4) -> np.ndarray:
    """Pixel averages of the phantom on the N x N grid, by supersampling (float64, [j][i])."""
    c = 0.5 * (n - 1)
    sub = (np.arange(supersample) + 0.5) / supersample - 0.5
    coords = ((np.arange(n)[:, None] - c) + sub[None, :]).reshape(-1) * pixel_mm
    X, Y = np.meshgrid(coords, coords, indexing="xy")
    img = np.zeros_like(X)
    for e in ellipses:
        img += e.value * _inside_ellipse(e, X, Y)
    img = img.reshape(n, supersample, n, supersample).mean(axis=(1, 3))
    return img


# ---------------------------------------------------------------------------
# Analytic line integrals and counts
# ---------------------------------------------------------------------------

def ray_table(g: Geometry):
    """Source positions and unit directions of every ray: arrays [n_views][n_channels]."""
    beta = g.start_angle_rad + g.arc_rad * np.arange(g.n_views) / g.n_views
    dgam = 2 * g.gamma_max / g.n_channels
    gam = (np.arange(g.n_channels) - 0.5 * (g.n_channels - 1)) * dgam
    sx = g.sad_mm * np.cos(beta)[:, None] * np.ones((1, g.n_channels))
    sy = g.sad_mm * np.sin(beta)[:, None] * np.ones((1, g.n_channels))
    theta = beta[:, None] + math.pi + gam[None, :]
    return sx, sy, np.cos(theta), np.sin(theta)


def analytic_sinogram(ellipses: list[Ellipse], g: Geometry) -> np.ndarray:
    """Exact line integrals of the ellipse phantom along every ray, [n_views][n_channels] (float64).

    A ray s + t d crosses an ellipse along the chord whose length is sqrt(disc) / A for the
    quadratic A t^2 + B t + C = 0 written in the ellipse's own frame.
    """
    sx, sy, dx, dy = ray_table(g)
    out = np.zeros_like(sx)
    for e in ellipses:
        c, s = math.cos(e.phi), math.sin(e.phi)
        px = c * (sx - e.cx) + s * (sy - e.cy)
        py = -s * (sx - e.cx) + c * (sy - e.cy)
        qx = c * dx + s * dy
        qy = -s * dx + c * dy
        A = qx * qx / e.a**2 + qy * qy / e.b**2
        B = 2 * (px * qx / e.a**2 + py * qy / e.b**2)
        C = px * px / e.a**2 + py * py / e.b**2 - 1
        disc = B * B - 4 * A * C
        chord = np.where(disc > 0, np.sqrt(np.maximum(disc, 0)) / A, 0.0)
        out += e.value * chord
    return out


# ---------------------------------------------------------------------------
# Helical acquisition (single-row fan beam, as on a helical tomotherapy unit)
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Ellipsoid:
    """An ellipse in the (x, y) plane extruded along z: semi-axis c in z (math.inf: a cylinder);
    the cross-section at z has semi-axes a r and b r with r = sqrt(1 - ((z - cz) / c)^2), and the
    value value + dvalue_dz (z - cz)."""
    cx: float
    cy: float
    cz: float
    a: float
    b: float
    c: float
    phi: float
    value: float
    dvalue_dz: float = 0.0

    def section(self, z: float) -> Ellipse | None:
        t = 0.0 if math.isinf(self.c) else (z - self.cz) / self.c
        if abs(t) >= 1.0:
            return None
        r = math.sqrt(1.0 - t * t)
        return Ellipse(self.cx, self.cy, self.a * r, self.b * r, self.phi, self.value + self.dvalue_dz * (z - self.cz))


def helical_view_z(g: Geometry, n_helical: int, pitch_mm: float, z0_mm: float) -> np.ndarray:
    """Source z of helical view h: z0 + pitch h / n_views (the table advances `pitch` per turn)."""
    return z0_mm + pitch_mm * np.arange(n_helical) / g.n_views


def helical_line_integrals(ellipsoids: list[Ellipsoid], g: Geometry, n_helical: int, pitch_mm: float,
                           z0_mm: float) -> np.ndarray:
    """Exact line integrals of a helical scan, [n_helical][n_channels] (float64): view h is the
    fan of geometry g at angle start + 2 pi h / n_views, in the plane z = helical_view_z(h), and
    sees the cross-sections of the ellipsoids there."""
    zs = helical_view_z(g, n_helical, pitch_mm, z0_mm)
    out = np.zeros((n_helical, g.n_channels))
    for h, z in enumerate(zs):
        gv = dataclasses.replace(g, n_views=1, start_angle_rad=g.start_angle_rad + 2 * math.pi * h / g.n_views)
        sec = [e for e in (q.section(float(z)) for q in ellipsoids) if e is not None]
        if sec:
            out[h] = analytic_sinogram(sec, gv)[0]
    return out


def random_helical_phantom(seed: int, *, scale: float = 1.0, length_mm: float = 60.0) -> list[Ellipsoid]:
    """Seeded helical phantom: random_phantom's body as a cylinder, its inserts as ellipsoids
    centred at U(-length/4, length/4) mm with z semi-axes U(10, length/2) mm."""
    rng = np.random.default_rng([seed, 7])
    ell = random_phantom(seed, low_contrast=True, scale=scale)
    out = [Ellipsoid(ell[0].cx, ell[0].cy, 0.0, ell[0].a, ell[0].b, math.inf, ell[0].phi, ell[0].value)]
    for e in ell[1:]:
        out.append(Ellipsoid(e.cx, e.cy, rng.uniform(-0.25, 0.25) * length_mm, e.a, e.b,
                             rng.uniform(10.0, 0.5 * length_mm), e.phi, e.value))
    return out


def poisson_counts(line_integrals: np.ndarray, i0: float, seed: int) -> np.ndarray:
    """Transmission counts y ~ Poisson(I0 exp(-l)), float32 (exact integers)."""
    rng = np.random.default_rng([seed, 1])
    lam = i0 * np.exp(-line_integrals)
    return rng.poisson(lam).astype(np.float32)


@dataclasses.dataclass
class Slice:
    geometry: Geometry
    ellipses: list
    truth: np.ndarray  # rasterized phantom, float64 [N][N], 1/mm
    line_integrals: np.ndarray  # analytic, float64 [n_views][n_channels]
    counts: np.ndarray  # float32 [n_views][n_channels]
    i0: float
    seed: int


def make_slice(g: Geometry, seed: int, i0: float, *, low_contrast: bool = False,
               supersample: int = 4) -> Slice:
    """One seeded slice: phantom, analytic sinogram and Poisson counts."""
    scale = min(1.0, g.fov_radius_mm / 200.0)
    ell = random_phantom(seed, low_contrast=low_contrast, scale=scale)
    truth = rasterize(ell, g.n, g.pixel_mm, supersample)
    li = analytic_sinogram(ell, g)
    counts = poisson_counts(li, i0, seed)
    return Slice(g, ell, truth, li, counts, i0, seed)


def random_batch_geometry(seed: int, *, sizes=(256, 512), views=(600, 900), channels=(520, 738)):
    """Per-slice geometry for a batch of helical-rebinned slices of uneven size.

    Image N drawn from `sizes` (400 mm FOV), views U{600..900}, channels U{520..738},
    I0 log-uniform in [1e3, 1e4].  Returns (Geometry, I0).
    """
    rng = np.random.default_rng([seed, 7])
    n = int(rng.choice(sizes))
    nv = int(rng.integers(views[0], views[1] + 1))
    nc = int(rng.integers(channels[0], channels[1] + 1))
    i0 = float(10 ** rng.uniform(3, 4))
    return Geometry(n=n, pixel_mm=400.0 / n, n_views=nv, n_channels=nc), i0


# ---------------------------------------------------------------------------
# Seeded initial parameters of the warm-start network
# ---------------------------------------------------------------------------

CNN_LAYERS = [(1, 32)] + [(32, 32)] * 6 + [(32, 1)]


def cnn_initial_params(seed: int, *, zero_last: bool = True, last_std: float = 0.0) -> np.ndarray:
    """Float32 parameter vector (layout: per layer W [out][in][3][3] then b [out]).

    Hidden layers: He-normal weights (std sqrt(2 / (9 in))), zero biases.  Last
    layer: zero (the network starts as the identity map) unless zero_last is
    False, then normal with std last_std (or He-normal when last_std is 0)."""
    rng = np.random.default_rng([seed, 11])
    parts = []
    for k, (c, o) in enumerate(CNN_LAYERS):
        std = math.sqrt(2.0 / (9 * c))
        last = k == len(CNN_LAYERS) - 1
        if last and zero_last:
            W = np.zeros((o, c, 3, 3))
        else:
            W = rng.normal(0.0, last_std if (last and last_std > 0) else std, (o, c, 3, 3))
        parts += [W.ravel(), np.zeros(o)]
    return np.concatenate(parts).astype(np.float32)
