"""Seeded synthetic inputs for the shallow water patch step.

This module only builds input arrays (bathymetry, initial surface, patch
layouts, request streams).  It contains none of the solver's arithmetic, and
both the HIP path and the reference solver used by the tests take their inputs
from here.

The paper's own runs (2011 Tohoku -> Crescent City, Seattle Fault -> Eagle
Harbor, Sec. 5) need earthquake deformation files and coastal elevation models
that are not available; these generators stand in for them with the shapes the
paper's runs have: a deep abyssal plain (about 4000 m) rising over a
continental shelf to a dry coast, a Gaussian sea-floor uplift as the source,
patch sizes up to 128 x 128 cells and three refinement levels.

Conventions: cell (i, j) with 1 <= i <= mx, 1 <= j <= my has centre
(x0 + (i - 1/2) dx, y0 + (j - 1/2) dy); arrays are indexed [j - 1, i - 1]
(row-major, x fastest).  b < 0 is below sea level.  Depth h = max(0, eta - b).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

G = 9.81
DRYTOL = 1e-3

BC_WALL, BC_EXTRAP, BC_USER = 0, 1, 2


@dataclass
class Problem:
    """Interior arrays of one patch plus its geometry."""
    name: str
    h: np.ndarray
    hu: np.ndarray
    hv: np.ndarray
    b: np.ndarray
    dx: float
    dy: float
    bc: tuple = (BC_WALL,) * 4
    nsteps: int = 0
    x0: float = 0.0
    y0: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def mx(self) -> int:
        return int(self.h.shape[1])

    @property
    def my(self) -> int:
        return int(self.h.shape[0])


def cell_centres(n: int, d: float, x0: float = 0.0) -> np.ndarray:
    return x0 + (np.arange(n, dtype=np.float64) + 0.5) * d


def shelf_profile(x: np.ndarray, x_s: float, width: float, deep: float = -4000.0,
                  coast: float = 50.0) -> np.ndarray:
    """Abyssal plain at `deep` rising by a tanh profile to `coast` metres."""
    return deep + (coast - deep) * 0.5 * (1.0 + np.tanh((x - x_s) / width))


def gaussian(xc: np.ndarray, yc: np.ndarray, amp: float, sigma: float, cx: float,
             cy: float) -> np.ndarray:
    X, Y = np.meshgrid(xc, yc)
    r2 = (X - cx) ** 2 + (Y - cy) ** 2
    return amp * np.exp(-r2 / (2.0 * sigma * sigma))


def depth_from_surface(eta: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Initial depth of a surface eta over bed b (0 where the bed is above eta)."""
    return np.maximum(0.0, eta - b)


def _roughen(b: np.ndarray, rough: float, rng: np.random.Generator) -> np.ndarray:
    xi = rng.uniform(-1.0, 1.0, size=b.shape)
    return b * (1.0 + rough * xi)


def gaussian_hump(n: int = 200, dx: float = 1000.0, depth: float = 4000.0,
                  amp: float = 1.0, sigma: float = 10e3, nsteps: int = 100) -> Problem:
    """Flat bottom at -depth, Gaussian surface hump at the centre, walls."""
    xc = cell_centres(n, dx)
    b = np.full((n, n), -depth)
    eta = gaussian(xc, xc, amp, sigma, 0.5 * n * dx, 0.5 * n * dx)
    h = depth_from_surface(eta, b)
    z = np.zeros_like(h)
    return Problem("gaussian_hump", h, z, z.copy(), b, dx, dx, (BC_WALL,) * 4, nsteps,
                   meta={"amp": amp, "sigma": sigma, "depth": depth})


def lake_at_rest_flat(n: int = 200, dx: float = 1000.0, depth: float = 4000.0) -> Problem:
    p = gaussian_hump(n, dx, depth, amp=0.0)
    p.name = "lake_at_rest_flat"
    return p


def dam_break_1d(n: int = 400, length: float = 400.0, h_left: float = 2.0,
                 h_right: float = 1.0, transpose: bool = False) -> Problem:
    """1D dam break on x in [-L/2, L/2], flat bed at 0, extrapolation ends.
    Embedded as an (my = 1, mx = n) patch, or (my = n, mx = 1) if transposed."""
    dx = length / n
    xc = cell_centres(n, dx, -0.5 * length)
    h = np.where(xc < 0.0, h_left, h_right).astype(np.float64)
    b = np.zeros(n)
    z = np.zeros(n)
    bc = (BC_EXTRAP,) * 4
    if transpose:
        return Problem("dam_break_y", h[:, None].copy(), z[:, None].copy(), z[:, None].copy(),
                       b[:, None].copy(), dx, dx, bc, 0, 0.0, -0.5 * length)
    return Problem("dam_break_x", h[None, :].copy(), z[None, :].copy(), z[None, :].copy(),
                   b[None, :].copy(), dx, dx, bc, 0, -0.5 * length, 0.0)


def shelf_grid(n: int, dx: float, seed: int, rough: float = 0.05, amp: float = 2.0,
               sigma: float = 30e3, src=None, bc=(BC_EXTRAP,) * 4, width: float = 20e3,
               x_s_frac: float = 0.75, nsteps: int = 0, name: str = "shelf") -> Problem:
    """Square n x n grid on [0, n dx]^2 with the tanh shelf along x, seeded
    multiplicative roughness, and a Gaussian uplift added to the surface."""
    L = n * dx
    x_s = x_s_frac * L
    xc = cell_centres(n, dx)
    b = np.broadcast_to(shelf_profile(xc, x_s, width)[None, :], (n, n)).copy()
    rng = np.random.default_rng(seed)
    if rough > 0.0:
        b = _roughen(b, rough, rng)
    if src is None:
        src = (0.5 * L, 0.5 * L)
    eta = gaussian(xc, xc, amp, sigma, src[0], src[1])
    h = depth_from_surface(eta, b)
    z = np.zeros_like(h)
    return Problem(name, h, z, z.copy(), b, dx, dx, tuple(bc), nsteps,
                   meta={"x_s": x_s, "width": width, "amp": amp, "sigma": sigma,
                         "src": src, "seed": seed, "rough": rough})


def shelf_4096(n: int = 4096, dx: float = 250.0, nsteps: int = 500) -> Problem:
    """4096^2 grid, dx = 250 m, shelf + 5% roughness (seed 2), 2 m source of
    sigma 30 km at the domain centre, extrapolation boundaries."""
    return shelf_grid(n, dx, seed=2, nsteps=nsteps, name=f"shelf_{n}")


def active_sea(n: int = 4096, dx: float = 250.0, seed: int = 6, depth: float = 4000.0) -> Problem:
    """A state with no quiet edge: flat sea floor at -depth, every cell wet,
    the surface and both velocities seeded uniform noise (+-0.5 m, +-0.3 m/s
    per cell, row-major), extrapolation boundaries.  Every edge carries
    waves, so a step can skip no Riemann solve."""
    rng = np.random.default_rng(seed)
    eta = rng.uniform(-0.5, 0.5, size=(n, n))
    u = rng.uniform(-0.3, 0.3, size=(n, n))
    v = rng.uniform(-0.3, 0.3, size=(n, n))
    b = np.full((n, n), -depth)
    h = eta - b
    return Problem(f"active_sea_{n}", h, h * u, h * v, b, dx, dx, (BC_EXTRAP,) * 4)


def shelf_walls(n: int = 2048, dx: float = 500.0, seed: int = 4, nsteps: int = 2000,
                amp: float = 2.0) -> Problem:
    """Wall-bounded shelf (mass drift is then pure numerics), source 60 km
    seaward of the shelf break at mid-height."""
    L = n * dx
    x_s = 0.75 * L
    return shelf_grid(n, dx, seed=seed, amp=amp, src=(x_s - 60e3, 0.5 * L),
                      bc=(BC_WALL,) * 4, nsteps=nsteps, name=f"shelf_walls_{n}")


# --------------------------------------------------------------------------
# Batched AMR-shaped patch sets.

@dataclass
class PatchSpec:
    mx: int
    my: int
    level: int          # 1-based refinement level
    dx: float
    x0: float
    y0: float
    tref: int           # substeps per coarse step (r^(level-1))


def amr_patch_set(npatch=(200, 800, 2000), dx1: float = 4000.0, ratio: int = 4,
                  L: float = 1024e3, size_lo: int = 16, size_hi: int = 96, seed: int = 3,
                  width: float = 20e3, x_s_frac: float = 0.75, amp: float = 2.0,
                  sigma: float = 30e3, rough: float = 0.05):
    """Patches of three refinement levels placed along the shelf.

    Level 1 windows lie anywhere in the domain, level 2 within 150 km of the
    shelf break, level 3 between 30 km seaward of the break and 20 km inland of
    the shoreline (so most level-3 patches hold a wet/dry coastline).  Side
    lengths are uniform in [size_lo, size_hi].  Each patch gets its own seeded
    roughness.  Returns (specs, problems) with one Problem per patch
    (extrapolation boundaries)."""
    rng = np.random.default_rng(seed)
    x_s = x_s_frac * L
    shore = x_s + width * np.arctanh(2.0 * 4000.0 / 4050.0 - 1.0)
    specs = []
    for lev, cnt in enumerate(npatch, start=1):
        dx = dx1 / ratio ** (lev - 1)
        for _ in range(cnt):
            mx = int(rng.integers(size_lo, size_hi + 1))
            my = int(rng.integers(size_lo, size_hi + 1))
            wx, wy = mx * dx, my * dx
            if lev == 1:
                lo, hi = 0.0, L - wx
            elif lev == 2:
                lo, hi = x_s - 150e3, x_s + 150e3 - wx
            else:
                lo, hi = x_s - 30e3, shore + 20e3 - wx
            x0 = float(rng.uniform(lo, hi))
            y0 = float(rng.uniform(0.0, L - wy))
            specs.append(PatchSpec(mx, my, lev, dx, x0, y0, ratio ** (lev - 1)))
    src = (x_s - 60e3, 0.5 * L)
    probs = []
    for k, s in enumerate(specs):
        xc = cell_centres(s.mx, s.dx, s.x0)
        yc = cell_centres(s.my, s.dx, s.y0)
        b = np.broadcast_to(shelf_profile(xc, x_s, width)[None, :], (s.my, s.mx)).copy()
        if rough > 0.0:
            b = _roughen(b, rough, np.random.default_rng([seed, k]))
        eta = gaussian(xc, yc, amp, sigma, src[0], src[1])
        h = depth_from_surface(eta, b)
        z = np.zeros_like(h)
        probs.append(Problem(f"patch{k}", h, z, z.copy(), b, s.dx, s.dx, (BC_EXTRAP,) * 4, 0,
                             s.x0, s.y0, meta={"level": s.level, "tref": s.tref}))
    return specs, probs


# --------------------------------------------------------------------------
# Scenario requests for the serving loop.

@dataclass
class Request:
    rid: int
    arrival: float       # seconds after the stream starts
    problem: Problem
    nsteps: int


def scenario(k: int, n: int | None = None, dx: float = 500.0, nsteps: int = 1000,
             n_lo: int = 256, n_hi: int = 2048) -> Problem:
    """Tsunami scenario k: seeded n x n shelf (no roughness), random source."""
    rng = np.random.default_rng(5000 + k)
    if n is None:
        n = int(rng.integers(n_lo, n_hi + 1))
    else:
        rng.integers(n_lo, n_hi + 1)
    L = n * dx
    x_s = float(rng.uniform(0.6, 0.85)) * L
    width = float(rng.uniform(10e3, 30e3))
    amp = float(rng.uniform(0.5, 5.0))
    sigma = float(rng.uniform(10e3, 50e3))
    cx = float(rng.uniform(0.2, 0.5)) * L
    cy = float(rng.uniform(0.3, 0.7)) * L
    xc = cell_centres(n, dx)
    b = np.broadcast_to(shelf_profile(xc, x_s, width)[None, :], (n, n)).copy()
    eta = gaussian(xc, xc, amp, sigma, cx, cy)
    h = depth_from_surface(eta, b)
    z = np.zeros_like(h)
    return Problem(f"scenario{k}", h, z, z.copy(), b, dx, dx, (BC_EXTRAP,) * 4, nsteps,
                   meta={"x_s": x_s, "width": width, "amp": amp, "sigma": sigma,
                         "src": (cx, cy)})


@dataclass
class ScenarioSpec:
    """Scenario k as its seeded parameters (the same draws as scenario(k)),
    for building the initial state where it is needed (on the device)."""
    name: str
    n: int
    dx: float
    nsteps: int
    x_s: float
    width: float
    amp: float
    sigma: float
    cx: float
    cy: float
    bc: tuple = (BC_EXTRAP,) * 4

    @property
    def mx(self) -> int:
        return self.n

    @property
    def my(self) -> int:
        return self.n

    @property
    def dy(self) -> float:
        return self.dx

    def device_state(self, device):
        """Initial depth and bed (FP64 torch tensors on `device`, (n, n)):
        the shelf of scenario() along x, the Gaussian source, h = max(eta - b, 0)."""
        import torch
        xc = (torch.arange(self.n, dtype=torch.float64, device=device) + 0.5) * self.dx
        bx = -4000.0 + (50.0 + 4000.0) * 0.5 * (1.0 + torch.tanh((xc - self.x_s) / self.width))
        b = bx[None, :].expand(self.n, self.n)
        gx = torch.exp(-((xc - self.cx) ** 2) / (2.0 * self.sigma * self.sigma))
        gy = torch.exp(-((xc - self.cy) ** 2) / (2.0 * self.sigma * self.sigma))
        eta = self.amp * (gy[:, None] * gx[None, :])
        return torch.clamp(eta - b, min=0.0), b


def scenario_spec(k: int, n: int | None = None, dx: float = 500.0, nsteps: int = 1000,
                  n_lo: int = 256, n_hi: int = 2048) -> ScenarioSpec:
    """The parameters of scenario(k, ...) without its arrays."""
    rng = np.random.default_rng(5000 + k)
    if n is None:
        n = int(rng.integers(n_lo, n_hi + 1))
    else:
        rng.integers(n_lo, n_hi + 1)
    L = n * dx
    x_s = float(rng.uniform(0.6, 0.85)) * L
    width = float(rng.uniform(10e3, 30e3))
    amp = float(rng.uniform(0.5, 5.0))
    sigma = float(rng.uniform(10e3, 50e3))
    cx = float(rng.uniform(0.2, 0.5)) * L
    cy = float(rng.uniform(0.3, 0.7)) * L
    return ScenarioSpec(f"scenario{k}", n, dx, nsteps, x_s, width, amp, sigma, cx, cy)


def request_stream(count: int = 1200, rate: float = 20.0, seed: int = 5, nsteps: int = 1000,
                   n_lo: int = 256, n_hi: int = 2048, dx: float = 500.0):
    """Poisson arrivals (exponential gaps of mean 1/rate) of scenario requests.
    Problems are generated lazily by the caller via scenario(rid, ...)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    sizes = [int(np.random.default_rng(5000 + k).integers(n_lo, n_hi + 1)) for k in range(count)]
    return [(k, float(t[k]), sizes[k]) for k in range(count)]


# --------------------------------------------------------------------------
# Nested AMR hierarchies (levels coupled by ghost filling and averaging).

@dataclass
class AmrPatch:
    """One patch of a hierarchy: interior cells i0 .. i0 + mx - 1, j0 .. j0 + my - 1
    in its level's global cell index (level l has n1 r^(l-1) cells a side);
    initial interior state, and the bed on the whole frame with two ghost
    layers, shape (my + 4, mx + 4)."""
    level: int
    i0: int
    j0: int
    mx: int
    my: int
    h: np.ndarray
    hu: np.ndarray
    hv: np.ndarray
    b_frame: np.ndarray


@dataclass
class AmrHierarchy:
    n1: int            # level-1 cells a side (the domain)
    dx1: float
    ratio: int         # refinement ratio in space and time between levels
    bc: tuple          # physical boundary codes of the domain (level 1)
    patches: list
    bed_kind: str = "shelf"
    depth: float = 2000.0

    def dx(self, level: int) -> float:
        return self.dx1 / self.ratio ** (level - 1)

    def levels(self) -> int:
        return max(p.level for p in self.patches)

    def bed_frame(self, level: int, i0: int, j0: int, mx: int, my: int) -> np.ndarray:
        """Bed of a patch of `level` with interior i0 .. i0 + mx - 1, j0 .. j0 +
        my - 1, on its frame with two ghost layers (the bathymetry a regridded
        patch is given)."""
        d = self.dx(level)
        xf = cell_centres(mx + 4, d, (i0 - 2) * d)
        yf = cell_centres(my + 4, d, (j0 - 2) * d)
        return _bed(self.bed_kind, xf, yf, self.n1 * self.dx1, self.depth)


def _bed(kind: str, xc, yc, L, depth):
    # each kind is separable, so the transcendental terms are taken per
    # column and per row and broadcast (the same values, cell for cell, as
    # taking them over the whole mesh)
    xc, yc = np.asarray(xc), np.asarray(yc)
    shape = (yc.size, xc.size)
    if kind == "flat":
        return np.full(shape, -depth)
    if kind == "bowl":  # deep everywhere, smooth, all wet
        cx = np.cos(2 * np.pi * xc / L)[None, :]
        cy = np.cos(2 * np.pi * yc / L)[:, None]
        return -depth + 0.25 * depth * cx * cy
    # "shelf": the tanh shelf along x with a dry coast past 0.8 L
    row = shelf_profile(xc, 0.7 * L, 0.05 * L, deep=-depth)
    return np.ascontiguousarray(np.broadcast_to(row[None, :], shape))


def amr_hierarchy(rects, n1: int = 48, dx1: float = 2000.0, ratio: int = 2,
                  bed: str = "shelf", depth: float = 2000.0, amp: float = 1.0,
                  sigma_frac: float = 0.08, src=(0.4, 0.5), u0: float = 0.0,
                  bc=(BC_EXTRAP,) * 4) -> AmrHierarchy:
    """A hierarchy from patch rectangles.  rects[l - 1] lists the (i0, j0, mx,
    my) of level l in that level's global index (level 1 normally one patch
    covering 0 .. n1 - 1).  Bed and initial surface are sampled at each
    level's own cell centres (ghost frame included for the bed); the surface
    is a Gaussian hump of amplitude amp at src (fractions of the domain),
    momenta u0 h in x.  The nesting is not checked here."""
    L = n1 * dx1
    patches = []
    for lev, lst in enumerate(rects, start=1):
        d = dx1 / ratio ** (lev - 1)
        for (i0, j0, mx, my) in lst:
            xf = cell_centres(mx + 4, d, (i0 - 2) * d)
            yf = cell_centres(my + 4, d, (j0 - 2) * d)
            bf = _bed(bed, xf, yf, L, depth)
            eta = gaussian(xf[2:-2], yf[2:-2], amp, sigma_frac * L, src[0] * L, src[1] * L)
            h = depth_from_surface(eta, bf[2:-2, 2:-2])
            hu = u0 * h
            patches.append(AmrPatch(lev, i0, j0, mx, my, h, hu, np.zeros_like(h), bf))
    return AmrHierarchy(n1, dx1, ratio, tuple(bc), patches, bed, depth)


def amr_three_levels(ratio: int = 2, bed: str = "shelf", amp: float = 1.0, u0: float = 0.0,
                     n1: int = 48) -> AmrHierarchy:
    """Small three-level test hierarchy: one level-1 patch, two level-2
    patches that abut (their shared side fills from each other), and two
    level-3 patches inside them, one straddling the level-2 seam.  Extents
    are multiples of the ratio, and every fine ghost cell lies over the
    interior of the level below."""
    r = ratio
    m = 2 if r == 1 else 1  # margin, in cells of the level below
    l2 = [((m + 3) * r, (m + 4) * r, 14 * r, 16 * r), ((m + 17) * r, (m + 4) * r, 10 * r, 20 * r)]
    l3 = [((m + 5) * r * r, (m + 7) * r * r, 6 * r * r, 6 * r * r),
          ((m + 14) * r * r, (m + 9) * r * r, 8 * r * r, 5 * r * r)]
    return amr_hierarchy([[(0, 0, n1, n1)], l2, l3], n1=n1, ratio=r, bed=bed, amp=amp, u0=u0)


def amr_nested(n1: int = 1024, dx1: float = 2000.0, ratio: int = 4, counts=(64, 128),
               sizes=(96, 160), seed: int = 11, amp: float = 2.0,
               depth: float = 2000.0) -> AmrHierarchy:
    """Seeded three-level hierarchy over the shelf: level 1 one n1 x n1 patch;
    counts[0] level-2 patches in the band 0.55 L .. 0.9 L across the shelf
    break and the coast, counts[1] level-3 patches inside them.  Side lengths
    are uniform in `sizes` (fine cells, multiples of the ratio); patches of a
    level do not overlap, and every patch's ghost cells lie over the interior
    of its parent."""
    rng = np.random.default_rng(seed)
    r = ratio
    rects = [[(0, 0, n1, n1)]]
    for lev, count in zip((2, 3), counts):
        parents = rects[-1]
        placed = []
        tries = 0
        while len(placed) < count and tries < 200 * count:
            tries += 1
            pi0, pj0, pmx, pmy = parents[int(rng.integers(len(parents)))]
            mx = int(rng.integers(sizes[0] // r, sizes[1] // r + 1)) * r
            my = int(rng.integers(sizes[0] // r, sizes[1] // r + 1)) * r
            lo_i = (pi0 * r + 2 + r - 1) // r  # ghost cells inside the parent
            hi_i = ((pi0 + pmx) * r - 2 - mx) // r
            lo_j = (pj0 * r + 2 + r - 1) // r
            hi_j = ((pj0 + pmy) * r - 2 - my) // r
            if lev == 2:  # the band across the shelf break and the coast
                lo_i = max(lo_i, int(0.55 * n1))
                hi_i = min(hi_i, int(0.9 * n1 * r - mx) // r)
            if hi_i < lo_i or hi_j < lo_j:
                continue
            i0 = int(rng.integers(lo_i, hi_i + 1)) * r
            j0 = int(rng.integers(lo_j, hi_j + 1)) * r
            if any(i0 < a + w and a < i0 + mx and j0 < b + h and b < j0 + my
                   for a, b, w, h in placed):
                continue
            placed.append((i0, j0, mx, my))
        rects.append(placed)
    return amr_hierarchy(rects, n1=n1, dx1=dx1, ratio=r, bed="shelf", depth=depth, amp=amp,
                         sigma_frac=0.04, src=(0.5, 0.5))


# --------------------------------------------------------------------------
# Latitude-longitude patches.

EARTH_RADIUS = 6.371e6


def latlon_basin(nx: int = 256, ny: int = 256, lon0: float = 140.0, lat0: float = -30.0,
                 dlon: float = 0.25, dlat: float = 0.25, depth: float = 4000.0,
                 amp: float = 2.0, sigma_deg: float = 2.0, src=None, shelf: bool = True,
                 bc=(BC_WALL,) * 4, name: str = "latlon_basin") -> Problem:
    """A basin on a latitude-longitude patch: cells dlon x dlat degrees from
    (lon0, lat0) at the lower-left corner; bed at -depth with, if `shelf`, a
    tanh rise to a dry coast over the last fifth in longitude; a Gaussian hump
    of amp metres and sigma_deg degrees (in both angles) at src (lon, lat;
    default the centre).  dx, dy are R dlon and R dlat in metres; the
    patch's latitudes are in meta (lat0, dlat)."""
    lon = lon0 + (np.arange(nx) + 0.5) * dlon
    lat = lat0 + (np.arange(ny) + 0.5) * dlat
    LON, LAT = np.meshgrid(lon, lat)
    if shelf:
        x_s = lon0 + 0.85 * nx * dlon
        b = shelf_profile(LON, x_s, 0.03 * nx * dlon, deep=-depth)
    else:
        b = np.full(LON.shape, -depth)
    if src is None:
        src = (lon0 + 0.5 * nx * dlon, lat0 + 0.5 * ny * dlat)
    eta = amp * np.exp(-((LON - src[0]) ** 2 + (LAT - src[1]) ** 2) / (2.0 * sigma_deg ** 2))
    h = depth_from_surface(eta, b)
    z = np.zeros_like(h)
    R = EARTH_RADIUS
    return Problem(name, h, z, z.copy(), b, R * np.deg2rad(dlon), R * np.deg2rad(dlat),
                   tuple(bc), 0, meta={"lon0": lon0, "lat0": lat0, "dlon": dlon, "dlat": dlat})
