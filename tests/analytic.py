"""Closed-form and textbook solutions used to pin the reference solver.

None of these reuse the solver's formulas: they are exact solutions of the
shallow water equations (Sec. 2, equations swe) in special cases.

* Stoker: dam break over a wet bed -- left rarefaction, middle state, right
  shock (Rankine-Hugoniot), middle depth by bisection.
* Ritter: dam break over a dry bed.
* d'Alembert: linearised 1D waves over a flat bed.
* Linearised 2D radially symmetric hump: Hankel-transform solution, summed over
  mirror images for reflecting walls.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special


def stoker_state(h_left: float, h_right: float, g: float = 9.81):
    """Middle depth/velocity and wave speeds for a wet dam break.

    The middle state connects to the left state through a 1-rarefaction
    (u_m = 2 (c_L - c_m)) and to the right state at rest through a 2-shock
    (u_m = (h_m - h_R) sqrt(g (h_m + h_R) / (2 h_m h_R)))."""
    cL = math.sqrt(g * h_left)

    def f(hm):
        cm = math.sqrt(g * hm)
        u_rare = 2.0 * (cL - cm)
        u_shock = (hm - h_right) * math.sqrt(g * (hm + h_right) / (2.0 * hm * h_right))
        return u_rare - u_shock

    lo, hi = h_right, h_left
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    hm = 0.5 * (lo + hi)
    cm = math.sqrt(g * hm)
    um = 2.0 * (cL - cm)
    shock = hm * um / (hm - h_right)
    return {"h_m": hm, "u_m": um, "shock": shock, "head": -cL, "tail": um - cm}


def stoker_profile(x: np.ndarray, t: float, h_left: float, h_right: float, g: float = 9.81):
    st = stoker_state(h_left, h_right, g)
    cL = math.sqrt(g * h_left)
    h = np.empty_like(x)
    u = np.empty_like(x)
    xi = x / t
    left = xi < st["head"]
    rare = (xi >= st["head"]) & (xi < st["tail"])
    mid = (xi >= st["tail"]) & (xi < st["shock"])
    right = xi >= st["shock"]
    h[left], u[left] = h_left, 0.0
    h[rare] = (2.0 * cL - xi[rare]) ** 2 / (9.0 * g)
    u[rare] = 2.0 / 3.0 * (cL + xi[rare])
    h[mid], u[mid] = st["h_m"], st["u_m"]
    h[right], u[right] = h_right, 0.0
    return h, u


def ritter_profile(x: np.ndarray, t: float, h_left: float, g: float = 9.81):
    cL = math.sqrt(g * h_left)
    xi = x / t
    h = np.where(xi < -cL, h_left, np.where(xi < 2.0 * cL, (2.0 * cL - xi) ** 2 / (9.0 * g), 0.0))
    u = np.where(xi < -cL, 0.0, np.where(xi < 2.0 * cL, 2.0 / 3.0 * (cL + xi), 0.0))
    return h, u


def dalembert_surface(x: np.ndarray, t: float, eta0, depth: float, g: float = 9.81):
    c = math.sqrt(g * depth)
    return 0.5 * (eta0(x - c * t) + eta0(x + c * t))


def radial_hump(r: np.ndarray, t: float, amp: float, sigma: float, depth: float,
                g: float = 9.81, kmax_sigmas: float = 12.0, nk: int = 4000):
    """Linear wave equation solution for an initial Gaussian surface at rest:
    eta(r, t) = A sigma^2 int_0^inf k exp(-sigma^2 k^2 / 2) J0(k r) cos(c k t) dk."""
    c = math.sqrt(g * depth)
    k = np.linspace(0.0, kmax_sigmas / sigma, nk)
    w = amp * sigma * sigma * k * np.exp(-0.5 * (sigma * k) ** 2) * np.cos(c * k * t)
    r = np.asarray(r, dtype=np.float64)
    out = np.empty(r.size)
    flat = r.ravel()
    for n0 in range(0, flat.size, 2048):
        rr = flat[n0:n0 + 2048]
        J = special.j0(np.outer(rr, k))
        out[n0:n0 + 2048] = integrate.simpson(J * w[None, :], x=k, axis=1)
    return out.reshape(r.shape)


def radial_hump_walls(xc: np.ndarray, yc: np.ndarray, t: float, amp: float, sigma: float,
                      depth: float, L: float, cx: float, cy: float, nimg: int = 1,
                      g: float = 9.81, nr: int = 6000):
    """Sum of mirror images of a source at (cx, cy) in the box [0, L]^2 with
    reflecting walls (surface is even across each wall).  The radial profile is
    evaluated once on a fine grid of r and interpolated (its scale is sigma,
    the grid step is far below it)."""
    X, Y = np.meshgrid(xc, yc)
    xs = sorted({s for k in range(-nimg, nimg + 1) for s in (cx + 2 * k * L, -cx + 2 * k * L)})
    ys = sorted({s for k in range(-nimg, nimg + 1) for s in (cy + 2 * k * L, -cy + 2 * k * L)})
    c = math.sqrt(g * depth)
    reach = c * t + 8.0 * sigma
    rgrid = np.linspace(0.0, reach, nr)
    prof = radial_hump(rgrid, t, amp, sigma, depth, g)
    eta = np.zeros_like(X)
    for sx in xs:
        for sy in ys:
            R = np.hypot(X - sx, Y - sy)
            near = R < reach
            if np.any(near):
                eta[near] += np.interp(R[near], rgrid, prof)
    return eta
