"""Pins of the reference solver's per-edge pieces against facts fixed by the
mathematics (not by retyping the solver):

* MC limiter values (textbook closed form of Phi_MC, Sec. 2 limiter);
* the f-waves of a wet edge sum to the jump of the flux of equations swe plus
  the bed source g * hbar * (b_R - b_L);
* a lake at rest (equal surface, no momentum) gives zero waves bit for bit
  (the solver's stated steady-state property, Sec. 2), also against a dry bank
  and with cells shallower than the dry tolerance;
* mirror symmetry x -> -x, bit for bit;
* speeds ordered s1 <= s2 <= s3;
* a first-order Godunov update of the two cells at Courant number <= 1 keeps
  both depths non-negative (the solver's stated positivity property);
* a wall edge against a dry bank acts like the explicit mirror state;
* water running off a dry bank it can reach takes no water out of the bank's
  empty cell: at the bound of the stationary jump that cell's middle depth is
  exactly 0, so its left-going mass flux is 0 (also mirrored).
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

G = 9.81
EPS = 1e-3


def test_mc_limiter_table(orc):
    # Phi_MC(theta) = max(0, min((1 + theta) / 2, 2, 2 theta))
    table = {-1.0: 0.0, 0.0: 0.0, 0.25: 0.5, 0.5: 0.75, 1.0: 1.0, 2.0: 1.5, 3.0: 2.0,
             10.0: 2.0, 1.0 / 3.0: 2.0 / 3.0}
    for th, v in table.items():
        assert orc.mc_limiter(th) == pytest.approx(v, abs=1e-15), th


def _flux(h, m, t):
    u = m / h
    return np.array([m, m * u + 0.5 * G * h * h, m * t / h])


wet_h = st.floats(min_value=0.01, max_value=6000.0)
mom = st.floats(min_value=-50.0, max_value=50.0)
bed = st.floats(min_value=-5000.0, max_value=100.0)


@settings(max_examples=400, deadline=None)
@given(wet_h, mom, mom, bed, wet_h, mom, mom, bed)
def test_fwaves_sum_to_flux_jump_plus_source(orc, hL, uL, vL, bL, hR, uR, vR, bR):
    mL, tL, mR, tR = hL * uL, hL * vL, hR * uR, hR * vR
    Z, s, kind, _ = orc.riemann((hL, mL, tL, bL), (hR, mR, tR, bR))
    assert kind == orc.EDGE_WET
    expect = _flux(hR, mR, tR) - _flux(hL, mL, tL)
    expect[1] += G * 0.5 * (hL + hR) * (bR - bL)
    total = Z.sum(axis=0)
    scale = np.array([abs(mL) + abs(mR), abs(_flux(hL, mL, tL)[1]) + abs(_flux(hR, mR, tR)[1])
                      + G * 0.5 * (hL + hR) * (abs(bL) + abs(bR)),
                      abs(mL * tL / hL) + abs(mR * tR / hR)]) + np.abs(Z).sum(axis=0)
    assert np.all(np.abs(total - expect) <= 1e-12 * scale + 1e-300), (total, expect)
    assert s[0] <= s[1] <= s[2]
    assert Z[1, 0] == 0.0


@settings(max_examples=300, deadline=None)
@given(wet_h, mom, mom, mom, mom, bed)
def test_fluctuations_split_the_flux_jump(orc, h, u, vL, vR, shift, b):
    # symmetric normal velocities give a shear wave of exactly zero speed; the
    # two fluctuations together must still carry the whole flux jump
    for left, right in (((h, h * u, h * vL, b), (h, -h * u, h * vR, b)),
                        ((h, h * u, h * vL, b), (h + abs(shift), h * vR, h * u, b - 1.0))):
        am, ap = orc.fluctuations(left, right)
        expect = _flux(right[0], right[1], right[2]) - _flux(left[0], left[1], left[2])
        expect[1] += G * 0.5 * (left[0] + right[0]) * (right[3] - left[3])
        # roundoff bound: the fluctuations are sums of the f-waves, which can
        # be much larger than their sum (the transverse momentum rides on
        # waves of size |Z|), so the scale includes sum_p |Z^p|
        Z, _, _, _ = orc.riemann(left, right)
        scale = (np.abs(_flux(*left[:3])) + np.abs(_flux(*right[:3]))
                 + G * (left[0] + right[0]) * abs(b) + np.abs(Z).sum(axis=0) + 1.0)
        assert np.all(np.abs(am + ap - expect) <= 1e-12 * scale)


@settings(max_examples=300, deadline=None)
@given(st.floats(min_value=-4000.0, max_value=-0.01), st.floats(min_value=-4000.0, max_value=-0.01),
       st.floats(min_value=-2.0, max_value=2.0))
def test_lake_at_rest_wet_wet_is_exactly_zero(orc, bL, bR, eta):
    hL, hR = max(0.0, eta - bL), max(0.0, eta - bR)
    # the depth must reproduce the surface exactly: use beds for which eta - b is exact
    bL, bR = eta - hL, eta - hR
    Z, s, kind, _ = orc.riemann((hL, 0.0, 0.0, bL), (hR, 0.0, 0.0, bR))
    if hL + bL == hR + bR:
        assert np.all(Z == 0.0)


@pytest.mark.parametrize("h_wet,b_wet,b_dry,h_dry", [
    (10.0, -10.0, 5.0, 0.0),        # wet cell against a high dry bank
    (4000.0, -4000.0, 50.0, 0.0),
    (0.5, -0.5, 0.0, 0.0),          # bank exactly at sea level
    (1.0, -1.0, 0.0005, 0.0),
])
def test_lake_at_rest_against_dry_bank(orc, h_wet, b_wet, b_dry, h_dry):
    for left, right in [((h_wet, 0, 0, b_wet), (h_dry, 0, 0, b_dry)),
                        ((h_dry, 0, 0, b_dry), (h_wet, 0, 0, b_wet))]:
        Z, s, kind, _ = orc.riemann(left, right)
        assert np.all(Z == 0.0)
        am, ap = orc.fluctuations(left, right)
        assert np.all(am == 0.0) and np.all(ap == 0.0)


def test_lake_at_rest_shallower_than_drytol(orc):
    # a wet cell next to a cell whose depth is below the dry tolerance but whose
    # surface is at the same level: no waves
    for hs in (1e-4, 5e-4, 1e-3):
        Z, s, kind, _ = orc.riemann((2.0, 0, 0, -2.0), (hs, 0, 0, -hs))
        assert np.all(Z == 0.0), hs
        Z, s, kind, _ = orc.riemann((hs, 0, 0, -hs), (2.0, 0, 0, -2.0))
        assert np.all(Z == 0.0), hs
    Z, s, kind, _ = orc.riemann((0.0, 0, 0, 1.0), (0.0, 0, 0, 3.0))
    assert kind == orc.EDGE_DRY and np.all(Z == 0.0) and np.all(s == 0.0)


@settings(max_examples=300, deadline=None)
@given(wet_h, mom, mom, st.floats(min_value=-100.0, max_value=100.0))
def test_uniform_state_gives_no_waves(orc, h, u, v, b):
    Z, s, kind, _ = orc.riemann((h, h * u, h * v, b), (h, h * u, h * v, b))
    assert np.all(Z == 0.0)


any_h = st.one_of(st.just(0.0), st.floats(min_value=0.0, max_value=0.002), wet_h)


@settings(max_examples=500, deadline=None)
@given(any_h, mom, mom, bed, any_h, mom, mom, bed)
def test_mirror_symmetry_bitwise(orc, hL, uL, vL, bL, hR, uR, vR, bR):
    # reflecting x -> -x swaps the sides and negates the normal momentum; the
    # mass and transverse flux components change sign, the normal momentum flux
    # does not, and the wave families 1 and 3 trade places
    mL, tL, mR, tR = hL * uL, hL * vL, hR * uR, hR * vR
    Z, s, kind, _ = orc.riemann((hL, mL, tL, bL), (hR, mR, tR, bR))
    Zm, sm, kindm, _ = orc.riemann((hR, -mR, tR, bR), (hL, -mL, tL, bL))
    flip = np.array([1.0, -1.0, 1.0])
    assert np.array_equal(sm, -s[::-1])
    assert np.array_equal(Zm, Z[::-1] * flip[None, :])
    swap = {orc.EDGE_WET: orc.EDGE_WET, orc.EDGE_DRY: orc.EDGE_DRY,
            orc.EDGE_WALL_R: orc.EDGE_WALL_L, orc.EDGE_WALL_L: orc.EDGE_WALL_R}
    assert kindm == swap[kind]


@settings(max_examples=600, deadline=None)
@given(any_h, mom, mom, bed, any_h, mom, mom, bed, st.floats(min_value=0.05, max_value=1.0))
def test_first_order_update_keeps_depth_nonnegative(orc, hL, uL, vL, bL, hR, uR, vR, bR, cfl):
    mL, tL, mR, tR = hL * uL, hL * vL, hR * uR, hR * vR
    Z, s, kind, _ = orc.riemann((hL, mL, tL, bL), (hR, mR, tR, bR))
    smax = np.abs(s).max()
    if smax == 0.0:
        return
    lam = cfl / smax
    am, ap = orc.fluctuations((hL, mL, tL, bL), (hR, mR, tR, bR))
    newL = hL - lam * am[0]
    newR = hR - lam * ap[0]
    tol = 1e-12 * max(hL, hR, 1.0)
    assert newL >= -tol and newR >= -tol


@settings(max_examples=300, deadline=None)
@given(st.floats(min_value=0.01, max_value=50.0), mom, mom, st.floats(min_value=-60.0, max_value=-1.0))
def test_wall_edge_matches_explicit_mirror(orc, h, u, v, bwet):
    # wet cell (depth h, bed bwet) against a dry bank far above its surface
    bank = bwet + h + 1000.0
    m, t = h * u, h * v
    Z, s, kind, _ = orc.riemann((h, m, t, bwet), (0.0, 0.0, 0.0, bank))
    assert kind == orc.EDGE_WALL_R
    am, ap = orc.fluctuations((h, m, t, bwet), (0.0, 0.0, 0.0, bank))
    Zm, sm, km, _ = orc.riemann((h, m, t, bwet), (h, -m, t, bwet))
    assert km == orc.EDGE_WET
    # the left-going part of the mirror problem is what the wet cell receives
    left = Zm[sm < 0].sum(axis=0) + 0.5 * Zm[sm == 0].sum(axis=0)
    assert np.allclose(am, left, rtol=0, atol=1e-12 * (abs(m) + G * h * h + abs(m * t / h) + 1))
    assert np.all(ap == 0.0)
    assert np.all(s >= -1e300) and np.all(s <= 0.0)


def test_wall_test_lets_water_over_low_bank(orc):
    # a fast flow toward a dry cell whose bed is below the run-up height floods it
    h, u = 1.0, 3.0
    hstar = (math.sqrt(G * h) + 0.5 * u) ** 2 / G
    Z, s, kind, _ = orc.riemann((h, h * u, 0.0, 0.0), (0.0, 0.0, 0.0, 0.9 * hstar))
    assert kind == orc.EDGE_WET
    Z, s, kind, _ = orc.riemann((h, h * u, 0.0, 0.0), (0.0, 0.0, 0.0, 1.1 * hstar))
    assert kind == orc.EDGE_WALL_R


def test_dry_front_speed(orc):
    # wet cell next to a dry bed at the same bed level: the front speed is u + 2c
    h, u = 2.0, 0.5
    Z, s, kind, _ = orc.riemann((h, h * u, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0))
    c = math.sqrt(G * h)
    assert s[2] == pytest.approx(u + 2 * c, rel=1e-15)
    assert s[0] == pytest.approx(u - c, rel=1e-15)


@settings(max_examples=400, deadline=None)
@given(st.floats(min_value=0.05, max_value=20.0), st.floats(min_value=0.0, max_value=4.0),
       st.floats(min_value=0.01, max_value=0.99), st.floats(min_value=-500.0, max_value=50.0))
def test_empty_cell_on_a_bank_loses_no_water(orc, hR, fr, rise, bR):
    # left: an empty cell on a bank whose bed lies below the right surface
    # (the water can reach it, no wall); right: water running away from it.
    # At the bound of the stationary jump the left middle depth is 0 in exact
    # arithmetic, so A-dQ carries no mass out of the empty cell: its depth
    # after a first-order update, 0 - lam * A-dQ[0], must not go below 0
    cR = math.sqrt(G * hR)
    uR = fr * cR
    bL = bR + rise * hR
    left, right = (0.0, 0.0, 0.0, bL), (hR, hR * uR, 0.0, bR)
    Z, s, kind, clamped = orc.riemann(left, right)
    assert kind == orc.EDGE_WET
    am, ap = orc.fluctuations(left, right)
    if clamped:
        assert am[0] <= 0.0, (am[0], Z[0])
    # the mirror image: the empty cell on the right
    am2, ap2 = orc.fluctuations((hR, -hR * uR, 0.0, bR), (0.0, 0.0, 0.0, bL))
    _, _, _, clamped2 = orc.riemann((hR, -hR * uR, 0.0, bR), (0.0, 0.0, 0.0, bL))
    if clamped2:
        assert ap2[0] <= 0.0, (ap2[0],)


def test_empty_cell_on_a_bank_grid_hits_the_bound(orc):
    # the same on a fixed grid of states, which reaches the bound many times
    hits = 0
    for hR in (0.3, 1.0, 2.5, 7.0):
        for fr in np.linspace(0.5, 3.5, 13):
            for rise in (0.05, 0.3, 0.6, 0.9):
                uR = fr * math.sqrt(G * hR)
                bR = -3.0
                bL = bR + rise * hR
                left, right = (0.0, 0.0, 0.0, bL), (hR, hR * uR, 0.0, bR)
                _, _, kind, clamped = orc.riemann(left, right)
                am, _ = orc.fluctuations(left, right)
                if clamped:
                    hits += 1
                    assert am[0] <= 0.0
                _, _, _, c2 = orc.riemann((hR, -hR * uR, 0.0, bR), (0.0, 0.0, 0.0, bL))
                _, ap2 = orc.fluctuations((hR, -hR * uR, 0.0, bR), (0.0, 0.0, 0.0, bL))
                if c2:
                    assert ap2[0] <= 0.0
    assert hits >= 20
