"""Pins of the reference latitude-longitude split step (an extension: capacity
kappa_j and parallel-edge lengths from the sphere's geometry): the
capacities telescope to the band's area; a sea at rest stays bitwise at
rest; mass on the sphere (sum of h kappa) is conserved to roundoff with walls;
a state independent of longitude stays so, with no zonal momentum; a
configuration mirrored about the equator stays mirrored; a thin band at the
equator reproduces the Cartesian step."""
import numpy as np
import pytest

import oracle as O
from paper_1901_06798_amd import workloads as W


@pytest.fixture(scope="module")
def P():
    O.lib()
    return O.params()


def setup(pb):
    q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b)
    g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
    O.ghost_fill_b(g, b)
    kap, ln = O.sphere_metric(pb.meta["lat0"], pb.meta["dlat"], pb.my, pb.bc)
    return q, b, g, kap, ln


def run(P, pb, dt, n):
    q, b, g, kap, ln = setup(pb)
    for _ in range(n):
        O.ghost_fill(g, q)
        out, _, _, nf = O.step_sphere(P, g, q, b, dt, kap, ln)
        assert nf == 0
        q[2:-2, 2:-2] = out[2:-2, 2:-2]
    return q, b, kap


def test_capacities_telescope_to_the_band_area():
    kap, ln = O.sphere_metric(-20.0, 0.5, 100)
    d = np.deg2rad(0.5)
    assert np.sum(kap[2:-2]) * d == pytest.approx(np.sin(np.deg2rad(30.0)) - np.sin(np.deg2rad(-20.0)),
                                                  rel=1e-14)
    assert np.all(kap > 0) and np.all(kap <= 1.0)
    assert ln[2] == pytest.approx(np.cos(np.deg2rad(-20.0)), rel=1e-15)


def test_sea_at_rest_stays_bitwise_at_rest(P):
    pb = W.latlon_basin(48, 40, lat0=30.0, amp=0.0)
    q, b, _ = run(P, pb, 20.0, 20)
    inner = q[2:-2, 2:-2]
    assert not inner[..., 1:].any()
    wet = inner[..., 0] > 0
    assert np.all((inner[..., 0] + b[2:-2, 2:-2])[wet] == 0.0)


def test_mass_on_the_sphere_is_conserved_with_walls(P):
    # long enough for the waves to reach the walls at both latitudes
    pb = W.latlon_basin(48, 40, lat0=40.0, shelf=False, amp=3.0)
    q0, _, _, kap, _ = setup(pb)
    m0 = np.sum(q0[2:-2, 2:-2, 0] * kap[2:-2, None])
    q, _, kap = run(P, pb, 20.0, 300)
    m1 = np.sum(q[2:-2, 2:-2, 0] * kap[2:-2, None])
    assert abs(m1 - m0) / m0 <= 1e-14
    assert np.abs(q[2:-2, 2:-2, 1]).max() > 1.0  # water moved
    assert np.abs(q[2, 2:-2, 2]).max() > 1.0 and np.abs(q[-3, 2:-2, 2]).max() > 1.0


def test_wall_ghost_rows_mirror_the_geometry():
    my = 30
    kap, ln = O.sphere_metric(50.0, 0.2, my, (O.BC_WALL,) * 4)
    g_kap, g_ln = O.sphere_metric(50.0, 0.2, my)
    assert kap[1] == kap[2] and kap[0] == kap[3] and ln[1] == ln[3] and ln[0] == ln[4]
    assert kap[my + 2] == kap[my + 1] and kap[my + 3] == kap[my]
    assert ln[my + 3] == ln[my + 1] and ln[my + 4] == ln[my]
    assert np.array_equal(kap[2:my + 2], g_kap[2:my + 2]) and np.array_equal(ln[2:my + 3], g_ln[2:my + 3])
    ekap, eln = O.sphere_metric(50.0, 0.2, my, (O.BC_EXTRAP,) * 4)
    assert np.array_equal(ekap, g_kap) and np.array_equal(eln, g_ln)


def test_longitude_independent_state_stays_so(P):
    pb = W.latlon_basin(24, 40, lat0=10.0, shelf=False, amp=0.0)
    lat = 10.0 + (np.arange(40) + 0.5) * 0.25
    pb.h = pb.h + 2.0 * np.exp(-((lat - 15.0) / 1.5) ** 2)[:, None]
    q, _, _ = run(P, pb, 20.0, 30)
    inner = q[2:-2, 2:-2]
    assert np.all(inner[..., 1] == 0.0)
    assert np.all(inner == inner[:, :1, :])
    assert np.abs(inner[..., 2]).max() > 1.0


def test_mirror_about_the_equator(P):
    pb = W.latlon_basin(30, 40, lat0=-5.0, dlat=0.25, shelf=False, amp=2.0,
                        src=(140.0 + 3.1, 0.0), sigma_deg=1.0)
    q, _, _ = run(P, pb, 20.0, 30)
    inner = q[2:-2, 2:-2]
    assert np.allclose(inner[..., 0], inner[::-1, :, 0], rtol=1e-13, atol=0)
    assert np.allclose(inner[..., 1], inner[::-1, :, 1], rtol=1e-12, atol=1e-12)
    assert np.allclose(inner[..., 2], -inner[::-1, :, 2], rtol=1e-12, atol=1e-12)
    assert np.abs(inner[..., 2]).max() > 0.1


def test_thin_equatorial_band_is_the_cartesian_step(P):
    pb = W.latlon_basin(40, 30, lat0=-0.0375, dlat=0.0025, dlon=0.0025, shelf=False,
                        amp=1.0, sigma_deg=0.01)
    qs, _, _ = run(P, pb, 0.5, 20)
    q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b)
    g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
    O.ghost_fill_b(g, b)
    for _ in range(20):
        O.ghost_fill(g, q)
        out, _, _, _ = O.step(P, g, q, b, 0.5)
        q[2:-2, 2:-2] = out[2:-2, 2:-2]
    for k in range(3):
        scale = np.abs(q[2:-2, 2:-2, k]).max()
        # kappa and len differ from 1 by at most (band half-width in radians)^2 / 2
        assert np.abs(qs[2:-2, 2:-2, k] - q[2:-2, 2:-2, k]).max() <= 1e-6 * scale
    assert np.abs(q[2:-2, 2:-2, 1]).max() > 0.01
