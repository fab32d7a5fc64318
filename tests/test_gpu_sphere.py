"""GPU tests of the latitude-longitude split step (swe_patch_step_sphere,
SphereSolver) against the reference step on the sphere: a basin at mid
latitudes with a wet/dry coast and walls, to the FP64 bar (relative 1e-12
per field) under a given dt sequence; a sea at rest stays bitwise at rest;
mass on the sphere is conserved to roundoff; the CFL rule on the device
keeps the Courant number within bounds."""
import numpy as np
import pytest

from paper_1901_06798_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.sphere import SphereSolver
    L.lib()
    return L, SphereSolver, torch


def reference(pb, dts, manning_n=0.0):
    import oracle as O
    O.lib()
    P = O.params(manning_n=manning_n)
    q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b)
    g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
    O.ghost_fill_b(g, b)
    kap, ln = O.sphere_metric(pb.meta["lat0"], pb.meta["dlat"], pb.my, pb.bc)
    for dt in dts:
        O.ghost_fill(g, q)
        out, _, c, nf = O.step_sphere(P, g, q, b, dt, kap, ln)
        assert nf == 0
        q[2:-2, 2:-2] = out[2:-2, 2:-2]
    return q


@pytest.mark.parametrize("lat0,bc,manning_n", [(20.0, W.BC_WALL, 0.0), (-50.0, W.BC_EXTRAP, 0.0),
                                               (35.0, W.BC_WALL, 0.025)])
def test_sphere_step_matches_the_reference(gpu, lat0, bc, manning_n):
    L, SphereSolver, torch = gpu
    pb = W.latlon_basin(150, 130, lat0=lat0, dlon=0.1, dlat=0.1, amp=3.0, sigma_deg=1.0,
                        bc=(bc,) * 4)
    print(f"case sphere basin 150x130 lat0={lat0} bc={bc} manning_n={manning_n}", flush=True)
    dts = [30.0] * 25
    s = SphereSolver(pb, L.params(manning_n=manning_n))
    s.run_forced(dts)
    torch.cuda.synchronize()
    ref = reference(pb, dts, manning_n)
    got = s.state()
    for k in range(3):
        want = ref[2:-2, 2:-2, k]
        err = np.abs(got[k] - want).max() / max(np.abs(want).max(), 1e-300)
        assert err <= 1e-12, (k, err)
    assert np.abs(got[2]).max() > 0.1


def test_sea_at_rest_and_mass_on_the_sphere(gpu):
    L, SphereSolver, torch = gpu
    rest = W.latlon_basin(96, 80, lat0=35.0, dlon=0.1, dlat=0.1, amp=0.0)
    s = SphereSolver(rest, L.params())
    s.run_forced([30.0] * 40)
    torch.cuda.synchronize()
    h, hu, hv = s.state()
    assert not hu.any() and not hv.any()
    wet = h > 0
    assert np.all((h + rest.b)[wet] == 0.0)
    hump = W.latlon_basin(96, 80, lat0=35.0, dlon=0.1, dlat=0.1, amp=3.0, shelf=False,
                          sigma_deg=1.0)
    s = SphereSolver(hump, L.params())
    m0 = s.mass()
    s.run_forced([30.0] * 150)
    torch.cuda.synchronize()
    assert abs(s.mass() - m0) / m0 <= 1e-13


def test_speeds_and_cfl_rule_on_the_sphere(gpu):
    L, SphereSolver, torch = gpu
    import oracle as O
    pb = W.latlon_basin(120, 100, lat0=55.0, dlon=0.05, dlat=0.05, amp=2.0, sigma_deg=0.5)
    print("case sphere speeds 120x100 lat0=55", flush=True)
    s = SphereSolver(pb, L.params())
    dt = torch.full((1,), 20.0, dtype=torch.float64, device=s.dev)
    s.enqueue_step(dt.data_ptr(), cfl=False)
    torch.cuda.synchronize()
    got = s.smax.cpu().numpy()
    O.lib()
    q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b)
    g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
    O.ghost_fill_b(g, b)
    O.ghost_fill(g, q)
    kap, ln = O.sphere_metric(pb.meta["lat0"], pb.meta["dlat"], pb.my, pb.bc)
    _, want, _, _ = O.step_sphere(O.params(), g, q, b, 20.0, kap, ln)
    assert np.allclose(got, want, rtol=1e-12, atol=0), (got, want)
    # the device CFL rule then keeps every accepted step within cfl_max
    s = SphereSolver(pb, L.params())
    dts = s.run(30)
    torch.cuda.synchronize()
    assert len(dts) == 30 and np.all(dts > 0)
    assert int(s.status[0].item()) & L.STATUS_CFL_EXCEEDED == 0


def test_heaviest_first_order_on_the_sphere_is_bitwise_index_order(gpu):
    L, SphereSolver, torch = gpu
    pb = W.latlon_basin(301, 257, lat0=-10.0, dlon=0.05, dlat=0.05, amp=2.0, sigma_deg=0.5)
    print("case sphere order 301x257", flush=True)
    a = SphereSolver(pb, L.params(), ordered=True, order_every=1)
    b = SphereSolver(pb, L.params(), ordered=False)
    da, db = a.run(30), b.run(30)
    torch.cuda.synchronize()
    assert np.array_equal(da, db)
    assert torch.equal(a.planes(), b.planes()) and torch.equal(a.status, b.status)
    n = L.swe_patch_tasks(a.pt)
    order = a.sched[:n].cpu().numpy()
    assert sorted(order.tolist()) == list(range(1, n + 1))


@pytest.mark.parametrize("nx,ny,lat0,dlat", [(7, 1, 60.0, 0.5), (61, 3, -70.0, 0.25),
                                             (125, 97, 72.0, 0.1), (64, 61, -5.0, 1.0)])
def test_small_and_high_latitude_patches(gpu, nx, ny, lat0, dlat):
    # one to three rows (a task shorter than its ghost frame), a ragged
    # strip, rows near 80 degrees (small capacities, large Courant factors)
    # and cells a degree tall across the equator
    L, SphereSolver, torch = gpu
    # a wall needs two cells beside it: one row takes extrapolation in y
    bc = (W.BC_WALL,) * 4 if ny >= 2 else (W.BC_WALL, W.BC_WALL, W.BC_EXTRAP, W.BC_EXTRAP)
    pb = W.latlon_basin(nx, ny, lat0=lat0, dlon=dlat, dlat=dlat, amp=1.5,
                        sigma_deg=max(2 * dlat, 0.3), shelf=nx > 40, bc=bc)
    print(f"case sphere small {nx}x{ny} lat0={lat0} dlat={dlat}", flush=True)
    s = SphereSolver(pb, L.params(), order_every=1)
    dts = s.run(12)
    torch.cuda.synchronize()
    assert int(s.status[0].item()) & (L.STATUS_NONFINITE | L.STATUS_CFL_EXCEEDED) == 0
    ref = reference(pb, dts)
    got = s.state()
    for k in range(3):
        want = ref[2:-2, 2:-2, k]
        scale = max(np.abs(want).max(), 1e-300)
        assert np.abs(got[k] - want).max() / scale <= 1e-12, (k,)


def test_first_step_speeds_on_the_sphere(gpu):
    # swe_speed_scan_sphere: the x-speeds are those the reference step reports
    # for the same state (bitwise: the same solves, scaled by the same 1 /
    # kappa); the y-speeds those of every y-edge of the initial state solved
    # by the reference Riemann solver, scaled by the mean of its two rows'
    # 1 / kappa; the first dt is cfl_desired over the larger Courant rate
    L, SphereSolver, torch = gpu
    import oracle as O
    pb = W.latlon_basin(60, 50, lat0=48.0, dlon=0.1, dlat=0.1, amp=2.0, sigma_deg=0.6,
                        bc=(W.BC_WALL, W.BC_EXTRAP, W.BC_WALL, W.BC_EXTRAP))
    s = SphereSolver(pb, L.params())
    s.smax.zero_()
    s.launch_scan()
    torch.cuda.synchronize()
    got = s.smax.cpu().numpy().copy()
    O.lib()
    P = O.params()
    q, b = O.new_state(pb.h, pb.hu, pb.hv, pb.b, bc=pb.bc)
    g = O.grid(pb.mx, pb.my, pb.dx, pb.dy, pb.bc)
    O.ghost_fill_b(g, b)
    O.ghost_fill(g, q)
    kap, ln = O.sphere_metric(pb.meta["lat0"], pb.meta["dlat"], pb.my, pb.bc)
    _, step_speeds, _, _ = O.step_sphere(P, g, q, b, 1.0, kap, ln)
    assert got[0] == step_speeds[0]
    sy = 0.0
    for j in range(2, pb.my + 3):          # edge between frame rows j - 1 and j
        a = 0.5 * (1.0 / kap[j - 1] + 1.0 / kap[j])
        for i in range(2, pb.mx + 2):
            lo, hi = q[j - 1, i], q[j, i]
            _, sp, _, _ = O.riemann((lo[0], lo[2], lo[1], b[j - 1, i]),
                                    (hi[0], hi[2], hi[1], b[j, i]), P)
            sy = max(sy, float(np.abs(sp).max()) * a)
    assert got[1] == sy
    s.initial_dt()
    torch.cuda.synchronize()
    rate = max(got[0] / pb.dx, got[1] / pb.dy)
    assert float(s.dt.item()) == P.cfl_desired / rate


def test_device_retake_on_the_sphere_equals_the_host_retake(gpu):
    # a first step 2.5 times the CFL step: the device redoes it (gated
    # swe_patch_retake_sphere) with the reduced dt, as the host loop does
    L, SphereSolver, torch = gpu
    pb = W.latlon_basin(90, 70, lat0=-30.0, dlon=0.1, dlat=0.1, amp=2.5, sigma_deg=0.8)
    print("case sphere retake 90x70", flush=True)
    host = SphereSolver(pb, L.params())
    host.initial_dt()
    big = 2.5 * float(host.dt.item())
    host.run(10, dt0=big)
    dev = SphereSolver(pb, L.params())
    dev.dt.fill_(big)
    dev.run_async(10)
    torch.cuda.synchronize()
    assert host.retakes >= 1
    assert int(dev.status[0].item()) & L.STATUS_RETAKEN
    assert not int(dev.status[0].item()) & L.STATUS_CFL_EXCEEDED
    for a, c in zip(host.state(), dev.state()):
        assert np.array_equal(a, c)


def test_mass_on_the_sphere_on_the_device(gpu):
    # swe_mass_sphere against sum(h kappa) dx dy of the same state on the host
    L, SphereSolver, torch = gpu
    from paper_1901_06798_amd.sphere import metric
    pb = W.latlon_basin(77, 41, lat0=60.0, dlon=0.2, dlat=0.2, amp=2.0, sigma_deg=1.0)
    s = SphereSolver(pb, L.params())
    s.run_forced([40.0] * 5)
    torch.cuda.synchronize()
    h = s.state()[0]
    kap = metric(pb.meta["lat0"], pb.meta["dlat"], pb.my, pb.bc)[2: pb.my + 2]
    want = float(np.sum(h * kap[:, None])) * pb.dx * pb.dy
    assert abs(s.mass() - want) <= 1e-14 * want
