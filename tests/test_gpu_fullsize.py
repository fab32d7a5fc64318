"""Parity at the headline size, in the launch configuration the bench times
(and at the size of the bench's latitude-longitude patch):
the 4096^2 shelf is advanced on the GPU (FP64 and FP32 surface deviation) far
enough for the wave to run up the coast; then one more step is checked on
sampled windows.  For each window the reference solver takes one step of the
window alone, its two ghost layers filled from the GPU's state before the
step (the big grid's extrapolation ghosts are the edge copies), with the dt
the GPU used.  A cell's new value depends only on its 5 x 5 neighbourhood,
so the window's interior must match the GPU's: FP64 to 1e-12 relative
(in practice bit for bit), FP32 to 1e-5 m of surface."""
import numpy as np
import pytest

from paper_1901_06798_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 4096
STEPS = 1500  # the source reaches the shoreline after ~1300 steps
WIN = 16


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.solver import PatchSolver
    L.lib()
    return L, PatchSolver, torch


@pytest.fixture(scope="module")
def shelf():
    return W.shelf_4096()


def windows(h, rng):
    """Window origins (interior coordinates): random, along the wet/dry line,
    around the source, and at the four domain sides and corners."""
    n = h.shape[0]
    out = [tuple(rng.integers(0, n - WIN, 2)) for _ in range(24)]
    wet = h > 1e-3
    edge = np.argwhere(wet[:, 1:] != wet[:, :-1])
    for k in rng.choice(len(edge), 8, replace=False):
        j, i = edge[k]
        out.append((int(np.clip(j - WIN // 2, 0, n - WIN)), int(np.clip(i - WIN // 2, 0, n - WIN))))
    c = n // 2
    out += [(c - WIN // 2 + d, c - WIN // 2 + e) for d, e in ((0, 0), (-200, 150), (300, -250), (-700, 40))]
    out += [(0, 0), (0, n - WIN), (n - WIN, 0), (n - WIN, n - WIN), (0, n // 3), (n - WIN, 2 * n // 3),
            (n // 5, 0), (3 * n // 5, n - WIN)]
    return out


def padded(a):
    # extrapolation ghosts of the big grid: edge copies, corners included
    return np.pad(a, 2, mode="edge")


def window_step(orc, P, state, b, j0, i0, dt, dx):
    qs = [padded(f)[j0: j0 + WIN + 4, i0: i0 + WIN + 4] for f in state]
    bw = padded(b)[j0: j0 + WIN + 4, i0: i0 + WIN + 4]
    q, bb = orc.new_state(qs[0][2:-2, 2:-2], qs[1][2:-2, 2:-2], qs[2][2:-2, 2:-2],
                          bw[2:-2, 2:-2])
    # ghost layers from the GPU's state (user boundaries: taken as given)
    for k in range(3):
        q[..., k] = qs[k]
    bb[...] = bw
    g = orc.grid(WIN, WIN, dx, dx, (orc.BC_USER,) * 4)
    out, _, _, nf = orc.step(P, g, q, bb, dt)
    assert nf == 0
    return out[2:-2, 2:-2]


@pytest.mark.parametrize("precision", [0, 1])
def test_fullsize_windows_match_reference(gpu, orc, shelf, precision):
    L, PatchSolver, torch = gpu
    p = L.params(precision=precision)
    print(f"case fullsize 4096^2 shelf precision={precision} steps={STEPS}", flush=True)
    s = PatchSolver(shelf, p)
    s.initial_dt()
    s.run_async(STEPS)
    torch.cuda.synchronize()
    before = s.state()
    dt = float(s.dt.item())
    # the step the bench times: swe_patch_step with dt from device memory
    s.enqueue_step(cfl=False)
    torch.cuda.synchronize()
    after = s.state()
    st = int(s.status[0].item())
    assert st & (L.STATUS_NONFINITE | L.STATUS_CFL_EXCEEDED) == 0
    b = shelf.b if precision == 0 else shelf.b.astype(np.float32).astype(np.float64)
    P = orc.params()
    rng = np.random.default_rng(7)
    worst = 0.0
    for j0, i0 in windows(before[0], rng):
        ref = window_step(orc, P, before, b, j0, i0, dt, shelf.dx)
        got = [f[j0: j0 + WIN, i0: i0 + WIN] for f in after]
        if precision == 0:
            for k in range(3):
                scale = max(np.abs(after[k]).max(), 1e-300)
                e = np.abs(got[k] - ref[..., k]).max() / scale
                worst = max(worst, e)
                assert e <= 1e-12, f"window ({j0}, {i0}) field {k}: {e:.3e}"
        else:
            eta_ref = ref[..., 0] + b[j0: j0 + WIN, i0: i0 + WIN]
            eta_got = got[0] + b[j0: j0 + WIN, i0: i0 + WIN]
            wet = (ref[..., 0] > 1e-2) & (got[0] > 1e-2)
            e = np.abs(eta_got - eta_ref)[wet].max() if wet.any() else 0.0
            worst = max(worst, e)
            assert e <= 1e-5, f"window ({j0}, {i0}): surface error {e:.3e} m"
    print(f"worst {'relative' if precision == 0 else 'surface (m)'} error {worst:.3e}", flush=True)


def test_fullsize_sphere_windows_match_reference(gpu, orc):
    # the bench's latitude-longitude patch (the paper's Pacific extent in
    # 2.05-minute cells), heaviest first, advanced 600 steps; the windows'
    # capacities and edge lengths are those of their own rows
    L, _, torch = gpu
    from paper_1901_06798_amd.sphere import SphereSolver
    d = 140.0 / N
    ny = int(round(96.0 / d))
    pb = W.latlon_basin(N, ny, lon0=-240.0, lat0=-31.0, dlon=d, dlat=d, amp=2.0, sigma_deg=1.0,
                        src=(-217.5, 38.0), bc=(W.BC_EXTRAP,) * 4)
    print(f"case fullsize sphere {N}x{ny}", flush=True)
    s = SphereSolver(pb, L.params())
    s.initial_dt()
    s.run_async(600)
    torch.cuda.synchronize()
    before = s.state()
    dt = float(s.dt.item())
    s.enqueue_step(cfl=False)
    torch.cuda.synchronize()
    after = s.state()
    assert int(s.status[0].item()) & (L.STATUS_NONFINITE | L.STATUS_CFL_EXCEEDED) == 0
    P = orc.params()
    rng = np.random.default_rng(8)
    wet = before[0] > 1e-3
    edge = np.argwhere(wet[:, 1:] != wet[:, :-1])
    src_j, src_i = int((38.0 + 31.0) / d), int((-217.5 + 240.0) / d)
    origins = [(int(rng.integers(0, ny - WIN)), int(rng.integers(0, N - WIN))) for _ in range(16)]
    origins += [(int(np.clip(j - WIN // 2, 0, ny - WIN)), int(np.clip(i - WIN // 2, 0, N - WIN)))
                for j, i in edge[rng.choice(len(edge), 6, replace=False)]]
    origins += [(src_j - WIN // 2 + dj, src_i - WIN // 2 + di)
                for dj, di in ((0, 0), (-60, 40), (80, -70), (150, 150))]
    origins += [(0, 0), (ny - WIN, N - WIN), (0, N // 2), (ny - WIN, 7), (ny // 2, 0)]
    worst = 0.0
    for j0, i0 in origins:
        qs = [padded(f)[j0: j0 + WIN + 4, i0: i0 + WIN + 4] for f in before]
        bw = padded(pb.b)[j0: j0 + WIN + 4, i0: i0 + WIN + 4]
        q, bb = orc.new_state(qs[0][2:-2, 2:-2], qs[1][2:-2, 2:-2], qs[2][2:-2, 2:-2],
                              bw[2:-2, 2:-2])
        for k in range(3):
            q[..., k] = qs[k]
        bb[...] = bw
        g = orc.grid(WIN, WIN, pb.dx, pb.dy, (orc.BC_USER,) * 4)
        kap, ln = orc.sphere_metric(-31.0 + j0 * d, d, WIN)
        out, _, _, nf = orc.step_sphere(P, g, q, bb, dt, kap, ln)
        assert nf == 0
        for k in range(3):
            scale = max(np.abs(after[k]).max(), 1e-300)
            e = np.abs(after[k][j0: j0 + WIN, i0: i0 + WIN] - out[2:-2, 2:-2, k]).max() / scale
            worst = max(worst, e)
            assert e <= 1e-12, f"window ({j0}, {i0}) field {k}: {e:.3e}"
    print(f"worst relative error {worst:.3e}", flush=True)
