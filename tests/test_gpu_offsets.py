"""Largest addresses: patches whose cells sit beyond 2^31 elements of their
pool (FP32 planes of more than 8 GiB), through swe_patch_step and
swe_batched_step, give bit for bit the results of the same patch at offset 0
(every index is 64-bit).  Also the empty batch and the empty reductions."""
import numpy as np
import pytest

from paper_1901_06798_amd import workloads as W

pytestmark = pytest.mark.gpu

BIG = (1 << 31) + 4096  # plane stride in elements, > 2^31


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.solver import patch_table
    L.lib()
    return L, patch_table, torch


def layout(pb):
    pitch = ((pb.mx + 4 + 15) // 16) * 16
    return pitch, pitch * (pb.my + 4)


def host_planes(pb, p, L):
    pitch, n = layout(pb)
    rows = pb.my + 4
    q = np.zeros((3, rows, pitch), np.float32)
    bb = np.zeros((rows, pitch), np.float32)
    inner = (slice(2, pb.my + 2), slice(2, pb.mx + 2))
    q[0][inner] = np.where(pb.h > 0, pb.h + pb.b - p.sea_level, pb.b - p.sea_level)
    q[1][inner] = pb.hu
    q[2][inner] = pb.hv
    bb[inner] = pb.b
    return q.reshape(3, n), bb.reshape(n)


def advance(L, torch, p, pt, table, qin, qout, b, steps, batched=False, plan=None):
    dev = qin.device
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    smax = torch.zeros(2, dtype=torch.float64, device=dev)
    status = torch.zeros(2, dtype=torch.int32, device=dev)
    queue = torch.zeros(2, dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    L.swe_speed_scan(p, table.data_ptr(), 1, pt.mx, pt.my, qin.data_ptr(), b.data_ptr(),
                     smax.data_ptr(), s)
    L.swe_cfl_reduce(p, table.data_ptr(), 1, 1, smax.data_ptr(), dt.data_ptr(),
                     status.data_ptr(), 0, 1, s)
    bufs = [qin, qout]
    for k in range(steps):
        a, c = bufs[k % 2], bufs[(k + 1) % 2]
        if batched:
            pl, items, tasks, sched = plan
            plain = tasks.data_ptr() + L.SWE_TASK_BYTES * (pl.ntasks - pl.nplain)
            L.swe_batched_step(p, table.data_ptr(), items.data_ptr(), pl.nitems,
                               tasks.data_ptr(), plain, pl.nplain, pl.nsub, a.data_ptr(),
                               c.data_ptr(), 0, a.numel(), b.data_ptr(), dt.data_ptr(),
                               smax.data_ptr(),
                               status.data_ptr(), queue.data_ptr(), sched, s)
        else:
            L.swe_patch_step(p, pt, a.data_ptr(), c.data_ptr(), b.data_ptr(), dt.data_ptr(),
                             smax.data_ptr(), status.data_ptr(), s)
        L.swe_cfl_reduce(p, table.data_ptr(), 1, 1, smax.data_ptr(), dt.data_ptr(),
                         status.data_ptr(), 0, 0, s)
    torch.cuda.synchronize()
    return bufs[steps % 2], int(status[0].item())


@pytest.mark.parametrize("batched", [False, True])
def test_offsets_beyond_2_31_elements(gpu, batched):
    L, patch_table, torch = gpu
    pb = W.gaussian_hump(100, 1000.0, sigma=8e3)
    p = L.params(precision=L.F32_DEV)
    pitch, n = layout(pb)
    q, bb = host_planes(pb, p, L)
    off = (1 << 31) + 512
    print(f"case offsets beyond 2^31 elements batched={batched} off={off} stride={BIG}",
          flush=True)
    dev = torch.device("cuda:0")
    steps = 6
    results = []
    for o, stride in ((0, n), (off, BIG)):
        size = o + 2 * stride + n
        qin = torch.empty(size, dtype=torch.float32, device=dev)
        qout = torch.empty(size, dtype=torch.float32, device=dev)
        b = torch.empty(o + n, dtype=torch.float32, device=dev)
        for k in range(3):
            qin[o + k * stride: o + k * stride + n].copy_(torch.from_numpy(q[k]))
            qout[o + k * stride: o + k * stride + n].zero_()
        b[o: o + n].copy_(torch.from_numpy(bb))
        pt = L.patch(pb.mx, pb.my, pitch, pb.dx, pb.dy, off=o, plane_stride=stride, bc=pb.bc)
        table = patch_table([pt]).to(dev)
        plan = None
        if batched:
            sched = L.schedule(seg=64, waves_per_group=4)
            pl = L.swe_batched_plan([pt], sched)
            plan = (pl, *pl.device(dev), sched)
        res, st = advance(L, torch, p, pt, table, qin, qout, b, steps, batched, plan)
        assert st & (L.STATUS_NONFINITE | L.STATUS_NEG_DEPTH) == 0
        results.append(torch.stack([res[o + k * stride: o + k * stride + n] for k in range(3)])
                       .cpu().numpy())
        del qin, qout, b, res
        torch.cuda.empty_cache()
    assert np.array_equal(results[0], results[1])
    # the step moved the water (the comparison is not of two untouched states)
    assert not np.array_equal(results[0][0], q[0])


def test_empty_batches(gpu):
    L, patch_table, torch = gpu
    dev = torch.device("cuda:0")
    p = L.params()
    z = torch.zeros(64, dtype=torch.float64, device=dev)
    st = torch.zeros(2, dtype=torch.int32, device=dev)
    q = torch.zeros(2, dtype=torch.int32, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    # zero patches / items: nothing is launched and nothing is written
    L.swe_ghost_fill(p, z.data_ptr(), 0, 1, 1, z.data_ptr(), z.data_ptr(), 1, s)
    L.swe_speed_scan(p, z.data_ptr(), 0, 1, 1, z.data_ptr(), z.data_ptr(), z.data_ptr(), s)
    L.swe_mass(p, z.data_ptr(), 0, z.data_ptr(), z.data_ptr(), z.data_ptr(), s)
    sched = L.schedule()
    L.swe_batched_step(p, z.data_ptr(), z.data_ptr(), 0, z.data_ptr(), z.data_ptr(), 0, 0,
                       z.data_ptr(), z[32:].data_ptr(), 0, 32, z.data_ptr(), z.data_ptr(),
                       z.data_ptr(), st.data_ptr(), q.data_ptr(), sched, s)
    torch.cuda.synchronize()
    assert int(st.abs().sum().item()) == 0 and int(q.abs().sum().item()) == 0
    assert float(z.abs().sum().item()) == 0.0
