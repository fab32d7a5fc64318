"""GPU tests of the batched step on the full AMR patch set (3000 patches,
200/800/2000 on levels 1-3, sides 16..96, 1/4/16 substeps per coarse step):
sampled patches of every level against the reference solver run patch by
patch with the device's step sizes (FP64, relative 1e-12); the coarse step
size against the CFL rule evaluated by the reference over all 3000 patches;
the captured coarse steps and another schedule bit for bit equal to the eager
run on every patch; the FP32 surface-deviation batched step within 1e-5 m of
the FP64 one on every cell wet in both."""
import numpy as np
import pytest

from helpers import interior, oracle_setup
from paper_1901_06798_amd import workloads as W

pytestmark = pytest.mark.gpu
NCOARSE = 2


@pytest.fixture(scope="module")
def full_set():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1901_06798_amd import _lib as L
    from paper_1901_06798_amd.batched import BatchedSolver
    L.lib()
    specs, probs = W.amr_patch_set()
    trefs = [s.tref for s in specs]
    print(f"case full AMR patch set: {len(probs)} patches, eager FP64", flush=True)
    bs = BatchedSolver(probs, L.params(), trefs=trefs, sched=L.schedule(seg=64, waves_per_group=4))
    bs.initial_dt()
    dts = bs.run(NCOARSE, record_dt=True)[:, 0]
    torch.cuda.synchronize()
    return L, BatchedSolver, torch, specs, probs, trefs, bs, dts


def sample(specs, per_level=8, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for lev in (1, 2, 3):
        ks = [k for k, s in enumerate(specs) if s.level == lev]
        big = max(ks, key=lambda k: specs[k].mx * specs[k].my)
        out += [big] + [int(k) for k in rng.choice(ks, per_level - 1, replace=False) if k != big]
    return out


def test_sampled_patches_match_the_reference(full_set, orc):
    L, BatchedSolver, torch, specs, probs, trefs, bs, dts = full_set
    assert bs.flags() == (0, 0)
    P = orc.params()
    ks = sample(specs)
    print(f"comparing {len(ks)} sampled patches over {NCOARSE} coarse steps", flush=True)
    for k in ks:
        g, q, b = oracle_setup(orc, probs[k])
        t = trefs[k]
        for dt in dts:
            orc.run(P, g, q, b, t, dt_forced=[dt / t] * t)
        for f, a in zip(range(3), bs.state(k)):
            ref = interior(q)[..., f]
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(a - ref).max() / scale <= 1e-12, (k, specs[k].level, f)
    # the sample holds moving water on every level
    for lev in (1, 2, 3):
        assert any(np.abs(bs.state(k)[1]).max() > 0.0 for k in ks if specs[k].level == lev)


def test_coarse_dt_follows_the_cfl_rule_over_all_patches(full_set, orc):
    # dt_1 = cfl_desired / max over patches of (max speed / dx) / tref, the
    # initial state scanned by the reference
    L, BatchedSolver, torch, specs, probs, trefs, bs, dts = full_set
    P = orc.params()
    rate = 0.0
    for k, pb in enumerate(probs):
        g, q, b = oracle_setup(orc, pb)
        sm = orc.speed_scan(P, g, q, b)
        rate = max(rate, max(sm[0] / g.dx, sm[1] / g.dy) / trefs[k])
    assert dts[0] == pytest.approx(P.cfl_desired / rate, rel=1e-15)
    assert np.all(dts > 0.0)


def test_graph_replay_and_another_schedule_equal_the_eager_run(full_set):
    L, BatchedSolver, torch, specs, probs, trefs, bs, dts = full_set
    print("case full AMR patch set: graph replay, seg 32 per substep, packed", flush=True)
    g = BatchedSolver(probs, L.params(), trefs=trefs, sched=L.schedule(seg=64, waves_per_group=4))
    g.initial_dt()
    g.capture(NCOARSE)
    g.replay()
    o = BatchedSolver(probs, L.params(), trefs=trefs, sched=L.schedule(seg=32, per_substep=1))
    o.initial_dt()
    o.run(NCOARSE)
    pk = BatchedSolver(probs, L.params(), trefs=trefs, sched=L.schedule(seg=0))
    pk.initial_dt()
    pk.run(NCOARSE)
    torch.cuda.synchronize()
    for k in range(len(probs)):
        want = bs.state(k)
        for a, c, d, w in zip(g.state(k), o.state(k), pk.state(k), want):
            assert np.array_equal(a, w) and np.array_equal(c, w) and np.array_equal(d, w), k


def test_fp32_batched_within_1e5_m_of_fp64(full_set):
    L, BatchedSolver, torch, specs, probs, trefs, bs, dts = full_set
    print("case full AMR patch set: FP32 deviation with the FP64 step sizes", flush=True)
    b32 = BatchedSolver(probs, L.params(precision=L.F32_DEV), trefs=trefs)
    d = torch.tensor(dts, dtype=torch.float64, device=b32.dev)
    for n in range(NCOARSE):
        b32.enqueue_step(cfl=False, dt_ptr=d.data_ptr() + 8 * n)
        b32.smax.zero_()
    torch.cuda.synchronize()
    assert b32.flags()[0] & (L.STATUS_NONFINITE | L.STATUS_NEG_DEPTH) == 0
    worst, wet = 0.0, 0
    for k in range(len(probs)):
        h64, h32 = bs.state(k)[0], b32.state(k)[0]
        both = (h64 > 1e-2) & (h32 > 1e-2)
        if both.any():
            worst = max(worst, float(np.abs(b32.surface(k) - bs.surface(k))[both].max()))
            wet += int(both.sum())
    print(f"FP32 batched: max surface difference {worst:.3e} m over {wet} wet cells", flush=True)
    assert wet > 1_000_000
    assert worst <= 1e-5
