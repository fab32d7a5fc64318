"""GPU tests of the batched-step autotuner: it picks the fastest candidate it
timed, leaves the state as it found it, and reuses a cached choice for a patch
set of the same shape."""
import json

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
    from paper_1901_06798_amd import autotune as A
    from paper_1901_06798_amd.batched import BatchedSolver
    L.lib()
    return L, A, BatchedSolver, torch


def small_set():
    specs, probs = W.amr_patch_set(npatch=(5, 8, 12), seed=9)
    return probs, [s.tref for s in specs]


CANDS = [(64, 0, 4, 0, 0), (32, 0, 4, 0, 0), (64, 8, 2, 1, 0), (32, 16, 8, 0, 0),
         (64, 0, 4, 0, 1)]


def test_tune_picks_fastest_keeps_state_and_caches(gpu, tmp_path):
    L, A, BatchedSolver, torch = gpu
    probs, trefs = small_set()
    p = L.params()
    cands = [L.schedule(seg=s, rows_per_task=r, waves_per_group=w, groups_per_cu=g,
                        per_substep=u) for s, r, w, g, u in CANDS]
    print("case autotune small AMR set, 5 candidates", flush=True)
    bs = BatchedSolver(probs, p, trefs=trefs)
    bs.initial_dt()
    bs.run(2)
    torch.cuda.synchronize()
    before = [bs.state(k) for k in range(len(probs))]
    cache = str(tmp_path / "tune.json")
    best = A.tune(bs, cands=cands, cache_path=cache)
    torch.cuda.synchronize()
    res = bs.tune_results
    assert len(res) == len(cands)
    assert A._sched_dict(best) == res[0][1]
    assert all(res[0][0] <= r[0] for r in res)
    # tuning restores the state it timed on
    for k in range(len(probs)):
        for a, c in zip(bs.state(k), before[k]):
            assert np.array_equal(a, c)
    # and the tuned schedule gives the same steps as the default one
    bs.run(3)
    ref = BatchedSolver(probs, p, trefs=trefs)
    ref.initial_dt()
    ref.run(5)
    torch.cuda.synchronize()
    for k in range(len(probs)):
        for a, c in zip(bs.state(k), ref.state(k)):
            assert np.array_equal(a, c), f"patch {k}"
    with open(cache) as f:
        stored = json.load(f)
    assert A.signature(bs) in stored
    assert stored[A.signature(bs)]["schedule"] == A._sched_dict(best)
    # a patch set of the same signature takes the cached choice without timing
    again = BatchedSolver(probs, p, trefs=trefs)
    got = A.tune(again, cands=cands, cache_path=cache)
    assert again.tune_results == []
    assert A._sched_dict(got) == A._sched_dict(best)
    assert A._sched_dict(again.sched) == A._sched_dict(best)
