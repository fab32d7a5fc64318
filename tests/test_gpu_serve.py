"""GPU tests of the scenario server: continuous batching with admission by
HBM footprint; each scenario's result is bit for bit its result alone."""
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
    from paper_1901_06798_amd.serve import Scenario, ScenarioServer
    from paper_1901_06798_amd.solver import PatchSolver
    L.lib()
    return L, ScenarioServer, Scenario, PatchSolver, torch


@pytest.mark.parametrize("precision", [1, 0])
def test_mix_equals_alone(gpu, precision):
    L, ScenarioServer, Scenario, PatchSolver, torch = gpu
    p = L.params(precision=precision)
    sizes = [64, 150, 96, 200, 80, 128, 64]
    steps = [40, 30, 50, 20, 40, 30, 25]
    reqs = [Scenario(k, 0.002 * k, W.scenario(k, n=n), steps[k]) for k, n in enumerate(sizes)]
    # budget for about two of the larger grids: later requests wait for memory
    srv = ScenarioServer(p, hbm_budget=3 * 7 * 208 * 208 * (4 if precision else 8),
                         max_slots=3, steps_per_round=10)
    out = srv.serve(reqs)
    torch.cuda.synchronize()
    assert out["requests"] == len(reqs)
    assert out["status_flags"] & (L.STATUS_NONFINITE | L.STATUS_NEG_DEPTH) == 0
    assert out["p99_ms"] >= out["p50_ms"] > 0
    for sc in out["done"]:
        s = PatchSolver(sc.problem, p)
        s.initial_dt()
        s.run_async(sc.nsteps)
        torch.cuda.synchronize()
        alone = s.surface()
        assert np.array_equal(sc.result["eta"], alone), f"request {sc.rid}"
