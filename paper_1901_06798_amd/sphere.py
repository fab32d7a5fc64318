"""One latitude-longitude patch on the GPU (swe_patch_step_sphere).

The patch's cells are dlon x dlat degrees from latitude lat0 (its first
interior row's lower edge); Problem.dx and dy are R dlon and R dlat in metres.
The capacities and edge length ratios come from the sphere's geometry: a row's
cells cover R^2 dlon (sin phi_top - sin phi_bottom), so its capacity (area over
the area of the same cells at the equator) is (sin phi_top - sin phi_bottom) /
dlat (angles in radians), and a parallel edge is cos(phi) times as long as at
the equator.  The CFL rule of the solver holds, on the device as for a
Cartesian patch: the step, the retake and the first step's speed scan report
speeds scaled by the edges' mean inverse capacity.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .solver import PatchSolver
from .workloads import Problem


def metric(lat0_deg: float, dlat_deg: float, my: int, bc=None) -> np.ndarray:
    """[kappa_0 .. kappa_{my+3}, len_0 .. len_{my+4}] of a patch with my rows.

    A wall side (bc = (xlo, xhi, ylo, yhi)) at ylo or yhi reflects the cells
    inside it, geometry included: the ghost rows beyond it take the capacities
    and edge lengths of the rows they mirror, so that the x-sweep of a ghost
    row is the mirror image of its interior row's and no mass crosses the wall.
    """
    rad = np.pi / 180.0
    j = np.arange(my + 5, dtype=np.float64)
    phi_edge = (lat0_deg + (j - 2.0) * dlat_deg) * rad   # lower edge of frame row j
    sin_e = np.sin(phi_edge)
    kap = (sin_e[1:] - sin_e[:-1]) / (dlat_deg * rad)
    ln = np.cos(phi_edge)
    if bc is not None and bc[2] == L.BC_WALL:
        kap[:2] = kap[3:1:-1]
        ln[:2] = ln[4:2:-1]
    if bc is not None and bc[3] == L.BC_WALL:
        kap[my + 2:] = kap[my + 1:my - 1:-1]
        ln[my + 3:] = ln[my + 1:my - 1:-1]
    return np.concatenate([kap, ln])


class SphereSolver(PatchSolver):
    """PatchSolver for a latitude-longitude patch (FP64 split step)."""

    def __init__(self, pb: Problem, params: L.swe_params | None = None, device: str = "cuda:0",
                 ordered: bool = True, order_every: int = 4):
        p = params or L.params()
        if p.precision != L.F64 or p.method != L.SPLIT:
            raise L.SweError("SphereSolver: FP64 split step only")
        for key in ("lat0", "dlat"):
            if key not in pb.meta:
                raise L.SweError(f"SphereSolver: the problem's meta needs {key!r}")
        lat0, dlat = pb.meta["lat0"], pb.meta["dlat"]
        # the ghost frame, two rows beyond each side, must stay off the poles
        if not (dlat > 0.0 and lat0 - 2.0 * dlat > -90.0 and lat0 + (pb.my + 2) * dlat < 90.0):
            raise L.SweError("SphereSolver: the patch with its ghost rows must not reach a pole")
        super().__init__(pb, p, device, ordered=ordered, order_every=order_every)
        m = metric(pb.meta["lat0"], pb.meta["dlat"], pb.my, pb.bc)
        self.metric = torch.from_numpy(m).to(self.dev)
        self.metric_ptr = self.metric.data_ptr()

    def launch_scan(self) -> None:
        # each edge's speed scaled by its inverse capacity, as the step reports it
        L.swe_speed_scan_sphere(self.p, self.pt_dev.data_ptr(), self.mx, self.my,
                                self.q[self.cur].data_ptr(), self.b.data_ptr(),
                                self.metric.data_ptr(), self.smax.data_ptr(), self.stream)

    def launch_step(self, qi: int, qo: int, dt: int, stream: int | None = None) -> None:
        st = self.stream if stream is None else stream
        L.swe_patch_step_sphere(self.p, self.pt, qi, qo, self.b.data_ptr(), dt,
                                self.smax.data_ptr(), self.status.data_ptr(),
                                self.metric.data_ptr(),
                                self.sched.data_ptr() if self.sched is not None else 0,
                                self.sched.numel() if self.sched is not None else 0,
                                self.launch, st)

    def launch_retake(self, qi: int, qo: int, retake: int, stream: int | None = None) -> None:
        L.swe_patch_retake_sphere(self.p, self.pt, qi, qo, self.b.data_ptr(),
                                  self.dt.data_ptr(), self.smax.data_ptr(),
                                  self.status.data_ptr(), self.metric.data_ptr(), retake,
                                  self.stream if stream is None else stream)

    def mass(self) -> float:
        """Water volume: sum of h kappa_j dx dy over the interior (on the device)."""
        out = torch.zeros(1, dtype=torch.float64, device=self.dev)
        L.swe_mass_sphere(self.p, self.pt_dev.data_ptr(), self.q[self.cur].data_ptr(),
                          self.metric.data_ptr(), out.data_ptr(), self.stream)
        return float(out.item())
