"""Replay of the GMRES loop from captured HIP graphs.

Every step replays the captured chunks of Krylov columns many times, with
direct launches and host synchronisations in between (Picard refresh, restart
residuals, chunk-state reads). Two solvers on the same input, one replaying
graphs and one launching every kernel directly, must agree bit for bit after
every step: FP64 and mixed precision, R1 and R2, a restart length that is not
a multiple of the chunk, a terrain-following mesh with hanging faces, and a
step count large enough that cycles span several chunks.
"""
import numpy as np
import pytest

from paper_2605_29598_amd import workloads as W

pytestmark = pytest.mark.gpu

HANG_TERRAIN = W.MeshSpec(8e3, 8e3, 4e3, 3, 3, 2, 3, terrain=W.BELL, h0=300, a=1.5e3, xc=4e3, yc=4e3,
                          ref_boxes=[(2.5e3, 5.5e3, 2.5e3, 5.5e3, 0, 2e3)])

CASES = {
    "slice_fp64_R2": (W.igw_slice(nx=8, nz=3, planetary=True).mesh, W.PhysSpec(f=1.03126e-4, slice=1),
                      W.NumSpec(dt=10.0, gmres_restart=11), "fp64"),
    "slice_mixed_R2": (W.igw_slice(nx=8, nz=3, planetary=True).mesh, W.PhysSpec(f=1.03126e-4, slice=1),
                       W.NumSpec(dt=10.0), "mixed"),
    "terrain_hanging_fp64_R1": (HANG_TERRAIN, W.PhysSpec(f=1e-4), W.NumSpec(dt=8.0, scheme=W.R1, gmres_restart=13),
                                "fp64"),
}


def _B():
    from paper_2605_29598_amd import binding as B
    return B


@pytest.mark.parametrize("name", list(CASES))
def test_graph_replay_bitwise_equals_direct_launches(name):
    B = _B()
    spec, phys, num, prec = CASES[name]
    mesh = B.Mesh(spec)
    pr = B.IMX_MIXED if prec == "mixed" else B.IMX_FP64
    q0 = W.initial_state(W.igw_slice(nx=8, nz=3, planetary=True) if spec.ny == 1 else W.tiny_box(),
                         mesh.node_coords())
    a = B.Solver(mesh, phys, num, precision=pr)
    b = B.Solver(mesh, phys, num, precision=pr)
    a.set_graphs(True)
    b.set_graphs(False)
    a.set_state(q0)
    b.set_state(q0)
    total = 0
    for step in range(4):
        sa, sb = a.step(1), b.step(1)
        assert sa.gmres_iters == sb.gmres_iters and sa.picard_iters == sb.picard_iters
        total += sa.gmres_iters
        qa, qb = a.get_state().cpu().numpy(), b.get_state().cpu().numpy()
        assert np.array_equal(qa, qb), (name, step)
    assert total > 16, total       # several chunks of 8 columns were replayed
