"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Operators (explicit residual, Schur complement apply) are compared element by
element on seeded inputs on meshes with several elements per direction,
periodic and wall faces, terrain-following geometry and hanging faces. The
implicit stage solve and whole IMEX-ARK2 steps are compared in parity mode
(fixed Picard / GMRES iteration counts, so both sides build the same Krylov
spaces) and in tolerance mode. FP64 bar: 1e-12 of each field's own maximum,
plus, for the momentum and velocity of states in near balance, a stated
cancellation floor (tests/bars.py); every field's error against its own
maximum is printed.
"""
import numpy as np
import pytest
import torch

from oracle import dg
from oracle.mesh import Mesh as OMesh, MeshDesc
from paper_2605_29598_amd import workloads as W
from tests.bars import check_state, check_tolerance_state, check_velocity

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _B():
    from paper_2605_29598_amd import binding as B
    return B


def _pair(spec, phys=None, num=None):
    B = _B()
    phys = phys or W.PhysSpec(f=1e-3)
    num = num or W.NumSpec(dt=5.0)
    gm = B.Mesh(spec)
    sol = B.Solver(gm, phys, num)
    om = OMesh(MeshDesc(**vars(spec)))
    oph = dg.Phys(**vars(phys))
    onum = dg.Numerics(**vars(num))
    return sol, om, oph, onum


def _cpu(t):
    return t.detach().cpu().numpy()


def relerr(gpu, ref):
    return np.abs(gpu - ref).max() / max(np.abs(ref).max(), 1e-300)


MESHES = {
    "periodic_r2": W.MeshSpec(4e3, 3e3, 2e3, 3, 2, 2, 2),
    "walls_r3": W.MeshSpec(4e3, 3e3, 2e3, 3, 2, 2, 3, periodic_x=0, periodic_y=0),
    "r1_periodic": W.MeshSpec(4e3, 3e3, 2e3, 4, 3, 2, 1),
    "r4_ragged": W.MeshSpec(5e3, 3e3, 2e3, 3, 1, 3, 4),       # E = 9, not a multiple of the 2 elements/block
    "terrain_r3": W.MeshSpec(8e3, 8e3, 4e3, 3, 3, 2, 3, terrain=W.GAUSS, h0=400, a=2e3, xc=4e3, yc=4e3),
    # conforming terrain-following meshes at other degrees: the Krylov passes
    # form their metric from the compact form (E = 18 and 15, ragged blocks)
    "terrain_r2": W.MeshSpec(8e3, 8e3, 4e3, 3, 3, 2, 2, terrain=W.BELL, h0=500, a=1.5e3, xc=3e3, yc=5e3),
    "terrain_r4": W.MeshSpec(10e3, 6e3, 4e3, 5, 3, 1, 4, terrain=W.GAUSS, h0=600, a=2e3, xc=6e3, yc=2e3,
                             periodic_x=0),
    "hanging_r2": W.MeshSpec(8e3, 8e3, 4e3, 4, 4, 2, 2,
                             ref_boxes=[(2e3, 6e3, 2e3, 6e3, 0, 2e3), (3.5e3, 4.5e3, 3.5e3, 4.5e3, 0, 0.5e3)]),
    "hanging_terrain_r4": W.MeshSpec(8e3, 8e3, 4e3, 3, 3, 2, 4, terrain=W.BELL, h0=300, a=1.5e3, xc=4e3, yc=4e3,
                                     ref_boxes=[(2.5e3, 5.5e3, 2.5e3, 5.5e3, 0, 2e3)]),
}


def _state(om, seed):
    return W.random_positive_state((om.E, om.Np), seed)


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("lateral", [False, True])
def test_explicit_residual_parity(name, lateral):
    spec = MESHES[name]
    # lateral: Rayleigh layers over the first and last quarter of x and third of y as well
    wx, wy = (spec.Lx / 4, spec.Ly / 3) if lateral else (0.0, 0.0)
    phys = W.PhysSpec(f=1.3e-3, sponge_zB=1e3, sponge_zT=4e3, sponge_lam=0.01, sponge_u=(3.0, -1.0, 0.0),
                      sponge_xw=wx, sponge_yw=wy)
    sol, om, oph, _ = _pair(spec, phys)
    q = _state(om, 11)
    TNS, TS = dg.explicit_residual(om, oph, q)
    Mw = om.W3 * om.detJ
    fNS, fS = sol.explicit_residual(q)
    fNS, fS = _cpu(fNS), _cpu(fS)
    for t in range(5):
        assert relerr(fNS[t], TNS[t] / Mw) < TOL, ("NS", t, relerr(fNS[t], TNS[t] / Mw))
    for t in range(4):
        assert relerr(fS[t], TS[t + 1] / Mw) < TOL, ("S", t, relerr(fS[t], TS[t + 1] / Mw))


@pytest.mark.parametrize("name", ["walls_r3", "terrain_r3", "hanging_r2", "hanging_terrain_r4"])
def test_explicit_residual_parity_sponge_target(name):
    """Damping layers relaxing the whole state towards a target state
    (imx_solver_set_sponge_target): every field's tendency against the oracle,
    with layers strong enough that the relaxation is a sizeable part of it;
    clearing the target restores the momentum-only form."""
    spec = MESHES[name]
    phys = W.PhysSpec(f=1.3e-3, sponge_zB=1e3, sponge_zT=4e3, sponge_lam=0.5, sponge_u=(3.0, -1.0, 0.0),
                      sponge_xw=spec.Lx / 4, sponge_yw=spec.Ly / 3)
    sol, om, oph, _ = _pair(spec, phys)
    q = _state(om, 11)
    target = q * (1.0 + 0.01 * np.random.default_rng(12).uniform(-1, 1, q.shape))
    Mw = om.W3 * om.detJ
    sol.set_sponge_target(target)
    oph.sponge_target = target
    TNS, TS = dg.explicit_residual(om, oph, q)
    fNS, fS = (_cpu(a) for a in sol.explicit_residual(q))
    for t in range(5):
        assert relerr(fNS[t], TNS[t] / Mw) < TOL, ("NS", t, relerr(fNS[t], TNS[t] / Mw))
    for t in range(4):
        assert relerr(fS[t], TS[t + 1] / Mw) < TOL, ("S", t, relerr(fS[t], TS[t + 1] / Mw))
    # the relaxation is visible in the density tendency, which has no other sponge part
    oph.sponge_target = None
    TNS0, _ = dg.explicit_residual(om, oph, q)
    assert np.abs(TNS[0] - TNS0[0]).max() > 1e-3 * np.abs(TNS[0]).max()
    sol.set_sponge_target(None)
    fNS0 = _cpu(sol.explicit_residual(q)[0])
    for t in range(5):
        assert relerr(fNS0[t], TNS0[t] / Mw) < TOL, ("NS momentum-only", t)


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("scheme", [dg.R1, dg.R2])
def test_schur_apply_parity(name, scheme):
    spec = MESHES[name]
    num = W.NumSpec(dt=7.0, scheme=scheme)
    sol, om, oph, onum = _pair(spec, W.PhysSpec(f=2e-3), num)
    rng = np.random.default_rng(5)
    shp = (om.E, om.Np)
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, shp)
    pk = 1e5 * (1 + 0.1 * rng.uniform(-1, 1, shp))
    uk = 10 * rng.uniform(-1, 1, (3,) + shp)
    p = 1e5 * (1 + 0.1 * rng.uniform(-1, 1, shp))
    S = dg.StageSystem(om, oph, rho, pk, uk, dg.A_IMP[1, 1], num.dt, scheme)
    ref = S.schur(p)
    sol.implicit_setup(rho, pk, uk)
    got = _cpu(sol.schur_apply(p))
    assert relerr(got, ref) < TOL, relerr(got, ref)


def _stage_inputs(om, oph, y, dt):
    """Stage-2 inputs of an ARK2 step built by the oracle from state y."""
    Mw = om.W3 * om.detJ
    TNS, TS = dg.explicit_residual(om, oph, y)
    a, at = dg.A_EXP[1, 0], dg.A_IMP[1, 0]
    rho = y[0] + dt * a * TNS[0] / Mw
    F = Mw * y[1:4] + dt * (a * TNS[1:4] + at * TS[1:4])
    F[2] -= dg.A_IMP[1, 1] * dt * oph.g * Mw * rho
    G0 = Mw * y[4] + dt * (a * TNS[4] + at * TS[4])
    _, _, _, u0, _, p0 = dg.primitives(y, oph.gamma)
    return rho, F, G0, p0, u0


@pytest.mark.parametrize("name", ["periodic_r2", "hanging_r2", "terrain_r3", "terrain_r2", "terrain_r4"])
@pytest.mark.parametrize("scheme", [dg.R1, dg.R2])
def test_implicit_solve_parity_fixed(name, scheme):
    spec = MESHES[name]
    num = W.NumSpec(dt=20.0, scheme=scheme, picard_max=3, gmres_max=14, gmres_restart=5, fixed_iterations=True)
    sol, om, oph, onum = _pair(spec, W.PhysSpec(f=1e-3), num)
    w = W.tiny_box()
    y = W.initial_state(w, om.node_coords())
    rho, F, G0, p0, u0 = _stage_inputs(om, oph, y, num.dt)
    pr, ur, st = dg.stage_solve(om, oph, onum, rho, F, G0, p0, u0, dg.A_IMP[1, 1])
    pg, ug, gst = sol.implicit_solve(rho, F, G0, p0, u0)
    assert gst.picard_iters == st["picard"] and gst.gmres_iters == st["gmres"]
    print(f"[parity] {name} R{scheme} p: err/own_max {relerr(_cpu(pg), pr):.3e}", flush=True)
    assert relerr(_cpu(pg), pr) < TOL
    check_velocity(_cpu(ug), ur, rho, np.abs(pr).max(), om, num.dt, tag=f"{name} R{scheme}")


def _run_steps(spec, phys, num, w, nsteps):
    sol, om, oph, onum = _pair(spec, phys, num)
    y0 = W.initial_state(w, om.node_coords())
    y = y0
    ost = []
    for _ in range(nsteps):
        y, st = dg.ark2_step(om, oph, onum, y)
        ost.append(st)
    sol.set_state(y0)
    gst = sol.step(nsteps)
    return _cpu(sol.get_state()), y, y0, gst, ost, sol


@pytest.mark.parametrize("scheme", [dg.R1, dg.R2])
def test_ark2_steps_parity_fixed(scheme):
    w = W.tiny_box(scheme=scheme)
    num = W.NumSpec(dt=2.0, scheme=scheme, picard_max=3, gmres_max=12, gmres_restart=8, fixed_iterations=True)
    g, o, y0, gst, ost, _ = _run_steps(w.mesh, w.phys, num, w, 3)
    check_state(g, o, OMesh(MeshDesc(**vars(w.mesh))), num.dt, 3, tag=f"tiny_box fixed R{scheme}")


def test_ark2_steps_tiny_box_tolerance_mode():
    """The tiny isothermal box (10x10x10 km, 4^3 elements, r = 2, 10 steps of 2 s, GMRES tol 1e-10)."""
    w = W.tiny_box()
    g, o, y0, gst, ost, sol = _run_steps(w.mesh, w.phys, w.num, w, 10)
    assert gst.gmres_iters == sum(s["gmres"] for s in ost)
    assert gst.picard_iters == sum(s["picard"] for s in ost)
    om = OMesh(MeshDesc(**vars(w.mesh)))
    check_state(g, o, om, w.num.dt, 10, tag="tiny_box tolerance mode")
    # discrete mass conservation on the GPU
    M0 = dg.total_mass(om, y0)
    assert abs(sol.total_mass() - M0) <= 1e-13 * M0


def test_hanging_terrain_steps_and_mass():
    spec = MESHES["hanging_terrain_r4"]
    w = W.tiny_box()
    num = W.NumSpec(dt=2.0, picard_max=2, gmres_max=10, gmres_restart=10, fixed_iterations=True)
    g, o, y0, gst, ost, sol = _run_steps(spec, W.PhysSpec(f=1e-4), num, w, 2)
    om = OMesh(MeshDesc(**vars(spec)))
    check_state(g, o, om, num.dt, 2, tag="hanging_terrain_r4 fixed")
    M0 = dg.total_mass(om, y0)
    assert abs(sol.total_mass() - M0) <= 1e-13 * M0


def test_step_is_deterministic():
    w = W.tiny_box()
    B = _B()
    gm = B.Mesh(w.mesh)
    q = W.initial_state(w, gm.node_coords())
    outs = []
    for _ in range(2):
        sol = B.Solver(gm, w.phys, w.num)
        sol.set_state(q)
        sol.step(2)
        outs.append(_cpu(sol.get_state()))
    assert np.array_equal(outs[0], outs[1])


# per-step bound of the binary32-inner path: each stage solve of either path
# ends at a binary64 residual and a Picard variation <= 1e-10 relative, so the
# two stage states differ by a few 1e-10 in the scales of tolerance_scales
# (momentum in p / c) and this accumulates over the steps
MIXED_PER_STEP = 1e-10


def test_mixed_precision_tiny_box_vs_oracle():
    """The tiny isothermal box in the mixed mode: binary32 Krylov inner loop inside binary64
    defect correction to the same tolerance, against the FP64 oracle."""
    B = _B()
    w = W.tiny_box()
    gm = B.Mesh(w.mesh)
    om = OMesh(MeshDesc(**vars(w.mesh)))
    y0 = W.initial_state(w, om.node_coords())
    sol = B.Solver(gm, w.phys, w.num, precision=B.IMX_MIXED, inner_tol=1e-3)
    sol.set_state(y0)
    st = sol.step(10)
    g = _cpu(sol.get_state())
    y = y0
    for _ in range(10):
        y, _ = dg.ark2_step(om, dg.Phys(**vars(w.phys)), dg.Numerics(**vars(w.num)), y)
    check_tolerance_state(g, y, MIXED_PER_STEP, 10, tag="tiny_box mixed")
    M0 = dg.total_mass(om, y0)
    assert abs(sol.total_mass() - M0) <= 1e-13 * M0


def test_mixed_precision_r3_affine_vs_oracle():
    """The binary32 Krylov loop on an r = 3 affine mesh (the one-wavefront-per-
    element pass 2), 4 steps of R1 against the FP64 oracle."""
    B = _B()
    w = W.tiny_box(degree=3, scheme=dg.R1)
    gm = B.Mesh(w.mesh)
    om = OMesh(MeshDesc(**vars(w.mesh)))
    y0 = W.initial_state(w, om.node_coords())
    sol = B.Solver(gm, w.phys, w.num, precision=B.IMX_MIXED, inner_tol=1e-3)
    sol.set_state(y0)
    sol.step(4)
    g = _cpu(sol.get_state())
    y = y0
    for _ in range(4):
        y, _ = dg.ark2_step(om, dg.Phys(**vars(w.phys)), dg.Numerics(**vars(w.num)), y)
    check_tolerance_state(g, y, MIXED_PER_STEP, 4, tag="tiny_box r3 mixed R1")


def test_ark2_steps_r3_affine_parity_fixed():
    """Fixed-count ARK2 steps on an r = 3 affine mesh (both Schur passes in
    their r = 3 forms), R2, against the oracle."""
    w = W.tiny_box(degree=3)
    num = W.NumSpec(dt=2.0, picard_max=3, gmres_max=12, gmres_restart=8, fixed_iterations=True)
    g, o, y0, gst, ost, _ = _run_steps(w.mesh, w.phys, num, w, 2)
    check_state(g, o, OMesh(MeshDesc(**vars(w.mesh))), num.dt, 2, tag="tiny_box r3 fixed")
