"""Oracle pins of the implicit stage system against the explicit weak forms.

The stage equations of Sec. 3 put a~_ll dt f_S(Y_l) on the implicit side: the
stage solve iterates the matrices A, R, B, C^k, D, M_g and the vectors f_g,
k^k, Lambda^k built from a lagged iterate (p^k, u^k), and never evaluates the
explicit T_S. When the lagged iterate is the state itself, each implicit term
must be the matching explicit term times -a~_ll dt:

    B p + f_g + R u              = -c T_S,m      (pressure, gravity, Coriolis)
    C^k u + M_g u + Lambda^k     = -c T_S,E      (enthalpy flux, gravity work,
                                                  lambda/2 [rho e])
    D p + k^k                    =  M (rho E)    (internal plus kinetic energy)

with c = a~_ll dt. The test states are chosen so that these hold to round-off:
density and velocity constant in each element (but jumping across faces, so
lambda and the jumps of rho e are nonzero on every face) and the pressure a
random polynomial per element. A sign or side error in Lambda^k, C^k, M_g or
k^k leaves a residual of the size of that term (checked below by planting
such errors in the oracle).

The stage equation itself is pinned at converged stages of whole ARK2 steps
from random states: with the Picard and GMRES loops converged to 1e-14,

    M (Y_l - y^n) - dt sum_{m<l} (a_lm T_NS + a~_lm T_S)(Y_m) - dt a~_ll T_S(Y_l) = 0

row by row to round-off, for l = 2, 3, R1 and R2, on walled, periodic,
terrain-following and hanging-face meshes, with T_NS and T_S from the explicit
residual. This ties every implicit operator to the explicit stiff part at a
general state, and it holds because both take their face values from the
traces of (rho, u, p); with face values from traces of the conserved
variables it fails at 1e-3 relative (planted below).

The Picard variation measure is pinned by closed forms on manufactured iterate
pairs.
"""
import math

import numpy as np
import pytest

from oracle import dg
from oracle.mesh import Mesh, MeshDesc
from paper_2605_29598_amd import workloads as W

STAGE_MESHES = {
    "walls_r2": MeshDesc(4e3, 3e3, 2e3, 2, 2, 2, 2, periodic_x=0, periodic_y=0),
    "periodic_r3": MeshDesc(4e3, 3e3, 2e3, 2, 2, 2, 3),
    "terrain_r2": MeshDesc(4e3, 4e3, 3e3, 2, 2, 2, 2, terrain=2, h0=300.0, a=1.5e3, xc=2e3, yc=2e3),
    "hanging_r2": MeshDesc(4e3, 4e3, 2e3, 2, 2, 2, 2, ref_boxes=[(2.5e3, 3e3, 0, 1e3, 1.2e3, 1.8e3)]),
    "hanging_terrain_r1": MeshDesc(4e3, 4e3, 3e3, 2, 2, 2, 1, terrain=1, h0=200.0, a=1e3, xc=2e3, yc=2e3,
                                   ref_boxes=[(0, 1e3, 0, 1e3, 0, 0.5e3)]),
}
IDENTITY_BAR = 1e-12
A_LL, DT = dg.A_IMP[1, 1], 3.0

_meshes = {}


def _mesh(name):
    if name not in _meshes:
        _meshes[name] = Mesh(STAGE_MESHES[name])
    return _meshes[name]


def _commuting_state(mesh, seed):
    """rho, u constant per element (jumping across faces), p random per node."""
    g = np.random.default_rng(seed)
    E, Np = mesh.E, mesh.Np
    rho = np.repeat(1.0 + 0.2 * g.uniform(-1, 1, (E, 1)), Np, axis=1)
    u = np.repeat(5.0 * g.uniform(-1, 1, (3, E, 1)), Np, axis=2)
    p = 1e5 * (1.0 + 0.05 * g.uniform(-1, 1, (E, Np)))
    return rho, u, p, W.conserved_from_primitive(rho, u, p)


def stage_term_residuals(mesh, phys, scheme, seed=21):
    """Relative residuals of the three term-by-term identities."""
    rho, u, p, q = _commuting_state(mesh, seed)
    _, TS = dg.explicit_residual(mesh, phys, q)
    S = dg.StageSystem(mesh, phys, rho, p, u, A_LL, DT, scheme)
    c = A_LL * DT
    Mw = mesh.W3 * mesh.detJ

    def rel(a, b):
        return float(np.abs(a - b).max() / max(np.abs(a).max(), np.abs(b).max()))
    return {"momentum": rel(S.B(p) + S.f_g() + S.R(u), -c * TS[1:4]),
            "energy": rel(S.C(u) + S.M_g(u) + S.Lam(), -c * TS[4]),
            "total_energy": rel(S.D(p) + S.k_vec(), Mw * q[4])}


@pytest.mark.parametrize("name", list(STAGE_MESHES))
@pytest.mark.parametrize("scheme", [dg.R1, dg.R2])
def test_stage_terms_equal_explicit_stiff_part(name, scheme):
    mesh = _mesh(name)
    res = stage_term_residuals(mesh, dg.Phys(f=1e-3, g=9.81), scheme)
    for key, v in res.items():
        assert v < IDENTITY_BAR, (key, v, res)


def test_lambda_term_is_not_negligible():
    """On the test states Lambda^k is a sizeable part of the energy identity
    (so dropping it or flipping its sign cannot hide under the bar)."""
    mesh = _mesh("periodic_r3")
    rho, u, p, q = _commuting_state(mesh, 21)
    S = dg.StageSystem(mesh, dg.Phys(f=1e-3, g=9.81), rho, p, u, A_LL, DT, dg.R2)
    lam, rest = np.abs(S.Lam()).max(), np.abs(S.C(u) + S.M_g(u) + S.Lam()).max()
    assert lam > 1e-3 * rest, (lam, rest)


def _planted(monkeypatch, what):
    """Plants one plausible mistake into the oracle's stage system."""
    S = dg.StageSystem
    if what == "lambda_sign":
        orig = S.Lam
        monkeypatch.setattr(S, "Lam", lambda self: -orig(self))
    elif what == "lambda_dropped":
        monkeypatch.setattr(S, "Lam", lambda self: np.zeros_like(self.p_k))
    elif what == "kinetic_half":
        orig = S.k_vec
        monkeypatch.setattr(S, "k_vec", lambda self: 0.5 * orig(self))
    elif what == "gravity_work_sign":
        orig = S.M_g
        monkeypatch.setattr(S, "M_g", lambda self, u: -orig(self, u))
    elif what == "coriolis_transposed":
        orig = S.R
        monkeypatch.setattr(S, "R", lambda self, u: -orig(self, u))
    elif what == "enthalpy_face_one_sided":
        # the centred enthalpy flux taken from this side only
        orig_fi = dg.face_integrals

        def one_sided(mesh, fields, flux, nout):
            if nout == 1 and fields.shape[0] == 4:
                return orig_fi(mesh, fields, lambda qA, qB, nS: flux(qA, None, nS), nout)
            return orig_fi(mesh, fields, flux, nout)
        monkeypatch.setattr(dg, "face_integrals", one_sided)
    else:
        raise ValueError(what)


@pytest.mark.parametrize("what", ["lambda_sign", "lambda_dropped", "kinetic_half", "gravity_work_sign",
                                  "coriolis_transposed", "enthalpy_face_one_sided"])
def test_stage_identity_detects_planted_mistakes(monkeypatch, what):
    """The identities have teeth: each planted mistake leaves a residual far
    above the bar."""
    mesh = _mesh("periodic_r3")
    _planted(monkeypatch, what)
    res = stage_term_residuals(mesh, dg.Phys(f=1e-3, g=9.81), dg.R2)
    assert max(res.values()) > 1e4 * IDENTITY_BAR, (what, res)


# --------------------------------------------------------- stage equation
STAGE_EQ_BAR = 1e-11


def stage_equation_residuals(mesh, scheme, seed=5):
    """Largest relative residual of the stage equation of each row at the
    converged stages 2 and 3 of one ARK2 step: the density row against
    M rho_l, the momentum and energy rows against dt a~_ll T_S(Y_l)."""
    q = W.random_positive_state((mesh.E, mesh.Np), seed, urms=5.0, rel=0.02)
    phys = dg.Phys(f=1e-4, g=9.81)
    num = dg.Numerics(dt=3.0, scheme=scheme, picard_tol=1e-14, gmres_tol=1e-14, picard_max=60, gmres_max=2000)
    _, st = dg.ark2_step(mesh, phys, num, q, return_stages=True)
    Ys, T = st["stages"], st["residuals"]
    Mw = mesh.W3 * mesh.detJ
    worst = np.zeros(5)
    for l in (1, 2):
        implicit = num.dt * dg.A_IMP[l, l] * T[l][1]
        res = Mw * (Ys[l] - q) - num.dt * sum(dg.A_EXP[l, m] * T[m][0] + dg.A_IMP[l, m] * T[m][1]
                                              for m in range(l)) - implicit
        scale = np.abs(implicit).reshape(5, -1).max(1)
        scale[0] = np.abs(Mw * Ys[l][0]).max()
        worst = np.maximum(worst, np.abs(res).reshape(5, -1).max(1) / scale)
    return worst


@pytest.mark.parametrize("name", list(STAGE_MESHES))
@pytest.mark.parametrize("scheme", [dg.R1, dg.R2])
def test_stage_equation_holds_at_converged_stages(name, scheme):
    worst = stage_equation_residuals(_mesh(name), scheme)
    assert worst.max() < STAGE_EQ_BAR, worst


def test_stage_equation_detects_conserved_face_traces(monkeypatch):
    """Planted: the explicit residual's face values from traces of the
    conserved variables (u_face = trace(m) / trace(rho)) while the stage
    operators take traces of u and p."""
    orig = dg.face_integrals
    gam = dg.Phys().gamma

    def conserved_traces(mesh, fields, flux, nout):
        if nout != 10:
            return orig(mesh, fields, flux, nout)
        rho, u, p = fields[0], fields[1:4], fields[4]
        q = np.concatenate([rho[None], rho * u, (p / (gam - 1) + 0.5 * rho * (u * u).sum(0))[None]])

        def prim(qq):
            uu = qq[1:4] / qq[0]
            pp = (gam - 1) * (qq[4] - 0.5 * qq[0] * (uu * uu).sum(0))
            return np.concatenate([qq[0][None], uu, pp[None]])
        return orig(mesh, q, lambda qA, qB, nS: flux(prim(qA), None if qB is None else prim(qB), nS), nout)
    monkeypatch.setattr(dg, "face_integrals", conserved_traces)
    worst = stage_equation_residuals(_mesh("terrain_r2"), dg.R2)
    assert worst.max() > 1e4 * STAGE_EQ_BAR, worst


# --------------------------------------------------------- Picard variation
def test_picard_variation_closed_forms():
    """delta = sqrt(sum M [dp^2 + gamma p rho |du|^2] / sum M p^2) with p the
    new iterate (velocity change weighted by the acoustic impedance rho c)."""
    mesh = Mesh(MeshDesc(3e3, 2e3, 1e3, 3, 2, 1, 3, periodic_x=0))
    Mw = mesh.W3 * mesh.detJ
    shp = (mesh.E, mesh.Np)
    gam = 1.4
    one = np.ones(shp)
    zero3 = np.zeros((3,) + shp)
    # (a) pressure only: the weights cancel, delta = |b - a| / |b| (new iterate in the denominator)
    d = dg.picard_variation(Mw, gam, one, 9e4 * one, zero3, 1e5 * one, zero3)
    assert abs(d - 0.1) < 1e-15
    # (b) velocity only, uniform: delta = rho c U / P with c^2 = gamma P / rho
    P, rho0, U = 8e4, 1.2, 0.3
    du = zero3.copy()
    du[1] = U
    d = dg.picard_variation(Mw, gam, rho0 * one, P * one, zero3, P * one, du)
    assert abs(d - rho0 * math.sqrt(gam * P / rho0) * U / P) < 1e-15
    # (c) both, with p_old != p_new: the impedance uses the new pressure
    P0, P1 = 7e4, 8e4
    d = dg.picard_variation(Mw, gam, rho0 * one, P0 * one, zero3, P1 * one, du)
    assert abs(d - math.sqrt((P1 - P0) ** 2 + gam * P1 * rho0 * U * U) / P1) < 1e-15
    # (d) the sums are integrals (mass weights), not node sums: p_new = 1 + x/L
    #     linear in x, a constant change dp; int (1 + x/L)^2 = L (8 - 1)/3 per unit area
    x = mesh.xq[..., 0]
    L = mesh.desc.Lx
    pn = 1.0 + x / L
    d = dg.picard_variation(Mw, gam, one, pn - 0.01, zero3, pn, zero3)
    assert abs(d - 0.01 * math.sqrt(1.0 / (7.0 / 3.0))) < 1e-14
