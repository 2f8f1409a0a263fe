"""Weak forms, stage systems and the IMEX-ARK2 step of the rotating IMEX-DG method.

Fields live in the nodal Q_r space with nodes at the Gauss-Legendre points
(Sec. 3); integrals use the same points, so values at quadrature points are
the nodal values and every mass-type matrix is diagonal (S = I in Sec. 3.1).
A field array has shape (..., E, Np) in the node order of oracle.mesh.

Numerical fluxes (Sec. 3): Rusanov with lambda = max(|u+.n|, |u-.n|) on the
advected quantities, centred averages on the pressure and enthalpy terms.
On a slip wall the outer state is the mirror state (rho, u - 2(u.n)n, p).
"""
from dataclasses import dataclass
import math
import numpy as np

from .mesh import Mesh

# --------------------------------------------------------------- constants
CHI = 2.0 - math.sqrt(2.0)
# Butcher tableaux of Sec. 3 (explicit: left, implicit: right), a32 = 1/2.
A_EXP = np.array([[0.0, 0.0, 0.0],
                  [CHI, 0.0, 0.0],
                  [0.5, 0.5, 0.0]])
A_IMP = np.array([[0.0, 0.0, 0.0],
                  [CHI / 2, CHI / 2, 0.0],
                  [0.5 - CHI / 4, 0.5 - CHI / 4, CHI / 2]])
B_W = np.array([0.5 - CHI / 4, 0.5 - CHI / 4, CHI / 2])
C_NODES = np.array([0.0, CHI, 1.0])

R1, R2 = 1, 2


@dataclass
class Phys:
    gamma: float = 1.4
    R: float = 287.0
    g: float = 9.81
    f: float = 0.0
    # Rayleigh sponge lambda(z) = lam * sin^2(pi/2 (z-zB)/(zT-zB)) for z >= zB,
    # relaxing the momentum towards rho * u_bg; lam = 0 switches it off. With
    # sponge_target (conserved state (5, E, Np)) the whole state relaxes
    # towards it instead.
    sponge_zB: float = 0.0
    sponge_zT: float = 1.0
    sponge_lam: float = 0.0
    sponge_u: tuple = (0.0, 0.0, 0.0)
    # lateral layers of the same sin^2 form over the first and last sponge_xw
    # of [0, Lx] and sponge_yw of [0, Ly] (0 = none); where layers overlap the
    # largest coefficient applies
    sponge_xw: float = 0.0
    sponge_yw: float = 0.0
    # vertical-slice model (Sec. 2, eq. vertical_slice): d/dy = 0 with v
    # prognostic, on a mesh with one periodic element in y; every step ends
    # with the projection onto fields constant in y (slice_project)
    slice: int = 0
    sponge_target: object = None


@dataclass
class Numerics:
    dt: float = 1.0
    scheme: int = R2
    picard_tol: float = 1e-10
    picard_max: int = 20
    gmres_tol: float = 1e-10
    gmres_restart: int = 30
    gmres_max: int = 500
    fixed_iterations: bool = False   # run exactly picard_max / gmres_max iterations


# ---------------------------------------------------- tensor-product helpers
def _r3(f, n):
    return f.reshape(f.shape[:-1] + (n, n, n))        # [..., k, j, i]


def apply_DT(G, d, D, n):
    """(D_d^T G)_i = sum_q G(q) l'_{i_d}(xi_{q_d}) along direction d."""
    g = _r3(G, n)
    if d == 0:
        out = np.einsum('...kjq,qi->...kji', g, D)
    elif d == 1:
        out = np.einsum('...kqi,qj->...kji', g, D)
    else:
        out = np.einsum('...qji,qk->...kji', g, D)
    return out.reshape(G.shape)


def trace(f, d, s, basis):
    """Values of the Q_r fields f on face (d, s) at the face GL points."""
    n = basis.n
    g, v = _r3(f, n), basis.face[s]
    if d == 0:
        t = np.einsum('...kji,i->...kj', g, v)
    elif d == 1:
        t = np.einsum('...kji,j->...ki', g, v)
    else:
        t = np.einsum('...kji,k->...ji', g, v)
    return t.reshape(f.shape[:-1] + (n * n,))


def lift(phi, d, s, basis):
    """out_i = psi_i(point) * phi(point) summed over the points of face (d, s)."""
    n = basis.n
    p, v = phi.reshape(phi.shape[:-1] + (n, n)), basis.face[s]
    if d == 0:
        out = np.einsum('...kj,i->...kji', p, v)
    elif d == 1:
        out = np.einsum('...ki,j->...kji', p, v)
    else:
        out = np.einsum('...ji,k->...kji', p, v)
    return out.reshape(phi.shape[:-1] + (n ** 3,))


def sub_interp(fv, sub, basis):
    """Face polynomial with GL values fv evaluated at the GL points of quarter sub."""
    n = basis.n
    h1, h2 = sub % 2, sub // 2
    p = fv.reshape(fv.shape[:-1] + (n, n))                # [b][a]
    out = np.einsum('...ba,xa,yb->...yx', p, basis.half[h1], basis.half[h2])
    return out.reshape(fv.shape)


def sub_interp_T(fv, sub, basis):
    """Transpose of sub_interp (coarse-side test functions at subface points)."""
    n = basis.n
    h1, h2 = sub % 2, sub // 2
    p = fv.reshape(fv.shape[:-1] + (n, n))                # [b'][a']
    out = np.einsum('...yx,xa,yb->...ba', p, basis.half[h1], basis.half[h2])
    return out.reshape(fv.shape)


def face_integrals(mesh: Mesh, fields, flux, nout):
    """sum over faces of K of int Fn psi_i dS, Fn the normal flux seen from K.

    fields: (nf, E, Np) Q_r fields whose traces the flux needs.
    flux(qA, qB, nS) -> (nout, F, Nf): normal flux on side A, with nS (F, Nf, 3)
    the outward area vector of side A; qB is None on a wall. The flux seen
    from side B is the negative (both sides share nS up to its sign).
    """
    b = mesh.basis
    out = np.zeros((nout, mesh.E, mesh.Np))
    W2 = mesh.W2
    for d, A, B in mesh.conf:
        if len(A) == 0:
            continue
        qA = trace(fields[:, A], d, 1, b)
        qB = trace(fields[:, B], d, 0, b)
        Fn = flux(qA, qB, mesh.nS[A, 2 * d + 1]) * W2
        np.add.at(out, (slice(None), A), lift(Fn, d, 1, b))
        np.add.at(out, (slice(None), B), -lift(Fn, d, 0, b))
    for d, s, sb, A, B in mesh.hang:
        qA = trace(fields[:, A], d, s, b)
        qB = sub_interp(trace(fields[:, B], d, 1 - s, b), sb, b)
        Fn = flux(qA, qB, mesh.nS[A, 2 * d + s]) * W2
        np.add.at(out, (slice(None), A), lift(Fn, d, s, b))
        np.add.at(out, (slice(None), B), -lift(sub_interp_T(Fn, sb, b), d, 1 - s, b))
    for d, s, A in mesh.wall:
        qA = trace(fields[:, A], d, s, b)
        Fn = flux(qA, None, mesh.nS[A, 2 * d + s]) * W2
        np.add.at(out, (slice(None), A), lift(Fn, d, s, b))
    return out


def weak_grad(mesh: Mesh, F):
    """int_K F . grad(psi_i) for a physical vector field F (3, E, Np)."""
    WJ = mesh.W3 * mesh.detJ
    G = np.einsum('eqdc,ceq->deq', mesh.Jinv, F) * WJ
    D = mesh.basis.deriv
    return sum(apply_DT(G[d], d, D, mesh.n) for d in range(3))


def _unit(nS):
    dS = np.sqrt((nS * nS).sum(-1))
    return nS / dS[..., None], dS


def _mirror(v, nh):
    """Reflect a vector field (3, F, Nf) in the wall with unit normal nh (F, Nf, 3)."""
    vn = np.einsum('cfp,fpc->fp', v, nh)
    return v - 2.0 * vn[None] * np.moveaxis(nh, -1, 0)


def primitives(q, gamma):
    rho, m, E = q[0], q[1:4], q[4]
    u = m / rho
    kin = 0.5 * (u * u).sum(0)
    p = (gamma - 1.0) * (E - rho * kin)
    return rho, m, E, u, kin, p


def sponge_coefficient(phys: Phys, xyz, Lx, Ly):
    """Rayleigh damping coefficient of eq. damping (Sec. 4.3) at points
    xyz (..., 3): the top layer lam sin^2(pi/2 (z - zB)/(zT - zB)) for z >= zB
    and, in the lateral buffer regions of widths sponge_xw and sponge_yw at
    both ends of [0, Lx] and [0, Ly], the same profile of the depth into the
    layer (0 at its inner edge, 1 at the boundary); the largest applies."""
    z = xyz[..., 2]
    if phys.sponge_lam == 0.0:
        return np.zeros_like(z)
    s = np.clip((z - phys.sponge_zB) / (phys.sponge_zT - phys.sponge_zB), 0.0, None)
    lam = np.where(z >= phys.sponge_zB, phys.sponge_lam * np.sin(0.5 * np.pi * s) ** 2, 0.0)
    for d, (w, ext) in enumerate(((phys.sponge_xw, Lx), (phys.sponge_yw, Ly))):
        if w <= 0.0:
            continue
        x = xyz[..., d]
        depth = np.where(x < w, (w - x) / w, np.where(x > ext - w, (x - (ext - w)) / w, 0.0))
        lam = np.maximum(lam, np.where(depth > 0.0, phys.sponge_lam * np.sin(0.5 * np.pi * depth) ** 2, 0.0))
    return lam


# --------------------------------------------------------- explicit residual
def explicit_residual(mesh: Mesh, phys: Phys, q):
    """T_NS(q) and T_S(q) as dual vectors (5, E, Np) (weak forms of Sec. 3).

    Non-stiff: advective fluxes m, m (x) u, kappa m with Rusanov dissipation on
    rho, m, rho*kappa (and the optional sponge). Stiff: pressure p I with a
    centred flux, enthalpy flux rho h u with Rusanov dissipation on rho e,
    gravity -rho g k and Coriolis -rho f k x u, and the gravity work -rho g w.

    Face values are formed from the traces of the nodal primitive fields
    (rho, u, p): the averages and jumps of Sec. 3 are written in rho, u, p, h,
    kappa and e, and the stage operators B and C act on the traces of the
    unknowns p and u, so T_S evaluated here at a converged stage is the same
    discrete operator as the one the stage equation was solved with (and the
    final update, whose implicit weights equal the last stage's, reproduces
    the stage solution). Taking the face values from traces of the conserved
    fields instead gives u_face = trace(m)/trace(rho), not trace(u): a linear
    difference about a stratified state that the update then fails to cancel.
    """
    gam = phys.gamma
    rho, m, E, u, kin, p = primitives(q, gam)
    WJ = mesh.W3 * mesh.detJ
    TNS = np.zeros((5, mesh.E, mesh.Np))
    TS = np.zeros((5, mesh.E, mesh.Np))
    TNS[0] = weak_grad(mesh, m)
    for c in range(3):
        TNS[1 + c] = weak_grad(mesh, m[c][None] * u)
    TNS[4] = weak_grad(mesh, kin[None] * m)
    for c in range(3):
        Fp = np.zeros((3, mesh.E, mesh.Np))
        Fp[c] = p
        TS[1 + c] = weak_grad(mesh, Fp)
    rhoh = gam / (gam - 1.0) * p
    TS[4] = weak_grad(mesh, rhoh[None] * u)
    TS[1] += WJ * rho * phys.f * u[1]
    TS[2] -= WJ * rho * phys.f * u[0]
    TS[3] -= WJ * rho * phys.g
    TS[4] -= WJ * rho * phys.g * u[2]
    if phys.sponge_lam != 0.0:
        lam = sponge_coefficient(phys, mesh.xq, mesh.desc.Lx, mesh.desc.Ly)
        if phys.sponge_target is None:
            for c in range(3):
                TNS[1 + c] -= WJ * lam * (m[c] - rho * phys.sponge_u[c])
        else:
            # Rayleigh relaxation of the whole conserved state (rho, rho u,
            # rho E) towards the target (the variables a damping layer acts on
            # are not stated in Sec. 4.3; this is the second of two readings)
            TNS -= WJ * lam * (q - phys.sponge_target)

    def flux(PA, PB, nS):
        # PA, PB: traces of (rho, u, p) on the two sides; slip walls mirror u
        nh, dS = _unit(nS)
        if PB is None:
            PB = PA.copy()
            PB[1:4] = _mirror(PA[1:4], nh)
        sides = []
        for P in (PA, PB):
            r, uu, pp = P[0], P[1:4], P[4]
            mm = r * uu
            kk = 0.5 * (uu * uu).sum(0)
            un = np.einsum('cfp,fpc->fp', uu, nh)
            sides.append((r, mm, uu, kk, pp, un))
        (rA, mA, uA, kA, pA, unA), (rB, mB, uB, kB, pB, unB) = sides
        lam = np.maximum(np.abs(unA), np.abs(unB))
        mnA = np.einsum('cfp,fpc->fp', mA, nS)
        mnB = np.einsum('cfp,fpc->fp', mB, nS)
        unSA = np.einsum('cfp,fpc->fp', uA, nS)
        unSB = np.einsum('cfp,fpc->fp', uB, nS)
        out = np.zeros((10,) + rA.shape)
        out[0] = 0.5 * (mnA + mnB) + 0.5 * lam * (rA - rB) * dS
        for c in range(3):
            out[1 + c] = 0.5 * (mA[c] * unSA + mB[c] * unSB) + 0.5 * lam * (mA[c] - mB[c]) * dS
        out[4] = 0.5 * (kA * mnA + kB * mnB) + 0.5 * lam * (rA * kA - rB * kB) * dS
        for c in range(3):
            out[6 + c] = 0.5 * (pA + pB) * nS[..., c]
        hA, hB = gam / (gam - 1.0) * pA, gam / (gam - 1.0) * pB
        out[9] = 0.5 * (hA * unSA + hB * unSB) + 0.5 * lam * (pA - pB) / (gam - 1.0) * dS
        return out

    Fc = face_integrals(mesh, np.concatenate([rho[None], u, p[None]]), flux, 10)
    TNS -= Fc[:5]
    TS -= Fc[5:]
    return TNS, TS


# ------------------------------------------------------------ stage system
class StageSystem:
    """Matrices of the stage-l system (Sec. 3) at Picard iterate (p^k, u^k).

    A u + R u + B p + f_g = f,    C^k u + M_g u + D p + k^k = g^k
    with c = a_ll dt, beta = c f and the lagged coefficients (rho h)^k,
    kappa^k, lambda^k taken from (p^k, u^k).
    """

    def __init__(self, mesh: Mesh, phys: Phys, rho_l, p_k, u_k, a_ll, dt, scheme):
        self.mesh, self.phys, self.scheme = mesh, phys, scheme
        self.rho_l, self.p_k, self.u_k = rho_l, p_k, u_k
        self.c = a_ll * dt
        self.beta = a_ll * dt * phys.f
        self.WJ = mesh.W3 * mesh.detJ
        gam = phys.gamma
        self.rhoh_k = gam / (gam - 1.0) * p_k

    # momentum-block matrices ------------------------------------------------
    def A(self, u):
        return self.WJ * self.rho_l * u

    def A_inv(self, v):
        """A_K = S^T W_rho S with S = I (Sec. 3.1): a pointwise division."""
        return v / (self.WJ * self.rho_l)

    def R(self, u):
        """R u = c f int rho_l (k x u) . phi."""
        kxu = np.stack([-u[1], u[0], np.zeros_like(u[0])])
        return self.c * self.phys.f * self.WJ * self.rho_l * kxu

    def IbJ_inv(self, u):
        """(I + beta J)^{-1} applied pointwise, with the closed form of Sec. 3.1."""
        b = self.beta
        s = 1.0 / (1.0 + b * b)
        return np.stack([s * (u[0] + b * u[1]), s * (-b * u[0] + u[1]), u[2]])

    def f_g(self):
        out = np.zeros((3,) + self.rho_l.shape)
        out[2] = self.c * self.phys.g * self.WJ * self.rho_l
        return out

    def B(self, p):
        """B p = c ( -int p div(phi) + int_dK {p} phi . n )."""
        mesh = self.mesh
        out = np.zeros((3, mesh.E, mesh.Np))
        for comp in range(3):
            Fp = np.zeros((3, mesh.E, mesh.Np))
            Fp[comp] = p
            out[comp] = -weak_grad(mesh, Fp)

        def flux(qA, qB, nS):
            pB = qA[0] if qB is None else qB[0]
            avg = 0.5 * (qA[0] + pB)
            return np.moveaxis(avg[..., None] * nS, -1, 0)

        out += face_integrals(mesh, p[None], flux, 3)
        return self.c * out

    # energy-block matrices --------------------------------------------------
    def C(self, w):
        """C^k w = c ( -int (rho h)^k w . grad psi + int_dK {(rho h)^k w} . n psi )."""
        mesh, gam = self.mesh, self.phys.gamma
        vol = -weak_grad(mesh, self.rhoh_k[None] * w)

        def flux(qA, qB, nS):
            nh, _ = _unit(nS)
            wA, hA = qA[0:3], gam / (gam - 1.0) * qA[3]
            if qB is None:
                wB, hB = _mirror(wA, nh), hA
            else:
                wB, hB = qB[0:3], gam / (gam - 1.0) * qB[3]
            fA = np.einsum('cfp,fpc->fp', hA[None] * wA, nS)
            fB = np.einsum('cfp,fpc->fp', hB[None] * wB, nS)
            return (0.5 * (fA + fB))[None]

        fields = np.concatenate([w, self.p_k[None]])
        face = face_integrals(mesh, fields, flux, 1)[0]
        return self.c * (vol + face)

    def D(self, p):
        return self.WJ * p / (self.phys.gamma - 1.0)

    def M_g(self, u):
        """[M_g u]_i = c g int rho_l (k . u) psi_i."""
        return self.c * self.phys.g * self.WJ * self.rho_l * u[2]

    def k_vec(self):
        """k_i = int rho_l kappa^k psi_i, kappa^k = |u^k|^2 / 2."""
        return self.WJ * self.rho_l * 0.5 * (self.u_k * self.u_k).sum(0)

    def Lam(self):
        """c int_dK lambda^k/2 ((rho e)^{k,-} - (rho e)^{k,+}) psi: the implicit
        Rusanov term on internal energy, lagged at iterate k."""
        mesh, gam = self.mesh, self.phys.gamma

        def flux(qA, qB, nS):
            nh, dS = _unit(nS)
            if qB is None:
                return np.zeros((1,) + qA.shape[1:])
            unA = np.abs(np.einsum('cfp,fpc->fp', qA[0:3], nh))
            unB = np.abs(np.einsum('cfp,fpc->fp', qB[0:3], nh))
            lam = np.maximum(unA, unB)
            return (0.5 * lam * (qA[3] - qB[3]) / (gam - 1.0) * dS)[None]

        fields = np.concatenate([self.u_k, self.p_k[None]])
        return self.c * face_integrals(mesh, fields, flux, 1)[0]

    # Schur complement ---------------------------------------------------------
    def schur(self, p):
        """R2: [D - (C^k + M_g)(A + R)^{-1} B] p, R1: [D - C^k A^{-1} B] p."""
        Bp = self.B(p)
        if self.scheme == R2:
            w = self.IbJ_inv(self.A_inv(Bp))
            return self.D(p) - self.C(w) - self.M_g(w)
        w = self.A_inv(Bp)
        return self.D(p) - self.C(w)

    def rhs(self, F, G0):
        """Right-hand side of the pressure system; F = f - f_g, G0 = g without
        the lagged implicit Rusanov term."""
        base = G0 - self.Lam() - self.k_vec()
        if self.scheme == R2:
            w = self.IbJ_inv(self.A_inv(F))
            return base - self.C(w) - self.M_g(w)
        w = self.A_inv(F - self.R(self.u_k))
        return base - self.M_g(self.u_k) - self.C(w)

    def recover_u(self, F, p):
        if self.scheme == R2:
            return self.IbJ_inv(self.A_inv(F - self.B(p)))
        return self.A_inv(F - self.R(self.u_k) - self.B(p))


# ------------------------------------------------------------------ GMRES
def gmres(apply, b, x0, Mw, tol, restart, maxit, fixed):
    """Restarted GMRES(m) (Saad, Alg. 6.9 with Givens rotations, modified
    Gram-Schmidt) in the inner product <a, b> = sum Mw a b.

    Stops when the Givens residual estimate falls to tol*|b| (unless `fixed`),
    after maxit matrix-vector products, or on an exact breakdown; the final
    residual is recomputed from the solution.
    Returns (x, iterations, |b - A x| / |b|).
    """
    def dot(a, c):
        return float(np.sum(Mw * a * c))

    bnorm = math.sqrt(dot(b, b))
    x = x0.copy()
    its = 0
    r = b - apply(x)
    beta = math.sqrt(dot(r, r))
    while True:
        if beta == 0.0 or its >= maxit or (not fixed and beta <= tol * bnorm):
            break
        m = restart
        V = [r / beta]
        H = np.zeros((m + 1, m))
        g = np.zeros(m + 1)
        g[0] = beta
        cs = np.zeros(m)
        sn = np.zeros(m)
        k = 0
        for j in range(m):
            w = apply(V[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = math.sqrt(dot(w, w))
            hnext = H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            if hnext == 0.0 or its >= maxit or (not fixed and abs(g[j + 1]) <= tol * bnorm):
                break
            V.append(w / hnext)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x = x + y[i] * V[i]
        r = b - apply(x)
        beta = math.sqrt(dot(r, r))
    rel = beta / bnorm if bnorm > 0 else 0.0
    return x, its, rel


# --------------------------------------------------------------- stage solve
def picard_variation(Mw, gamma, rho_l, p_old, u_old, p_new, u_new):
    """Relative variation of consecutive Picard iterates (u, p).

    The velocity change is put in pressure units with the acoustic impedance
    rho c (c^2 = gamma p / rho), so both unknowns count:
    delta^2 = sum Mw [dp^2 + gamma p rho |du|^2] / sum Mw p^2.
    """
    dp = p_new - p_old
    du = u_new - u_old
    num = np.sum(Mw * (dp * dp + gamma * p_new * rho_l * (du * du).sum(0)))
    den = np.sum(Mw * p_new * p_new)
    return math.sqrt(float(num) / float(den))


def stage_solve(mesh, phys, num: Numerics, rho_l, F, G0, p0, u0, a_ll):
    """Picard iteration of Sec. 3 on the stage system (R1 or R2), started from
    the previous stage and stopped on the relative variation of the iterates."""
    Mw = mesh.W3 * mesh.detJ
    p, u = p0, u0
    stats = {"picard": 0, "gmres": 0, "variation": 0.0}
    for k in range(num.picard_max):
        S = StageSystem(mesh, phys, rho_l, p, u, a_ll, num.dt, num.scheme)
        b = S.rhs(F, G0) / Mw
        pn, its, _ = gmres(lambda x: S.schur(x) / Mw, b, p, Mw, num.gmres_tol,
                           num.gmres_restart, num.gmres_max, num.fixed_iterations)
        un = S.recover_u(F, pn)
        stats["picard"] += 1
        stats["gmres"] += its
        var = picard_variation(Mw, phys.gamma, rho_l, p, u, pn, un)
        stats["variation"] = var
        p, u = pn, un
        if not num.fixed_iterations and var <= num.picard_tol:
            break
    return p, u, stats


# ------------------------------------------------------------------ ARK2 step
def ark2_step(mesh: Mesh, phys: Phys, num: Numerics, y, return_stages=False):
    """One IMEX-ARK2 step (Sec. 3): explicit density, implicit (u, p) stages,
    final update with the shared weights b. With return_stages the stage
    states Y_1..Y_3 and their explicit residuals (T_NS, T_S) are returned as
    well (stats["stages"], stats["residuals"])."""
    gam, dt = phys.gamma, num.dt
    Mw = mesh.W3 * mesh.detJ
    Ys = [y]
    T = [explicit_residual(mesh, phys, y)]
    stats = {"picard": 0, "gmres": 0}
    for l in (1, 2):                       # stages 2 and 3 (0-based index l)
        rho_l = y[0] + dt * sum(A_EXP[l, m] * T[m][0][0] for m in range(l)) / Mw
        F = Mw * y[1:4] + dt * sum(A_EXP[l, m] * T[m][0][1:4] + A_IMP[l, m] * T[m][1][1:4]
                                   for m in range(l))
        G0 = Mw * y[4] + dt * sum(A_EXP[l, m] * T[m][0][4] + A_IMP[l, m] * T[m][1][4]
                                  for m in range(l))
        a_ll = A_IMP[l, l]
        F = F - StageSystem(mesh, phys, rho_l, rho_l, y[1:4], a_ll, dt, num.scheme).f_g()
        _, _, _, u0, _, p0 = primitives(Ys[l - 1], gam)
        p, u, st = stage_solve(mesh, phys, num, rho_l, F, G0, p0, u0, a_ll)
        stats["picard"] += st["picard"]
        stats["gmres"] += st["gmres"]
        Yl = np.empty_like(y)
        Yl[0] = rho_l
        Yl[1:4] = rho_l * u
        Yl[4] = p / (gam - 1.0) + 0.5 * rho_l * (u * u).sum(0)
        Ys.append(Yl)
        T.append(explicit_residual(mesh, phys, Yl))
    ynew = y + dt * sum(B_W[l] * (T[l][0] + T[l][1]) for l in range(3)) / Mw
    if phys.slice:
        ynew = slice_project(mesh, ynew)
    if return_stages:
        stats["stages"], stats["residuals"] = Ys, T
    return ynew, stats


def slice_project(mesh: Mesh, q):
    """L2 projection of nodal fields (..., E, Np) onto the functions that are
    constant in y within each element: the y-lines of nodes are replaced by
    their Gauss-weighted mean sum_j w_j f_j / sum_j w_j, which is the exact
    integral mean of the degree-r polynomial in y (so element integrals, and
    the mass, are unchanged). On a slice mesh this imposes d/dy = 0 of the
    vertical-slice equations on the discrete state."""
    n, w = mesh.n, mesh.basis.w
    g = q.reshape(q.shape[:-1] + (n, n, n))                    # [..., k, j, i]
    m = np.einsum('...kji,j->...ki', g, w) / w.sum()
    return np.broadcast_to(m[..., :, None, :], g.shape).reshape(q.shape).copy()


def total_mass(mesh: Mesh, q):
    return float(np.sum(mesh.W3 * mesh.detJ * q[0]))
