"""A resting column with its volume and face integrals on Q Gauss points per
direction (test infrastructure for the spectrum study).

The oracle evaluates every integral with the (r+1)-point Gauss-Legendre rule
at the nodes (collocation). This module evaluates the same weak forms of
T_NS + T_S on a periodic 1 x 1 x nz column of boxes with slip walls at the
bottom and top, interpolating the nodal state to Q points per direction:
Q = r + 1 reproduces the oracle (checked in the test), Q > r + 1 integrates
the nonlinear and variable-coefficient products more exactly
(over-integration). Face values come from the traces of the nodal primitive
fields (rho, u, p), as in the method; the volume integrands from the
conserved state at the Q points. It is written for flat boxes only.
"""
import numpy as np

from oracle.basis import Basis1D, gauss_legendre, lagrange_derivatives, lagrange_values

GAM = 1.4


def prim(q):
    rho, m, E = q[0], q[1:4], q[4]
    u = m / rho
    k = 0.5 * (u * u).sum(0)
    p = (GAM - 1) * (E - rho * k)
    return rho, m, E, u, k, p


def nodal_prims(qq):
    """(rho, u, p) of a nodal conserved state (5, ...)."""
    rho = qq[0]
    u = qq[1:4] / rho
    p = (GAM - 1) * (qq[4] - 0.5 * rho * (u * u).sum(0))
    return np.concatenate([rho[None], u, p[None]])


def cons(P):
    """Conserved state from (rho, u, p) (5, ...)."""
    rho, u, p = P[0], P[1:4], P[4]
    return np.concatenate([rho[None], rho * u, (p / (GAM - 1) + 0.5 * rho * (u * u).sum(0))[None]])


def face_flux(qA, qB, nS, wall):
    """Rusanov / centred fluxes (10 comps) as the oracle: 0..4 NS, 6..8 pressure, 9 enthalpy.
    qA, qB: (5, ...), nS: 3-vector (uniform)."""
    nS = np.asarray(nS, float)
    dS = np.sqrt((nS * nS).sum())
    nh = nS / dS
    if wall:
        qB = qA.copy()
        mn = np.einsum('c...,c->...', qA[1:4], nh)
        qB[1:4] = qA[1:4] - 2 * mn[None] * nh.reshape(3, *([1] * mn.ndim))
    rA, mA, EA, uA, kA, pA = prim(qA)
    rB, mB, EB, uB, kB, pB = prim(qB)
    unA = np.einsum('c...,c->...', uA, nh)
    unB = np.einsum('c...,c->...', uB, nh)
    lam = np.maximum(np.abs(unA), np.abs(unB))
    mnA = np.einsum('c...,c->...', mA, nS)
    mnB = np.einsum('c...,c->...', mB, nS)
    unSA = np.einsum('c...,c->...', uA, nS)
    unSB = np.einsum('c...,c->...', uB, nS)
    out = np.zeros((10,) + rA.shape)
    out[0] = 0.5 * (mnA + mnB) + 0.5 * lam * (rA - rB) * dS
    for c in range(3):
        out[1 + c] = 0.5 * (mA[c] * unSA + mB[c] * unSB) + 0.5 * lam * (mA[c] - mB[c]) * dS
    out[4] = 0.5 * (kA * mnA + kB * mnB) + 0.5 * lam * (rA * kA - rB * kB) * dS
    for c in range(3):
        out[6 + c] = 0.5 * (pA + pB) * nS[c]
    hA, hB = GAM / (GAM - 1) * pA, GAM / (GAM - 1) * pB
    out[9] = 0.5 * (hA * unSA + hB * unSB) + 0.5 * lam * (pA - pB) / (GAM - 1) * dS
    return out


class Column:
    def __init__(self, n, Q, h, nz, grav=9.81, fcor=0.0):
        self.n, self.Q, self.h, self.nz, self.g, self.f = n, Q, h, nz, grav, fcor
        xn = Basis1D(n - 1).x
        self.xn = xn
        self.wn = Basis1D(n - 1).w
        xq, wq = gauss_legendre(Q)
        self.wq = wq
        self.L = lagrange_values(xn, xq)          # [Q, n]
        self.D = lagrange_derivatives(xn, xq)     # [Q, n]
        self.F = lagrange_values(xn, np.array([0.0, 1.0]))   # [2, n]
        hx, hy, hz = h
        self.M = np.einsum('k,j,i->kji', self.wn, self.wn, self.wn) * hx * hy * hz

    def quad(self, q):          # nodal (5, nz, n,n,n)[k,j,i] -> quad (5, nz, c,b,a)
        L = self.L
        return np.einsum('fekji,ai,bj,ck->fecba', q, L, L, L)

    def residual(self, q):
        n, Q, (hx, hy, hz), nz = self.n, self.Q, self.h, self.nz
        L, D, F, wq = self.L, self.D, self.F, self.wq
        qq = q.reshape(5, nz, n, n, n)
        Pn = nodal_prims(qq)
        Vq = self.quad(qq)
        rho, m, E, u, k, p = prim(Vq)
        J = hx * hy * hz
        Wq = np.einsum('c,b,a->cba', wq, wq, wq) * J
        # flux vectors per output: (10, 3, nz, c, b, a): 0..4 NS, 6..8 pressure, 9 enthalpy
        Fl = np.zeros((10, 3) + rho.shape)
        Fl[0] = m
        for c in range(3):
            Fl[1 + c] = m[c][None] * u
        Fl[4] = k[None] * m
        for c in range(3):
            Fl[6 + c, c] = p
        Fl[9] = (GAM / (GAM - 1) * p)[None] * u
        T = np.zeros((10, nz, n, n, n))
        WF = Fl * Wq
        T += np.einsum('tecba,ai,bj,ck->tekji', WF[:, 0], D, L, L) / hx
        T += np.einsum('tecba,ai,bj,ck->tekji', WF[:, 1], L, D, L) / hy
        T += np.einsum('tecba,ai,bj,ck->tekji', WF[:, 2], L, L, D) / hz
        # sources
        S = np.zeros((10,) + rho.shape)
        S[6] = rho * self.f * u[1]
        S[7] = -rho * self.f * u[0]
        S[8] = -rho * self.g
        S[9] = -rho * self.g * u[2]
        T += np.einsum('tecba,ai,bj,ck->tekji', S * Wq, L, L, L)
        # faces: traces at the quad points of each face
        W2 = lambda w1, w2: np.einsum('b,a->ba', w1, w2)
        # x faces (periodic, one element): A = element at x=1, B = same element at x=0
        tA = cons(np.einsum('fekji,i,bj,ck->fecb', Pn, F[1], L, L))
        tB = cons(np.einsum('fekji,i,bj,ck->fecb', Pn, F[0], L, L))
        fl = face_flux(tA, tB, [hy * hz, 0, 0], False) * np.einsum('c,b->cb', wq, wq)
        T -= np.einsum('tecb,i,bj,ck->tekji', fl, F[1], L, L)
        T += np.einsum('tecb,i,bj,ck->tekji', fl, F[0], L, L)
        # y faces
        tA = cons(np.einsum('fekji,ai,j,ck->feca', Pn, L, F[1], L))
        tB = cons(np.einsum('fekji,ai,j,ck->feca', Pn, L, F[0], L))
        fl = face_flux(tA, tB, [0, hx * hz, 0], False) * np.einsum('c,a->ca', wq, wq)
        T -= np.einsum('teca,ai,j,ck->tekji', fl, L, F[1], L)
        T += np.einsum('teca,ai,j,ck->tekji', fl, L, F[0], L)
        # z faces: interior between e (top, s=1) and e+1 (bottom, s=0); walls at the ends
        top = cons(np.einsum('fekji,ai,bj,k->feba', Pn, L, L, F[1]))
        bot = cons(np.einsum('fekji,ai,bj,k->feba', Pn, L, L, F[0]))
        wba = np.einsum('b,a->ba', wq, wq)
        nS = [0, 0, hx * hy]
        if nz > 1:
            fl = face_flux(top[:, :-1], bot[:, 1:], nS, False) * wba
            T[:, :-1] -= np.einsum('teba,ai,bj,k->tekji', fl, L, L, F[1])
            T[:, 1:] += np.einsum('teba,ai,bj,k->tekji', fl, L, L, F[0])
        fl = face_flux(top[:, -1:], None, nS, True) * wba
        T[:, -1:] -= np.einsum('teba,ai,bj,k->tekji', fl, L, L, F[1])
        fl = face_flux(bot[:, :1], None, [0, 0, -hx * hy], True) * wba
        T[:, :1] -= np.einsum('teba,ai,bj,k->tekji', fl, L, L, F[0])
        TNS = T[:5]
        TS = np.concatenate([np.zeros((1,) + T.shape[1:]), T[6:]])
        return TNS.reshape(5, nz, n ** 3), TS.reshape(5, nz, n ** 3)

    def rhs(self, q):
        TNS, TS = self.residual(q)
        return ((TNS + TS).reshape(5, self.nz, self.n, self.n, self.n) / self.M).reshape(q.shape)


