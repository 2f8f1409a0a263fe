"""Independent dense brute-force evaluation of the DG weak forms on tiny meshes.

Nothing here uses the oracle's tensor contractions, face tables or geometry:
- basis functions are full 3D Lagrange products evaluated point by point,
  their reference gradients and the mesh Jacobian come from complex-step
  differentiation (exact to rounding for analytic functions);
- face area vectors are cross products of the two tangent vectors;
- the element across a face is found by searching which leaf's flat box holds a
  point just outside the face; a face whose neighbour is finer is integrated
  over its four quarters.
Only the list of leaves (their flat boxes, in the project's element order) and
the analytic surface/Gal-Chen definitions are taken as inputs.
"""
import math
import numpy as np

HC = 1e-30          # complex-step size


def gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1), 0.5 * w


def gll(n):
    inner = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots()
    return 0.5 * (np.concatenate(([-1.0], np.sort(inner.real), [1.0])) + 1)


def lag(nodes, x):
    """Lagrange polynomials of `nodes` at scalar x (real or complex): vector."""
    n = len(nodes)
    v = np.ones(n, dtype=complex)
    for i in range(n):
        for m in range(n):
            if m != i:
                v[i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return v


class Dense:
    def __init__(self, mesh_desc, leaves, degree):
        """leaves: (base[E,3], level[E], sub[E,3]) in element order."""
        self.desc = mesh_desc
        self.base, self.level, self.sub = leaves
        self.E = len(self.level)
        self.r = degree
        self.n = degree + 1
        self.Np = self.n ** 3
        self.h0 = np.array([mesh_desc.Lx / mesh_desc.nx, mesh_desc.Ly / mesh_desc.ny,
                            mesh_desc.Lz / mesh_desc.nz])
        self.nodes, self.wts = gl(self.n)
        self.lo = np.array([(self.base[e] + self.sub[e] / 2.0 ** self.level[e]) * self.h0
                            for e in range(self.E)])
        self.hi = np.array([(self.base[e] + (self.sub[e] + 1) / 2.0 ** self.level[e]) * self.h0
                            for e in range(self.E)])
        self._setup()

    # ------------------------------------------------------------ geometry
    def surface(self, x, y):
        d = self.desc
        dx, dy = x - d.xc, y - d.yc
        if d.periodic_x:
            dx = dx - d.Lx * np.round(np.real(dx) / d.Lx)
        if d.periodic_y:
            dy = dy - d.Ly * np.round(np.real(dy) / d.Ly)
        r2 = (dx * dx + dy * dy) / d.a ** 2
        if d.terrain == 1:
            return d.h0 / (1 + r2)
        if d.terrain == 2:
            return d.h0 * np.exp(-r2)
        return 0.0 * x

    def X(self, e, xi):
        """Physical point of reference point xi (possibly complex) in element e."""
        L = self.level[e]
        eta = (self.sub[e] + xi) / 2.0 ** L
        flat = (self.base[e] + eta) * self.h0
        if self.desc.terrain == 0:
            return flat
        g = gll(self.n)
        b = self.base[e]
        zsum = 0.0
        la, lb, lc = lag(g, eta[0]), lag(g, eta[1]), lag(g, eta[2])
        for a in range(self.n):
            xa = (b[0] + g[a]) * self.h0[0]
            for bb in range(self.n):
                yb = (b[1] + g[bb]) * self.h0[1]
                h = self.surface(xa, yb)
                for c in range(self.n):
                    zeta = (b[2] + g[c]) * self.h0[2]
                    zg = h + zeta * (self.desc.Lz - h) / self.desc.Lz
                    zsum = zsum + zg * la[a] * lb[bb] * lc[c]
        return np.array([flat[0], flat[1], zsum])

    def jac(self, e, xi):
        J = np.zeros((3, 3))
        for d in range(3):
            dxi = np.zeros(3, dtype=complex)
            dxi[d] = 1j * HC
            J[:, d] = np.imag(self.X(e, xi.astype(complex) + dxi)) / HC
        return J

    # --------------------------------------------------------------- basis
    def psi(self, xi):
        lx, ly, lz = (lag(self.nodes, xi[0]), lag(self.nodes, xi[1]), lag(self.nodes, xi[2]))
        return np.einsum('k,j,i->kji', lz, ly, lx).reshape(-1)

    def psi_real(self, xi):
        return np.real(self.psi(np.asarray(xi, dtype=complex)))

    def grad_ref(self, xi):
        G = np.zeros((self.Np, 3))
        for d in range(3):
            dxi = np.zeros(3, dtype=complex)
            dxi[d] = 1j * HC
            G[:, d] = np.imag(self.psi(xi.astype(complex) + dxi)) / HC
        return G

    # ---------------------------------------------------------- neighbours
    def locate(self, flat):
        d = self.desc
        p = flat.copy()
        Ls = np.array([d.Lx, d.Ly, d.Lz])
        for c, per in ((0, d.periodic_x), (1, d.periodic_y)):
            if per:
                p[c] = p[c] % Ls[c]
        for c in range(3):
            if p[c] < 0 or p[c] > Ls[c]:
                return -1
        for e in range(self.E):
            if np.all(self.lo[e] <= p) and np.all(p <= self.hi[e]):
                return e
        return -1

    def ref_in(self, e, flat):
        """Reference coordinates of flat point in element e (periodic image)."""
        d = self.desc
        p = flat.copy()
        Ls = np.array([d.Lx, d.Ly, d.Lz])
        for c, per in ((0, d.periodic_x), (1, d.periodic_y)):
            if per:
                while p[c] < self.lo[e][c] - 1e-9 * Ls[c]:
                    p[c] += Ls[c]
                while p[c] > self.hi[e][c] + 1e-9 * Ls[c]:
                    p[c] -= Ls[c]
        return (p - self.lo[e]) / (self.hi[e] - self.lo[e])

    # ---------------------------------------------------------------- setup
    def _setup(self):
        n, Np = self.n, self.Np
        x, w = self.nodes, self.wts
        self.vol = []
        for e in range(self.E):
            V, G, WJ, Xp = [], [], [], []
            for k in range(n):
                for j in range(n):
                    for i in range(n):
                        xi = np.array([x[i], x[j], x[k]])
                        J = self.jac(e, xi)
                        V.append(self.psi_real(xi))
                        G.append(self.grad_ref(xi) @ np.linalg.inv(J))   # physical gradients
                        WJ.append(w[i] * w[j] * w[k] * np.linalg.det(J))
                        Xp.append(np.real(self.X(e, xi.astype(complex))))
            self.vol.append((np.array(V), np.array(G), np.array(WJ), np.array(Xp)))
        self.faces = []
        for e in range(self.E):
            recs = []
            for d in range(3):
                t1, t2 = [c for c in range(3) if c != d]
                for s in range(2):
                    # probe the element across at the face centre
                    size = self.hi[e] - self.lo[e]
                    centre = 0.5 * (self.lo[e] + self.hi[e])
                    probe = centre.copy()
                    probe[d] = (self.hi[e][d] + 1e-6 * size[d]) if s == 1 else (self.lo[e][d] - 1e-6 * size[d])
                    probe[t1] = self.lo[e][t1] + 0.25 * size[t1]
                    probe[t2] = self.lo[e][t2] + 0.25 * size[t2]
                    nb = self.locate(probe)
                    finer = nb >= 0 and self.level[nb] > self.level[e]
                    quarters = [(0, 0), (1, 0), (0, 1), (1, 1)] if finer else [None]
                    for qd in quarters:
                        pts = []
                        for b in range(n):
                            for a in range(n):
                                xi = np.zeros(3)
                                xi[d] = s
                                ta, tb = x[a], x[b]
                                wq = w[a] * w[b]
                                if qd is not None:
                                    ta, tb = 0.5 * (qd[0] + ta), 0.5 * (qd[1] + tb)
                                    wq = 0.25 * wq
                                xi[t1], xi[t2] = ta, tb
                                J = self.jac(e, xi)
                                area = np.cross(J[:, t1], J[:, t2])
                                # orient outward
                                out = np.zeros(3)
                                out[d] = 1.0 if s == 1 else -1.0
                                if np.dot(area, J @ out) < 0:
                                    area = -area
                                flat = self.lo[e] + xi * (self.hi[e] - self.lo[e])
                                step = flat.copy()
                                step[d] += (1e-6 if s == 1 else -1e-6) * (self.hi[e][d] - self.lo[e][d])
                                nbp = self.locate(step)
                                if nbp >= 0:
                                    xin = self.ref_in(nbp, flat)
                                    xin[d] = 0.0 if s == 1 else 1.0
                                    if self.level[nbp] >= self.level[e]:
                                        # conforming or finer: neighbour's face coordinate is exact
                                        pass
                                    vn = self.psi_real(xin)
                                else:
                                    vn = None
                                pts.append((self.psi_real(xi), nbp, vn, wq, area))
                        recs.append(pts)
            self.faces.append(recs)

    # ------------------------------------------------------------ helpers
    def eval_vol(self, f):
        """Values of nodal field f (E, Np) at the volume points of each element."""
        return np.array([self.vol[e][0] @ f[e] for e in range(self.E)])

    # ------------------------------------------------------- linear blocks
    def mass_blocks(self, coef):
        """Per-element sum_q WJ coef psi_i psi_j; coef (E, Nq)."""
        return [self.vol[e][0].T @ (self.vol[e][2][:, None] * coef[e][:, None] * self.vol[e][0])
                for e in range(self.E)]

    def assemble_scalar_mass(self, coef):
        N = self.E * self.Np
        M = np.zeros((N, N))
        for e, blk in enumerate(self.mass_blocks(coef)):
            s = slice(e * self.Np, (e + 1) * self.Np)
            M[s, s] = blk
        return M

    def assemble_B(self, c_dt):
        """B[(c,e,i),(e',j)] = c_dt(-int psi_j d_c psi_i + int_dK {psi_j} psi_i n_c)."""
        E, Np = self.E, self.Np
        B = np.zeros((3 * E * Np, E * Np))
        for e in range(E):
            V, G, WJ, _ = self.vol[e]
            for c in range(3):
                rows = slice(c * E * Np + e * Np, c * E * Np + (e + 1) * Np)
                B[rows, e * Np:(e + 1) * Np] += -c_dt * (G[:, :, c].T @ (WJ[:, None] * V))
            for pts in self.faces[e]:
                for (v, nb, vn, wq, area) in pts:
                    for c in range(3):
                        r0 = c * E * Np + e * Np
                        if nb < 0:
                            B[r0:r0 + Np, e * Np:(e + 1) * Np] += c_dt * wq * area[c] * np.outer(v, v)
                        else:
                            B[r0:r0 + Np, e * Np:(e + 1) * Np] += 0.5 * c_dt * wq * area[c] * np.outer(v, v)
                            B[r0:r0 + Np, nb * Np:(nb + 1) * Np] += 0.5 * c_dt * wq * area[c] * np.outer(v, vn)
        return B

    def assemble_C(self, c_dt, rhoh_nodal):
        """C[(e,i),(c,e',j)] = c_dt(-int rhoh psi_j d_c psi_i + int_dK {rhoh psi_j n_c} psi_i)."""
        E, Np = self.E, self.Np
        C = np.zeros((E * Np, 3 * E * Np))
        for e in range(E):
            V, G, WJ, _ = self.vol[e]
            hq = V @ rhoh_nodal[e]
            for c in range(3):
                cols = slice(c * E * Np + e * Np, c * E * Np + (e + 1) * Np)
                C[e * Np:(e + 1) * Np, cols] += -c_dt * (G[:, :, c].T @ ((WJ * hq)[:, None] * V))
            for pts in self.faces[e]:
                for (v, nb, vn, wq, area) in pts:
                    if nb < 0:
                        continue          # mirror state: {rho h w}.n = 0 on a slip wall
                    h_own = v @ rhoh_nodal[e]
                    h_nb = vn @ rhoh_nodal[nb]
                    for c in range(3):
                        c0 = c * E * Np
                        C[e * Np:(e + 1) * Np, c0 + e * Np:c0 + (e + 1) * Np] += 0.5 * c_dt * wq * area[c] * h_own * np.outer(v, v)
                        C[e * Np:(e + 1) * Np, c0 + nb * Np:c0 + (nb + 1) * Np] += 0.5 * c_dt * wq * area[c] * h_nb * np.outer(v, vn)
        return C

    def assemble_vector_mass(self, coef):
        """Block-diagonal over the 3 components."""
        Ms = self.assemble_scalar_mass(coef)
        N = Ms.shape[0]
        A = np.zeros((3 * N, 3 * N))
        for c in range(3):
            A[c * N:(c + 1) * N, c * N:(c + 1) * N] = Ms
        return A

    def assemble_R(self, cf, rho_nodal):
        """R[(i,a),(j,b)] = cf int rho (k x e_b) . e_a psi_j psi_i."""
        Ms = self.assemble_scalar_mass(self.eval_vol(rho_nodal))
        N = Ms.shape[0]
        R = np.zeros((3 * N, 3 * N))
        # k x e_x = e_y, k x e_y = -e_x
        R[N:2 * N, 0:N] = cf * Ms
        R[0:N, N:2 * N] = -cf * Ms
        return R

    def assemble_Mg(self, cg, rho_nodal):
        Ms = self.assemble_scalar_mass(self.eval_vol(rho_nodal))
        N = Ms.shape[0]
        Mg = np.zeros((N, 3 * N))
        Mg[:, 2 * N:3 * N] = cg * Ms
        return Mg

    # ---------------------------------------------------- nonlinear vectors
    @staticmethod
    def _nodal_prims(q, gamma):
        """(rho, u, p) at the nodes of every element: (5, E, Np)."""
        rho = q[0]
        u = q[1:4] / rho
        p = (gamma - 1) * (q[4] - 0.5 * rho * (u * u).sum(0))
        return np.concatenate([rho[None], u, p[None]])

    @staticmethod
    def _face_state(v, P, e, gamma):
        """Conserved state at a face point from the traces of the nodal
        primitives (the face values of the method: averages and jumps of rho,
        u, p and of what is formed from them)."""
        r = v @ P[0, e]
        u = np.array([v @ P[1 + c, e] for c in range(3)])
        p = v @ P[4, e]
        return np.concatenate([[r], r * u, [p / (gamma - 1) + 0.5 * r * (u @ u)]])

    def explicit_residual(self, q, gamma, g, f):
        """T_NS and T_S (5, E, Np) by direct point-by-point quadrature."""
        E, Np = self.E, self.Np
        TNS = np.zeros((5, E, Np))
        TS = np.zeros((5, E, Np))

        def prim(s):
            rho, m, Et = s[0], s[1:4], s[4]
            u = m / rho
            k = 0.5 * u @ u
            p = (gamma - 1) * (Et - rho * k)
            return rho, m, Et, u, k, p

        P = self._nodal_prims(q, gamma)
        for e in range(E):
            V, G, WJ, _ = self.vol[e]
            for qp in range(V.shape[0]):
                s = np.array([V[qp] @ q[fd, e] for fd in range(5)])
                rho, m, Et, u, k, p = prim(s)
                gr = G[qp]                       # (Np, 3)
                TNS[0, e] += WJ[qp] * gr @ m
                for c in range(3):
                    TNS[1 + c, e] += WJ[qp] * gr @ (m[c] * u)
                    TS[1 + c, e] += WJ[qp] * gr[:, c] * p
                TNS[4, e] += WJ[qp] * gr @ (k * m)
                TS[4, e] += WJ[qp] * gr @ (gamma / (gamma - 1) * p * u)
                ps = V[qp]
                TS[1, e] += WJ[qp] * rho * f * u[1] * ps
                TS[2, e] -= WJ[qp] * rho * f * u[0] * ps
                TS[3, e] -= WJ[qp] * rho * g * ps
                TS[4, e] -= WJ[qp] * rho * g * u[2] * ps
            for pts in self.faces[e]:
                for (v, nb, vn, wq, area) in pts:
                    dS = np.linalg.norm(area)
                    nh = area / dS
                    sA = self._face_state(v, P, e, gamma)
                    if nb < 0:
                        sB = sA.copy()
                        mB = sA[1:4] - 2 * (sA[1:4] @ nh) * nh
                        sB[1:4] = mB
                    else:
                        sB = self._face_state(vn, P, nb, gamma)
                    rA, mA, EA, uA, kA, pA = prim(sA)
                    rB, mB, EB, uB, kB, pB = prim(sB)
                    lam = max(abs(uA @ nh), abs(uB @ nh))
                    fl = np.zeros(10)
                    fl[0] = 0.5 * (mA + mB) @ area + 0.5 * lam * (rA - rB) * dS
                    for c in range(3):
                        fl[1 + c] = 0.5 * (mA[c] * (uA @ area) + mB[c] * (uB @ area)) + 0.5 * lam * (mA[c] - mB[c]) * dS
                        fl[6 + c] = 0.5 * (pA + pB) * area[c]
                    fl[4] = 0.5 * (kA * (mA @ area) + kB * (mB @ area)) + 0.5 * lam * (rA * kA - rB * kB) * dS
                    hA, hB = gamma / (gamma - 1) * pA, gamma / (gamma - 1) * pB
                    fl[9] = 0.5 * (hA * (uA @ area) + hB * (uB @ area)) + 0.5 * lam * (pA - pB) / (gamma - 1) * dS
                    TNS[:, e] -= wq * fl[:5, None] * v[None, :]
                    TS[1:, e] -= wq * fl[6:, None] * v[None, :]
        return TNS, TS

    def euler_total_residual(self, q, gamma):
        """Textbook DG residual of the full Euler equations (no sources):
        int F(q) : grad psi - int_dK (F^ . n) psi with the flux tensor
        F = (m, m u^T + p I, (E + p) u) and the Rusanov flux
        F^ . n = {F(q) . n} + lambda/2 (q^- - q^+), lambda = max |u^+- . n|
        applied to every conserved variable, rho E included; slip walls by
        the mirror state; face states from the traces of the nodal
        primitives. Written in total-energy form, without the split of the
        energy flux and its dissipation into advective and stiff parts."""
        E, Np = self.E, self.Np
        out = np.zeros((5, E, Np))
        P = self._nodal_prims(q, gamma)

        def flux_tensor(s):
            rho, m, Et = s[0], s[1:4], s[4]
            u = m / rho
            p = (gamma - 1) * (Et - 0.5 * rho * (u @ u))
            Fm = np.zeros((5, 3))
            Fm[0] = m
            Fm[1:4] = np.outer(m, u) + p * np.eye(3)
            Fm[4] = (Et + p) * u
            return Fm, u

        for e in range(E):
            V, G, WJ, _ = self.vol[e]
            for qp in range(V.shape[0]):
                s = np.array([V[qp] @ q[fd, e] for fd in range(5)])
                Fm, _ = flux_tensor(s)
                out[:, e] += WJ[qp] * (Fm @ G[qp].T)
            for pts in self.faces[e]:
                for (v, nb, vn, wq, area) in pts:
                    dS = np.linalg.norm(area)
                    nh = area / dS
                    sA = self._face_state(v, P, e, gamma)
                    if nb < 0:
                        sB = sA.copy()
                        sB[1:4] = sA[1:4] - 2 * (sA[1:4] @ nh) * nh
                    else:
                        sB = self._face_state(vn, P, nb, gamma)
                    FA, uA = flux_tensor(sA)
                    FB, uB = flux_tensor(sB)
                    lam = max(abs(uA @ nh), abs(uB @ nh))
                    Fn = 0.5 * (FA + FB) @ area + 0.5 * lam * (sA - sB) * dS
                    out[:, e] -= wq * Fn[:, None] * v[None, :]
        return out

    def lam_vector(self, c_dt, u_nodal, p_nodal, gamma):
        """c_dt int_dK lambda/2 ((rho e)^- - (rho e)^+) psi, lambda from u traces."""
        out = np.zeros((self.E, self.Np))
        for e in range(self.E):
            for pts in self.faces[e]:
                for (v, nb, vn, wq, area) in pts:
                    if nb < 0:
                        continue
                    dS = np.linalg.norm(area)
                    nh = area / dS
                    uA = np.array([v @ u_nodal[c, e] for c in range(3)])
                    uB = np.array([vn @ u_nodal[c, nb] for c in range(3)])
                    lam = max(abs(uA @ nh), abs(uB @ nh))
                    pA, pB = v @ p_nodal[e], vn @ p_nodal[nb]
                    out[e] += c_dt * wq * 0.5 * lam * (pA - pB) / (gamma - 1) * dS * v
        return out

    def mass_total(self, rho):
        return sum(np.sum(self.vol[e][2] * (self.vol[e][0] @ rho[e])) for e in range(self.E))
