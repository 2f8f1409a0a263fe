"""Hexahedral box mesh with static nested 2:1 refinement and its geometry.

Sec. 3 discretises on a hexahedral mesh T_h; Sec. 4.3 deforms a box with the
Gal-Chen terrain-following map over a hill and refines it locally, leaving
hanging (non-conforming) faces at every level boundary.

Element order (shared convention of the whole project): base cells are
numbered with the vertical index fastest, b = bz + nz*(bx + nx*by); the leaves
of a refined base cell follow it depth first, children numbered
c = cz + 2*(cx + 2*cy). Node order inside an element: i + n*(j + n*k) with the
x index i fastest. Faces: f = 2*d + s for direction d (0 x, 1 y, 2 z) and side
s (0 lower, 1 upper). A face's (r+1)^2 points are numbered a + n*b with a, b
the indices along the two other directions in increasing order.

Refinement: box i (i = 0, 1, ...) refines every level-i leaf whose flat box
overlaps it with positive volume. Meshes that break 2:1 balance are rejected.
"""
from dataclasses import dataclass, field
import numpy as np

from .basis import Basis1D, lagrange_values, lagrange_derivatives

BOUNDARY, CONFORMING, FINE_SIDE, COARSE_SIDE = 0, 1, 2, 3
TERRAIN_FLAT, TERRAIN_BELL, TERRAIN_GAUSS = 0, 1, 2
TANGENTS = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


@dataclass
class MeshDesc:
    Lx: float
    Ly: float
    Lz: float
    nx: int
    ny: int
    nz: int
    degree: int
    periodic_x: int = 1
    periodic_y: int = 1
    terrain: int = TERRAIN_FLAT
    h0: float = 0.0
    a: float = 1.0
    xc: float = 0.0
    yc: float = 0.0
    ref_boxes: list = field(default_factory=list)   # [(x0,x1,y0,y1,z0,z1), ...]


def terrain_height(desc, x, y):
    """Surface height h(x, y): the bell of Sec. 4.3 or a Gaussian hill.

    In a periodic direction the distance to the hill centre is the minimum
    image distance, so the surface is continuous across the periodic seam.
    """
    dx = x - desc.xc
    dy = y - desc.yc
    if desc.periodic_x:
        dx = dx - desc.Lx * np.round(dx / desc.Lx)
    if desc.periodic_y:
        dy = dy - desc.Ly * np.round(dy / desc.Ly)
    r2 = (dx * dx + dy * dy) / (desc.a * desc.a)
    if desc.terrain == TERRAIN_BELL:
        return desc.h0 / (1.0 + r2)
    if desc.terrain == TERRAIN_GAUSS:
        return desc.h0 * np.exp(-r2)
    return np.zeros_like(x)


def galchen_z(desc, x, y, zeta):
    """Gal-Chen map of the flat height zeta in [0, H] over the surface h."""
    h = terrain_height(desc, x, y)
    return h + zeta * (desc.Lz - h) / desc.Lz


class Mesh:
    def __init__(self, desc: MeshDesc):
        self.desc = desc
        self.r = desc.degree
        self.n = n = desc.degree + 1
        self.Np = n ** 3
        self.Nf = n ** 2
        self.basis = Basis1D(desc.degree)
        self.h0 = np.array([desc.Lx / desc.nx, desc.Ly / desc.ny, desc.Lz / desc.nz])
        self.nbase = np.array([desc.nx, desc.ny, desc.nz])
        self.periodic = (bool(desc.periodic_x), bool(desc.periodic_y), False)
        self._build_leaves()
        self._build_faces()
        self._build_geometry()
        self._build_face_lists()

    # ------------------------------------------------------------------ leaves
    def _overlaps(self, base, level, sub, box):
        lo = (base + sub / 2.0 ** level) * self.h0
        hi = (base + (sub + 1) / 2.0 ** level) * self.h0
        blo = np.array(box[0::2], dtype=float)
        bhi = np.array(box[1::2], dtype=float)
        return bool(np.all(lo < bhi) and np.all(blo < hi))

    def _build_leaves(self):
        d = self.desc
        nref = len(d.ref_boxes)
        bases, levels, subs = [], [], []

        def visit(base, level, sub):
            if level < nref and self._overlaps(base, level, sub, d.ref_boxes[level]):
                for cy in range(2):
                    for cx in range(2):
                        for cz in range(2):
                            visit(base, level + 1, 2 * sub + np.array([cx, cy, cz]))
            else:
                bases.append(base.copy())
                levels.append(level)
                subs.append(sub.copy())

        for by in range(d.ny):
            for bx in range(d.nx):
                for bz in range(d.nz):
                    visit(np.array([bx, by, bz]), 0, np.zeros(3, dtype=int))
        self.elem_base = np.array(bases, dtype=np.int64)
        self.elem_level = np.array(levels, dtype=np.int64)
        self.elem_sub = np.array(subs, dtype=np.int64)
        self.E = len(levels)
        self.Lmax = int(self.elem_level.max()) if self.E else 0
        # origin and size of every leaf in units of the finest level
        scale = 2 ** self.Lmax
        self.size = (2 ** (self.Lmax - self.elem_level)).astype(np.int64)
        self.origin = self.elem_base * scale + self.elem_sub * self.size[:, None]
        self.nfine = self.nbase * scale
        owner = -np.ones(tuple(self.nfine), dtype=np.int64)
        for e in range(self.E):
            o, s = self.origin[e], self.size[e]
            owner[o[0]:o[0] + s, o[1]:o[1] + s, o[2]:o[2] + s] = e
        assert (owner >= 0).all()
        self.owner = owner

    def _lookup(self, P):
        return self.owner[P[0], P[1], P[2]]

    # ------------------------------------------------------------------- faces
    def _build_faces(self):
        E = self.E
        kind = np.zeros((E, 6), dtype=np.int64)
        nbr = -np.ones((E, 6, 4), dtype=np.int64)
        sub = -np.ones((E, 6), dtype=np.int64)
        for e in range(E):
            o, s, L = self.origin[e], self.size[e], self.elem_level[e]
            for d in range(3):
                t1, t2 = TANGENTS[d]
                for side in range(2):
                    f = 2 * d + side
                    P = o.copy()
                    P[d] = o[d] + s if side == 1 else o[d] - 1
                    if P[d] < 0 or P[d] >= self.nfine[d]:
                        if d < 2 and self.periodic[d]:
                            P[d] %= self.nfine[d]
                        else:
                            kind[e, f] = BOUNDARY
                            continue
                    nb = self._lookup(P)
                    Lnb = self.elem_level[nb]
                    if Lnb == L:
                        kind[e, f] = CONFORMING
                        nbr[e, f, 0] = nb
                    elif Lnb == L - 1:
                        kind[e, f] = FINE_SIDE
                        nbr[e, f, 0] = nb
                        h1 = (o[t1] - self.origin[nb][t1]) // s
                        h2 = (o[t2] - self.origin[nb][t2]) // s
                        sub[e, f] = h1 + 2 * h2
                    elif Lnb == L + 1:
                        kind[e, f] = COARSE_SIDE
                        for h2 in range(2):
                            for h1 in range(2):
                                Q = P.copy()
                                Q[t1] = o[t1] + h1 * (s // 2)
                                Q[t2] = o[t2] + h2 * (s // 2)
                                nq = self._lookup(Q)
                                if self.elem_level[nq] != L + 1:
                                    raise ValueError("mesh is not 2:1 balanced")
                                nbr[e, f, h1 + 2 * h2] = nq
                    else:
                        raise ValueError("mesh is not 2:1 balanced")
        self.face_kind, self.face_nbr, self.face_sub = kind, nbr, sub

    # ---------------------------------------------------------------- geometry
    def _map(self, e_idx, xi):
        """Physical points and Jacobians of elements e_idx at reference points xi.

        xi: (P, 3) reference points in [0,1]^3. Returns X (E', P, 3) and
        J (E', P, 3, 3) with J[..., c, d] = dx_c / dxi_d.
        """
        d = self.desc
        lev = self.elem_level[e_idx].astype(float)
        scale = 2.0 ** (-lev)                                   # (E',)
        base = self.elem_base[e_idx].astype(float)
        subc = self.elem_sub[e_idx].astype(float)
        # base-cell local coordinates eta in [0,1]^3
        eta = (subc[:, None, :] + xi[None, :, :]) * scale[:, None, None]
        flat = (base[:, None, :] + eta) * self.h0[None, None, :]
        Ep, P = eta.shape[0], eta.shape[1]
        X = np.empty((Ep, P, 3))
        J = np.zeros((Ep, P, 3, 3))
        X[..., 0] = flat[..., 0]
        X[..., 1] = flat[..., 1]
        J[..., 0, 0] = self.h0[0] * scale[:, None]
        J[..., 1, 1] = self.h0[1] * scale[:, None]
        if d.terrain == TERRAIN_FLAT:
            X[..., 2] = flat[..., 2]
            J[..., 2, 2] = self.h0[2] * scale[:, None]
            return X, J
        # isoparametric: degree-r interpolant of the Gal-Chen height at the
        # Gauss-Lobatto points of the base cell, restricted to the leaf
        g = self.basis.gll
        n = self.n
        gx = (base[:, 0, None] + g[None, :]) * self.h0[0]      # (E', n)
        gy = (base[:, 1, None] + g[None, :]) * self.h0[1]
        gz = (base[:, 2, None] + g[None, :]) * self.h0[2]
        zg = galchen_z(d, gx[:, :, None, None], gy[:, None, :, None], gz[:, None, None, :])  # [e,a,b,c]
        Lv = [lagrange_values(g, eta[..., c].ravel()).reshape(Ep, P, n) for c in range(3)]
        Ld = [lagrange_derivatives(g, eta[..., c].ravel()).reshape(Ep, P, n) for c in range(3)]
        X[..., 2] = np.einsum('eabc,epa,epb,epc->ep', zg, Lv[0], Lv[1], Lv[2])
        J[..., 2, 0] = np.einsum('eabc,epa,epb,epc->ep', zg, Ld[0], Lv[1], Lv[2]) * scale[:, None]
        J[..., 2, 1] = np.einsum('eabc,epa,epb,epc->ep', zg, Lv[0], Ld[1], Lv[2]) * scale[:, None]
        J[..., 2, 2] = np.einsum('eabc,epa,epb,epc->ep', zg, Lv[0], Lv[1], Ld[2]) * scale[:, None]
        return X, J

    def _chunks(self, chunk=2048):
        for s in range(0, self.E, chunk):
            yield np.arange(s, min(s + chunk, self.E))

    def volume_points(self):
        x = self.basis.x
        n = self.n
        k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing='ij')
        return np.stack([x[i.ravel()], x[j.ravel()], x[k.ravel()]], axis=1)

    def face_points(self, d, side, sub=None):
        """Reference points (in the element) of the GL points of face (d, side).

        With sub = (h1, h2) the points are those of that quarter of the face.
        """
        x = self.basis.x
        n = self.n
        b, a = np.meshgrid(np.arange(n), np.arange(n), indexing='ij')
        ta, tb = x[a.ravel()], x[b.ravel()]
        if sub is not None:
            ta = 0.5 * (sub[0] + ta)
            tb = 0.5 * (sub[1] + tb)
        pts = np.empty((n * n, 3))
        t1, t2 = TANGENTS[d]
        pts[:, d] = float(side)
        pts[:, t1] = ta
        pts[:, t2] = tb
        return pts

    def _build_geometry(self):
        n, Np, Nf = self.n, self.Np, self.Nf
        w = self.basis.w
        k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing='ij')
        self.W3 = (w[i] * w[j] * w[k]).ravel()                # tensor GL weights
        b, a = np.meshgrid(np.arange(n), np.arange(n), indexing='ij')
        self.W2 = (w[a] * w[b]).ravel()
        self.xq = np.empty((self.E, Np, 3))
        self.detJ = np.empty((self.E, Np))
        self.Jinv = np.empty((self.E, Np, 3, 3))                # [d][c] = dxi_d/dx_c
        self.nS = np.empty((self.E, 6, Nf, 3))                  # outward area vector / ref. area
        vp = self.volume_points()
        for idx in self._chunks():
            X, J = self._map(idx, vp)
            self.xq[idx] = X
            self.detJ[idx] = np.linalg.det(J)
            self.Jinv[idx] = np.linalg.inv(J)
            for d in range(3):
                for side in range(2):
                    _, Jf = self._map(idx, self.face_points(d, side))
                    cof = np.linalg.det(Jf)[..., None, None] * np.linalg.inv(Jf)   # detJ J^-1
                    sign = 1.0 if side == 1 else -1.0
                    self.nS[idx, 2 * d + side] = sign * cof[..., d, :]
        if (self.detJ <= 0).any():
            raise ValueError("inverted element")

    # ------------------------------------------------------------ face groups
    def _build_face_lists(self):
        """Unique face entities, grouped so each group can be processed at once.

        conforming: side A is the element whose upper face (d, 1) it is.
        hanging: one entity per fine subface; side A is the fine element and the
                 area vector is the fine element's.
        boundary: one-sided wall faces.
        """
        self.conf = []       # (d, A[], B[])
        self.hang = []       # (d, sA, sub, A[], B[])  A fine, B coarse
        self.wall = []       # (d, s, A[])
        kind, nbr, sub = self.face_kind, self.face_nbr, self.face_sub
        for d in range(3):
            A = np.nonzero(kind[:, 2 * d + 1] == CONFORMING)[0]
            self.conf.append((d, A, nbr[A, 2 * d + 1, 0]))
            for s in range(2):
                f = 2 * d + s
                Wl = np.nonzero(kind[:, f] == BOUNDARY)[0]
                if len(Wl):
                    self.wall.append((d, s, Wl))
                for sb in range(4):
                    A = np.nonzero((kind[:, f] == FINE_SIDE) & (sub[:, f] == sb))[0]
                    if len(A):
                        self.hang.append((d, s, sb, A, nbr[A, f, 0]))

    # ------------------------------------------------------------- utilities
    def node_coords(self):
        """[3][E][Np] physical coordinates of the nodes (the GL points)."""
        return np.ascontiguousarray(self.xq.transpose(2, 0, 1))

    def mass_weights(self):
        """Diagonal of the (collocated) mass matrix: W_q detJ_q."""
        return self.W3[None, :] * self.detJ
