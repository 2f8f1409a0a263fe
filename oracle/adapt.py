"""Solution transfer between two refinements of one base grid (test
infrastructure: the plain reference for dynamic adaptivity).

The paper refines statically (Sec. 4.3, nested 2:1 refinement regions around
the hill). Dynamic adaptivity changes the refinement during a run: leaves are
split (refinement) or merged (coarsening), and the discrete solution moves
with them. The transfer written here follows from the DG space of Sec. 3:

* a leaf that exists in both meshes keeps its nodal values;
* a new leaf inside an old, coarser leaf (refinement, one or two levels)
  takes the old leaf's polynomial evaluated at its own nodes: the old
  solution restricted to the new leaf is a polynomial of the same degree, so
  this is exact;
* a new leaf that covers old, finer leaves (coarsening) takes the L2
  projection of the old solution onto its polynomial space, with the
  mass-matrix quadrature of Sec. 3 (the Gauss-Legendre rule at the nodes,
  weights W detJ): for each new node i,
      c_i = (sum over old leaves K' inside, over their nodes q,
             W detJ(q) u(q) l_i(x_q)) / (W detJ(i))
  with l_i the new leaf's Lagrange polynomial at the old node x_q.

Both directions keep the integral of every conserved field (the
Gauss-Legendre rule is exact for l_i times det J, degree <= 2r), and a
coarsening undoes a refinement on affine elements.
Fields are arrays (..., E, Np) in the node order of oracle.mesh.
"""
import numpy as np

from .basis import lagrange_values
from .mesh import Mesh


def _key(mesh, e):
    return (tuple(int(v) for v in mesh.elem_base[e]), int(mesh.elem_level[e]),
            tuple(int(v) for v in mesh.elem_sub[e]))


def _eval(u, n, px, py, pz, x):
    """Values of the nodal fields u (..., Np) of one element at the tensor
    points (px_i, py_j, pz_k) of its reference cube."""
    Lx, Ly, Lz = lagrange_values(x, px), lagrange_values(x, py), lagrange_values(x, pz)
    g = u.reshape(u.shape[:-1] + (n, n, n))                      # [..., c, b, a] = z, y, x
    v = np.einsum('...cba,ia,jb,kc->...kji', g, Lx, Ly, Lz)
    return v.reshape(u.shape)


def transfer(src: Mesh, dst: Mesh, q):
    """Fields q (..., src.E, Np) on `src` transferred onto `dst`; both meshes
    share the box, the base grid, the degree and the terrain."""
    assert src.n == dst.n and np.array_equal(src.nbase, dst.nbase)
    n, x = src.n, src.basis.x
    index = {_key(src, e): e for e in range(src.E)}
    by_base = {}
    for e in range(src.E):
        by_base.setdefault(tuple(int(v) for v in src.elem_base[e]), []).append(e)
    Msrc = src.W3 * src.detJ
    Mdst = dst.W3 * dst.detJ
    out = np.zeros(q.shape[:-2] + (dst.E, dst.Np))
    for t in range(dst.E):
        base, lt, st = _key(dst, t)
        st = np.array(st)
        done = False
        # the same leaf, or an old leaf that contains it (refinement)
        for lf in range(lt, -1, -1):
            d = lt - lf
            sf = st >> d
            e = index.get((base, lf, tuple(int(v) for v in sf)))
            if e is None:
                continue
            pos = st - (sf << d)
            px, py, pz = ((pos[c] + x) / 2.0 ** d for c in range(3))
            out[..., t, :] = q[..., e, :] if d == 0 else _eval(q[..., e, :], n, px, py, pz, x)
            done = True
            break
        if done:
            continue
        # old leaves inside it (coarsening): L2 projection
        acc = np.zeros(q.shape[:-2] + (dst.Np,))
        for e in by_base.get(base, []):
            lf = int(src.elem_level[e])
            if lf <= lt:
                continue
            m = lf - lt
            sf = np.array(src.elem_sub[e])
            if not np.array_equal(sf >> m, st):
                continue
            pos = sf - (st << m)
            # the new leaf's Lagrange polynomials at the old leaf's nodes
            Lx, Ly, Lz = (lagrange_values(x, (pos[c] + x) / 2.0 ** m) for c in range(3))
            g = (Msrc[e] * q[..., e, :]).reshape(q.shape[:-2] + (n, n, n))
            acc += np.einsum('...cba,ai,bj,ck->...kji', g, Lx, Ly, Lz).reshape(acc.shape)
        out[..., t, :] = acc / Mdst[t]
    return out
