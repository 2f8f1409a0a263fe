"""1D building blocks of the tensor-product nodal DG space (Sec. 3).

The discrete solution on each hexahedron is a Q_r polynomial written in the
Lagrange basis of its values at the (r+1)^3 tensor Gauss-Legendre points
(Sec. 3, nodal formulation). Integrals use the same (r+1)-point Gauss-Legendre
rule in each direction, so the nodal-to-quadrature interpolation matrix S of
Sec. 3.1 is the identity and the element mass matrices are diagonal.

The geometry of deformed elements is the degree-r interpolant of the mesh
map at the Gauss-Lobatto points of the element (isoparametric map); those
points include the element faces, so two elements that share a face agree on
it.

All reference coordinates are on [0, 1].
"""
import numpy as np


def gauss_legendre(n):
    """n-point Gauss-Legendre points and weights on [0, 1] (exact to degree 2n-1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto(n):
    """n-point Gauss-Lobatto points on [0, 1]: the endpoints and the roots of P'_{n-1}."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs at least 2 points")
    inner = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots()
    x = np.concatenate(([-1.0], np.sort(inner.real), [1.0]))
    return 0.5 * (x + 1.0)


def lagrange_values(nodes, x):
    """L[k, i] = l_i(x_k), the Lagrange polynomials of `nodes` evaluated at points x."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(x), n))
    for i in range(n):
        for m in range(n):
            if m != i:
                L[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return L


def lagrange_derivatives(nodes, x):
    """D[k, i] = l_i'(x_k), by the product rule applied to the Lagrange product."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for l in range(n):
                if l != i and l != m:
                    term *= (x - nodes[l]) / (nodes[i] - nodes[l])
            D[:, i] += term
    return D


class Basis1D:
    """Tables for degree r: GL nodes/weights, derivative matrix, face values.

    deriv[q, i]  = l_i'(xi_q)           (derivative of node basis at GL points)
    face[s, i]   = l_i(s), s in {0, 1}   (trace of the node basis on each face)
    half[h, a, i] = l_i((h + xi_a) / 2)  (node basis at the GL points of half h,
                                          used for hanging subfaces)
    """

    def __init__(self, r):
        self.r = r
        self.n = r + 1
        self.x, self.w = gauss_legendre(self.n)
        self.deriv = lagrange_derivatives(self.x, self.x)
        self.face = lagrange_values(self.x, np.array([0.0, 1.0]))
        self.half = np.stack([lagrange_values(self.x, 0.5 * (h + self.x)) for h in (0, 1)])
        self.gll = gauss_lobatto(self.n)
