"""Diagnostics of Sec. 4: effective resolution, Courant numbers, error norms,
and the geostrophic-imbalance measure of the planetary-scale wave test.

H = min diam(K); C = r c dt sqrt(d) / H and C_adv = r U dt sqrt(d) / H; discrete
l2 / l_inf errors over sample points and the experimental order of
convergence EOC = log(e2/e1) / log(h2/h1).

Test infrastructure: imported only by the tests, the smoke check and the
CPU baseline of the benchmark.
"""
import math
import numpy as np


def courant(r, speed, dt, H, d):
    return r * speed * dt * math.sqrt(d) / H


def box_diameter(*h):
    return math.sqrt(sum(x * x for x in h))


def l2_error(a, b):
    return float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)))


def linf_error(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def eoc(e1, e2, h1, h2):
    return math.log(e2 / e1) / math.log(h2 / h1)


def dofs_per_scalar(n_cells, r, d=3):
    return n_cells * (r + 1) ** d


def broken_x_derivative(mesh, f):
    """d f / d x of the element-local Q_r polynomial of a nodal field f (E, Np)
    at the element's own nodes (no face terms): the reference derivatives
    d f / d xi_d = sum_i l_i'(xi_q) f_i along each direction, combined with the
    inverse Jacobian, d f / d x = sum_d (d xi_d / d x) d f / d xi_d."""
    n = mesh.n
    D = mesh.basis.deriv                       # D[q, i] = l_i'(xi_q)
    g = f.reshape(f.shape[:-1] + (n, n, n))    # [e][k][j][i]
    dxi = [np.einsum('ekji,qi->ekjq', g, D).reshape(f.shape),
           np.einsum('ekji,qj->ekqi', g, D).reshape(f.shape),
           np.einsum('ekji,qk->eqji', g, D).reshape(f.shape)]
    return sum(mesh.Jinv[:, :, d, 0] * dxi[d] for d in range(3))


def geostrophic_imbalance(mesh, q, f_cor, gamma):
    """Departure from geostrophic balance of the x momentum (eq. egeo,
    Sec. 4.2, planetary-scale test): the domain mean of |(1/rho) dp/dx - f v|,
    int |.| dV / int dV with the Gauss-Legendre rule of the elements. On a
    vertical slice (one element in y) this is the paper's area mean over
    x and z; dp/dx is the element-local derivative of the discrete pressure."""
    rho = q[0]
    v = q[2] / rho
    kin = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / rho
    p = (gamma - 1.0) * (q[4] - kin)
    WJ = mesh.W3 * mesh.detJ
    val = np.abs(broken_x_derivative(mesh, p) / rho - f_cor * v)
    return float((WJ * val).sum() / WJ.sum())
