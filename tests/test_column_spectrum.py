"""The growing grid-scale mode of the resting stratified column is not an
aliasing effect.

About a resting, stratified, wall-bounded column the semi-discrete operator
M^{-1}(T_NS + T_S) of the scheme as read has eigenvalues with a positive real
part (the mode that makes long runs over stratified rest states grow). A
plausible cause would be the collocated (r+1)-point quadrature of the
nonlinear and variable-coefficient products. The column variant of
tests/bruteforce/column.py integrates the same weak forms on Q points per
direction; with Q = r + 1 it reproduces the oracle's residual, and with
Q = r + 3 the largest real part is unchanged to 0.5 %: over-integration does
not remove the mode.
"""
import numpy as np

from oracle import dg
from oracle.mesh import Mesh, MeshDesc
from paper_2605_29598_amd import workloads as W
from tests.bruteforce.column import Column


def _spectrum(r, Q, nz, h):
    om = Mesh(MeshDesc(h, h, h * nz, 1, 1, nz, r))
    w = W.orography()
    x, y, z = om.node_coords()
    rho, p = W.primitive_background(w, x, y, z)              # N = 0.01, theta_ref = 293.15 K
    q0 = W.conserved_from_primitive(rho, np.zeros((3,) + rho.shape), p)
    col = Column(r + 1, Q, (h, h, h), nz, grav=9.81)
    flat = q0.reshape(-1)
    scale = np.abs(q0).reshape(5, -1).max(1)
    per = q0.size // 5
    J = np.zeros((flat.size, flat.size))
    for k in range(flat.size):
        fld = k // per
        eps = 1e-7 * (scale[fld] if fld in (0, 4) else scale[0])
        qp, qm = flat.copy(), flat.copy()
        qp[k] += eps
        qm[k] -= eps
        J[:, k] = (col.rhs(qp.reshape(q0.shape)) - col.rhs(qm.reshape(q0.shape))).reshape(-1) / (2 * eps)
    return np.linalg.eigvals(J)


def test_column_variant_reproduces_the_oracle():
    r, nz, h = 3, 3, 2e3
    om = Mesh(MeshDesc(h, h, h * nz, 1, 1, nz, r))
    q = W.random_positive_state((om.E, om.Np), 3)
    TNS, TS = dg.explicit_residual(om, dg.Phys(f=1e-4, g=9.81), q)
    a, b = Column(r + 1, r + 1, (h, h, h), nz, grav=9.81, fcor=1e-4).residual(q)
    assert np.abs(a - TNS).max() < 1e-13 * np.abs(TNS).max()
    assert np.abs(b[1:] - TS[1:]).max() < 1e-13 * np.abs(TS[1:]).max()


def test_growing_mode_survives_over_integration():
    r, nz, h = 2, 4, 2e3
    collocated = _spectrum(r, r + 1, nz, h).real.max()
    over = _spectrum(r, r + 3, nz, h).real.max()
    # an e-folding time of about 2.3 h on 2 km elements at r = 2, either way
    assert collocated > 5e-5 and over > 5e-5, (collocated, over)
    assert abs(over - collocated) < 0.01 * collocated, (collocated, over)
