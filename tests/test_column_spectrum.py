"""The resting stratified column: the linearised operator and long steps.

About a resting, stratified, wall-bounded column the semi-discrete operator
M^{-1}(T_NS + T_S) has a few eigenvalues with a small positive real part:
the scheme is centred at rest (lambda = |u.n| vanishes) and the discrete rest
state is not exactly balanced. The column variant of
tests/bruteforce/column.py integrates the same weak forms on Q points per
direction; with Q = r + 1 it reproduces the oracle's residual. On 2 km
elements at r = 2 the largest real part is 3.6e-5 1/s (an e-folding time of
about 7.6 h), and over-integration (Q = r + 3) changes it by about 13 %: it is
not an aliasing effect of the collocated quadrature.

With face values taken from traces of the conserved variables instead of
(rho, u, p) the same column has 1.2e-4 1/s, and the ARK2 step, whose stage
operators then differ from the T_S of its final update, grows a perturbation
of the resting column tenfold every few minutes at dt = 8 s. The last test
runs the oracle's ARK2 steps on the column of the Sec. 4.3 benchmark (16 km,
2 km elements, r = 4) at that dt and requires the rest state to stay at rest.
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


def test_rest_column_spectrum_is_nearly_neutral():
    r, nz, h = 2, 4, 2e3
    collocated = _spectrum(r, r + 1, nz, h).real.max()
    over = _spectrum(r, r + 3, nz, h).real.max()
    # e-folding times above 5 h on 2 km elements at r = 2, either way
    assert 0 < collocated < 5e-5 and 0 < over < 5e-5, (collocated, over)
    assert abs(over - collocated) < 0.2 * collocated, (collocated, over)


def test_rest_column_stays_at_rest_at_dt_8():
    om = Mesh(MeshDesc(4e3, 4e3, 16e3, 1, 1, 8, 4))
    w = W.hill_benchmark(rotating=False)
    w.U = 0.0
    q = W.initial_state(w, om.node_coords())
    num = dg.Numerics(dt=8.0)
    wmax = []
    for _ in range(100):
        q, _ = dg.ark2_step(om, dg.Phys(), num, q)
        wmax.append(np.abs(q[3] / q[0]).max())
    # the discrete imbalance of the analytic rest state drives w of a few
    # 1e-6 m/s at once; it must not grow (face values from conserved traces:
    # 1.8e-4 m/s after these 800 s and rising)
    assert max(wmax) < 2e-5, max(wmax)
    assert max(wmax[50:]) < 5 * max(wmax[:50]), (max(wmax[:50]), max(wmax[50:]))
