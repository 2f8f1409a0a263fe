"""CPU checks of the slice runner's host-side sampling: a state whose w and
p' are polynomials of degree <= r in x and z is sampled exactly at arbitrary
points (the element lookup, the reference coordinates and the Lagrange
evaluation of the runner's own code)."""
import numpy as np

from oracle.mesh import Mesh, MeshDesc
from paper_2605_29598_amd import experiments as X
from paper_2605_29598_amd import workloads as W


def test_sample_slice_reproduces_polynomials():
    w = W.igw_slice(nx=6, nz=10)
    spec = w.mesh
    mesh = Mesh(MeshDesc(**vars(spec)))
    coords = mesh.node_coords()
    x, y, z = coords
    s, t = x / spec.Lx, z / spec.Lz
    wv = 0.01 * (1 + 2 * s - 3 * t * t + s * t)                # degree 2 in x and z
    delta = W.GRAV / (W.RGAS * 250.0)
    pp = 5.0 * (s - 0.5) * t ** 3                               # p' of degree 3
    p = W.P_REF * np.exp(-delta * z) + pp
    rho = 1.0 + 0.1 * s
    u = np.zeros((3,) + x.shape)
    u[2] = wv
    q = W.conserved_from_primitive(rho, u, p)
    rng = np.random.default_rng(3)
    XS, ZS = rng.uniform(0, spec.Lx, 500), rng.uniform(0, spec.Lz, 500)
    gw, gp = X.sample_slice(q, coords, spec, spec.degree + 1, W.GAMMA, XS, ZS)
    sx, tz = XS / spec.Lx, ZS / spec.Lz
    assert np.abs(gw - 0.01 * (1 + 2 * sx - 3 * tz * tz + sx * tz)).max() < 1e-12
    assert np.abs(gp - 5.0 * (sx - 0.5) * tz ** 3).max() < 1e-9     # p' ~ 1: Pa-scale cancellation of 1e5
