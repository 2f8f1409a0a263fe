"""Pins of the oracle's geostrophic-imbalance measure (eq. egeo, Sec. 4.2,
planetary-scale test) against closed forms.

* p linear in x, constant rho, v linear in z with the sign change of
  (1/rho) dp/dx - f v at z = Lz/4 (an element boundary, so the Gauss rule
  integrates the piecewise linear integrand exactly): the mean of
  c |1 - 4 z/Lz| over the domain is 5c/4 (a wrong sign on f v gives 3c,
  multiplying by rho instead of dividing gives a different c).
* On a terrain-following mesh: p linear in x gives |b|/rho exactly, and p
  linear in z gives dp/dx = 0 (the inverse Jacobian must undo the terrain
  slope of the reference coordinates).
* A sinusoidal pressure: mean of |A k cos(k x)| / rho = 2 A k / (pi rho).
"""
import math

import numpy as np
import pytest

from oracle.diagnostics import geostrophic_imbalance, broken_x_derivative
from oracle.mesh import Mesh, MeshDesc
from paper_2605_29598_amd import workloads as W

F = 1.03126e-4


def _state(rho, u, p):
    return W.conserved_from_primitive(rho, u, p)


@pytest.mark.parametrize("r", [1, 3, 4])
def test_piecewise_linear_closed_form(r):
    Lx, Ly, Lz = 40e3, 10e3, 8e3
    mesh = Mesh(MeshDesc(Lx, Ly, Lz, 4, 1, 8, r))
    x, y, z = mesh.node_coords()
    rho0, c = 2.0, 3e-3
    b = c * rho0                             # (1/rho) dp/dx = c
    p = 1e5 + b * (x - Lx / 2)
    u = np.zeros((3,) + x.shape)
    u[1] = 4.0 * c * (z / Lz) / F            # f v = 4 c z / Lz
    q = _state(np.full_like(x, rho0), u, p)
    e = geostrophic_imbalance(mesh, q, F, W.GAMMA)
    assert abs(e - 1.25 * c) < 1e-12 * c, e


@pytest.mark.parametrize("r", [2, 4])
def test_terrain_following_mesh(r):
    d = MeshDesc(8e3, 8e3, 4e3, 3, 3, 2, r, terrain=W.GAUSS, h0=400.0, a=2e3, xc=4e3, yc=4e3)
    mesh = Mesh(d)
    x, y, z = mesh.node_coords()
    rho0, b = 1.5, 0.02
    u = np.zeros((3,) + x.shape)
    q = _state(np.full_like(x, rho0), u, 1e5 + b * x)
    assert abs(geostrophic_imbalance(mesh, q, F, W.GAMMA) - b / rho0) < 1e-12 * b / rho0
    # a pressure that varies with height only has no x derivative, although its
    # reference-coordinate derivatives along xi_0 do not vanish over the hill
    pz = 1e5 - b * z
    assert np.abs(broken_x_derivative(mesh, pz)).max() < 1e-10 * b
    assert np.abs(np.einsum('ekji,qi->ekjq', pz.reshape(mesh.E, r + 1, r + 1, r + 1),
                            mesh.basis.deriv)).max() > 1e-3 * b


def test_sinusoid_converges():
    Lx = 100e3
    mesh = Mesh(MeshDesc(Lx, 5e3, 5e3, 16, 1, 1, 4))
    x, y, z = mesh.node_coords()
    A, rho0 = 50.0, 1.2
    k = 2 * math.pi / Lx
    q = _state(np.full_like(x, rho0), np.zeros((3,) + x.shape), 1e5 + A * np.sin(k * x))
    exact = 2 * A * k / (math.pi * rho0)
    assert abs(geostrophic_imbalance(mesh, q, F, W.GAMMA) - exact) < 1e-5 * exact


# ----------------------------------------------------- vertical-slice projection
def test_slice_projection_closed_forms():
    """The projection onto y-constant fields (vertical-slice model, Sec. 2):
    a y-invariant field is unchanged up to rounding, the result is constant
    along every y-line of nodes, a field polynomial in y of degree <= r is
    replaced by its exact element mean in y, and the mass is unchanged."""
    from oracle import dg
    r = 4
    Lx, Ly, Lz = 30e3, 20e3, 10e3
    mesh = Mesh(MeshDesc(Lx, Ly, Lz, 3, 1, 2, r))
    x, y, z = mesh.node_coords()
    f0 = np.sin(x / 7e3) + z / Lz
    q = np.stack([f0] * 5)
    assert np.abs(dg.slice_project(mesh, q) - q).max() < 4e-16 * np.abs(q).max()
    g = dg.slice_project(mesh, q + np.sin(y / 3e3)).reshape(5, mesh.E, r + 1, r + 1, r + 1)
    assert (g == g[:, :, :, :1, :]).all()            # the same value on every y-line node
    t = y / Ly                                       # one element in y: t in (0, 1)
    fy = f0 * (1.0 + 3.0 * t ** 4 - 2.0 * t)         # degree 4 in y: mean factor 1 + 3/5 - 1
    got = dg.slice_project(mesh, fy[None])[0]
    assert np.abs(got - f0 * 0.6).max() < 1e-13 * np.abs(f0).max()
    # rho: mass unchanged
    rho = 1.0 + 0.3 * np.cos(2 * np.pi * t) * np.exp(-z / 5e3)
    qq = W.conserved_from_primitive(rho, np.zeros((3,) + x.shape), 1e5 + 0 * x)
    assert abs(dg.total_mass(mesh, dg.slice_project(mesh, qq)) - dg.total_mass(mesh, qq)) \
        < 1e-14 * dg.total_mass(mesh, qq)
