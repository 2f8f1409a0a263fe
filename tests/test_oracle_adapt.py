"""Pins of the oracle's solution transfer (dynamic adaptivity).

Closed forms: a field that is one polynomial of degree <= r in each
coordinate over the whole box lies in the DG space of every refinement of an
affine mesh, so refinement (evaluation) and coarsening (L2 projection) must
both reproduce it exactly at the new nodes, evaluated here from the formula.
Invariants: the integral of every field is kept by both directions, on flat
and terrain-following meshes; coarsening undoes refinement on affine meshes.
"""
import numpy as np
import pytest

from oracle import adapt
from oracle.mesh import Mesh, MeshDesc

L = 4e3
ONE = [(1e3, 3e3, 1e3, 3e3, 0.0, 1e3)]
TWO = [(0.5e3, 3.5e3, 0.5e3, 2.5e3, 0.0, 1.5e3), (1.2e3, 2.2e3, 1.1e3, 1.9e3, 0.0, 0.6e3)]
MOVED = [(2e3, 4e3, 0.0, 2e3, 0.5e3, 2e3)]


def _mesh(r, boxes, terrain=0):
    return Mesh(MeshDesc(L, L, 2e3, 4, 4, 2, r, terrain=terrain, h0=250.0, a=1.2e3, xc=2e3, yc=2e3,
                         ref_boxes=list(boxes)))


def _poly(xyz, r):
    x, y, z = xyz[0] / L, xyz[1] / L, xyz[2] / 2e3
    return np.stack([1.0 + x ** r - 0.5 * y * z,
                     x * y ** (r - 1) + z ** r,
                     0.3 + (x - 0.2) * (y + 0.1) * (z - 0.7),
                     x ** r * y ** r * z ** r,
                     2.0 - y ** r + x * z])


@pytest.mark.parametrize("r", [1, 2, 3])
@pytest.mark.parametrize("a,b", [((), ONE), ((), TWO), (ONE, TWO), (ONE, MOVED), (TWO, MOVED)])
def test_polynomials_transfer_exactly(r, a, b):
    ma, mb = _mesh(r, a), _mesh(r, b)
    for src, dst in ((ma, mb), (mb, ma)):
        q = _poly(src.node_coords(), r)
        got = adapt.transfer(src, dst, q)
        ref = _poly(dst.node_coords(), r)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), (r, len(src.desc.ref_boxes))


@pytest.mark.parametrize("terrain", [0, 2])
@pytest.mark.parametrize("a,b", [((), TWO), (ONE, MOVED), (TWO, MOVED)])
def test_integrals_are_kept(terrain, a, b):
    ma, mb = _mesh(3, a, terrain), _mesh(3, b, terrain)
    rng = np.random.default_rng(7)
    for src, dst in ((ma, mb), (mb, ma)):
        q = 1.0 + rng.uniform(-0.5, 0.5, (5, src.E, src.Np))
        got = adapt.transfer(src, dst, q)
        I0 = (src.W3 * src.detJ * q).sum(axis=(1, 2))
        I1 = (dst.W3 * dst.detJ * got).sum(axis=(1, 2))
        assert np.abs(I1 - I0).max() < 1e-13 * np.abs(I0).max(), (I0, I1)


def test_coarsening_undoes_refinement():
    coarse, fine = _mesh(3, ()), _mesh(3, TWO)
    q = np.random.default_rng(3).uniform(-1, 1, (5, coarse.E, coarse.Np))
    back = adapt.transfer(fine, coarse, adapt.transfer(coarse, fine, q))
    assert np.abs(back - q).max() < 1e-13


def test_unchanged_leaves_are_copied():
    ma, mb = _mesh(2, ONE), _mesh(2, MOVED)
    q = np.random.default_rng(1).uniform(-1, 1, (2, ma.E, ma.Np))
    got = adapt.transfer(ma, mb, q)
    ka = {adapt._key(ma, e): e for e in range(ma.E)}
    same = 0
    for t in range(mb.E):
        e = ka.get(adapt._key(mb, t))
        if e is not None:
            assert np.array_equal(got[:, t], q[:, e])
            same += 1
    assert 0 < same < mb.E
