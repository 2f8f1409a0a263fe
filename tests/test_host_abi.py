"""CPU tests of the C-ABI library: symbols, host mesh construction, errors.

The library's mesh and geometry are built by its own C++ code on the host;
they are compared here with the oracle's independent construction (element
order, node coordinates, mass-matrix diagonal), so the GPU parity tests can
feed both sides the same node-ordered inputs.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle.mesh import Mesh as OMesh, MeshDesc
from paper_2605_29598_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "imexdg.h")


def _binding():
    from paper_2605_29598_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libimexdg.so not built")
    return B


def test_all_declared_symbols_exported():
    B = _binding()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(imx_[a-z_]+)\s*\(", text))
    assert len(declared) >= 18
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(B.SIGNATURES), declared ^ set(B.SIGNATURES)


MESHES = [
    W.MeshSpec(4e3, 3e3, 2e3, 3, 2, 2, 2),
    W.MeshSpec(4e3, 3e3, 2e3, 2, 1, 2, 3, periodic_x=0, periodic_y=0),
    W.MeshSpec(8e3, 8e3, 4e3, 3, 3, 2, 3, terrain=W.GAUSS, h0=400, a=2e3, xc=4e3, yc=4e3),
    W.MeshSpec(8e3, 8e3, 4e3, 4, 4, 2, 2, terrain=W.BELL, h0=300, a=1.5e3, xc=4e3, yc=4e3,
               ref_boxes=[(2e3, 6e3, 2e3, 6e3, 0, 2e3), (3.5e3, 4.5e3, 3.5e3, 4.5e3, 0, 0.5e3)]),
    W.MeshSpec(4e3, 4e3, 2e3, 2, 2, 2, 4, ref_boxes=[(0, 1e3, 0, 1e3, 0, 0.5e3)]),
]


@pytest.mark.parametrize("spec", MESHES, ids=range(len(MESHES)))
def test_host_mesh_matches_oracle(spec):
    B = _binding()
    m = B.Mesh(spec)
    o = OMesh(MeshDesc(**vars(spec)))
    assert m.E == o.E and m.Np == o.Np
    assert m.deformed == (spec.terrain != W.FLAT)
    assert m.n_hanging == int((o.face_kind == 3).sum())
    xyz = m.node_coords()
    assert np.abs(xyz - o.node_coords()).max() < 1e-9 * max(spec.Lx, spec.Lz)
    wj = m.mass_diag()
    WJo = o.W3 * o.detJ
    assert np.abs(wj - WJo).max() < 1e-12 * WJo.max()


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_compact_terrain_metric_reproduces_the_mapped_geometry(degree):
    """Mesh creation forms the compact terrain metric of every terrain-following
    element (per element: J22 and the two slopes over phi on the element's plane,
    J22 on the side faces, phi per level) and fails unless its products reproduce
    the mapped W cof(J), W detJ and n dS to 1e-12 of their largest entry. Each
    creation below is that check, on a uniform mesh with walls, a refined mesh
    with two nested boxes and, at r = 4, the non-conforming hill of Sec. 4.3."""
    B = _binding()
    specs = [W.MeshSpec(8e3, 6e3, 4e3, 4, 3, 2, degree, terrain=W.GAUSS, h0=600, a=1.5e3, xc=3e3, yc=4e3,
                        periodic_x=0),
             W.MeshSpec(8e3, 8e3, 4e3, 4, 4, 2, degree, terrain=W.BELL, h0=400, a=1e3, xc=4e3, yc=4e3,
                        ref_boxes=[(2e3, 6e3, 2e3, 6e3, 0, 2e3), (3e3, 5e3, 3e3, 5e3, 0, 1e3)])]
    if degree == 4:
        specs.append(W.hill_benchmark(nonconforming=True).mesh)
    for spec in specs:
        m = B.Mesh(spec)
        assert m.deformed


def test_config_sizes():
    B = _binding()
    m = B.Mesh(W.orography(32, 32, 12, 4, refined=True).mesh)
    assert m.E == 14304 and m.Np == 125 and m.deformed
    m = B.Mesh(W.igw_channel().mesh)
    assert m.E == 48000 and m.Np == 64 and not m.deformed


def test_invalid_meshes_rejected():
    B = _binding()
    with pytest.raises(B.IMXError) as e:
        B.Mesh(W.MeshSpec(4e3, 4e3, 2e3, 2, 2, 2, 2,
                          ref_boxes=[(0, 1e3, 0, 1e3, 0, 0.5e3), (0, 0.5e3, 0, 0.5e3, 0, 0.2e3)]))
    assert e.value.code == B.IMX_EINVAL and "balanced" in str(e.value)
    with pytest.raises(B.IMXError):
        B.Mesh(W.MeshSpec(4e3, 4e3, 2e3, 2, 2, 2, 5))
    with pytest.raises(B.IMXError):
        B.Mesh(W.MeshSpec(4e3, 4e3, 2e3, 0, 2, 2, 2))


def test_lateral_sponge_widths_validated():
    """Negative lateral sponge widths and layers that would overlap across the
    domain are refused before any device call."""
    B = _binding()
    num = B.num_struct(W.NumSpec())
    m = B.Mesh(W.MeshSpec(4e3, 2e3, 2e3, 2, 2, 2, 2))
    for xw, yw in ((-1.0, 0.0), (0.0, -1.0), (2.1e3, 0.0), (0.0, 1.1e3)):
        ph = B.phys_struct(W.PhysSpec(sponge_lam=0.01, sponge_zB=1e3, sponge_zT=2e3, sponge_xw=xw, sponge_yw=yw))
        out = ctypes.c_void_p()
        code = B.lib().imx_solver_create(m.h, ctypes.byref(ph), ctypes.byref(num), None, ctypes.byref(out))
        assert code == B.IMX_EINVAL and b"sponge" in B.lib().imx_last_error(), (xw, yw)


def test_sponge_layer_validated():
    """A sponge with its top at or below its base, or with a negative or
    non-finite strength, is refused before any device call."""
    B = _binding()
    num = B.num_struct(W.NumSpec())
    m = B.Mesh(W.MeshSpec(4e3, 2e3, 2e3, 2, 2, 2, 2))
    for lam, zB, zT in ((0.01, 1e3, 1e3), (0.01, 2e3, 1e3), (-0.01, 1e3, 2e3), (math.inf, 1e3, 2e3),
                        (math.nan, 1e3, 2e3)):
        ph = B.phys_struct(W.PhysSpec(sponge_lam=lam, sponge_zB=zB, sponge_zT=zT))
        out = ctypes.c_void_p()
        code = B.lib().imx_solver_create(m.h, ctypes.byref(ph), ctypes.byref(num), None, ctypes.byref(out))
        assert code == B.IMX_EINVAL and b"sponge" in B.lib().imx_last_error(), (lam, zB, zT)


def test_slice_model_needs_a_slice_mesh():
    """The vertical-slice model is refused on a mesh with two elements in y
    (the check runs on the host before any device call)."""
    B = _binding()
    num = B.num_struct(W.NumSpec())
    for spec in (W.MeshSpec(4e3, 4e3, 2e3, 2, 2, 2, 2),
                 W.MeshSpec(4e3, 4e3, 2e3, 2, 1, 2, 2, periodic_y=0),
                 W.MeshSpec(8e3, 8e3, 4e3, 3, 1, 2, 2, terrain=W.GAUSS, h0=300, a=2e3, xc=4e3, yc=4e3)):
        m = B.Mesh(spec)
        ph = B.phys_struct(W.PhysSpec(slice=1))
        out = ctypes.c_void_p()
        code = B.lib().imx_solver_create(m.h, ctypes.byref(ph), ctypes.byref(num), None, ctypes.byref(out))
        assert code == B.IMX_EINVAL and b"slice" in B.lib().imx_last_error()


def test_transfer_plan_host_checks():
    """imx_transfer_workspace_bytes builds the leaf map on the host: sizes for
    refinements of one grid, refusal of different grids or of leaves more than
    two levels apart."""
    B = _binding()
    base = dict(Lx=4e3, Ly=4e3, Lz=2e3, nx=4, ny=4, nz=2, degree=2)
    a = B.Mesh(W.MeshSpec(**base))
    b = B.Mesh(W.MeshSpec(**base, ref_boxes=[(1e3, 3e3, 1e3, 3e3, 0.0, 1e3)]))
    n = ctypes.c_size_t()
    assert B.lib().imx_transfer_workspace_bytes(a.h, b.h, ctypes.byref(n)) == B.IMX_OK
    # leaf map, two W detJ arrays and the tables
    assert n.value >= 8 * (a.E + b.E) * a.Np
    other = B.Mesh(W.MeshSpec(**dict(base, nx=5)))
    assert B.lib().imx_transfer_workspace_bytes(a.h, other.h, ctypes.byref(n)) == B.IMX_EINVAL
    assert b"base grid" in B.lib().imx_last_error()
    deep = B.Mesh(W.MeshSpec(**base, ref_boxes=[(0.2e3, 3.8e3, 0.2e3, 3.8e3, 0.0, 1.8e3),
                                                 (1.1e3, 2.9e3, 1.1e3, 2.9e3, 0.0, 0.9e3),
                                                 (1.6e3, 2.4e3, 1.6e3, 2.4e3, 0.0, 0.3e3)]))
    assert B.lib().imx_transfer_workspace_bytes(a.h, deep.h, ctypes.byref(n)) == B.IMX_EINVAL
