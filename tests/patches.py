"""Patches of base-cell columns cut out of a large mesh, for sampled parity.

An operator value on an element depends only on elements within a small face
distance, so the oracle can evaluate it on a patch of (2R+1)^2 base-cell
columns (same cells, same refinement, same terrain) built as a mesh of its
own, with its own walls at the patch edge. Elements of the patch are matched
to the large mesh by centroid.
"""
import numpy as np
from scipy.spatial import cKDTree

from oracle.mesh import Mesh as OMesh, MeshDesc

R = 2   # patch half-width in base cells


def columns(om, lo, hi):
    """Elements of a patch whose base cell column lies in [lo, hi]^2."""
    b = om.elem_base
    return np.nonzero((b[:, 0] >= lo) & (b[:, 0] <= hi) & (b[:, 1] >= lo) & (b[:, 1] <= hi))[0]


def patch_for(ms, xyz_full, cen_full, centre, r=R):
    """Oracle mesh of the columns around base cell `centre` of mesh spec `ms`
    and the index in the large mesh of each of its elements. xyz_full are the
    large mesh's node coordinates [3][E][Np], cen_full its element centroids."""
    dx, dy = ms.Lx / ms.nx, ms.Ly / ms.ny
    x0, y0 = (centre[0] - r) * dx, (centre[1] - r) * dy
    n = 2 * r + 1
    # candidate elements of the large mesh: those in the patch columns
    bx = np.floor(np.mod(cen_full[0], ms.Lx) / dx).astype(int)
    by = np.floor(np.mod(cen_full[1], ms.Ly) / dy).astype(int)
    sel = np.nonzero((np.mod(bx - centre[0] + r, ms.nx) <= 2 * r) & (np.mod(by - centre[1] + r, ms.ny) <= 2 * r))[0]
    boxes = [(b[0] - x0, b[1] - x0, b[2] - y0, b[3] - y0, b[4], b[5]) for b in ms.ref_boxes]
    # the hill image nearest to the patch (the large mesh measures the distance
    # to the hill by minimum image in its periodic directions)
    xc = ms.xc + (ms.Lx * np.round((x0 + n * dx / 2 - ms.xc) / ms.Lx) if ms.periodic_x else 0.0)
    yc = ms.yc + (ms.Ly * np.round((y0 + n * dy / 2 - ms.yc) / ms.Ly) if ms.periodic_y else 0.0)
    pd = MeshDesc(n * dx, n * dy, ms.Lz, n, n, ms.nz, ms.degree, 0, 0, ms.terrain, ms.h0, ms.a,
                  xc - x0, yc - y0, boxes)
    om = OMesh(pd)
    px = om.node_coords()
    cen = px.mean(axis=2)
    full_c = np.stack([np.mod(cen_full[0, sel], ms.Lx), np.mod(cen_full[1, sel], ms.Ly), cen_full[2, sel]], 1)
    mine = np.stack([np.mod(cen[0] + x0, ms.Lx), np.mod(cen[1] + y0, ms.Ly), cen[2]], 1)
    dist, j = cKDTree(full_c).query(mine)
    assert dist.max() < 1e-3, dist.max()
    idx = sel[j]
    assert len(np.unique(idx)) == om.E
    # same geometry: node coordinates agree after the shift (modulo the periods)
    fx = xyz_full[:, idx]
    per = lambda d, L: np.abs(np.mod(d + L / 2, L) - L / 2).max()
    assert per(px[0] + x0 - fx[0], ms.Lx) < 1e-6 and per(px[1] + y0 - fx[1], ms.Ly) < 1e-6
    assert np.abs(px[2] - fx[2]).max() < 1e-6
    return om, idx
