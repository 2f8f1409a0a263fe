"""The patch reasoning behind the full-size sampled parity tests, checked on
the oracle alone: on meshes small enough to evaluate whole (periodic, terrain,
two refinement levels), the explicit residual on the 3x3 centre columns and
the Schur complement on the centre column of a 5x5-column patch equal the
values on the whole mesh."""
import numpy as np
import pytest

from oracle import dg
from oracle.mesh import Mesh as OMesh, MeshDesc
from paper_2605_29598_amd import workloads as W
from tests.patches import R, columns, patch_for

SPECS = {
    "periodic_flat_r2": W.MeshSpec(9e3, 8e3, 3e3, 9, 8, 3, 2),
    "terrain_r3": W.MeshSpec(9e3, 9e3, 3e3, 9, 9, 2, 3, terrain=W.GAUSS, h0=300, a=700.0, xc=2e3, yc=2e3),
    "refined_terrain_r2": W.MeshSpec(12e3, 12e3, 4e3, 8, 8, 2, 2, terrain=W.BELL, h0=300, a=1.5e3, xc=6e3, yc=6e3,
                                     ref_boxes=[(4.5e3, 7.5e3, 4.5e3, 7.5e3, 0, 2e3),
                                                (5.5e3, 6.5e3, 5.5e3, 6.5e3, 0, 1e3)]),
}
CENTRES = {"periodic_flat_r2": [(4, 4), (0, 7)], "terrain_r3": [(4, 4), (0, 0)],
           "refined_terrain_r2": [(4, 4), (3, 5)]}


@pytest.mark.parametrize("name", list(SPECS))
def test_patch_reproduces_whole_mesh(name):
    spec = SPECS[name]
    om_full = OMesh(MeshDesc(**vars(spec)))
    xyz = om_full.node_coords()
    cen = xyz.mean(axis=2)
    ph = dg.Phys(f=1e-3, sponge_zB=1e3, sponge_zT=3e3, sponge_lam=0.01, sponge_u=(2.0, 0.0, 0.0))
    q = W.random_positive_state((om_full.E, om_full.Np), 3)
    TNS, TS = dg.explicit_residual(om_full, ph, q)
    rng = np.random.default_rng(4)
    shp = (om_full.E, om_full.Np)
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, shp)
    pk = 1e5 * (1 + 0.1 * rng.uniform(-1, 1, shp))
    uk = 10 * rng.uniform(-1, 1, (3,) + shp)
    p = 1e5 * (1 + 0.1 * rng.uniform(-1, 1, shp))
    Sf = dg.StageSystem(om_full, ph, rho, pk, uk, dg.A_IMP[1, 1], 5.0, dg.R2).schur(p)
    for centre in CENTRES[name]:
        om, idx = patch_for(spec, xyz, cen, centre)
        PNS, PS = dg.explicit_residual(om, ph, q[:, idx])
        c1 = columns(om, R - 1, R + 1)
        assert np.allclose(PNS[:, c1], TNS[:, idx[c1]], rtol=0, atol=1e-12 * np.abs(TNS).max())
        assert np.allclose(PS[:, c1], TS[:, idx[c1]], rtol=0, atol=1e-12 * np.abs(TS).max())
        Sp = dg.StageSystem(om, ph, rho[idx], pk[idx], uk[:, idx], dg.A_IMP[1, 1], 5.0, dg.R2).schur(p[idx])
        c0 = columns(om, R, R)
        assert np.allclose(Sp[c0], Sf[idx[c0]], rtol=0, atol=1e-12 * np.abs(Sf).max())
        # and the patch edge does differ (the comparison is not vacuous)
        edge = columns(om, 0, 2 * R)
        assert len(edge) > len(c1) > len(c0) > 0
