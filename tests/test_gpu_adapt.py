"""GPU parity of the solution transfer (dynamic adaptivity) against the oracle.

imx_transfer_state moves the conserved state between two refinements of one
grid (refinement, coarsening, a moved refinement box, two levels at once), on
flat and terrain-following meshes and degrees 2-4; the result is compared
with oracle.adapt.transfer node by node, and the integrals of the five
conserved fields are checked with the oracle's mass weights.
"""
import numpy as np
import pytest

from oracle import adapt
from oracle.mesh import Mesh as OMesh, MeshDesc
from paper_2605_29598_amd import workloads as W

pytestmark = pytest.mark.gpu

ONE = [(1e3, 3e3, 1e3, 3e3, 0.0, 1e3)]
TWO = [(0.5e3, 3.5e3, 0.5e3, 2.5e3, 0.0, 1.5e3), (1.2e3, 2.2e3, 1.1e3, 1.9e3, 0.0, 0.6e3)]
MOVED = [(2e3, 4e3, 0.0, 2e3, 0.5e3, 2e3)]
CASES = [("refine2", (), TWO), ("coarsen2", TWO, ()), ("moved", ONE, MOVED), ("moved2", TWO, MOVED)]


def _spec(r, boxes, terrain):
    return W.MeshSpec(4e3, 4e3, 2e3, 4, 4, 2, r, terrain=terrain, h0=250.0, a=1.2e3, xc=2e3, yc=2e3,
                      ref_boxes=list(boxes))


@pytest.mark.parametrize("r", [2, 3, 4])
@pytest.mark.parametrize("terrain", [W.FLAT, W.GAUSS])
@pytest.mark.parametrize("name,a,b", CASES)
def test_transfer_matches_oracle(r, terrain, name, a, b):
    from paper_2605_29598_amd import binding as B
    sa, sb = _spec(r, a, terrain), _spec(r, b, terrain)
    ga, gb = B.Mesh(sa), B.Mesh(sb)
    oa, ob = OMesh(MeshDesc(**vars(sa))), OMesh(MeshDesc(**vars(sb)))
    q = W.random_positive_state((oa.E, oa.Np), 5)
    got = B.transfer_state(ga, gb, q).cpu().numpy()
    ref = adapt.transfer(oa, ob, q)
    for t in range(5):
        err = np.abs(got[t] - ref[t]).max() / np.abs(ref[t]).max()
        print(f"[transfer] {name} r={r} terrain={terrain} field {t}: {err:.2e}", flush=True)
        assert err < 1e-12, (t, err)
    I0 = (oa.W3 * oa.detJ * q).sum(axis=(1, 2))
    I1 = (ob.W3 * ob.detJ * got).sum(axis=(1, 2))
    assert np.abs(I1 - I0).max() <= 1e-13 * np.abs(I0).max()


def test_transfer_round_trip_on_affine_mesh():
    from paper_2605_29598_amd import binding as B
    sa, sb = _spec(3, (), W.FLAT), _spec(3, TWO, W.FLAT)
    ga, gb = B.Mesh(sa), B.Mesh(sb)
    q = W.random_positive_state((ga.E, ga.Np), 9)
    back = B.transfer_state(gb, ga, B.transfer_state(ga, gb, q)).cpu().numpy()
    assert np.abs(back - q).max() <= 1e-13 * np.abs(q).max()


def test_adaptive_run_follows_the_bubble():
    """A refinement box that follows a warm bubble carried by a 20 m/s wind
    for 400 s: it is moved at least once, every transfer keeps the total mass
    to round-off, and the box advances downstream."""
    from paper_2605_29598_amd import adaptive
    recs, summary = adaptive.run(200, 20, w=W.advected_bubble(nx=8, ny=4, nz=4, degree=2))
    print("[adaptive]", summary, flush=True)
    moves = [r for r in recs if r["remeshed"]]
    assert len(moves) >= 2, recs
    assert summary["max_transfer_mass_rel_change"] < 1e-13
    assert abs(summary["mass_rel_change"]) < 1e-13
    assert moves[-1]["box_x_km"][1] > moves[0]["box_x_km"][1]
