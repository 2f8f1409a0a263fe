"""Host logic of the adaptive runs: the column indicator and the choice of
the refinement box (no GPU)."""
import numpy as np

from oracle.mesh import Mesh as OMesh, MeshDesc
from paper_2605_29598_amd import adaptive, workloads as W


def test_box_covers_the_feature_and_moves_with_it():
    w = W.advected_bubble(nx=8, ny=4, nz=4, degree=2)
    om = OMesh(MeshDesc(**vars(w.mesh)))
    coords = om.node_coords()
    boxes = []
    for xc in (8e3, 14e3):
        w.pert_xc = xc
        q = W.initial_state(w, coords)
        ind, ztop = adaptive.column_indicator(q, coords, w, w.mesh)
        box = adaptive.choose_box(ind, ztop, w.mesh)
        # the columns around the bubble centre are flagged, with one column of padding
        assert box[0] < xc - 2e3 and box[1] > xc + 2e3
        assert box[2] < 10e3 - 2e3 and box[3] > 10e3 + 2e3
        assert box[4] == 0.0 and 4e3 < box[5] <= 10e3
        boxes.append(box)
    assert abs((boxes[1][0] - boxes[0][0]) - 5e3) < 1.0     # one 5 km base column further
    # an unperturbed state selects nothing
    w.pert = "none"
    q = W.initial_state(w, coords)
    ind, ztop = adaptive.column_indicator(q, coords, w, w.mesh)
    assert adaptive.choose_box(ind, ztop, w.mesh) is None
