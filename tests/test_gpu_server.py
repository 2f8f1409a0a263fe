"""GPU tests of the ensemble server: a member's result does not depend on what
runs beside it, the memory pool bounds what runs at once, and a request that
can never fit is rejected.

Members are integrations of different meshes (uniform periodic box, hanging
faces, terrain), degrees and schemes. Each is run alone through a plain
solver and inside a mix on the server; the final states must agree bit for
bit, and one member is also checked against the oracle at the FP64 bar.
"""
import time

import numpy as np
import pytest

from oracle import dg
from oracle.mesh import Mesh as OMesh, MeshDesc
from paper_2605_29598_amd import workloads as W
from tests.bars import check_state

pytestmark = pytest.mark.gpu


def _B():
    from paper_2605_29598_amd import binding as B
    return B


def _members():
    tiny = W.tiny_box()
    hang = W.MeshSpec(8e3, 8e3, 4e3, 4, 4, 2, 2,
                      ref_boxes=[(2e3, 6e3, 2e3, 6e3, 0, 2e3)])
    terr = W.MeshSpec(8e3, 8e3, 4e3, 3, 3, 2, 3, terrain=W.GAUSS, h0=400, a=2e3, xc=4e3, yc=4e3)
    # affine members of three degrees next to a terrain-following one, long
    # enough to overlap on the device: every element kernel then runs on
    # compute units whose LDS another kernel (other degree, other tables) has
    # just used
    box3 = W.MeshSpec(12e3, 12e3, 10e3, 10, 10, 6, 3)
    box4 = W.MeshSpec(12e3, 12e3, 10e3, 8, 8, 5, 4)
    out = [
        (tiny.mesh, tiny.phys, tiny.num, 4),
        (hang, W.PhysSpec(f=1e-4), W.NumSpec(dt=2.0, scheme=dg.R1), 3),
        (terr, W.PhysSpec(f=1e-4), W.NumSpec(dt=2.0), 3),
        (tiny.mesh, tiny.phys, W.NumSpec(dt=1.0), 5),
        (box3, W.PhysSpec(f=1e-4), W.NumSpec(dt=2.0), 6),
        (box4, W.PhysSpec(f=1e-4), W.NumSpec(dt=2.0), 6),
    ]
    return [(spec, ph, nm, W.initial_state(tiny, OMesh(MeshDesc(**vars(spec))).node_coords()), n)
            for spec, ph, nm, n in out]


def _alone(spec, ph, nm, q0, n):
    B = _B()
    sol = B.Solver(B.Mesh(spec), ph, nm)
    sol.set_state(q0)
    sol.step(n)
    return sol.get_state().cpu().numpy()


def _drain(sv, limit_s=120.0):
    t0 = time.time()
    while True:
        r, w = sv.tick()
        if r == 0 and w == 0:
            return
        assert time.time() - t0 < limit_s, "server did not drain"
        time.sleep(0.002)


@pytest.mark.parametrize("graphs", [False, True])
def test_mix_equals_alone_bitwise(graphs):
    B = _B()
    mem = _members()
    ref = [_alone(*m) for m in mem]
    sv = B.Server(pool_bytes=4 << 30, max_running=6)
    # with graphs the members replay their Krylov chunks from HIP graphs
    sv.set_graphs(graphs)
    ids = [sv.submit(*m) for m in mem]
    _drain(sv)
    st = sv.query()
    assert st.completed == len(mem) and st.rejected == 0 and st.pool_bytes_in_use == 0
    for rid, r, m in zip(ids, ref, mem):
        q, ms = sv.result(rid)
        assert ms.status == B.IMX_OK and ms.steps_done == m[4]
        assert np.array_equal(q, r), rid
        assert ms.p99_step_ms >= ms.p50_step_ms > 0


def test_member_matches_oracle():
    B = _B()
    w = W.tiny_box()
    om = OMesh(MeshDesc(**vars(w.mesh)))
    y0 = W.initial_state(w, om.node_coords())
    sv = B.Server(pool_bytes=1 << 30, max_running=2)
    rid = sv.submit(w.mesh, w.phys, w.num, y0, 3)
    _drain(sv)
    q, ms = sv.result(rid)
    y = y0
    for _ in range(3):
        y, _ = dg.ark2_step(om, dg.Phys(**vars(w.phys)), dg.Numerics(**vars(w.num)), y)
    # same stopping tests on both sides, so the same iteration counts: the
    # FP64 parity bars apply
    check_state(q, y, om, w.num.dt, 3, tag="served member")


def test_pool_budget_bounds_concurrency():
    """The pool holds the two largest members but not three: peak usage stays
    within the pool, every member still completes, later members wait."""
    B = _B()
    mem = _members()
    need = [B.member_pool_bytes(B.Mesh(m[0]), m[1], m[2]) for m in mem]
    big = sorted(need)[-2:]
    pool = sum(big) + 4096
    assert pool < sum(need)
    sv = B.Server(pool_bytes=pool, max_running=8)
    ids = [sv.submit(*m) for m in mem]
    r, w = sv.tick()
    assert r >= 1 and r + w == len(mem) and w >= 1
    peak_running = r
    t0 = time.time()
    while True:
        r, w = sv.tick()
        peak_running = max(peak_running, r)
        st = sv.query()
        assert st.pool_bytes_in_use <= pool
        if r == 0 and w == 0:
            break
        assert time.time() - t0 < 120
        time.sleep(0.002)
    st = sv.query()
    assert st.completed == len(mem) and st.pool_bytes_peak <= pool and st.pool_bytes_in_use == 0
    assert peak_running < len(mem)
    for rid, m in zip(ids, mem):
        q, ms = sv.result(rid)
        assert ms.status == B.IMX_OK and ms.steps_done == m[4]


def test_oversized_request_rejected():
    B = _B()
    spec, ph, nm, q0, n = _members()[0]
    need = B.member_pool_bytes(B.Mesh(spec), ph, nm)
    sv = B.Server(pool_bytes=need - 4096, max_running=2)
    with pytest.raises(B.IMXError) as e:
        sv.submit(spec, ph, nm, q0, n)
    assert e.value.code == B.IMX_EREJECT
    assert sv.query().rejected == 1
