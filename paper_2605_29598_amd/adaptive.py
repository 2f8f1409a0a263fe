"""Dynamic adaptivity on the library: a refinement box that follows a feature.

The paper refines statically (Sec. 4.3: nested 2:1 regions around the hill).
Here the refinement changes during the run: every `every` steps an indicator
(the largest potential-temperature deviation from the unperturbed background
per base column) selects the base cells to refine, a new mesh is built with one
refinement box covering them, and the conserved state is moved onto it by
imx_transfer_state (copy on kept leaves, exact evaluation on refined ones,
L2 projection on coarsened ones; every conserved integral kept). The step
itself is imx_step on the current mesh.

    python -m paper_2605_29598_amd.adaptive --steps 200 --every 10
"""
import argparse
import json
import sys
import time

import numpy as np

from . import workloads as W


def potential_temperature(rho, p):
    return p / (rho * W.RGAS) * (W.P_REF / p) ** (W.RGAS / W.CP)


def column_indicator(q, coords, w, spec):
    """Largest potential-temperature deviation |theta - theta_background| over
    the nodes of every base column, as an array [nx][ny], and the largest
    height at which a node's deviation exceeds a tenth of the global maximum.
    (theta is carried with the flow; the density deviation would also flag
    the sound waves that the initial imbalance sends through the box.)"""
    x, y, z = coords
    rho_bg, p_bg = W.primitive_background(w, x, y, z)
    kin = 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / q[0]
    p = (W.GAMMA - 1.0) * (q[4] - kin)
    dev = np.abs(potential_temperature(q[0], p) - potential_temperature(rho_bg, p_bg))   # [E][Np]
    cen = coords.mean(axis=2)                                    # element centres [3][E]
    bx = np.clip((cen[0] / (spec.Lx / spec.nx)).astype(int), 0, spec.nx - 1)
    by = np.clip((cen[1] / (spec.Ly / spec.ny)).astype(int), 0, spec.ny - 1)
    ind = np.zeros((spec.nx, spec.ny))
    np.maximum.at(ind, (bx, by), dev.max(axis=1))
    big = dev > 0.1 * dev.max()
    ztop = float(z[big].max()) if big.any() else 0.0
    return ind, ztop


def choose_box(ind, ztop, spec, frac=0.25, floor=1e-6):
    """Refinement box over the base columns whose indicator reaches `frac` of
    its maximum, padded by one column (clipped to the domain), from the ground
    to one base layer above `ztop`; None if nothing stands out (the largest
    deviation below `floor` K, the round-off of an unperturbed state)."""
    if ind.max() <= floor:
        return None
    ix, iy = np.nonzero(ind >= frac * ind.max())
    hx, hy, hz = spec.Lx / spec.nx, spec.Ly / spec.ny, spec.Lz / spec.nz
    x0 = max(0, ix.min() - 1) * hx
    x1 = min(spec.nx, ix.max() + 2) * hx
    y0 = max(0, iy.min() - 1) * hy
    y1 = min(spec.ny, iy.max() + 2) * hy
    z1 = min(spec.Lz, (np.floor(ztop / hz) + 2) * hz)
    # shrink by a small margin so that the box overlaps exactly these base cells
    e = 1e-6 * min(hx, hy, hz)
    return (x0 + e, x1 - e, y0 + e, y1 - e, 0.0, z1 - e)


def run(nsteps, every, w=None, out=sys.stdout):
    import torch
    from . import binding as B
    w = w or W.advected_bubble()
    spec = w.mesh
    mesh = B.Mesh(spec)
    sol = B.Solver(mesh, w.phys, w.num)
    coords = mesh.node_coords()
    sol.set_state(W.initial_state(w, coords))
    mass0 = sol.total_mass()
    box, done, t0 = None, 0, time.perf_counter()
    records = []
    while done < nsteps:
        # adapt: indicator on the current state, new box, new mesh, transfer
        q = sol.get_state().cpu().numpy()
        ind, ztop = column_indicator(q, coords, w, spec)
        nbox = choose_box(ind, ztop, spec)
        moved = nbox != box
        if moved:
            nspec = W.MeshSpec(**{**vars(spec), "ref_boxes": [nbox] if nbox else []})
            nmesh = B.Mesh(nspec)
            m_before = sol.total_mass()
            qn = B.transfer_state(mesh, nmesh, sol.get_state())
            nsol = B.Solver(nmesh, w.phys, w.num)
            nsol.set_state(qn)
            m_after = nsol.total_mass()
            del sol
            torch.cuda.empty_cache()
            sol, mesh, box = nsol, nmesh, nbox
            coords = mesh.node_coords()
        n = min(every, nsteps - done)
        st = sol.step(n)
        done += n
        rec = {"step": done, "t_s": done * w.num.dt, "elements": mesh.E,
               "box_x_km": None if box is None else [round(box[0] / 1e3, 3), round(box[1] / 1e3, 3)],
               "remeshed": bool(moved),
               "transfer_mass_rel_change": (m_after - m_before) / m_before if moved else 0.0,
               "mass_rel_change": (sol.total_mass() - mass0) / mass0,
               "picard": st.picard_iters, "gmres": st.gmres_iters}
        records.append(rec)
        print(json.dumps(rec), file=out, flush=True)
    summary = {"steps": done, "wall_s": time.perf_counter() - t0, "remeshes": sum(r["remeshed"] for r in records),
               "max_transfer_mass_rel_change": max(abs(r["transfer_mass_rel_change"]) for r in records),
               "mass_rel_change": records[-1]["mass_rel_change"]}
    return records, summary


def main(argv=None):
    ap = argparse.ArgumentParser(description="adaptive run: a refinement box following a bubble")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--nx", type=int, default=16)
    ap.add_argument("--ny", type=int, default=8)
    ap.add_argument("--nz", type=int, default=4)
    ap.add_argument("--degree", type=int, default=2)
    a = ap.parse_args(argv)
    _, summary = run(a.steps, a.every, w=W.advected_bubble(a.nx, a.ny, a.nz, a.degree))
    print("SUMMARY " + json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
