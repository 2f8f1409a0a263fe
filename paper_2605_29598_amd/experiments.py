"""Long integrations of the vertical-slice inertia-gravity-wave tests of
Secs. 4.1 and 4.2 on the library, with the geostrophic-imbalance measure (eq. egeo).

    python -m paper_2605_29598_amd.experiments planetary --hours 96
    python -m paper_2605_29598_amd.experiments reference --hours 8

`planetary`: 60000 x 10 km channel, a = 1000 km, dt = 10 s (the paper runs
96 h and reports an imbalance below 1e-7 m s^-2). `reference`: 6000 x 10 km,
a = 100 km, dt = 0.5 s, 8 h. Both on 300 x 20 elements at r = 4 with one
periodic element in y. One JSON line per reporting interval (model time,
imbalance, relative mass change, largest velocity components, iterations
and wall time per step) and a
summary line at the end. A run can be continued from a saved state
(--load / --save: a .npy file of the conserved state, the step count in a
sidecar .json).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import workloads as W


def run(kind, hours, every_hours, scheme, precision, load=None, save=None, out=sys.stdout):
    import torch
    from . import binding as B
    w = W.igw_slice(planetary=(kind == "planetary"), scheme=scheme)
    mesh = B.Mesh(w.mesh)
    prec = B.IMX_MIXED if precision == "mixed" else B.IMX_FP64
    sol = B.Solver(mesh, w.phys, w.num, precision=prec)
    step0 = 0
    if load:
        q0 = np.load(load, allow_pickle=False)
        with open(os.path.splitext(load)[0] + ".json") as f:
            step0 = int(json.load(f)["step"])
    else:
        q0 = W.initial_state(w, mesh.node_coords())
    sol.set_state(q0)
    dofs = 5 * mesh.E * mesh.Np
    mass0 = float((mesh.mass_diag() * W.initial_state(w, mesh.node_coords())[0]).sum())
    nsteps = int(round(hours * 3600.0 / w.num.dt))
    every = max(1, int(round(every_hours * 3600.0 / w.num.dt)))
    done, series, wall = 0, [], 0.0
    rec = {"t_h": step0 * w.num.dt / 3600.0, "egeo": sol.geo_imbalance()}
    series.append(rec)
    print(json.dumps(rec), file=out, flush=True)
    while done < nsteps:
        n = min(every, nsteps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sol.step(n)
        torch.cuda.synchronize()
        dt_wall = time.perf_counter() - t0
        wall += dt_wall
        done += n
        q = sol.get_state().cpu().numpy()
        rec = {"t_h": (step0 + done) * w.num.dt / 3600.0, "egeo": sol.geo_imbalance(),
               "mass_rel": (sol.total_mass() - mass0) / mass0,
               "max_abs_u": float(np.abs(q[1] / q[0]).max()), "max_abs_v": float(np.abs(q[2] / q[0]).max()),
               "max_abs_w": float(np.abs(q[3] / q[0]).max()),
               "picard_per_step": st.picard_iters / n, "gmres_per_step": st.gmres_iters / n,
               "ms_per_step": 1e3 * dt_wall / n}
        series.append(rec)
        print(json.dumps(rec), file=out, flush=True)
    if save:
        np.save(save, sol.get_state().cpu().numpy(), allow_pickle=False)
        with open(os.path.splitext(save)[0] + ".json", "w") as f:
            json.dump({"step": step0 + done}, f)
    summary = {"workload": w.name, "scheme": "R%d" % scheme, "precision": precision,
               "hours": (step0 + done) * w.num.dt / 3600.0, "steps": done, "dt": w.num.dt,
               "egeo_max": max(r["egeo"] for r in series), "egeo_final": series[-1]["egeo"],
               "dof_updates_per_s": dofs * done / wall if wall > 0 else None,
               "ms_per_step": 1e3 * wall / done if done else None, "wall_s": wall}
    print(json.dumps({"summary": summary}), file=out, flush=True)
    return summary, series


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("kind", choices=["planetary", "reference"])
    ap.add_argument("--hours", type=float, default=None)
    ap.add_argument("--every-hours", type=float, default=None)
    ap.add_argument("--scheme", choices=["R1", "R2"], default="R2")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--load", default=None)
    ap.add_argument("--save", default=None)
    a = ap.parse_args(argv)
    hours = a.hours if a.hours is not None else (96.0 if a.kind == "planetary" else 8.0)
    every = a.every_hours if a.every_hours is not None else (1.0 if a.kind == "planetary" else 0.25)
    run(a.kind, hours, every, W.R1 if a.scheme == "R1" else W.R2, a.precision, a.load, a.save)


if __name__ == "__main__":
    main()
