"""HBM traffic per kernel class from rocprofv3 counter runs.

Two `rocprofv3 --pmc` passes over the same command give FETCH_SIZE and
WRITE_SIZE (KiB per dispatch). Each is scaled by what the same counter reads
for a plain device copy of known size (run with `bench.py --copy-probe`), so
the result is in bytes of HBM traffic. The summary is keyed by the kernel
classes the solver's own timers use and stamped with a hash of the kernel
sources: a summary taken from other kernels is not used.

    python -m paper_2605_29598_amd.profiling \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \
        --copy-bytes 1073741824 --out profiles/pmc_traffic_<workload>.json

Any other counters (occupancy, VALU and LDS activity, instruction counts) are
averaged per kernel and printed as a markdown table:

    python -m paper_2605_29598_amd.profiling counters A.csv [B.csv ...] [--match REGEX]

The busy fractions and occupancy that say what bounds each kernel (VALUBusy,
LdsUtil, LDSBankConflict, OccupancyPercent) are kept per kernel, stamped with
the same hash, for the bench line's roofline object:

    python -m paper_2605_29598_amd.profiling limiters A.csv [B.csv ...] [--match REGEX] \
        --out profiles/pmc_limiters_<workload>.json
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))

# kernel-name stem -> class reported by the solver's timers
CLASSES = {
    "k_explicit": "explicit", "k_explicit_gc": "explicit", "k_pass1": "pass1", "k_mv1": "pass1", "k_mv1_gc": "pass1", "k_pass2": "pass2",
    "k_mv2": "pass2",
    "k_mv2w": "pass2", "k_lambda": "lambda", "k_dots": "dots", "k_axpy_norm": "ortho", "k_lincomb": "lincomb",
}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "vec.hip"):
        with open(os.path.join(_HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _load(path, counter):
    per = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def _stem(name):
    m = re.search(r"(k_[a-z0-9_]+)", name)
    return m.group(1) if m else name


def _copy_factor(path, counter, nbytes):
    per = _load(path, counter)
    # the copy of nbytes is the dispatch with the largest count
    best = max((max(v), k) for k, v in per.items())[0]
    return nbytes / (best * 1024.0), best


def summarize(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes):
    ff, fraw = _copy_factor(copy_fetch_csv, "FETCH_SIZE", copy_bytes)
    wf, wraw = _copy_factor(copy_write_csv, "WRITE_SIZE", copy_bytes)
    F, Wr = _load(fetch_csv, "FETCH_SIZE"), _load(write_csv, "WRITE_SIZE")
    kernels, classes = {}, collections.defaultdict(lambda: [0.0, 0])
    for name, v in F.items():
        w = Wr.get(name, [0.0])
        fb = ff * 1024.0 * sum(v) / len(v)
        wb = wf * 1024.0 * sum(w) / len(w)
        kernels[name] = {"dispatches": len(v), "fetch_bytes": fb, "write_bytes": wb, "bytes_per_dispatch": fb + wb}
        c = CLASSES.get(_stem(name))
        if c:
            classes[c][0] += (fb + wb) * len(v)
            classes[c][1] += len(v)
    return {
        "kernel_source_hash": kernel_source_hash(),
        "calibration": {"copy_bytes": copy_bytes, "fetch_KiB": fraw, "write_KiB": wraw,
                        "fetch_factor": ff, "write_factor": wf},
        "kernels": {c: {"bytes_per_launch": b / n, "dispatches": n} for c, (b, n) in classes.items()},
        "per_kernel": kernels,
    }


def counter_means(paths, match=None):
    """Per kernel (those whose name matches `match`, if given): the number of
    dispatches, the compiler's resources as the profiler reports them, and the
    mean value per dispatch of every counter in the given rocprofv3 CSVs."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    res = {}
    for path in paths:
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if match and not re.search(match, r["Kernel_Name"]):
                    continue
                k = r["Kernel_Name"].split("(")[0].replace("void ", "")
                per[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
                res[k] = (r["VGPR_Count"], r["Accum_VGPR_Count"], r["SGPR_Count"], r["LDS_Block_Size"],
                          r["Workgroup_Size"])
    out = {}
    for k in sorted(per):
        rec = {"dispatches": max(len(v) for v in per[k].values()),
               "resources": dict(zip(("VGPR", "AGPR", "SGPR", "LDS B", "WG"), res[k]))}
        rec["counters"] = {c: sum(v) / len(v) for c, v in sorted(per[k].items())}
        out[k] = rec
    return out


def counter_table(paths, match=None):
    """Mean value per dispatch of every counter in the given rocprofv3 CSVs,
    per kernel (kernels whose name matches `match`, if given), as a table."""
    means = counter_means(paths, match)
    names = sorted({c for v in means.values() for c in v["counters"]})
    head = ["kernel", "dispatches", "VGPR", "AGPR", "SGPR", "LDS B", "WG"] + names
    rows = ["| " + " | ".join(head) + " |", "|---" * len(head) + "|"]
    for k, v in means.items():
        cells = [f"`{k}`", str(v["dispatches"])] + list(v["resources"].values())
        for c in names:
            x = v["counters"].get(c)
            cells.append("" if x is None else f"{x:.4g}")
        rows.append("| " + " | ".join(cells) + " |")
    return "\n".join(rows)


# counters that say what bounds an element kernel, and how each reads
LIMITER_COUNTERS = ("VALUBusy", "LdsUtil", "LDSBankConflict", "OccupancyPercent")


def limiter_record(paths, match=None, command=""):
    """Busy fractions and occupancy per kernel from rocprofv3 counter CSVs,
    stamped with the kernel sources' hash (used only while the sources hash to
    it). waves_per_simd = OccupancyPercent x 32 / 100 / 4 (32 wave slots per
    compute unit, 4 SIMDs)."""
    rec = {"kernel_source_hash": kernel_source_hash(), "command": command, "kernels": {}}
    for k, v in counter_means(paths, match).items():
        c = {n: v["counters"][n] for n in LIMITER_COUNTERS if n in v["counters"]}
        if "OccupancyPercent" in c:
            c["waves_per_simd"] = c["OccupancyPercent"] * 32 / 100 / 4
        rec["kernels"][k] = {"dispatches": v["dispatches"], **c}
    return rec


WORKLOADS = {
    "igw_channel_120x40x10_r3": lambda W: W.igw_channel(),
    "orography_64x64x24_r4": lambda W: W.orography(),
    "orography_amr_32x32x12_r4": lambda W: W.orography(32, 32, 12, 4, refined=True),
}


def operators(name, reps=20, seed=1):
    """Per-launch time and algorithmic bandwidth of the explicit residual and
    the two Schur passes (R2) on a full workload, from the solver's HIP-event
    timers: `reps` Schur applies and `reps` // 4 explicit residuals on seeded
    inputs, after a warm-up."""
    import numpy as np
    import torch
    from . import binding as B
    from . import workloads as W
    w = WORKLOADS[name](W)
    mesh = B.Mesh(w.mesh)
    sol = B.Solver(mesh, w.phys, w.num)
    rng = np.random.default_rng(seed)
    shp = (mesh.E, mesh.Np)
    sol.implicit_setup(1 + 0.1 * rng.uniform(size=shp), 1e5 * (1 + 0.1 * rng.uniform(size=shp)),
                       rng.uniform(-1, 1, size=(3,) + shp))
    p = torch.from_numpy(1e5 * (1 + 0.1 * rng.uniform(size=shp))).cuda()
    q = torch.from_numpy(W.initial_state(w, mesh.node_coords())).cuda()
    for _ in range(3):
        sol.schur_apply(p)
        sol.explicit_residual(q)
    torch.cuda.synchronize()
    sol.timing(True)
    for _ in range(reps):
        sol.schur_apply(p)
    for _ in range(max(1, reps // 4)):
        sol.explicit_residual(q)
    torch.cuda.synchronize()
    rep = sol.timing_report()
    out = {"workload": name, "elements": mesh.E, "nodes_per_element": mesh.Np, "deformed": bool(mesh.deformed),
           "coarse_hanging_faces": mesh.n_hanging, "kernels": {}}
    for k in ("pass1", "pass2", "explicit"):
        ms, by, n = rep[k]
        us = 1e3 * ms / n
        out["kernels"][k] = {"launches": n, "avg_launch_us": us, "algorithmic_MB_per_launch": by / n / 1e6,
                             "GB_per_s": by / ms / 1e6, "frac_of_hbm_peak": by / ms / 1e6 / 8000.0}
    return out


def steps(name, nsteps=3, mixed=False):
    """Whole ARK2 steps of a workload from its initial state: one untimed step,
    then `nsteps` timed ones (wall clock around synchronised calls)."""
    import time
    import torch
    from . import binding as B
    from . import workloads as W
    w = WORKLOADS[name](W)
    mesh = B.Mesh(w.mesh)
    sol = B.Solver(mesh, w.phys, w.num, precision=B.IMX_MIXED if mixed else B.IMX_FP64)
    sol.set_state(W.initial_state(w, mesh.node_coords()))
    sol.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = sol.step(nsteps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / nsteps
    dofs = 5 * mesh.E * mesh.Np
    return {"workload": name, "precision": "fp32_inner" if mixed else "fp64", "elements": mesh.E, "dofs": dofs,
            "dt": w.num.dt, "ms_per_step": 1e3 * dt, "dof_updates_per_s": dofs / dt,
            "gmres_per_step": st.gmres_iters / nsteps, "picard_per_step": st.picard_iters / nsteps}


def run(name, nsteps, mixed=False, scheme=None, out=None, every=10, dt=None):
    """A workload run to its stated length from its initial state, one step at
    a time: per step the Picard and GMRES iterations, the wall time, max|w|
    (diagnostic, from the device state) and, every `every` steps, the total
    mass; one JSON line per step to `out` and a progress line to stdout."""
    import time
    import torch
    from . import binding as B
    from . import workloads as W
    w = WORKLOADS[name](W)
    if scheme is not None:
        w.num.scheme = scheme
    if dt is not None:
        # the sponge strength is stated as lambda dt; keep lambda itself
        w.num.dt = dt
    mesh = B.Mesh(w.mesh)
    sol = B.Solver(mesh, w.phys, w.num, precision=B.IMX_MIXED if mixed else B.IMX_FP64)
    sol.set_state(W.initial_state(w, mesh.node_coords()))
    m0 = sol.total_mass()
    fh = open(out, "w") if out else None
    recs = []
    t_run = time.perf_counter()
    status = "ok"
    for k in range(nsteps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            st = sol.step(1)
        except B.IMXError as e:
            status = f"step {k + 1}: {e}"
            print(status, flush=True)
            break
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        q = sol.get_state()
        wmax = float((q[3] / q[0]).abs().max())
        rec = {"step": k + 1, "ms": ms, "picard": st.picard_iters, "gmres": st.gmres_iters, "max_w": wmax}
        if (k + 1) % every == 0 or k + 1 == nsteps:
            rec["mass_rel_change"] = (sol.total_mass() - m0) / m0
            print(json.dumps(rec), flush=True)
        recs.append(rec)
        if fh:
            fh.write(json.dumps(rec) + "\n")
            fh.flush()
    wall = time.perf_counter() - t_run
    dofs = 5 * mesh.E * mesh.Np
    n = len(recs)
    summary = {"workload": name, "precision": "fp32_inner" if mixed else "fp64",
               "scheme": "R1" if w.num.scheme == B.IMX_R1 else "R2", "dt": w.num.dt,
               "steps_asked": nsteps, "steps_done": n, "status": status, "elements": mesh.E, "dofs": dofs,
               "wall_s": wall}
    if n:
        ms = [r["ms"] for r in recs]
        summary.update({
            "mean_ms_per_step": sum(ms) / n, "dof_updates_per_s": dofs * n / (sum(ms) * 1e-3),
            "gmres_per_step_first10": sum(r["gmres"] for r in recs[:10]) / min(n, 10),
            "gmres_per_step_last10": sum(r["gmres"] for r in recs[-10:]) / min(n, 10),
            "picard_per_step_first10": sum(r["picard"] for r in recs[:10]) / min(n, 10),
            "picard_per_step_last10": sum(r["picard"] for r in recs[-10:]) / min(n, 10),
            "max_w_first": recs[0]["max_w"], "max_w_last": recs[-1]["max_w"],
            "max_w_max": max(r["max_w"] for r in recs),
            "mass_rel_change_last": recs[-1].get("mass_rel_change")})
    if fh:
        fh.close()
    return summary


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "run":
        ap = argparse.ArgumentParser(description="a workload run to its stated length, logged per step")
        ap.add_argument("mode")
        ap.add_argument("--workload", choices=list(WORKLOADS), required=True)
        ap.add_argument("--steps", type=int, required=True)
        ap.add_argument("--mixed", action="store_true")
        ap.add_argument("--scheme", choices=["R1", "R2"], default=None)
        ap.add_argument("--out", default=None, help="per-step JSON lines")
        ap.add_argument("--dt", type=float, default=None, help="time step instead of the workload's")
        a = ap.parse_args()
        sch = None if a.scheme is None else (1 if a.scheme == "R1" else 2)
        print("SUMMARY " + json.dumps(run(a.workload, a.steps, a.mixed, sch, a.out, dt=a.dt)), flush=True)
        return
    if len(sys.argv) > 1 and sys.argv[1] == "steps":
        ap = argparse.ArgumentParser(description="ARK2 step rate of a full workload")
        ap.add_argument("mode")
        ap.add_argument("--workload", choices=list(WORKLOADS), required=True)
        ap.add_argument("--steps", type=int, default=3)
        ap.add_argument("--mixed", action="store_true")
        a = ap.parse_args()
        print(json.dumps(steps(a.workload, a.steps, a.mixed)))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "operators":
        ap = argparse.ArgumentParser(description="operator timings on a full workload")
        ap.add_argument("mode")
        ap.add_argument("--workload", choices=list(WORKLOADS), required=True)
        ap.add_argument("--reps", type=int, default=20)
        a = ap.parse_args()
        print(json.dumps(operators(a.workload, a.reps)))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        ap = argparse.ArgumentParser(description="per-kernel mean of rocprofv3 counters")
        ap.add_argument("mode")
        ap.add_argument("csv", nargs="+")
        ap.add_argument("--match", default=None, help="regular expression on the kernel name")
        a = ap.parse_args()
        print(counter_table(a.csv, a.match))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "limiters":
        ap = argparse.ArgumentParser(description="busy fractions and occupancy per kernel, hash-stamped")
        ap.add_argument("mode")
        ap.add_argument("csv", nargs="+")
        ap.add_argument("--match", default=None, help="regular expression on the kernel name")
        ap.add_argument("--out", required=True)
        ap.add_argument("--command", default="")
        a = ap.parse_args()
        with open(a.out, "w") as fh:
            json.dump(limiter_record(a.csv, a.match, a.command), fh, indent=1)
        return
    ap = argparse.ArgumentParser()
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--out"):
        ap.add_argument(a, required=True)
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    rec = summarize(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes)
    rec["command"] = a.command
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
