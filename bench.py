"""Benchmark: IMEX-ARK2 steps of the stratified rotating flow over orography on one MI355X.

Workload: 60x60x20 km Gal-Chen box over a Gaussian hill (h0 = 400 m,
half-width 2 km), 64x64x24 hexahedra of degree 4 (98,304 elements, 61.44 M DoF
over the 5 conserved fields, per-point Jacobians stored), theta_ref =
293.15 K, N = 0.01 1/s, U = 10 m/s, f = 1e-4 1/s, Rayleigh sponge above 12 km
with lambda dt = 1.2, dt = 4 s, R2 treatment, GMRES(30) / Picard tolerance
1e-10, binary64. A step is one whole IMEX-ARK2 step (three explicit
residuals, two implicit stages with their Picard and GMRES iterations, stage
combinations, final update and mass check) on device-resident state.

Prints one JSON line: DoF-updates/s (5 E Np per step); the roofline of the
Schur-complement apply (pass 1 + pass 2, the operator that dominates the
step) and every kernel class, timed on the same steps as the headline (the
state at the start of the timed region is kept and the steps are replayed
with a HIP event pair around every launch: the solver is deterministic, so
the replay does the same iterations); the same steps with the binary32
Krylov inner loop; the rotating IGW channel as a second workload; the served
ensemble; and the CPU oracle on the host's cores on a bounded sample of the
same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DoF-updates/s per IMEX step (FP64 vs FP32-inner); operator GB/s; p99 latency"
OPERATORS = ("explicit", "pass1", "pass2", "lambda")


def measured_traffic(workload, classes):
    """HBM bytes per launch (summed over `classes`) from the committed
    rocprofv3 --pmc summary of this workload, if the kernels have not changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    from paper_2605_29598_amd.profiling import kernel_source_hash
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    tot = 0.0
    for c in classes:
        k = rec.get("kernels", {}).get(c)
        if k is None:
            return None
        tot += k["bytes_per_launch"]
    return tot


def measured_limiters(workload, stems):
    """Busy fractions and occupancy of the binary64 kernels behind the timed
    classes ({class: kernel-name pattern}; the most dispatched match is taken)
    from the committed counter record of this workload, if the kernels have not
    changed since it was taken: what bounds them, beside the HBM fraction."""
    path = os.path.join(ROOT, "profiles", f"pmc_limiters_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    from paper_2605_29598_amd.profiling import kernel_source_hash
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    out = {}
    for cls, stem in stems.items():
        cands = [(v["dispatches"], k) for k, v in rec.get("kernels", {}).items() if stem in k and "double" in k]
        if not cands:
            return None
        k = max(cands)[1]
        out[cls] = {"kernel": k, **{c: x for c, x in rec["kernels"][k].items() if c != "dispatches"}}
    return out


def _oracle_worker(args):
    """One host process: the oracle's ARK2 steps on its own copy of the sample."""
    spec, phys, num, steps = args
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import dg
    from oracle.mesh import Mesh as OMesh, MeshDesc
    from paper_2605_29598_amd import workloads as W
    with threadpool_limits(1):
        w = W.orography()
        w.mesh = W.MeshSpec(**spec)
        om = OMesh(MeshDesc(**spec))
        q = W.initial_state(w, om.node_coords())
        ph, nm = dg.Phys(**phys), dg.Numerics(**num)
        t0 = time.perf_counter()
        for _ in range(steps):
            q, _ = dg.ark2_step(om, ph, nm, q)
        el = time.perf_counter() - t0
    return 5 * om.E * om.Np * steps, el


def cpu_baseline(procs=None, n=2, steps=1):
    """The oracle (plain numpy, one thread per process) on the host's cores:
    `procs` processes (all cores the process may use, at most 16, the CPU
    share of one GPU on the box) each advance their own copy of an n x n x 24
    element piece of the orography box (same element size, degree, dt,
    physics and tolerances, the hill at its centre, periodic) by `steps` ARK2
    steps; the rate is the total DoF updates over the wall time of the pool."""
    import multiprocessing as mp
    from paper_2605_29598_amd import workloads as W
    if procs is None:
        procs = max(1, min(len(os.sched_getaffinity(0)), 16))
    w = W.orography()
    spec = dict(vars(w.mesh))
    spec.update(Lx=60e3 * n / 64, Ly=60e3 * n / 64, nx=n, ny=n, xc=30e3 * n / 64, yc=30e3 * n / 64)
    job = (spec, dict(vars(w.phys)), dict(vars(w.num)), steps)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_worker, [job] * procs)
    wall = time.perf_counter() - t0
    dof_updates = sum(r[0] for r in res)
    per_proc = [r[1] for r in res]
    return {"value": dof_updates / wall, "unit": "DoF-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} processes x 1 thread, each {steps} ARK2 step(s) of its own {n}x{n}x24-element "
                      f"piece of the orography box ({n * n * 24} elements, r = 4, same element size, dt, "
                      f"physics, tolerances; hill at the centre, periodic); wall {wall:.1f} s, "
                      f"per-process step time {min(per_proc):.1f}-{max(per_proc):.1f} s"}


def field_errors(a, b, gamma=1.4):
    """Max error per conserved field against its own maximum, and against the
    tolerance-mode scale (momentum in p / c: two solves that stop at a relative
    tolerance tol may differ by tol p / c in momentum)."""
    import numpy as np
    rho = np.abs(b[0]).max()
    kin = 0.5 * (b[1] ** 2 + b[2] ** 2 + b[3] ** 2) / b[0]
    p = np.abs((gamma - 1.0) * (b[4] - kin)).max()
    c = math.sqrt(gamma * p / rho)
    scale = [rho, p / c, p / c, p / c, np.abs(b[4]).max()]
    names = ["rho", "rho_u", "rho_v", "rho_w", "rho_E"]
    own = {names[t]: float(np.abs(a[t] - b[t]).max() / np.abs(b[t]).max()) for t in range(5)}
    tol = {names[t]: float(np.abs(a[t] - b[t]).max() / scale[t]) for t in range(5)}
    return {"vs_own_max": own, "vs_tolerance_scale": tol}


def timed_steps(sol, steps):
    """Wall time of `steps` steps with nothing else queued; iteration counts."""
    import torch
    torch.cuda.synchronize()
    picard = gmres = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        st = sol.step(1)
        picard += st.picard_iters
        gmres += st.gmres_iters
    torch.cuda.synchronize()
    return time.perf_counter() - t0, picard, gmres


def kernel_replay(sol, q_start, steps):
    """The same steps again from the saved state with a HIP event pair around
    every launch on the solver's stream: {class: (ms, bytes, launches)} and
    the iteration counts of the replay."""
    import torch
    sol.set_state(q_start)
    torch.cuda.synchronize()
    sol.timing(True)
    picard = gmres = 0
    for _ in range(steps):
        st = sol.step(1)
        picard += st.picard_iters
        gmres += st.gmres_iters
    torch.cuda.synchronize()
    rep = sol.timing_report()
    sol.timing(False)
    return rep, picard, gmres


def roofline_of(rep, classes, steps, traffic, note):
    ms = sum(rep[c][0] for c in classes)
    by = sum(rep[c][1] for c in classes)
    n = rep[classes[0]][2]
    achieved = by / (ms * 1e-3) / 1e9
    return {"kernel": " + ".join(classes), "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "avg_launch_us": 1e3 * ms / max(n, 1), "algorithmic_bytes_per_launch": by / max(n, 1),
            "launches_per_step": n / steps, "timing": note}


def kernels_block(rep, steps):
    out = {}
    for k, v in rep.items():
        if not v[2]:
            continue
        gbs = v[1] / (v[0] * 1e-3) / 1e9 if v[0] > 0 else 0.0
        out[k] = {"ms_per_step": round(v[0] / steps, 3), "GB_per_s": round(gbs, 1),
                  "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 3), "avg_launch_us": round(1e3 * v[0] / v[2], 1),
                  "launches_per_step": round(v[2] / steps, 1)}
    return out


def run_workload(w, args, precision, ref_state=None, replay=True):
    """Warm-up, timed steps, and (replay) the kernel-timed replay of the same
    steps. Returns the result block and the final state."""
    import torch
    from paper_2605_29598_amd import binding as B
    mesh = B.Mesh(w.mesh)
    sol = B.Solver(mesh, w.phys, w.num, device="cuda:0", precision=precision, inner_tol=1e-3)
    q0 = W_initial(w, mesh)
    sol.set_state(q0)
    dofs = 5 * mesh.E * mesh.Np
    for i in range(args.warmup):
        sol.step(1)
    q_start = sol.get_state().clone()
    el, picard, gmres = timed_steps(sol, args.steps)
    final = sol.get_state().cpu().numpy()
    out = {"value": dofs * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
           "iterations_per_step": {"picard": picard / args.steps, "gmres": gmres / args.steps},
           "elements": mesh.E, "degree": w.mesh.degree, "dofs": dofs, "mass": sol.total_mass()}
    rep = None
    if replay:
        rep, rp, rg = kernel_replay(sol, q_start, args.steps)
        same = (rp, rg) == (picard, gmres) and bool((sol.get_state().cpu().numpy() == final).all())
        out["kernels"] = kernels_block(rep, args.steps)
        out["kernels_timing"] = ("HIP event pair around every launch on the solver stream, on a replay of the "
                                 "timed steps from their saved start state; replay identical to the timed "
                                 f"steps (iterations and final state bitwise): {same}")
    if ref_state is not None:
        out["max_rel_error_vs_fp64"] = field_errors(final, ref_state)
    del sol
    torch.cuda.empty_cache()
    return out, final, rep


def W_initial(w, mesh):
    from paper_2605_29598_amd import workloads as W
    return W.initial_state(w, mesh.node_coords())


def served_run(args):
    """The served ensemble: requests from a seeded Poisson trace are submitted
    at their arrival times to the server (pool = the HBM budget) and advanced
    concurrently; the same requests are also run one at a time in arrival
    order through a plain solver (a queue alone), whose member times give the
    serial makespan under the same arrivals."""
    import numpy as np
    import torch
    from paper_2605_29598_amd import binding as B
    from paper_2605_29598_amd import workloads as W

    # members are scaled down from the full ensemble (E uniform in 2k-200k, 50
    # steps, Poisson arrivals at 2/s); the arrival rate is scaled up by the same
    # factor as the work per member, so the offered load matches the full trace
    from paper_2605_29598_amd import ensemble
    e_lo, e_hi = 2000, 24000
    rate = ensemble.scaled_rate(e_lo, e_hi, args.serve_steps)
    trace = W.served_trace(n_requests=args.serve_requests, rate_per_s=rate, elem_min=e_lo, elem_max=e_hi,
                           steps=args.serve_steps, seed=5)
    meshes, q0s, dofs = [], [], []
    for r in trace:
        m = B.Mesh(r.workload.mesh)
        meshes.append(m)
        q0s.append(W.initial_state(r.workload, m.node_coords()))
        dofs.append(5 * m.E * m.Np)
    total = float(sum(d * r.steps for d, r in zip(dofs, trace)))

    # queue alone: each member's whole life (solver, upload, steps, download) in arrival order
    dur, alone_steps, finals = [], [], []
    for r, m, q0 in zip(trace, meshes, q0s):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol = B.Solver(m, r.workload.phys, r.workload.num)
        sol.set_state(torch.from_numpy(q0).cuda())
        for _ in range(r.steps):
            a = time.perf_counter()
            sol.step(1)
            alone_steps.append(1e3 * (time.perf_counter() - a))
        finals.append(sol.get_state().cpu().numpy())
        torch.cuda.synchronize()
        dur.append(time.perf_counter() - t0)
        del sol
    end, lat = 0.0, []
    for r, d in zip(trace, dur):
        end = max(end, r.arrival_s) + d
        lat.append(end - r.arrival_s)
    serial = {"dof_updates_per_s": total / (end - trace[0].arrival_s), "makespan_s": end - trace[0].arrival_s,
              "step_ms_p50": float(np.percentile(alone_steps, 50)), "step_ms_p99": float(np.percentile(alone_steps, 99)),
              "request_latency_s_p50": float(np.percentile(lat, 50)),
              "request_latency_s_p99": float(np.percentile(lat, 99))}
    print(f"serve: queue alone makespan {serial['makespan_s']:.2f} s", file=sys.stderr, flush=True)

    def served(precision):
        out, qs = ensemble.serve(trace, q0s, dofs, precision, args.serve_pool_gb, args.serve_slots)
        if precision == B.IMX_FP64:
            out["max_abs_diff_vs_alone"] = max(float(np.abs(q - f).max()) for q, f in zip(qs, finals))
        else:
            out["max_rel_error_vs_fp64_alone_tolerance_scale"] = max(
                max(field_errors(q, f)["vs_tolerance_scale"].values()) for q, f in zip(qs, finals))
        print(f"serve: {'fp64' if precision == B.IMX_FP64 else 'mixed'} makespan {out['makespan_s']:.2f} s",
              file=sys.stderr, flush=True)
        return out

    fp64 = served(B.IMX_FP64)
    mixed = served(B.IMX_MIXED)
    return {"workload": f"{len(trace)} requests, Poisson arrivals at {rate:.1f}/s (the full ensemble's 2/s scaled "
                        f"by its work per member), IGW channel or orography members, elements uniform 2k-24k, "
                        f"degree 2-4, {args.serve_steps} ARK2 steps each",
            "dof_updates": total, "queue_alone_fp64": serial, "served_fp64": fp64, "served_fp32_inner": mixed,
            "speedup_served_fp64_vs_queue": fp64["dof_updates_per_s"] / serial["dof_updates_per_s"],
            "speedup_served_fp32_inner_vs_queue": mixed["dof_updates_per_s"] / serial["dof_updates_per_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scheme", default="R2", choices=["R1", "R2"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-inner comparison run")
    ap.add_argument("--no-channel", action="store_true", help="skip the IGW channel run")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-ensemble run")
    ap.add_argument("--serve-only", action="store_true", help="run only the served-ensemble comparison")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-steps", type=int, default=20)
    # one running member per hardware queue of the process (HIP's default of 4):
    # 4, 8 and 12 slots give the same throughput, more slots only queue longer
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-pool-gb", type=int, default=64)
    ap.add_argument("--cpu-procs", type=int, default=None)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only a 1 GiB device-to-device copy, the calibration run for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2605_29598_amd import binding as B
    from paper_2605_29598_amd import workloads as W

    if args.copy_probe:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes": n, "GB_per_s_read_plus_write": 2 * n / el / 1e9}))
        return
    if args.serve_only:
        print(json.dumps({"served": served_run(args)}))
        return

    scheme = B.IMX_R1 if args.scheme == "R1" else B.IMX_R2
    w = W.orography(scheme=scheme)
    head, ref_state, rep = run_workload(w, args, B.IMX_FP64)
    print(f"bench: {w.name} fp64 {head['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    note = (f"HIP events on the solver stream around every launch, on a replay of the {args.steps} timed steps "
            f"from their saved start state")
    traffic = measured_traffic(w.name, ["pass1", "pass2"])
    roof = roofline_of(rep, ["pass1", "pass2"], args.steps, traffic,
                       note + "; one Schur-complement apply = one pass-1 and one pass-2 launch")
    roof["limiters"] = measured_limiters(w.name, {"pass1": "k_mv1", "pass2": "k_mv2<"})
    operators = {}
    for name, cls in (("schur_apply", ["pass1", "pass2"]), ("explicit_residual", ["explicit"]),
                      ("picard_refresh", ["lambda"])):
        r = roofline_of(rep, cls, args.steps, measured_traffic(w.name, cls), note)
        operators[name] = {k: r[k] for k in ("achieved", "frac", "avg_launch_us", "algorithmic_bytes_per_launch",
                                             "launches_per_step", "traffic")}
    kern = head.pop("kernels")
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        # the paper's unit counts DoF per scalar variable (E Np): the same rate over 5 fields
        "dof_updates_per_s_per_variable": head["value"] / 5.0,
        "config": {"workload": w.name, "elements": head["elements"], "degree": head["degree"], "dofs": head["dofs"],
                   "dt": w.num.dt, "scheme": args.scheme, "precision": "fp64",
                   "gmres_restart": w.num.gmres_restart, "tolerances": [w.num.picard_tol, w.num.gmres_tol]},
        "roofline": roof,
        "operators": operators,
        "iterations_per_step": head["iterations_per_step"],
        "kernels": kern,
        "kernels_timing": head["kernels_timing"],
        "dominant_class_by_time": max(kern, key=lambda k: kern[k]["ms_per_step"]),
        "mass": head["mass"],
    }
    if not args.no_mixed:
        mixed, _, _ = run_workload(w, args, B.IMX_MIXED, ref_state=ref_state, replay=False)
        mixed["inner_tol"] = 1e-3
        mixed["dof_updates_per_s_per_variable"] = mixed["value"] / 5.0
        for k in ("elements", "degree", "dofs", "mass"):
            mixed.pop(k, None)
        out["fp32_inner"] = mixed
        print(f"bench: {w.name} fp32-inner {mixed['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    if not args.no_channel:
        wc = W.igw_channel(scheme=scheme)
        ch, _, crep = run_workload(wc, args, B.IMX_FP64)
        ch["workload"] = wc.name
        ch["schur_apply"] = roofline_of(crep, ["pass1", "pass2"], args.steps, None, note)
        ch["schur_apply"].pop("timing")
        out["igw_channel"] = ch
        print(f"bench: {wc.name} fp64 {ch['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
    if not args.no_serve:
        out["served"] = served_run(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_procs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
