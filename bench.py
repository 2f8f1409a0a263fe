"""Benchmark: IMEX-ARK2 steps of the rotating inertia-gravity-wave channel on one MI355X.

Workload: 3000x1000x10 km channel, 120x40x10 hexahedra of degree 3 (48,000
elements, 15.36 M DoF over the 5 conserved fields), N = 0.01 1/s, theta0 =
300 K, U = 20 m/s, f = 1e-4 1/s, dt = 20 s, R2 treatment, GMRES / Picard
tolerance 1e-10, binary64. A step is one whole IMEX-ARK2 step (three explicit
residuals, two implicit stages with their Picard and GMRES iterations, stage
combinations, final update and mass check) on device-resident state.

Prints one JSON line: DoF-updates/s (5 E Np per step), the roofline of the
kernel class that takes the most device time in the timed region (algorithmic
bytes / HIP-event time on the solver stream), and the CPU oracle timed on a
bounded sample of the same workload.
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


def measured_traffic(kind):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if the
    kernels have not changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    from paper_2605_29598_amd.profiling import kernel_source_hash
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kind)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(seconds_budget=30.0):
    """Oracle (plain numpy, one thread) on a 12x4x10-element piece of the same
    channel: identical element size, degree, dt, physics and tolerances."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import dg
    from oracle.mesh import Mesh as OMesh, MeshDesc
    from paper_2605_29598_amd import workloads as W

    w = W.igw_channel()
    nx, ny = 12, 4
    w.mesh.Lx, w.mesh.Ly = 3000e3 * nx / 120, 1000e3 * ny / 40
    w.mesh.nx, w.mesh.ny = nx, ny
    w.pert_xc = w.mesh.Lx / 2
    om = OMesh(MeshDesc(**vars(w.mesh)))
    q = W.initial_state(w, om.node_coords())
    ph, num = dg.Phys(**vars(w.phys)), dg.Numerics(**vars(w.num))
    steps, t_total = 0, 0.0
    with threadpool_limits(1):
        while steps < 4 and t_total < seconds_budget:
            t0 = time.perf_counter()
            q, _ = dg.ark2_step(om, ph, num, q)
            t_total += time.perf_counter() - t0
            steps += 1
    dofs = 5 * om.E * om.Np
    return {"value": dofs * steps / t_total, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} ARK2 steps of a {nx}x{ny}x10-element piece of the channel "
                      f"({om.E} elements, r=3, same dt/physics/tolerances), numpy on 1 thread, "
                      f"{t_total:.1f} s"}


def field_errors(a, b, gamma=1.4):
    """Max error per conserved field, relative to rho, p/c (momentum) and rho E scales."""
    import numpy as np
    rho = np.abs(b[0]).max()
    kin = 0.5 * (b[1] ** 2 + b[2] ** 2 + b[3] ** 2) / b[0]
    p = np.abs((gamma - 1.0) * (b[4] - kin)).max()
    c = math.sqrt(gamma * p / rho)
    scale = [rho, p / c, p / c, p / c, np.abs(b[4]).max()]
    names = ["rho", "rho_u", "rho_v", "rho_w", "rho_E"]
    return {names[t]: float(np.abs(a[t] - b[t]).max() / scale[t]) for t in range(5)}


def kernel_pass(sol, steps):
    """{class: (ms, algorithmic bytes, launches)} over `steps` further steps,
    and their GMRES iteration count."""
    import torch
    torch.cuda.synchronize()
    sol.timing(True)
    gm = 0
    for _ in range(steps):
        gm += sol.step(1).gmres_iters
    torch.cuda.synchronize()
    rep = sol.timing_report()
    sol.timing(False)
    return rep, gm


def mixed_run(w, mesh, q0, args, ref_state, dofs):
    """Same steps with the binary32 Krylov inner loop (binary64 defect
    correction to the same tolerance), timed the same way."""
    import torch
    from paper_2605_29598_amd import binding as B
    sol = B.Solver(mesh, w.phys, w.num, device="cuda:0", precision=B.IMX_MIXED, inner_tol=1e-3)
    sol.set_state(q0)
    for _ in range(args.warmup):
        sol.step(1)
    torch.cuda.synchronize()
    gm = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gm += sol.step(1).gmres_iters
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    err = field_errors(sol.get_state().cpu().numpy(), ref_state)
    rep, _ = kernel_pass(sol, args.steps)
    return {"value": dofs * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
            "gmres_inner_per_step": gm / args.steps, "inner_tol": 1e-3,
            "max_rel_error_vs_fp64": err,
            "kernels_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in rep.items() if v[2]}}


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
    e_lo, e_hi = 2000, 24000
    rate = 2.0 * ((2000 + 200000) / (e_lo + e_hi)) * (50.0 / args.serve_steps)
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
        print(f"serve: alone {r.workload.name} {dur[-1]:.2f} s", file=sys.stderr, flush=True)
    end, lat = 0.0, []
    for r, d in zip(trace, dur):
        end = max(end, r.arrival_s) + d
        lat.append(end - r.arrival_s)
    serial = {"dof_updates_per_s": total / (end - trace[0].arrival_s), "makespan_s": end - trace[0].arrival_s,
              "step_ms_p50": float(np.percentile(alone_steps, 50)), "step_ms_p99": float(np.percentile(alone_steps, 99)),
              "request_latency_s_p50": float(np.percentile(lat, 50)),
              "request_latency_s_p99": float(np.percentile(lat, 99))}

    def served(precision):
        sv = B.Server(pool_bytes=args.serve_pool_gb << 30, max_running=args.serve_slots)
        ids, i, t0 = [], 0, time.perf_counter()
        first = None
        while True:
            now = time.perf_counter() - t0
            while i < len(trace) and trace[i].arrival_s <= now:
                r = trace[i]
                ids.append((sv.submit(r.workload.mesh, r.workload.phys, r.workload.num, q0s[i], r.steps,
                                      precision=precision), time.perf_counter() - t0))
                first = first if first is not None else ids[-1][1]
                i += 1
            nr, nw = sv.tick()
            if i == len(trace) and nr == 0 and nw == 0:
                break
            time.sleep(0.0005)
        makespan = time.perf_counter() - t0 - first
        st = sv.query()
        lat, worst = [], 0.0
        for k, (rid, t_sub) in enumerate(ids):
            q, ms = sv.result(rid)
            if ms.status != B.IMX_OK:
                msg = B.lib().imx_last_error().decode(errors="replace")
                raise RuntimeError(f"served member {k} ({trace[k].workload.name}) failed with status {ms.status} "
                                   f"after {ms.steps_done} steps: {msg}")
            lat.append(1e-3 * (ms.queue_ms + ms.run_ms))
            if precision == B.IMX_FP64:
                worst = max(worst, float(np.abs(q - finals[k]).max()))
            else:
                worst = max(worst, max(field_errors(q, finals[k]).values()))
        out = {"dof_updates_per_s": total / makespan, "makespan_s": makespan,
               "step_ms_p50": st.p50_step_ms, "step_ms_p99": st.p99_step_ms,
               "request_latency_s_p50": float(np.percentile(lat, 50)),
               "request_latency_s_p99": float(np.percentile(lat, 99)),
               "pool_gb": args.serve_pool_gb, "pool_peak_gb": st.pool_bytes_peak / 2 ** 30,
               "slots": args.serve_slots, "completed": st.completed}
        if precision == B.IMX_FP64:
            out["max_abs_diff_vs_alone"] = worst
        else:
            out["max_rel_error_vs_fp64_alone"] = worst
        del sv
        print(f"serve: {'fp64' if precision == B.IMX_FP64 else 'mixed'} makespan {makespan:.2f} s",
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
    ap.add_argument("--profile-steps", action="store_true", help="print progress per step")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-ensemble run")
    ap.add_argument("--serve-only", action="store_true", help="run only the served-ensemble comparison")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-steps", type=int, default=20)
    # one running member per hardware queue of the process (HIP's default of 4):
    # 4, 8 and 12 slots give the same throughput, more slots only queue longer
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-pool-gb", type=int, default=64)
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
    w = W.igw_channel(scheme=B.IMX_R1 if args.scheme == "R1" else B.IMX_R2)
    mesh = B.Mesh(w.mesh)
    sol = B.Solver(mesh, w.phys, w.num, device="cuda:0")
    q0 = W.initial_state(w, mesh.node_coords())
    sol.set_state(q0)
    dofs = 5 * mesh.E * mesh.Np
    for i in range(args.warmup):
        sol.step(1)
        if args.profile_steps:
            print(f"warmup step {i} done", file=sys.stderr, flush=True)

    # timed region: K steps with nothing but the solver's own work queued
    torch.cuda.synchronize()
    picard = gmres = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = sol.step(1)
        picard += st.picard_iters
        gmres += st.gmres_iters
        if args.profile_steps:
            print(f"step {i}: picard {st.picard_iters} gmres {st.gmres_iters}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ref_state = sol.get_state().cpu().numpy()
    # kernel timing: the next K steps with a HIP event pair around every launch
    # on the solver's stream (the events themselves add ~7% to a step)
    rep, k_gmres = kernel_pass(sol, args.steps)

    ms_per_step = 1e3 * elapsed / args.steps
    value = dofs * args.steps / elapsed
    dom = max(rep, key=lambda k: rep[k][0])
    ms, by, n = rep[dom]
    achieved = by / (ms * 1e-3) / 1e9
    traffic = measured_traffic(dom)
    kernels = {k: {"ms_per_step": round(v[0] / args.steps, 3),
                   "GB_per_s": round(v[1] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else 0,
                   "frac_of_hbm_peak": round(v[1] / (v[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 3) if v[0] > 0 else 0,
                   "avg_launch_us": round(1e3 * v[0] / v[2], 1),
                   "launches_per_step": round(v[2] / args.steps, 1)} for k, v in rep.items() if v[2]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "elements": mesh.E, "degree": w.mesh.degree, "dofs": dofs,
                   "dt": w.num.dt, "scheme": args.scheme, "precision": "fp64",
                   "gmres_restart": w.num.gmres_restart, "tolerances": [w.num.picard_tol, w.num.gmres_tol]},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_us": 1e3 * ms / max(n, 1), "algorithmic_bytes_per_launch": by / max(n, 1),
                     "timing": f"HIP events on the solver stream around every launch, over {args.steps} steps "
                               f"following the timed ones"},
        "iterations_per_step": {"picard": picard / args.steps, "gmres": gmres / args.steps},
        "kernels": kernels,
        "mass": sol.total_mass(),
    }
    if not args.no_mixed:
        out["fp32_inner"] = mixed_run(w, mesh, q0, args, ref_state, dofs)
    if not args.no_serve:
        out["served"] = served_run(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
