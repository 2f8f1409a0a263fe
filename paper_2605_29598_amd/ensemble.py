"""Served ensembles on the library's server (imx_server_*).

A trace of requests (workloads.served_trace: Poisson arrivals, IGW channel
and orography members of different sizes and degrees) is submitted at its
arrival times to one server whose pool is the HBM budget; the server admits
members as slots and memory free up and advances them concurrently. Reported:
aggregate DoF-updates/s over the makespan, p50/p99 step latency, request
latency (queue + run), pool use. For comparison each member can also be run
alone through a plain solver.

    python -m paper_2605_29598_amd.ensemble serve [--precision fp64|mixed] [--requests 64] [--steps 50]
    python -m paper_2605_29598_amd.ensemble alone [--requests 64] [--steps 3]
    python -m paper_2605_29598_amd.ensemble graphs-ab --requests 24 --elem-max 24000 --steps 20 --pool-gb 64

`graphs-ab` serves the trace four times in one process, alternating direct
launches and Krylov-chunk graph replay, and checks that the final states are
bitwise equal.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import workloads as W


def scaled_rate(elem_min, elem_max, steps):
    """Arrival rate of a trace scaled down from the full ensemble (elements
    uniform in 2k-200k, 50 steps, arrivals at 2/s): scaled up by the same factor
    as the work per member, so that the offered load relative to the work is
    the same."""
    return 2.0 * ((2000 + 200000) / (elem_min + elem_max)) * (50.0 / steps)


def prepare(trace, log=None):
    """Node coordinates and initial states of every member (host)."""
    from . import binding as B
    q0s, dofs = [], []
    for k, r in enumerate(trace):
        m = B.Mesh(r.workload.mesh)
        q0s.append(W.initial_state(r.workload, m.node_coords()))
        dofs.append(5 * m.E * m.Np)
        del m
        if log:
            print(json.dumps({"prepared": k, "member": r.workload.name, "dofs": dofs[-1]}), file=log, flush=True)
    return q0s, dofs


def serve(trace, q0s, dofs, precision, pool_gb, slots, log=None, graphs=False):
    """Submits every request at its arrival time and ticks the server until
    all are done; returns the aggregate figures and the final states. With
    `graphs` the members replay their Krylov chunks from HIP graphs."""
    from . import binding as B
    total = float(sum(d * r.steps for d, r in zip(dofs, trace)))
    sv = B.Server(pool_bytes=int(pool_gb) << 30, max_running=slots)
    sv.set_graphs(graphs)
    ids, i, t0, first, done = [], 0, time.perf_counter(), None, set()
    while True:
        now = time.perf_counter() - t0
        while i < len(trace) and trace[i].arrival_s <= now:
            r = trace[i]
            rid = sv.submit(r.workload.mesh, r.workload.phys, r.workload.num, q0s[i], r.steps, precision=precision)
            ids.append((rid, time.perf_counter() - t0))
            first = first if first is not None else ids[-1][1]
            i += 1
        nr, nw = sv.tick()
        if log:
            st = sv.query()
            if st.completed > len(done):
                done = set(range(st.completed))
                print(json.dumps({"t_s": round(time.perf_counter() - t0, 2), "completed": st.completed,
                                  "running": nr, "waiting": nw,
                                  "pool_in_use_gb": round(st.pool_bytes_in_use / 2 ** 30, 2)}), file=log, flush=True)
        if i == len(trace) and nr == 0 and nw == 0:
            break
        time.sleep(0.0005)
    makespan = time.perf_counter() - t0 - first
    st = sv.query()
    lat, finals, status = [], [], []
    for k, (rid, t_sub) in enumerate(ids):
        q, ms = sv.result(rid)
        status.append(int(ms.status))
        if ms.status != B.IMX_OK:
            msg = B.lib().imx_server_last_error(sv.h).decode(errors="replace")
            raise RuntimeError(f"served member {k} ({trace[k].workload.name}) failed with status {ms.status} "
                               f"after {ms.steps_done} steps: {msg}")
        lat.append(1e-3 * (ms.queue_ms + ms.run_ms))
        finals.append(q)
    out = {"dof_updates": total, "dof_updates_per_s": total / makespan, "makespan_s": makespan,
           "step_ms_p50": st.p50_step_ms, "step_ms_p99": st.p99_step_ms,
           "request_latency_s_p50": float(np.percentile(lat, 50)),
           "request_latency_s_p99": float(np.percentile(lat, 99)),
           "pool_gb": pool_gb, "pool_peak_gb": st.pool_bytes_peak / 2 ** 30, "slots": slots,
           "completed": st.completed, "graphs": bool(graphs)}
    del sv
    return out, finals


def alone(trace, q0s, dofs, steps, warmup=1, log=None):
    """Each member alone on a plain solver: `warmup` steps, then `steps`
    timed ones; the member's rate and its serial share of the ensemble (its
    stated steps at that rate)."""
    import torch
    from . import binding as B
    rows = []
    for k, (r, q0) in enumerate(zip(trace, q0s)):
        m = B.Mesh(r.workload.mesh)
        sol = B.Solver(m, r.workload.phys, r.workload.num)
        sol.set_state(torch.from_numpy(q0).cuda())
        sol.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol.step(steps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        rows.append({"member": r.workload.name, "dofs": dofs[k], "ms_per_step": ms})
        if log:
            print(json.dumps(rows[-1]), file=log, flush=True)
        del sol, m
        torch.cuda.empty_cache()
    serial_s = sum(r.steps * row["ms_per_step"] * 1e-3 for r, row in zip(trace, rows))
    total = float(sum(d * r.steps for d, r in zip(dofs, trace)))
    return {"members": rows, "serial_seconds_of_steps": serial_s, "dof_updates_per_s_alone": total / serial_s}


def main(argv=None):
    ap = argparse.ArgumentParser(description="served ensemble at the stated shape")
    ap.add_argument("mode", choices=["serve", "alone", "graphs-ab"])
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--elem-min", type=int, default=2000)
    ap.add_argument("--elem-max", type=int, default=200000)
    ap.add_argument("--rate", type=float, default=None,
                    help="arrivals per second (default: 2/s scaled by the work per member)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--pool-gb", type=int, default=200)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--alone-steps", type=int, default=3)
    ap.add_argument("--graphs", action="store_true", help="members replay their Krylov chunks from HIP graphs")
    a = ap.parse_args(argv)
    from . import binding as B
    rate = a.rate if a.rate is not None else scaled_rate(a.elem_min, a.elem_max, a.steps)
    trace = W.served_trace(n_requests=a.requests, rate_per_s=rate, elem_min=a.elem_min, elem_max=a.elem_max,
                           steps=a.steps, seed=5)
    q0s, dofs = prepare(trace, log=sys.stdout)
    if a.mode == "graphs-ab":
        prec = B.IMX_MIXED if a.precision == "mixed" else B.IMX_FP64
        runs, ref = [], None
        for graphs in (False, True, False, True):
            out, finals = serve(trace, q0s, dofs, prec, a.pool_gb, a.slots, graphs=graphs)
            ref = finals if ref is None else ref
            out["bitwise_equal_to_first_run"] = all(np.array_equal(x, y) for x, y in zip(ref, finals))
            runs.append(out)
            print(json.dumps({k: out[k] for k in ("graphs", "dof_updates_per_s", "makespan_s", "step_ms_p50",
                                                  "step_ms_p99", "bitwise_equal_to_first_run")}), flush=True)
        out = {"runs": runs, "precision": a.precision}
    elif a.mode == "serve":
        prec = B.IMX_MIXED if a.precision == "mixed" else B.IMX_FP64
        out, _ = serve(trace, q0s, dofs, prec, a.pool_gb, a.slots, log=sys.stdout, graphs=a.graphs)
        out["precision"] = a.precision
    else:
        out = alone(trace, q0s, dofs, a.alone_steps, log=sys.stdout)
    out.update({"requests": a.requests, "steps": a.steps, "elements": [a.elem_min, a.elem_max], "rate": rate})
    print("SUMMARY " + json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
