"""Benchmark of the MCS Stokes hot path on one MI355X.

A step is one pass of the whole path on one synthetic problem that is already
resident in HBM: element matrices and static condensation, smoother / embedding
/ multigrid setup (mcs_condense), load assembly and the preconditioned MINRES
solve with pressure normalisation (mcs_solve).  The metric is the paper's
DOF-iterations per second of the solve phase, #D * #IT / t_sol, with #D the
free dofs of V_h x hat V_h x Q_h and t_sol the solve time without setup (the
paper separates t_sup and t_sol).  Setup and total times are reported beside it.

Prints one JSON line.  Extra objects:
  roofline      the coloured block Gauss-Seidel phase kernel (the dominant
                kernel): algorithmic bytes per launch / its average launch
                duration, timed live with HIP events around every launch
                inside the timed steps (mcs_timer_*), against 8 TB/s HBM.
  cpu_baseline  the FP64 oracle timed on the host on a bounded sample of the
                same workload recipe (a smaller cube, a few MINRES iterations),
                single threaded.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)

WORKLOADS = {
    # name: (workload key in workloads.py, precision, description)
    "cube16_k3": ("cube16_k3", 0, "unit cube 16^3 x 6 tets (24,576), k=3, nu=1, curl of 8 random sin^2 modes, FP64, tol 1e-10"),
    "cube32_k4_mixed": ("cube32_k4_lognormal", 1, "unit cube 32^3 x 6 tets (196,608), k=4, lognormal nu (1e3 contrast), random smooth f, FP32 inner + FP64 refinement, tol 1e-10"),
    "cube32_k4_fp64": ("cube32_k4_lognormal", 0, "unit cube 32^3 x 6 tets (196,608), k=4, lognormal nu (1e3 contrast), random smooth f, FP64, tol 1e-10"),
    "square8_k2": ("square8_k2", 0, "unit square 8x8 x 2 triangles, k=2, nu=1, FP64, tol 1e-10"),
    "cube16_k3_additive": ("cube16_k3", 0, "unit cube 16^3 x 6 tets (24,576), k=3, nu=1, curl of 8 random sin^2 modes, "
                                           "FP64, tol 1e-10; additive auxiliary-space preconditioner with the facet "
                                           "block-Jacobi smoother"),
    "channel_k3": ("channel_k3", 0, "plane channel 4 x 1 x 1 (40 x 10 x 10 cells x 6 tets = 24,000), k=3, nu=1e-3, "
                                    "parabolic profile as Dirichlet data on the inlet and z = 0, 1, no-slip plates, "
                                    "outlet Gamma_NT at x = 4, FP64, tol 1e-10"),
    "cube16_k3_full": ("cube16_k3", 0, "unit cube 16^3 x 6 tets (24,576), k=3, nu=1, curl of 8 random sin^2 modes, "
                                       "FP64, tol 1e-10; full-system auxiliary-space preconditioner (overlapping "
                                       "facet blocks on A, no bubble factorisation in the preconditioner)"),
    "serve": ("serve", 1, "serving stream: requests on unit cubes of T ~ logU[1e3, 2e5] tets (n = max(2, round((T/6)^(1/3)))), "
                          "k uniform in {2,3,4,5}, per-tet lognormal nu clipped to 1e3 contrast, random smooth forces, "
                          "tol 1e-8, FP32 inner + FP64 refinement; closed-loop saturation first, then Poisson arrivals "
                          "at 0.7 x the saturated rate; continuous batching under an HBM arena budget"),
    "batch256_mixed": ("batch", 1, "batch of 256 unit-cube problems, n^3 x 6 tets with n = round(exp(U[ln 4, ln 16])), "
                                   "k uniform in {2,3,4}, nu = exp(N(0, 0.5^2)) per problem, random smooth forces; "
                                   "FP32 inner MINRES + FP64 refinement per problem, tol 1e-8; iterations of all "
                                   "groups replayed from one captured HIP graph"),
}


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (calibrated against a plain copy), or None when no record
    covers this kernel and workload or the kernel source changed since."""
    import glob
    import hashlib
    if precision != 0:
        return None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json"))):
        rec = json.load(open(path))
        if not rec["kernel"].startswith(kernel) or workload not in rec.get("workloads", [rec.get("workload")]):
            continue
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
            return None
        return round(rec["traffic_bytes_per_launch"])
    return None


def device_copy_gbs(dev, mib=2048, reps=10):
    """Bytes moved (read + write) per second by a plain device-to-device copy
    of `mib` MiB, outside the timed region: the practical HBM rate the
    roofline fraction can be read against."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 8 / (ms / 1e3) / 1e9


def device_read_gbs(dev, mib=4096, reps=10):
    """Bytes read per second by a plain device reduction (torch sum) over `mib`
    MiB, outside the timed region: the practical rate of a read-only stream,
    against which read-dominated kernels such as the colour phase can be set."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    a.sum()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        a.sum()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a
    return n * 8 / (ms / 1e3) / 1e9


def cpu_baseline(seconds_hint=20.0):
    """Time the oracle (as it stands) on a bounded sample in a child process:
    the same cube recipe (k=3, nu=1, curl modes) on 3^3 x 6 tets, 40 MINRES
    iterations; single-threaded BLAS.  Returns the cpu_baseline object."""
    code = r'''
import sys, time, json
sys.path.insert(0, %r)
import numpy as np, workloads as W
from oracle.system import GlobalSystem
from oracle.precond import Preconditioner
from oracle.minres import minres
wl = W.workload("cube16_k3", n=3)
m = wl["mesh"]
gs = GlobalSystem(m.vertices, m.elements, wl["nu"], wl["k"], wl["f_lattice"])
pc = Preconditioner(gs, m.lattice)
K = gs.assemble_K(); b = gs.assemble_rhs()
t = time.perf_counter()
x, info = minres(lambda v: K @ v, pc.apply, b, tol=1e-30, max_it=40)
dt = time.perf_counter() - t
print(json.dumps({"ndof": gs.n_dof, "its": info["iterations"], "t": dt}))
''' % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=600)
    if out.returncode != 0:
        return {"value": None, "unit": "DOF-iterations/s", "cores": 1, "kind": "oracle",
                "sample": "failed: " + out.stderr[-300:]}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["ndof"] * r["its"] / r["t"], "unit": "DOF-iterations/s", "cores": 1,
            "kind": "oracle",
            "sample": f"FP64 oracle MINRES, {r['its']} iterations on the 3^3 x 6-tet cube of the same "
                      f"recipe (k=3, nu=1, {r['ndof']} dofs), {r['t']:.1f} s, 1 thread"}


def run_batch(args, precision, desc):
    """Batch of independent problems (mcs_batch_*): a step is condensation +
    solve of every member.  value = sum_i #D_i #IT_i / t_sol (batch wall time of
    the solve phase).  The timed steps replay the captured graph; the roofline
    of the smoother kernel comes from one more solve of the same batch with the
    kernel timer on (launch by launch)."""
    import torch
    import workloads as W
    from paper_2207_08481_amd import Batch
    log("batch members (host)")
    specs = W.batch_members(256, seed=5)
    members = [W.batch_member(sp) for sp in specs]
    dev = "cuda:0"
    b = Batch([(m["mesh"].vertices, m["mesh"].elements, m["mesh"].lattice) for m in members],
              [m["k"] for m in members], precision=precision, tol=1e-8, max_it=5000)
    log(f"planned: {b.info.n_problems} problems, {b.info.n_groups} groups, {b.info.n_dof_total} dofs, "
        f"workspace {b.info.workspace_bytes / 1e9:.1f} GB")
    b.bind(dev)
    nus = [torch.as_tensor(m["nu"], device=dev) for m in members]
    fs = [torch.as_tensor(m["f_lattice"], device=dev) for m in members]
    ndofs = [mi.n_dof for mi in b.members]

    def step():
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        b.condense(nus)
        ev1.record()
        torch.cuda.synchronize()
        xs, infos = b.solve(fs)
        bad = [i for i, inf in enumerate(infos) if inf["status"] != 0]
        its = sum(inf["iterations"] for inf in infos)
        dofits = sum(n * inf["iterations"] for n, inf in zip(ndofs, infos))
        t_sol = infos[0]["t_solve_ms"]
        log(f"step: setup {ev0.elapsed_time(ev1):.1f} ms, solve {t_sol:.1f} ms, member iterations "
            f"min {min(i['iterations'] for i in infos)} max {max(i['iterations'] for i in infos)}, "
            f"not converged {len(bad)}")
        return ev0.elapsed_time(ev1), t_sol, dofits, its, infos

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_sup = t_sol = dofits = 0.0
    its = 0
    infos = None
    for _ in range(args.steps):
        ts, tsol, di, it, infos = step()
        t_sup += ts
        t_sol += tsol
        dofits += di
        its += it
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log("roofline solve (kernel timer on)")
    b.timer_enable(True)
    b.solve(fs)
    kms, klaunch, kbytes = b.timer_read()
    b.timer_enable(False)
    avg_launch_ms = kms / max(klaunch, 1)
    bytes_per_launch = kbytes / max(klaunch, 1)
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    rel = [inf["rel_residual"] for inf in infos]
    out = {
        "metric": "DOF-iterations/s of preconditioned MCS solve",
        "value": dofits / (t_sol / 1e3),
        "unit": "DOF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_problems": b.info.n_problems, "n_dof_total": b.info.n_dof_total,
                   "groups": b.info.n_groups, "member_iterations_sum": its / args.steps,
                   "solves_per_s": b.info.n_problems / (t_sol / args.steps / 1e3),
                   "t_sup_ms": t_sup / args.steps, "t_sol_ms": t_sol / args.steps,
                   "max_rel_residual": max(rel),
                   "not_converged": sum(1 for inf in infos if inf["status"] != 0),
                   "smoother_launch_per_group": b.launch_configs(1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_smooth_y2, FP32 (one colour of one block Gauss-Seidel sweep, two columns of the "
                               "row block per thread, all groups)",
                     "avg_launch_us": round(avg_launch_ms * 1e3, 2), "launches": klaunch,
                     "bytes_per_launch": int(bytes_per_launch),
                     "note": "measured in one extra launch-by-launch solve of the same batch"},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def run_serve(args, precision, desc):
    """Serving stream (mcs_server_*).  Phase 1 (closed loop): n_closed
    requests submitted at once; saturated solves/s = n_closed / makespan.
    Phase 2 (open loop): n_open requests with Poisson arrivals at 0.7 x the
    saturated rate; value = completed solves / elapsed, with p50/p99 of the
    per-request latency (submit -> solution on the host, planning included)."""
    import threading
    import numpy as np
    import workloads as W
    from paper_2207_08481_amd import Problem, Server
    rng = np.random.default_rng(7)
    n_closed, n_open = args.serve_closed, args.serve_requests
    specs = W.serving_requests(n_closed + n_open, seed=6)
    log(f"serving: generating {len(specs)} requests (host)")
    reqs = []
    for sp in specs:
        r = W.serving_request(sp)
        m = r["mesh"]
        r["n_dof"] = Problem(m.vertices, m.elements, m.lattice, r["k"]).n_dof
        reqs.append(r)
    srv = Server(int(args.serve_arena_gb * (1 << 30)), max_inflight=args.serve_inflight, max_batch=64,
                 precision=precision, tol=1e-8, max_it=5000)

    def submit(r):
        m = r["mesh"]
        return srv.submit(m.vertices, m.elements, m.lattice, r["k"], r["nu"], r["f_lattice"])

    results = {}

    def waiter(i, rid, n_dof):
        results[i] = srv.wait(rid, n_dof)[1]
        r = results[i]
        log(f"request {i} (n={specs[i]['n']}, k={specs[i]['k']}) done: status {r['status']}, "
            f"{r['iterations']} its, batch {r['batch_size']}, latency {r['latency_ms']:.0f} ms")

    # phase 1: closed loop
    log(f"closed loop: {n_closed} requests at once")
    t0 = time.perf_counter()
    ths = []
    for i in range(n_closed):
        rid = submit(reqs[i])
        th = threading.Thread(target=waiter, args=(i, rid, reqs[i]["n_dof"]))
        th.start()
        ths.append(th)
    for th in ths:
        th.join()
    sat = n_closed / (time.perf_counter() - t0)
    log(f"saturated: {sat:.3f} solves/s")
    # phase 2: Poisson arrivals
    lam = 0.7 * sat
    log(f"open loop: {n_open} requests, Poisson rate {lam:.3f}/s")
    gaps = rng.exponential(1.0 / lam, n_open)
    t0 = time.perf_counter()
    t_next = t0
    ths = []
    for j in range(n_open):
        i = n_closed + j
        t_next += gaps[j]
        dt = t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        rid = submit(reqs[i])
        th = threading.Thread(target=waiter, args=(i, rid, reqs[i]["n_dof"]))
        th.start()
        ths.append(th)
        if (j + 1) % 8 == 0:
            log(f"submitted {j + 1}/{n_open}, completed {sum(1 for q in results if q >= n_closed)}")
    for th in ths:
        th.join()
    wall = time.perf_counter() - t0
    lat = np.array([results[n_closed + j]["latency_ms"] for j in range(n_open)])
    qms = np.array([results[n_closed + j]["queue_ms"] for j in range(n_open)])
    bsz = np.array([results[n_closed + j]["batch_size"] for j in range(n_open)])
    its = np.array([results[n_closed + j]["iterations"] for j in range(n_open)])
    ndof = np.array([reqs[n_closed + j]["n_dof"] for j in range(n_open)])
    ok = sum(1 for j in range(n_open) if results[n_closed + j]["status"] == 0)
    st = srv.stats()
    srv.close()
    out = {
        "metric": "solves/s of served MCS solves (p50/p99 latency beside)",
        "value": n_open / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": n_open,
        "warmup": n_closed,
        "ms_per_step": wall * 1e3 / n_open,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "requests_open_loop": n_open, "requests_closed_loop": n_closed,
                   "saturated_solves_per_s": sat, "arrival_rate_per_s": lam,
                   "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
                   "queue_ms_p50": float(np.percentile(qms, 50)), "mean_batch_size": float(bsz.mean()),
                   "dof_iterations_per_s": float((ndof * its).sum() / wall), "converged": ok,
                   "arena_gb": args.serve_arena_gb, "arena_peak_gb": st["arena_peak"] / 1e9,
                   "max_inflight": args.serve_inflight, "batches": st["batches"]},
        "roofline": None,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube16_k3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (calibrates "
                         "FETCH_SIZE / WRITE_SIZE counters against a plain copy of known size)")
    ap.add_argument("--serve-requests", type=int, default=32, help="serve: open-loop requests")
    ap.add_argument("--serve-closed", type=int, default=12, help="serve: closed-loop requests")
    ap.add_argument("--serve-arena-gb", type=float, default=200.0, help="serve: HBM budget (GB)")
    ap.add_argument("--serve-inflight", type=int, default=3, help="serve: concurrent micro-batches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no multi-GPU "
              "path (no sharding or collectives); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2207_08481_amd import Problem

    key, precision, desc = WORKLOADS[args.workload]
    log(f"workload {args.workload}")
    if key == "batch":
        return run_batch(args, precision, desc)
    if key == "serve":
        return run_serve(args, precision, desc)
    wl = W.workload(key)
    mesh = wl["mesh"]
    k = wl["k"]
    dev = "cuda:0"
    smoother = 1 if args.workload.endswith("_additive") else 2 if args.workload.endswith("_full") else 0
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, k, precision=precision,
                 tol=1e-10, max_it=5000, autotune=1, smoother=smoother, face_bc=wl.get("face_bc")).bind(dev)
    if wl.get("g_lattice") is not None:
        pb.set_dirichlet(wl["g_lattice"])
    nu = torch.as_tensor(wl["nu"], device=dev)
    f = torch.as_tensor(wl["f_lattice"], device=dev)
    ndof = pb.n_dof
    log(f"planned: {ndof} dofs, workspace {pb.info.workspace_bytes / 1e9:.1f} GB")

    def step():
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        pb.condense(nu)
        ev1.record()
        x, si = pb.solve(f)
        torch.cuda.synchronize()
        last["x"] = x
        log(f"step: setup {ev0.elapsed_time(ev1):.1f} ms, {si['iterations']} iterations, "
            f"solve {si['t_solve_ms']:.1f} ms, rel {si['rel_precond_residual']:.2e}")
        return ev0.elapsed_time(ev1), si

    last = {}

    for _ in range(args.warmup):
        step()
    # kernel timer over the timed steps, sampling one sweep call and one
    # operator apply in eight so that its event records barely slow the solve
    period = 8
    pb.timer_enable(True, period=period)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_sup = t_sol = 0.0
    its = 0
    infos = []
    for _ in range(args.steps):
        ts, si = step()
        t_sup += ts
        t_sol += si["t_solve_ms"]
        its += si["iterations"]
        infos.append(si)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed = {kern: pb.timer_read(kern) for kern in ("smooth", "kapply")}
    pb.timer_enable(False)

    exact_err = None
    if key == "channel_k3":
        # the channel flow lies in the discrete spaces: point values of the
        # solution (with the lifted inflow data) against the exact one
        import numpy as np
        sol = wl["solution"]
        pts = np.random.default_rng(1).dirichlet(np.ones(4), size=3)
        u, p = pb.eval(last["x"], pts)
        X = np.einsum("pj,ejr->epr", pts, mesh.vertices[mesh.elements])
        exact_err = {"u_max_abs": float(np.abs(u.cpu().numpy() - sol.u(X)).max()),
                     "p_max_abs": float(np.abs(p.cpu().numpy() - sol.p(X)).max())}

    copy_gbs = device_copy_gbs(dev)
    read_gbs = device_read_gbs(dev)
    value = ndof * its / (t_sol / 1e3)

    def roof(kern, name, traffic):
        kms, klaunch, kbytes = timed[kern]
        avg_launch_ms = kms / klaunch
        bytes_per_launch = kbytes / klaunch
        achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
                "avg_launch_us": round(avg_launch_ms * 1e3, 2), "launches": klaunch,
                "bytes_per_launch": int(bytes_per_launch),
                # one call in `period` is timed: the kernel's share of the solve
                # is estimated from the sampled calls scaled by the period
                "est_share_of_t_sol": round(kms * period / t_sol, 4), "sample_period": period,
                "device_copy_gbs": round(copy_gbs, 1), "frac_of_device_copy": round(achieved / copy_gbs, 4),
                "device_read_gbs": round(read_gbs, 1), "frac_of_device_read": round(achieved / read_gbs, 4)}

    kapply_name = "k_elem_apply (operator apply K x)"
    if smoother == 0:
        # the block Gauss-Seidel colour phase dominates the multiplicative solve
        # every bench mesh is 3D with k <= 4: the two-column colour phase
        roofline = roof("smooth", "k_smooth_y2 (one colour of one block Gauss-Seidel sweep, two columns of the "
                        "row block per thread)", measured_traffic("k_smooth_y2", args.workload, precision))
        secondary = roof("kapply", kapply_name, measured_traffic("k_elem_apply", args.workload, precision))
    elif smoother == 2:
        # overlapping block Gauss-Seidel on the whole velocity block
        roofline = roof("smooth", "k_full_smooth (one colour of one overlapping block Gauss-Seidel sweep on A)",
                        measured_traffic("k_full_smooth", args.workload, precision))
        secondary = roof("kapply", kapply_name, measured_traffic("k_elem_apply", args.workload, precision))
    else:
        # no Gauss-Seidel phases: the operator apply is the largest kernel
        roofline = roof("kapply", kapply_name, measured_traffic("k_elem_apply", args.workload, precision))
        secondary = None
    out = {
        "metric": "DOF-iterations/s of preconditioned MCS solve",
        "value": value,
        "unit": "DOF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_dof": ndof, "tets": mesh.n_elements, "order": k,
                   "iterations_per_solve": its / args.steps,
                   "t_sup_ms": t_sup / args.steps, "t_sol_ms": t_sol / args.steps,
                   "rel_precond_residual": infos[-1]["rel_precond_residual"],
                   "rel_residual": infos[-1]["rel_residual"],
                   "outer_steps": infos[-1]["outer_steps"],
                   "smoother_launch": pb.launch_config(0 if precision == 0 else 1)},
        "roofline": roofline,
    }
    if exact_err is not None:
        out["config"]["error_vs_exact_solution"] = exact_err
    if secondary:
        out["roofline_secondary"] = secondary
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    if args.copy_calib_mb:
        n = args.copy_calib_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
