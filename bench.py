"""Benchmark of the MCS Stokes hot path on one MI355X.

Default workload: the 32^3 x 6-tet cube at order k = 4 with lognormal
viscosity and a random smooth force, FP32 inner MINRES with FP64 iterative
refinement (the largest single-GPU configuration).  A complete solve of it
takes about 40 s, so a step there is a fixed block of complete inner MINRES
iterations on the resident condensed problem: one refinement step of
`--block` (100) inner FP32 iterations from the FP64 residual of b, followed by
the FP64 update and residual r = b - K x, i.e. the work of a solve at a
refinement cadence of one FP64 residual per `--block` inner iterations (the
complete solve needs one per ~240).  One complete solve of the same problem
runs first, untimed, and is reported in `config` (iterations, refinement
steps, t_sol, residuals).

The metric is the paper's DOF-iterations per second of the solve phase,
#D * #IT / t_sol, with #D the free dofs of V_h x hat V_h x Q_h and #IT the
MINRES iterations (inner iterations summed over refinement steps); the setup
(element matrices, condensation, smoother and multigrid setup) is done once
before the timed region (the paper separates t_sup and t_sol).

Other workloads (`--workload`) time complete solves (condensation + solve per
step), batches and the serving stream.  The default line also carries the
16^3 k = 3 FP64 solve as `secondary_workload`.

Prints one JSON line.  Extra objects:
  roofline      the coloured block Gauss-Seidel phase kernel (the dominant
                kernel): algorithmic bytes per launch / its average launch
                duration, timed live with HIP events around the launches of
                sampled sweep calls inside the timed steps (mcs_timer_*),
                against 8 TB/s HBM; the byte count of the packed-storage model
                is given beside it (`model_packed`).
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded sample of
                the same workload recipe (a smaller cube, one complete MINRES
                solve), with all host cores and with one thread.
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
    # name: (workload key in workloads.py, precision, description, solve tolerance)
    "cube32_k4_mixed": ("cube32_k4_lognormal", 1, "unit cube 32^3 x 6 tets (196,608), k=4, lognormal nu (1e3 "
                        "contrast), random smooth f, FP32 inner MINRES + FP64 refinement, tol 1e-8", 1e-8),
    "cube16_k3": ("cube16_k3", 0, "unit cube 16^3 x 6 tets (24,576), k=3, nu=1, curl of 8 random sin^2 modes, FP64, "
                  "tol 1e-10", 1e-10),
    "cube32_k4_fp64": ("cube32_k4_lognormal", 0, "unit cube 32^3 x 6 tets (196,608), k=4, lognormal nu (1e3 "
                       "contrast), random smooth f, FP64, tol 1e-10", 1e-10),
    "square8_k2": ("square8_k2", 0, "unit square 8x8 x 2 triangles, k=2, nu=1, FP64, tol 1e-10", 1e-10),
    "cube64_k1": ("cube64_k1", 0, "unit cube 64^3 x 6 tets (1,572,864), lowest order k=1 (H(div) omega, Sec. 7), "
                               "nu=1, curl of 8 random sin^2 modes, FP64, tol 1e-10", 1e-10),
    "cube16_k3_additive": ("cube16_k3", 0, "unit cube 16^3 x 6 tets (24,576), k=3, nu=1, curl of 8 random sin^2 "
                                           "modes, FP64, tol 1e-10; additive auxiliary-space preconditioner with the "
                                           "facet block-Jacobi smoother", 1e-10),
    "channel_k3": ("channel_k3", 0, "plane channel 4 x 1 x 1 (40 x 10 x 10 cells x 6 tets = 24,000), k=3, nu=1e-3, "
                                    "parabolic profile as Dirichlet data on the inlet and z = 0, 1, no-slip plates, "
                                    "outlet Gamma_NT at x = 4, FP64, tol 1e-10", 1e-10),
    "channel_k1": ("channel_k1", 0, "plane channel 4 x 1 x 1 (160 x 40 x 40 cells x 6 tets = 1,536,000), lowest order "
                                    "k=1 (H(div) omega, Sec. 7), nu=1e-3, parabolic profile as Dirichlet data on the "
                                    "inlet and z = 0, 1, no-slip plates, outlet Gamma_NT at x = 4, FP64, tol 1e-10",
                   1e-10),
    "cube16_k3_l1": ("cube16_k3", 0, "unit cube 16^3 x 6 tets (24,576), k=3, nu=1, curl of 8 random sin^2 modes, "
                                     "FP64, tol 1e-10; multiplicative auxiliary-space preconditioner with facet block "
                                     "l1-Jacobi sweeps (no colour phases)", 1e-10),
    "cube32_k4_mixed_l1": ("cube32_k4_lognormal", 1, "unit cube 32^3 x 6 tets (196,608), k=4, lognormal nu (1e3 "
                           "contrast), random smooth f, FP32 inner MINRES + FP64 refinement, tol 1e-8; facet block "
                           "l1-Jacobi sweeps", 1e-8),
    "cube16_k3_full": ("cube16_k3", 0, "unit cube 16^3 x 6 tets (24,576), k=3, nu=1, curl of 8 random sin^2 modes, "
                                       "FP64, tol 1e-10; full-system auxiliary-space preconditioner (overlapping "
                                       "facet blocks on A, no bubble factorisation in the preconditioner)", 1e-10),
    "serve": ("serve", 1, "serving stream: requests on unit cubes of T ~ logU[1e3, 2e5] tets (n = max(2, "
                          "round((T/6)^(1/3)))), k uniform in {2,3,4,5}, per-tet lognormal nu clipped to 1e3 contrast, "
                          "random smooth forces, tol 1e-8, FP32 inner + FP64 refinement; closed-loop saturation "
                          "first, then Poisson arrivals at 0.7 x the saturated rate; continuous batching under an "
                          "HBM arena budget", 1e-8),
    "batch256_mixed": ("batch", 1, "batch of 256 unit-cube problems, n^3 x 6 tets with n = round(exp(U[ln 4, ln 16])), "
                                   "k uniform in {2,3,4}, nu = exp(N(0, 0.5^2)) per problem, random smooth forces; "
                                   "FP32 inner MINRES + FP64 refinement per problem, tol 1e-8; iterations of all "
                                   "groups replayed from one captured HIP graph", 1e-8),
}


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (calibrated against a plain copy), or None when no record
    covers this kernel and workload or the kernel source changed since."""
    import glob
    import hashlib
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


def host_cpu():
    """(logical CPUs the process may use, CPU model name from lscpu)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return n, model


def cpu_baseline(key="cube32_k4_lognormal", n=2, tol=1e-10):
    """Time the oracle (as it stands) on a bounded sample in a child process:
    the workload recipe `key` on the n^3 x 6-tet cube, one complete FP64 MINRES
    solve at `tol` (setup untimed), once with the BLAS thread pools at the
    host's thread share (OMP_NUM_THREADS if set, else all logical CPUs) and
    once with one thread.  Returns the cpu_baseline object (the all-thread run;
    the one-thread run beside it)."""
    nproc, model = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc) or nproc)
    code = r"""
import sys, time, json
sys.path.insert(0, %r)
import numpy as np, workloads as W
from threadpoolctl import threadpool_limits
from oracle.system import GlobalSystem
from oracle.precond import Preconditioner
from oracle.minres import minres
wl = W.workload(%r, n=%d)
m = wl["mesh"]
gs = GlobalSystem(m.vertices, m.elements, wl["nu"], wl["k"], wl["f_lattice"])
pc = Preconditioner(gs, m.lattice)
K = gs.assemble_K(); b = gs.assemble_rhs()
out = {"ndof": gs.n_dof, "tets": int(m.n_elements), "k": int(wl["k"])}
for label, th in (("all", %d), ("one", 1)):
    with threadpool_limits(th):
        t = time.perf_counter()
        x, info = minres(lambda v: K @ v, pc.apply, b, tol=%r, max_it=3000)
        out[label] = {"its": info["iterations"], "t": time.perf_counter() - t, "threads": th}
print(json.dumps(out))
""" % (ROOT, key, n, threads, tol)
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), OPENBLAS_NUM_THREADS=str(threads),
               MKL_NUM_THREADS=str(threads))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)
    if out.returncode != 0:
        return {"value": None, "unit": "DOF-iterations/s", "cores": threads, "kind": "oracle",
                "sample": "failed: " + out.stderr[-300:]}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    a, o = r["all"], r["one"]
    return {"value": r["ndof"] * a["its"] / a["t"], "unit": "DOF-iterations/s", "cores": a["threads"],
            "kind": "oracle",
            "sample": f"FP64 oracle, one complete preconditioned MINRES solve to tol {tol:g} ({a['its']} iterations, "
                      f"{a['t']:.1f} s) on the {n}^3 x 6-tet cube of the same recipe ({r['tets']} tets, "
                      f"k={r['k']}, {r['ndof']} dofs); setup not timed",
            "host_logical_cpus": nproc, "host_cpu_model": model,
            "one_thread": {"value": r["ndof"] * o["its"] / o["t"], "iterations": o["its"], "seconds": o["t"]}}


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
                   "arena_gib": args.serve_arena_gb, "arena_peak_gib": st["arena_peak"] / (1 << 30),
                   "max_inflight": args.serve_inflight, "batches": st["batches"]},
        "roofline": None,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def smooth_bytes_per_facet(nfb, nd, w):
    """Algorithmic bytes of one facet block of the colour phase kernel (the
    count its device counters use): the facet's rows of A^d of both
    neighbours, the packed D_F^{-1}, the vectors and the facet record."""
    return (2 * nfb * nd + nfb * (nfb + 1) // 2 + 4 * nd + 5 * nfb) * w + 16


def roofline(pb, timed, kern, name, t_sol_ms, period, copy_gbs, read_gbs, traffic, precision):
    """Roofline object of one timed kernel: `achieved` on the kernel's own
    algorithmic byte count, and beside it (`model_packed`) the count of the
    packed-storage model (symmetric matrices read once as packed triangles:
    per sweep every element's A^d once plus every facet's D_F; per operator
    apply every element's A_T = (A^d, H, A_oo) once; vectors not counted)."""
    kms, klaunch, kbytes = timed[kern]
    avg_launch_ms = kms / klaunch
    bytes_per_launch = kbytes / klaunch
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    info = pb.info
    w = 8 if precision == 0 else 4
    dim = pb.dim
    nfb, nb = info.n_fb, info.n_bub
    nd = (dim + 1) * nfb
    ne, nff = pb.n_elements, info.n_free_facets
    if kern == "smooth":
        facets_per_launch = kbytes / smooth_bytes_per_facet(nfb, nd, w) / klaunch
        packed = facets_per_launch * (ne * w * nd * (nd + 1) / 2 / nff + w * nfb * (nfb + 1) / 2)
        model_note = ("per colour launch: (facets of the colour) x (n_e S_d / n_ff + S_D), S = w n(n+1)/2; "
                      "the kernel's own count reads the facet's full rows of A^d of both neighbours, since "
                      "a colour-ordered Gauss-Seidel sweep needs every off-diagonal facet block of A^d "
                      "twice (once in the colour phase of each of its two facets)")
    else:
        na = nb + nd
        packed = ne * w * na * (na + 1) / 2
        model_note = "per element: the packed A_T = (A^d, H, A_oo), w n_A (n_A + 1) / 2 with n_A = n_b + n_d"
    ach_p = packed / (avg_launch_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
            "avg_launch_us": round(avg_launch_ms * 1e3, 2), "launches": klaunch,
            "bytes_per_launch": int(bytes_per_launch),
            "model_packed": {"bytes_per_launch": int(packed), "achieved": round(ach_p, 1),
                             "frac": round(ach_p / HBM_PEAK_GBS, 4), "model": model_note},
            # one call in `period` is timed: the kernel's share of the solve
            # is estimated from the sampled calls scaled by the period
            "est_share_of_t_sol": round(kms * period / t_sol_ms, 4), "sample_period": period,
            "device_copy_gbs": round(copy_gbs, 1), "frac_of_device_copy": round(achieved / copy_gbs, 4),
            "device_read_gbs": round(read_gbs, 1), "frac_of_device_read": round(achieved / read_gbs, 4)}


def run_single(args, name, steps, warmup, block):
    """One problem of workload `name`.  block = 0: a step is condensation +
    complete solve.  block > 0: condensation and one complete solve first
    (reported, untimed), then a step is one refinement step of `block` inner
    iterations (see the module docstring).  Returns the JSON object."""
    import torch
    import workloads as W
    from paper_2207_08481_amd import Problem

    key, precision, desc, tol = WORKLOADS[name]
    log(f"workload {name}")
    wl = W.workload(key)
    mesh = wl["mesh"]
    k = wl["k"]
    dev = "cuda:0"
    smoother = (1 if name.endswith("_additive") else 2 if name.endswith("_full") else
                3 if name.endswith("_l1") else 0)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, k, precision=precision,
                 tol=tol, max_it=5000, autotune=1, smoother=smoother, face_bc=wl.get("face_bc")).bind(dev)
    if wl.get("g_lattice") is not None:
        pb.set_dirichlet(wl["g_lattice"])
    nu = torch.as_tensor(wl["nu"], device=dev)
    f = torch.as_tensor(wl["f_lattice"], device=dev)
    ndof = pb.n_dof
    log(f"planned: {ndof} dofs, workspace {pb.info.workspace_bytes / 1e9:.1f} GB")
    last = {}

    def condense():
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        pb.condense(nu)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def full_step():
        ts = condense()
        x, si = pb.solve(f)
        torch.cuda.synchronize()
        last["x"] = x
        log(f"step: setup {ts:.1f} ms, {si['iterations']} iterations, "
            f"solve {si['t_solve_ms']:.1f} ms, rel {si['rel_precond_residual']:.2e}")
        return ts, si

    full = None
    if block:
        t_sup = condense()
        b = pb.load(f)
        if not args.no_complete_solve:
            x, si = pb.solve_rhs(b)
            torch.cuda.synchronize()
            full = {"iterations": si["iterations"], "outer_steps": si["outer_steps"], "t_sol_ms": si["t_solve_ms"],
                    "t_sup_ms": t_sup, "tol": tol, "rel_precond_residual": si["rel_precond_residual"],
                    "rel_residual": si["rel_residual"],
                    "dof_iterations_per_s": ndof * si["iterations"] / (si["t_solve_ms"] / 1e3)}
            log(f"complete solve: setup {t_sup:.1f} ms, {si['iterations']} iterations in {si['outer_steps']} "
                f"refinement steps, solve {si['t_solve_ms']:.1f} ms, rel residual {si['rel_residual']:.2e}")
            del x
        pb.set_solve_options(0.0, block, 0.0, 1)

        def step():
            x, si = pb.solve_rhs(b, allow_max_it=True)
            torch.cuda.synchronize()
            assert si["iterations"] == block and si["status"] in (0, -5), si
            log(f"step: {si['iterations']} inner iterations + FP64 residual, solve {si['t_solve_ms']:.1f} ms")
            return 0.0, si
    else:
        step = full_step

    for _ in range(warmup):
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
    for _ in range(steps):
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
    # block steps: whole-step wall time (the timed region holds only the
    # steps); complete-solve steps: the solve phase without the condensation
    value = ndof * its / (wall if block else t_sol / 1e3)

    info = pb.info
    # the two-column colour phase serves the 3D blocks of 6, 12, 22 and (FP32)
    # 35 dofs with one facet per workgroup; two facets per workgroup and the
    # other blocks take the one-column kernel
    two_col = (pb.dim == 3 and (info.n_fb in (6, 12, 22) or (info.n_fb == 35 and precision == 1))
               and pb.launch_config(0 if precision == 0 else 1)["facets_per_block"] == 1)
    smooth_kernel = "k_smooth_y2" if two_col else "k_smooth_y"

    def roof(kern, kname):
        kfull = {"smooth": smooth_kernel, "kapply": "k_elem_apply"}[kern]
        if kern == "smooth" and smoother == 2:
            kfull = "k_full_smooth"
        return roofline(pb, timed, kern, kname, t_sol, period, copy_gbs, read_gbs,
                        measured_traffic(kfull, name, precision), precision)

    wname = "FP64" if precision == 0 else "FP32"
    kapply_name = f"k_elem_apply, {wname} (operator apply K x)"
    secondary = None
    if smoother == 0:
        # the block Gauss-Seidel colour phase dominates the multiplicative solve
        roof_main = roof("smooth", f"k_smooth_y2, {wname} (one colour of one block Gauss-Seidel sweep, two "
                                   "columns of the row block per thread)" if two_col else
                         f"k_smooth_y, {wname} (one colour of one block Gauss-Seidel sweep, one row of A^d per "
                         "thread)")
        secondary = roof("kapply", kapply_name)
    elif smoother == 2:
        roof_main = {**roof("smooth", "k_full_smooth (one colour of one overlapping block Gauss-Seidel sweep "
                                      "on A)"), "model_packed": None}
        secondary = roof("kapply", kapply_name)
    else:
        # no Gauss-Seidel phases (additive, l1): the operator apply is timed
        roof_main = roof("kapply", kapply_name)
    cfg = {"workload": desc, "n_dof": ndof, "tets": mesh.n_elements, "order": k,
           "iterations_per_step": its / steps, "t_sol_ms_per_step": t_sol / steps,
           "rel_precond_residual": infos[-1]["rel_precond_residual"],
           "smoother_launch": pb.launch_config(0 if precision == 0 else 1),
           "apply_launch": pb.apply_config(0 if precision == 0 else 1)}
    if block:
        cfg["step"] = (f"one refinement step: {block} inner FP32 MINRES iterations from the FP64 residual of b, "
                       "then the FP64 update, residual b - K x and its norm")
        cfg["complete_solve"] = full
    else:
        cfg["step"] = "mcs_condense + complete mcs_solve"
        cfg.update({"iterations_per_solve": its / steps, "t_sup_ms": t_sup / steps, "t_sol_ms": t_sol / steps,
                    "rel_residual": infos[-1]["rel_residual"], "outer_steps": infos[-1]["outer_steps"]})
    if exact_err is not None:
        cfg["error_vs_exact_solution"] = exact_err
    out = {
        "metric": "DOF-iterations/s of preconditioned MCS solve",
        "value": value,
        "unit": "DOF-iterations/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": roof_main,
    }
    if secondary:
        out["roofline_secondary"] = secondary
    pb.close()
    del pb
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube32_k4_mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--block", type=int, default=100,
                    help="cube32_k4_mixed: inner iterations per step (0: a step is a complete solve)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 16^3 k = 3 FP64 line beside the default")
    ap.add_argument("--no-complete-solve", action="store_true",
                    help="block steps without the untimed complete solve first (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (calibrates "
                         "FETCH_SIZE / WRITE_SIZE counters against a plain copy of known size)")
    ap.add_argument("--serve-requests", type=int, default=32, help="serve: open-loop requests")
    ap.add_argument("--serve-closed", type=int, default=12, help="serve: closed-loop requests")
    ap.add_argument("--serve-arena-gb", type=float, default=200.0, help="serve: HBM budget (GiB)")
    ap.add_argument("--serve-inflight", type=int, default=3, help="serve: concurrent micro-batches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no multi-GPU "
              "path (no sharding or collectives); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    key, precision, desc, tol = WORKLOADS[args.workload]
    if key == "batch":
        return run_batch(args, precision, desc)
    if key == "serve":
        return run_serve(args, precision, desc)
    block = args.block if args.workload == "cube32_k4_mixed" else 0
    out = run_single(args, args.workload, args.steps, args.warmup, block)
    if args.workload == "cube32_k4_mixed" and not args.no_secondary:
        # the 16^3 k = 3 FP64 solve beside the default line (complete solves)
        sec = run_single(args, "cube16_k3", max(1, min(args.steps, 3)), 1, 0)
        out["secondary_workload"] = {kk: sec[kk] for kk in ("value", "unit", "steps", "ms_per_step", "dtype",
                                                            "config", "roofline", "roofline_secondary")}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        if key == "cube16_k3":
            out["cpu_baseline"] = cpu_baseline("cube16_k3", n=3)
        else:
            out["cpu_baseline"] = cpu_baseline("cube32_k4_lognormal", n=2)
    print(json.dumps(out), flush=True)
    if args.copy_calib_mb:
        dev = "cuda:0"
        n = args.copy_calib_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
