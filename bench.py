"""Throughput of the alpha-circulant preconditioned Richardson sweep on one MI355X.

One step = one converged solve of the composite collocation system (Alg. 2:
u initialised to (u0, ..., u0), then sweeps of residual, alpha-scaled DFT over
the L steps with the M x M eigenbasis transform, L*M shifted spatial solves,
and the back-transform, until the stop rule holds).  The metric counts every
sweep: value = B*L*M*N * (sweeps in the timed region) / (wall time).

Prints ONE JSON line.  Default workload: 2D heat, nu = 1e-2, 256 x 256 periodic
5-point stencil, L = 64 steps of dt = 1e-3, M = 3 Radau IIA nodes, 16 seeded
Fourier modes, adaptive alpha (Alg. 2), batched COCG inner solves, FP64.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

# Algorithmic bytes per unit of work of each kernel class as the textbook
# (unfused) form of each step counts them: per complex element and inner
# iteration for the Krylov kernels, per real space-time DOF for the
# transforms; cs = bytes of one complex element of the inner solves (16 or 8),
# half-spectrum factor h = (L/2 + 1)/L on the complex terms.  The roofline's
# `achieved` uses the bytes each kernel's own algorithm must move (the
# library's statistics: e.g. 4 cs / 6 cs per element and pass for the fused
# COCG pass, which never writes s or A r); `achieved_unfused_bytes` divides
# these larger counts by the same time, a measure of the fusion, not of
# bandwidth (it can exceed the peak).
#   fwd_residual_dft_l: residual (read u 8, write r 8) + transform (read r 8,
#                       write cs h)
#   bwd_idft_l_update:  read cs h, read and write u 16
#   cocg_pass:          10 cs per element and iteration (x, r, p, s, w traffic
#                       of the two-kernel form); cocg_init 3 cs
#   bicgstab_wg:        250 / 16 cs per element and iteration
#   fft_inner:          6 cs per element in 2D (rows, columns, rows), 2 cs in 1D


def survey_bytes(name, s, w, cs):
    h = (w.L // 2 + 1) / w.L
    per = {"fwd_residual_dft_l": 24.0 + cs * h, "bwd_idft_l_update": 16.0 + cs * h,
           "cocg_pass": 10.0 * cs, "cocg_init": 3.0 * cs, "bicgstab_wg": 250.0 / 16.0 * cs}.get(name)
    return s["bytes"] if per is None else per * s["elements"]


def roofline_of(stats, w, cs):
    """The dominant kernel class of a timed run against the 8 TB/s HBM peak:
    achieved = the kernel's algorithmic bytes / its summed launch time (HIP
    events on the plan's stream); also the unfused byte count over the same
    time, and the counter traffic when a record for these sources exists."""
    if not stats:
        return None
    name, s = max(stats.items(), key=lambda kv: kv[1]["ms"])
    if s["ms"] <= 0:
        return None
    sec = s["ms"] * 1e-3
    unf = survey_bytes(name, s, w, cs)
    ach = s["bytes"] / sec / 1e9
    out = {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_for(name, w.name, w.precision),
           "launches": s["launches"], "avg_launch_us": round(1e3 * s["ms"] / s["launches"], 2),
           "bytes_per_launch": s["bytes"] / s["launches"],
           "achieved_unfused_bytes": round(unf / sec / 1e9, 1), "unfused_bytes_per_launch": unf / s["launches"],
           "share_of_kernel_time": round(s["ms"] / sum(v["ms"] for v in stats.values()), 3)}
    tr = out["traffic"]
    if tr:
        out["achieved_traffic"] = round(tr * s["launches"] / sec / 1e9, 1)
        out["frac_traffic"] = round(out["achieved_traffic"] / HBM_PEAK_GBS, 4)
    return out


def host_info():
    """CPU model and the cores this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "usable_cores": usable}


_BARRIER = None


def _pool_init(barrier):
    global _BARRIER
    _BARRIER = barrier


def _oracle_job(name):
    """One oracle solve of workload `name` in a worker process (one thread);
    returns its wall-clock start and end after all workers met at a barrier."""
    from paper_2103_12571_amd import workloads as wl
    w = wl.WORKLOADS[name]
    u0 = wl.initial_batch(w)
    _BARRIER.wait()
    t0 = time.time()
    oracle_solution(w, u0)
    return t0, time.time()


def oracle_all_cores(name, procs):
    """The oracle as it stands (one thread per process: numpy's FFTs and
    batched 3 x 3 solves do not thread) run as `procs` concurrent independent
    solves of the same workload, one per core; returns the span from the first
    start to the last end.  Spawned workers, started before this process
    touches the GPU."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    bar = ctx.Barrier(procs)
    with ctx.Pool(procs, initializer=_pool_init, initargs=(bar,)) as pool:
        spans = pool.map(_oracle_job, [name] * procs, chunksize=1)
    return max(b for _, b in spans) - min(a for a, _ in spans)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat2d_256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-speedup", action="store_true", help="skip the mixed-vs-FP64 comparison")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel events in the timed region")
    ap.add_argument("--copy-probe", action="store_true", help="only run a plain device copy (counter scale)")
    ap.add_argument("--no-gmres", action="store_true", help="skip the outer-GMRES comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (row a7) timing")
    ap.add_argument("--no-small", action="store_true", help="skip the 1D configurations (heat1d_64, adv1d_4096)")
    ap.add_argument("--all-configs", action="store_true",
                    help="also time every workload once against the oracle (adds about a minute)")
    ap.add_argument("--only", choices=["small", "speedup", "adjoint"],
                    help="run one block alone, without the oracle, and print its JSON (for profiling)")
    return ap.parse_args()


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2103_12571_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload, precision):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    for r in rec.get("records", []):
        if (r.get("kernel") == kernel and r.get("workload") == workload and r.get("precision") == precision
                and r.get("source_sha") == source_hash()):
            return r.get("bytes_per_launch")
    return None


def cpu_legs(w, u0):
    """The oracle on the host before the GPU is touched: one thread (median of
    three whole solves) and all usable cores (one concurrent solve per core,
    at most 16)."""
    ts = []
    ref = None
    for _ in range(3):
        t0 = time.perf_counter()
        ref = oracle_solution(w, u0)
        ts.append(time.perf_counter() - t0)
    host = host_info()
    procs = max(1, min(16, host["usable_cores"]))
    span = oracle_all_cores(w.name, procs)
    return {"t1": sorted(ts)[1], "procs": procs, "span": span, "host": host, "ref": ref}


def run_solves(plan, u, w, n, timing):
    import torch
    plan.reset_stats()
    plan.set_timing(timing)
    sweeps = 0
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        _, info = plan.solve(u, tol=w.tol, stop=w.stop, max_iter=50,
                             alphas=[w.alpha] if w.alpha > 0 else None)
        sweeps += info["iterations"]
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_timing(False)
    return t1 - t0, sweeps, infos, plan.stats()


def oracle_solution(w, u0):
    import numpy as np
    import oracle
    from paper_2103_12571_amd import workloads as wl
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel, order=w.order)
    tau = oracle.radau_right_nodes(w.M)
    Q = oracle.collocation_matrix(tau)
    b = None
    if w.source:
        b = wl.source_values(w, w.t0 + (np.arange(w.L)[:, None] + tau[None, :]) * w.dt)
    return np.stack([oracle.sequential_solve(op, Q, w.dt, u0[i], w.L, backend="spectral",
                                             forcing=None if b is None else b[i])
                     for i in range(w.batch)])


def speedup_block(np, torch, wl, plan_for, with_oracle):
    """Time to solution of the FP64 and the mixed (complex64 inner) paths on
    the 2D heat 1024^2, L = 32 workload, for both inner solvers (batched COCG
    and the spatial-FFT direct solve), each to its own stop rule, with the
    relative l2 error of each result against the oracle checked after."""
    base = wl.WORKLOADS["heat2d_1024_mixed"]
    # Stop rules calibrated offline (the fastest of tol in {5e-8, 2e-7, 1e-6}
    # and inner tau in {1e-9, 1e-8} (FP64) / {1e-6, 3e-7} (complex64) that
    # lands below 1e-8 relative l2; the error is checked after the fact):
    # FP64 uses Alg. 2 (COCG; the FFT solve is exact), mixed the
    # residual-relative alpha (COCG tau = 1e-6; FFT in complex64).
    paths = {
        "cocg": {"fp64": base.with_(precision="fp64", inner="cocg", inner_tol=1e-8, tol=1e-6),
                 "mixed": base.with_(precision="mixed", inner="cocg", inner_tol=1e-6, tol=2e-7)},
        "fft": {"fp64": base.with_(precision="fp64", inner="fft", inner_tol=1e-15, tol=5e-8),
                "mixed": base.with_(precision="mixed", inner="fft", inner_tol=1e-7, tol=5e-8)},
    }
    u0 = wl.initial_batch(base)
    ref = None
    res = {"workload": base.name, "dof": base.dof, "target_rel_l2": 1e-8}
    if with_oracle:
        t0 = time.perf_counter()
        ref = oracle_solution(base, u0)
        res["oracle_time_s"] = time.perf_counter() - t0
    for inner, pp in paths.items():
        out = {}
        for name, w in pp.items():
            plan = plan_for(w)
            plan.set_u0(torch.as_tensor(u0, device="cuda"))
            u = torch.empty(plan.shape, dtype=torch.float64, device="cuda")
            print("bench: %s %s path on %s" % (inner, name, w.name), file=sys.stderr, flush=True)
            run_solves(plan, u, w, 1, False)  # warm-up
            el, sw, infos, _ = run_solves(plan, u, w, 2, False)
            _, _, _, st = run_solves(plan, u, w, 1, True)  # kernel timing in a run of its own
            r = {"time_to_solution_s": el / 2, "sweeps": sw / 2, "inner_tol": w.inner_tol,
                 "dof_sweeps_per_s": w.dof * sw / el,
                 "alphas": [float("%.3e" % a) for a in infos[-1]["alpha"]],
                 "inner_iters_mean": [round(v, 1) for v in infos[-1]["inner_mean"]],
                 "inner_iters_max": infos[-1]["inner_max"],
                 "inner_fail": infos[-1]["inner_fail"],
                 "roofline": roofline_of(st, w, 16 if name == "fp64" else 8)}
            if ref is not None:
                r["rel_l2_vs_oracle"] = float(np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref))
            out[name] = r
            del plan, u
            torch.cuda.empty_cache()
        out["speedup"] = out["fp64"]["time_to_solution_s"] / out["mixed"]["time_to_solution_s"]
        res[inner] = out
    # the same comparison with the outer flexible GMRES (COCG inner, default
    # alpha from each path's inner tolerance), to a relative residual of 1e-9
    out = {}
    for name, w in (("fp64", base.with_(precision="fp64", inner="cocg", inner_tol=1e-12)),
                    ("mixed", base.with_(precision="mixed", inner="cocg", inner_tol=1e-6))):
        plan = plan_for(w)
        plan.set_u0(torch.as_tensor(u0, device="cuda"))
        u = torch.empty(plan.shape, dtype=torch.float64, device="cuda")
        print("bench: outer GMRES %s path on %s" % (name, w.name), file=sys.stderr, flush=True)
        plan.solve_gmres(u, restart=10, tol=1e-9, max_steps=40)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            _, info = plan.solve_gmres(u, restart=10, tol=1e-9, max_steps=40)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 2
        r = {"time_to_solution_s": el, "steps": info["steps"], "inner_tol": w.inner_tol,
             "alpha": float("%.3e" % info["alpha"][0]), "res_rel": info["res_rel"],
             "inner_iters_mean": [round(v, 1) for v in info["inner_mean"]]}
        if ref is not None:
            r["rel_l2_vs_oracle"] = float(np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref))
        out[name] = r
        del plan, u
        torch.cuda.empty_cache()
    out["speedup"] = out["fp64"]["time_to_solution_s"] / out["mixed"]["time_to_solution_s"]
    res["cocg_outer_gmres"] = out
    return res


def gmres_block(np, torch, w, plan, u0, ref, richardson_s):
    """The same workload solved by flexible GMRES(10) with C_alpha as right
    preconditioner (default alpha), to a relative residual of 1e-12, beside
    the Richardson time; error against the oracle when it was computed."""
    u = torch.empty(plan.shape, dtype=torch.float64, device="cuda")
    plan.solve_gmres(u, restart=10, tol=1e-12, max_steps=60)  # warm-up (workspace allocation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 3
    for _ in range(n):
        _, info = plan.solve_gmres(u, restart=10, tol=1e-12, max_steps=60)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / n
    r = {"restart": 10, "tol_rel_residual": 1e-12, "time_to_solution_s": el, "steps": info["steps"],
         "alpha": float("%.3e" % info["alpha"][0]), "res_rel": info["res_rel"],
         "inner_iters_mean": [round(v, 1) for v in info["inner_mean"]],
         "richardson_time_to_solution_s": richardson_s, "speedup_vs_richardson": richardson_s / el}
    if ref is not None:
        r["rel_l2_vs_oracle"] = float(np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref))
    return r


def adjoint_block(np, torch, wl, plan_for, with_oracle):
    """Row a7 at the adjoint workload (2D advection-diffusion 512^2, nu = 5e-3,
    v = (1, 0.5), L = 64, M = 3, B = 8, complex64 inner solves): forward solve,
    adjoint solve of C^T lambda = e_{L,M} (x) (u_{L,M} - u_target) and both
    gradients, timed to the gradients; instance 0 against the oracle.
    u_target is the final value of the same problem from a seeded u0* (each
    side with its own solver, before the timed region).  The
    same with the spatial-FFT direct inner solve (exact for this periodic
    constant-coefficient operator) under "fft_inner"."""
    w = wl.WORKLOADS["advdiff2d_512_adj"]
    u0 = wl.initial_batch(w)
    us = wl.target_initial_batch(w)
    al = [w.alpha] if w.alpha > 0 else None

    def run(wk):
        plan = plan_for(wk)
        # u_target = the model's final value from u0* (outside the timed region)
        plan.set_u0(torch.as_tensor(us, device="cuda"))
        ut_u, _ = plan.solve(tol=wk.tol, stop=wk.stop, max_iter=50, alphas=al)
        utd = ut_u[:, -1, -1, :].clone()
        del ut_u
        plan.set_u0(torch.as_tensor(u0, device="cuda"))

        def once():
            u, info = plan.solve(tol=wk.tol, stop=wk.stop, max_iter=50, alphas=al)
            lam, ainfo = plan.adjoint_solve(u[:, -1, -1, :] - utd, tol=wk.tol, max_iter=50)
            gu0, gnu = plan.grad(u, lam)
            return u, lam, gu0, gnu, info, ainfo

        print("bench: adjoint on %s (%s inner)" % (wk.name, wk.inner), file=sys.stderr, flush=True)
        once()  # warm-up
        plan.reset_stats()  # kernel timing in a run of its own
        plan.set_timing(True)
        once()
        torch.cuda.synchronize()
        plan.set_timing(False)
        st = plan.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 2
        for _ in range(n):
            u, lam, gu0, gnu, info, ainfo = once()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / n
        sw = info["iterations"] + ainfo["iterations"]
        res = {"workload": wk.name, "dof": wk.dof, "batch": wk.batch, "precision": wk.precision, "inner": wk.inner,
               "time_to_gradient_s": el, "forward_sweeps": info["iterations"], "adjoint_sweeps": ainfo["iterations"],
               "dof_sweeps_per_s": wk.dof * sw / el,
               "inner_fail": {"forward": info["inner_fail"], "adjoint": ainfo["inner_fail"]},
               "roofline": roofline_of(st, wk, 16 if wk.precision == "fp64" else 8)}
        out = (u[0].cpu().numpy(), lam[0].cpu().numpy(), gu0[0].cpu().numpy(), float(gnu[0]))
        del plan
        torch.cuda.empty_cache()
        return res, out

    res, got = run(w)
    res_fft, got_fft = run(w.with_(inner="fft"))
    if with_oracle:
        import oracle
        op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel, order=w.order)
        Q = oracle.collocation_matrix(oracle.radau_right_nodes(w.M))
        t1 = time.perf_counter()
        Uo = oracle.sequential_solve(op, Q, w.dt, u0[0], w.L, backend="spectral")
        uto = oracle.sequential_solve(op, Q, w.dt, us[0], w.L, backend="spectral")[-1, -1]
        lo = oracle.adjoint_solve(op, Q, w.dt, Uo[-1, -1] - uto, w.L, backend="spectral")
        g0, gn = oracle.gradients(op, Q, w.dt, Uo, lo)
        res["oracle_instance_time_s"] = time.perf_counter() - t1
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        for r_, (uu, ll, gg, gv) in ((res, got), (res_fft, got_fft)):
            r_["instance0_rel_l2_vs_oracle"] = {"u": rel(uu, Uo), "lambda": rel(ll, lo), "dJ_du0": rel(gg, g0),
                                                "dJ_dnu": abs(gv - gn) / abs(gn)}
    res["fft_inner"] = res_fft
    return res


def small_configs_block(np, torch, wl, plan_for, with_oracle):
    """The 1D configurations beside the headline: heat1d_64 (768 DOF, fixed
    alpha = 1e-3, relative residual 1e-12) is launch-latency bound, so it is
    reported in microseconds per sweep; adv1d_4096 (1.6 M DOF, complex
    vectors of 25 MB that stay in the 256 MB Infinity Cache) with the
    BiCGStab inner solve and with the spatial-FFT direct solve, whose
    bandwidth is "effective" (cache-resident, not HBM)."""
    out = {}
    for key, w, reps in (("heat1d_64", wl.WORKLOADS["heat1d_64"], 20),
                         ("adv1d_4096", wl.WORKLOADS["adv1d_4096"], 3),
                         ("adv1d_4096+fft", wl.WORKLOADS["adv1d_4096"].with_(inner="fft", inner_tol=1e-15), 10)):
        print("bench: config %s" % key, file=sys.stderr, flush=True)
        u0 = wl.initial_batch(w)
        plan = plan_for(w)
        plan.set_u0(torch.as_tensor(u0, device="cuda"))
        u = torch.empty(plan.shape, dtype=torch.float64, device="cuda")
        run_solves(plan, u, w, 1, False)
        best = None
        for _ in range(reps):
            el, sw, infos, _ = run_solves(plan, u, w, 1, False)
            best = el if best is None else min(best, el)
        _, _, _, st = run_solves(plan, u, w, 1, True)
        info = infos[-1]
        r = {"dof": w.dof, "inner": w.inner, "sweeps": sw, "gpu_time_to_solution_s": best,
             "us_per_sweep": round(1e6 * best / sw, 2), "dof_sweeps_per_s": w.dof * sw / best,
             "inner_iters_mean": [round(v, 1) for v in info["inner_mean"]], "inner_iters_max": info["inner_max"],
             "inner_fail": info["inner_fail"]}
        if key != "heat1d_64":
            rf = roofline_of(st, w, 16)
            if rf:
                rf["bound"] = ("instruction issue (one workgroup per system, vectors in registers and LDS; "
                               "HBM bytes are b read and x, r written once per solve)"
                               if rf["kernel"] == "bicgstab_wg" else "effective (Infinity Cache resident)")
            r["effective_bandwidth"] = rf
        if with_oracle:
            t0 = time.perf_counter()
            ref = oracle_solution(w, u0)
            r["oracle_time_s"] = time.perf_counter() - t0
            r["speedup_vs_oracle_1core"] = r["oracle_time_s"] / best
            r["rel_l2_vs_oracle"] = float(np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref))
        out[key] = r
        del plan, u
        torch.cuda.empty_cache()
    return out


def copy_bandwidth(torch):
    """GB/s of a plain 2 GiB device-to-device copy (read + write counted), the
    practical streaming ceiling on this part."""
    x = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        y.copy_(x)
    b.record()
    b.synchronize()
    gbps = 5 * 2 * x.numel() * 8 / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbps


def all_configs(np, torch, wl, plan_for):
    """Every workload once: GPU time to solution (best of 2 after a warm-up),
    sweeps, error against the oracle, and the oracle's time."""
    out = {}
    runs = []
    for name, w in wl.WORKLOADS.items():
        runs.append((name, w))
        if w.inner != "fft":  # the spatial-FFT direct inner solve on the same problem (any grid size)
            runs.append((name + "+fft", w.with_(inner="fft", inner_tol=1e-15 if w.precision == "fp64" else 1e-7)))
    for name, w in runs:
        print("bench: config %s" % name, file=sys.stderr, flush=True)
        u0 = wl.initial_batch(w)
        plan = plan_for(w)
        plan.set_u0(torch.as_tensor(u0, device="cuda"))
        if w.source:
            plan.set_forcing(torch.as_tensor(wl.source_values(w, plan.node_times(w.t0)), device="cuda"))
        u = torch.empty(plan.shape, dtype=torch.float64, device="cuda")
        run_solves(plan, u, w, 1, False)
        best = None
        for _ in range(2):
            el, sw, infos, _ = run_solves(plan, u, w, 1, False)
            best = el if best is None else min(best, el)
        t0 = time.perf_counter()
        ref = oracle_solution(w, u0)
        t_or = time.perf_counter() - t0
        out[name] = {"dof": w.dof, "precision": w.precision, "inner": w.inner, "sweeps": sw,
                     "gpu_time_to_solution_s": best, "dof_sweeps_per_s": w.dof * sw / best,
                     "rel_l2_vs_oracle": float(np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)),
                     "oracle_time_s": t_or, "speedup_vs_oracle": t_or / best}
        if w.init in ("heat_exact", "adv_exact"):
            out[name]["max_err_vs_exact"] = float(np.max(np.abs(u[0, -1, -1].cpu().numpy()
                                                               - wl.exact_solution(w, w.t0 + w.L * w.dt))))
        del plan, u
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the sweep on a single MI355X "
              "(sharding the time steps across GPUs is designed, not implemented).", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    from paper_2103_12571_amd import workloads as wl

    w = wl.WORKLOADS[args.workload]
    u0 = wl.initial_batch(w)
    cpu = None
    if not args.no_cpu_baseline and not args.copy_probe and not args.only:
        print("bench: oracle on the host (one thread, then all cores)", file=sys.stderr, flush=True)
        cpu = cpu_legs(w, u0)

    import torch
    from paper_2103_12571_amd import binding
    from paper_2103_12571_amd.stencil import plan_for

    binding.lib()
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float64, device="cuda")  # 2 GiB
        x.fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": x.numel() * 8, "copies": 3}))
        return
    if args.only:
        block = {"small": small_configs_block, "speedup": speedup_block, "adjoint": adjoint_block}[args.only]
        print(json.dumps({args.only: block(np, torch, wl, plan_for, False)}), flush=True)
        return

    plan = plan_for(w)
    u0_d = torch.as_tensor(u0, device="cuda")
    plan.set_u0(u0_d)
    u = torch.empty(plan.shape, dtype=torch.float64, device="cuda")
    print("bench: workload %s DOF=%d warmup=%d steps=%d" % (w.name, w.dof, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    if args.warmup:
        run_solves(plan, u, w, args.warmup, False)
    elapsed, sweeps, infos, stats = run_solves(plan, u, w, args.steps, not args.no_timing)
    value = w.dof * sweeps / elapsed
    print("bench: timed %.3f s, %d sweeps" % (elapsed, sweeps), file=sys.stderr, flush=True)

    # dominant kernel and its roofline
    cs = 16 if w.precision == "fp64" else 8
    roofline = roofline_of(stats, w, cs)
    if roofline is not None:
        cp = copy_bandwidth(torch)
        roofline["copy_probe_GBps"] = round(cp, 1)
        roofline["frac_of_copy"] = round(roofline["achieved"] / cp, 4)
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3), "bytes": v["bytes"],
                   "GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 and v["bytes"] > 0 else None}
               for k, v in stats.items()}

    u_gpu = u.cpu().numpy()
    last = infos[-1]
    out = {
        "metric": "space-time DOF*sweeps/s",
        "value": value,
        "unit": "DOF*sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.precision == "fp64" else "f64 outer / c64 inner",
        "data": "synthetic",
        "config": {"workload": w.name, "pde": w.kind, "nx": w.nx, "ny": w.ny, "L": w.L, "M": w.M,
                   "batch": w.batch, "dof": w.dof, "dt": w.dt, "nu": w.nu, "inner": w.inner,
                   "inner_tol": w.inner_tol, "precision": w.precision,
                   "alpha_rule": "fixed %g" % w.alpha if w.alpha > 0 else "Alg. 2",
                   "stop": w.stop, "tol": w.tol, "sweeps_per_step": sweeps / args.steps,
                   "alphas": [float("%.3e" % a) for a in last["alpha"]],
                   "inner_iters_mean": [round(v, 1) for v in last["inner_mean"]],
                   "inner_iters_max": last["inner_max"],
                   "inner_fail": last["inner_fail"]},
        "roofline": roofline,
        "kernels": kernels,
    }

    ref = None
    out["gpu_time_to_solution_s"] = elapsed / args.steps
    if cpu is not None:
        ref = cpu["ref"]
        spp = sweeps / args.steps
        out["cpu_baseline"] = {
            "value": w.dof * spp * cpu["procs"] / cpu["span"], "unit": "DOF*sweeps/s", "cores": cpu["procs"],
            "kind": "oracle",
            "sample": "%d concurrent whole solves of the workload, one per core (one thread each: the oracle's "
                      "FFTs and batched M x M solves do not thread), sequential collocation over all L steps "
                      "with per-Fourier-mode solves; %.3f s from the first start to the last end; converted "
                      "with the GPU's %.1f sweeps per solve (equal result)" % (cpu["procs"], cpu["span"], spp),
            "host": cpu["host"],
            "aggregate_s_per_solve": cpu["span"] / cpu["procs"],
            "one_core": {"value": w.dof * spp / cpu["t1"], "cores": 1, "time_to_solution_s": cpu["t1"],
                         "sample": "one whole solve, median of 3"}}
        out["parity"] = {"rel_l2_vs_oracle": float(np.linalg.norm(u_gpu - ref) / np.linalg.norm(ref))}
    if not args.no_small:
        out["small_configs"] = small_configs_block(np, torch, wl, plan_for, cpu is not None)
    if not args.no_gmres:
        print("bench: outer GMRES on %s" % w.name, file=sys.stderr, flush=True)
        out["outer_gmres"] = gmres_block(np, torch, w, plan, u0, ref, elapsed / args.steps)
    if not args.no_speedup:
        out["mixed_vs_fp64"] = speedup_block(np, torch, wl, plan_for, cpu is not None)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_block(np, torch, wl, plan_for, cpu is not None)
    if args.all_configs:
        out["configs"] = all_configs(np, torch, wl, plan_for)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
