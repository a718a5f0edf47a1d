"""Every parameter set of Table 1 (Sec. 5.1) and Table 2 (Sec. 5.2) on the GPU.

Table 1: the heat problem (eq. (heat), with its source) and the upwind
advection problem (eq. (advection)) at the three tolerances each, solved by
the parallel method over L steps, with the exact spatial-FFT inner solve and
with the Krylov inner solve (COCG for heat, BiCGStab for advection).  The
result at T is within the set's tolerance of the exact solution and within
1e-10 (relative l2) of the oracle's sequential collocation solution.

Table 2: the same problems over 64 steps of dT = T64 / 64 as a moving window
of 4 x 16 steps.  (a) With the table's inner tolerance tilde-tau for the
Krylov inner solves (the advection sets have tilde-tau below tau), Alg. 2's
alpha and a stop at a tenth of the set's tolerance: the result is within the
tolerance of the exact solution and of the oracle.  (b) Converged with the
exact inner solve: within 1e-10 of the oracle as well.
"""
import functools

import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu

SETS = [("heat", 1e-5), ("heat", 1e-9), ("heat", 1e-12), ("adv", 1e-5), ("adv", 1e-9), ("adv", 1e-12)]
IDS = ["%s_%g" % s for s in SETS]


def _oracle_parts(w):
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel, order=w.order)
    tau = oracle.radau_right_nodes(w.M)
    return op, oracle.collocation_matrix(tau), tau


def _source(w, tau, first_step, nsteps):
    if not w.source:
        return None
    t = w.t0 + (first_step + np.arange(nsteps)[:, None] + np.asarray(tau)[None, :]) * w.dt
    return wl.source_values(w, t)[0]


@functools.lru_cache(maxsize=None)
def _oracle_solution(w, nsteps):
    """Sequential collocation over nsteps steps of w (oracle), [nsteps, M, N]."""
    op, Q, tau = _oracle_parts(w)
    u0 = wl.initial_batch(w)[0]
    return oracle.sequential_solve(op, Q, w.dt, u0, nsteps, backend="spectral",
                                   forcing=_source(w, tau, 0, nsteps))


def _plan(w):
    p = plan_for(w)
    p.set_u0(dev(wl.initial_batch(w)))
    return p


def _krylov(problem):
    return "cocg" if problem == "heat" else "bicgstab"


@pytest.mark.parametrize("inner", ["fft", "krylov"])
@pytest.mark.parametrize("problem,tol", SETS, ids=IDS)
def test_table1_parameter_set(problem, tol, inner):
    need_gpu()
    # the parallel method's inner tolerance is tighter than the sequential
    # solver's tau of the table (its error floor scales with L tau / alpha)
    tight = tol < 1e-10
    kw = dict(tol=1e-13 if tight else 1e-11)
    if inner == "fft":
        kw.update(inner="fft", inner_tol=1e-15)
    else:
        kw.update(inner=_krylov(problem), inner_tol=(1e-13 if problem == "heat" else 1e-14) if tight else
                  (1e-12 if problem == "heat" else 1e-13))
    w = wl.table1_workload(problem, tol, **kw)
    say("table 1", w.name, inner, "N", w.nx, "order", w.order, "M", w.M, "L", w.L)
    p = _plan(w)
    if w.source:
        p.set_forcing(dev(wl.source_values(w, p.node_times(w.t0))))
    u, info = p.solve(tol=w.tol, max_iter=40)
    u = host(u)[0]
    T = w.t0 + w.L * w.dt
    ex = float(np.max(np.abs(u[-1, -1] - wl.exact_solution(w, T))))
    ref = _oracle_solution(w.with_(inner="fft", inner_tol=1e-15, tol=1e-13), w.L)
    e = rel_l2(u, ref)
    say("  sweeps", info["iterations"], "alphas", ["%.2e" % a for a in info["alpha"]],
        "inner mean", ["%.0f" % v for v in info["inner_mean"]], "fails", info["inner_fail_total"],
        "| exact err %.2e oracle err %.2e" % (ex, e))
    assert info["converged"]
    assert ex < tol
    assert e < 1e-10


def _windows(w, W):
    p = _plan(w)
    tau = np.asarray(p.collocation()[0])
    src = None
    if w.source:
        src = dev(np.stack([wl.source_values(w, w.t0 + (k * w.L + np.arange(w.L)[:, None] + tau[None, :]) * w.dt)
                            for k in range(W)]))
    u, infos = p.solve_windows(W, sources=src, tol=w.tol, max_iter=40)
    return host(u)[0], infos


@pytest.mark.parametrize("problem,tol", SETS, ids=IDS)
def test_table2_windows_with_the_tables_inner_tolerance(problem, tol):
    """(a) Krylov inner solves at the table's tilde-tau, Alg. 2, stop at tol / 10."""
    need_gpu()
    L, W = 16, 4
    w = wl.table2_workload(problem, tol, L=L, inner=_krylov(problem), tol=tol / 10)
    say("table 2 (a)", w.name, "N", w.nx, "order", w.order, "M", w.M, "dT %.3g" % w.dt,
        "tilde-tau %.0e" % w.inner_tol)
    u, infos = _windows(w, W)
    T = w.t0 + W * L * w.dt
    ex = float(np.max(np.abs(u[-1, -1] - wl.exact_solution(w, T))))
    ref = _oracle_solution(w.with_(L=W * L, inner="fft", inner_tol=1e-15, tol=1e-13), W * L)[-L:]
    eo = float(np.max(np.abs(u - ref)))
    say("  sweeps per window", [i["iterations"] for i in infos], "fails", [i["inner_fail_total"] for i in infos],
        "| exact err %.2e, max err vs oracle %.2e" % (ex, eo))
    assert all(i["converged"] for i in infos)
    assert ex < tol
    # within the set's tolerance of the oracle, down to the FP64 round-off that
    # both sides carry: the stiffest set (heat, 1e-12: 350^2 points, 6th-order
    # differences, dT |lambda_max| ~ 3e3) agrees to about 2e-12 even when
    # converged with the exact inner solve (test (b))
    assert eo < max(tol, 1e-11 * float(np.max(np.abs(ref))))


@pytest.mark.parametrize("problem,tol", SETS, ids=IDS)
def test_table2_windows_converged(problem, tol):
    """(b) The exact inner solve and a tight stop: the windows reproduce the
    sequential collocation solution over 64 steps."""
    need_gpu()
    L, W = 16, 4
    w = wl.table2_workload(problem, tol, L=L, inner="fft", inner_tol=1e-15, tol=1e-13 if tol < 1e-10 else 1e-12)
    say("table 2 (b)", w.name)
    u, infos = _windows(w, W)
    T = w.t0 + W * L * w.dt
    ex = float(np.max(np.abs(u[-1, -1] - wl.exact_solution(w, T))))
    ref = _oracle_solution(w.with_(L=W * L, tol=1e-13), W * L)[-L:]
    e = rel_l2(u, ref)
    say("  sweeps per window", [i["iterations"] for i in infos], "| exact err %.2e oracle err %.2e" % (ex, e))
    assert all(i["converged"] for i in infos)
    assert ex < tol
    assert e < 1e-10
