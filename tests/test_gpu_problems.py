"""The two test problems of Sec. 5 on the GPU: the heat equation with its
source (eq. (heat), the source entering w through aao_set_forcing) and the
advection equation with upwind differences (eq. (advection)), against the
oracle; the moving window of Sec. 5.2 against sequential collocation.  Every
parameter set of Tables 1 and 2 runs in test_gpu_tables.py."""
import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say, torch

pytestmark = pytest.mark.gpu


def _oracle(w, u0, b):
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel, order=w.order)
    tau = oracle.radau_right_nodes(w.M)
    Q = oracle.collocation_matrix(tau)
    return op, Q, tau


def _oracle_source(w, tau):
    t = w.t0 + (np.arange(w.L)[:, None] + np.asarray(tau)[None, :]) * w.dt
    return wl.source_values(w, t)


def _solve(w, tol=None):
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    if w.source:
        p.set_forcing(dev(wl.source_values(w, p.node_times(w.t0))))
    u, info = p.solve(tol=w.tol if tol is None else tol, stop=w.stop, max_iter=50)
    return host(u), info, u0, p


HEAT = wl.WORKLOADS["heat2d_table1"]
ADV = wl.WORKLOADS["adv2d_table1"]


@pytest.mark.parametrize("name,w", [
    ("heat_24x20_o4_M2_cocg", HEAT.with_(nx=24, ny=20, L=8, tol=1e-12, inner_tol=1e-13)),
    ("heat_16_o6_M3_cocg", HEAT.with_(nx=16, ny=16, L=4, M=3, order=6, tol=1e-12, inner_tol=1e-13)),
    ("heat_32_o2_M1_fft", HEAT.with_(nx=32, ny=32, L=8, M=1, order=2, inner="fft", inner_tol=1e-15, tol=1e-12)),
    ("heat_16_o4_M2_mixed", HEAT.with_(nx=16, ny=16, L=8, precision="mixed", inner_tol=1e-6, tol=1e-10)),
])
def test_forced_heat_parity(name, w):
    need_gpu()
    say("forced heat", name)
    u, info, u0, _ = _solve(w)
    op, Q, tau = _oracle(w, u0, None)
    b = _oracle_source(w, tau)[0]
    ref = oracle.sequential_solve(op, Q, w.dt, u0[0], w.L, backend="spectral", forcing=b)
    e = rel_l2(u[0], ref)
    say("  sweeps", info["iterations"], "err %.2e" % e)
    assert e < (1e-8 if w.precision == "mixed" else 1e-10)


def test_forced_residual_matches_oracle():
    need_gpu()
    w = HEAT.with_(nx=12, ny=10, L=4, M=3, order=4)
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    frc = wl.source_values(w, p.node_times(w.t0))
    p.set_forcing(dev(frc))
    U = np.random.default_rng(5).standard_normal((1, w.L, w.M, w.N))
    r, rel = p.residual(dev(U))
    op, Q, tau = _oracle(w, u0, None)
    b = _oracle_source(w, tau)[0]
    ref = oracle.residual(op, Q, w.dt, u0[0], U[0], forcing=b)
    assert rel_l2(host(r)[0], ref) < 1e-13
    wref = oracle.assemble_w(u0[0], w.L, w.M, b, Q, w.dt)
    assert abs(rel - np.linalg.norm(ref) / np.linalg.norm(wref)) < 1e-12 * rel
    p.set_forcing(None)  # source removed: back to w = (1 (x) u0, 0, ...)
    r0, _ = p.residual(dev(U))
    assert rel_l2(host(r0)[0], oracle.residual(op, Q, w.dt, u0[0], U[0])) < 1e-13


@pytest.mark.parametrize("name,w", [
    ("adv_20_o1_M2_bicg", ADV.with_(nx=20, ny=20, L=8, order=1, tol=1e-12, inner_tol=1e-13)),
    ("adv_18x14_o3_M3_bicg", ADV.with_(nx=18, ny=14, L=4, M=3, order=3, tol=1e-12, inner_tol=1e-13)),
    ("adv_24_o5_M2_bicg", ADV.with_(nx=24, ny=24, L=8, order=5, tol=1e-12, inner_tol=1e-13)),
    ("adv_32_o4_M2_fft", ADV.with_(nx=32, ny=32, L=8, order=4, inner="fft", inner_tol=1e-15, tol=1e-12)),
])
def test_upwind_advection_parity(name, w):
    need_gpu()
    say("upwind advection", name)
    u, info, u0, _ = _solve(w)
    op, Q, _ = _oracle(w, u0, None)
    ref = oracle.sequential_solve(op, Q, w.dt, u0[0], w.L, backend="spectral")
    e = rel_l2(u[0], ref)
    say("  sweeps", info["iterations"], "err %.2e" % e)
    assert e < 1e-10


def test_moving_window_equals_sequential():
    """Four windows of L = 4 steps reproduce steps 13-16 of the sequential
    collocation solution over 16 steps (Sec. 5.2's moving window)."""
    need_gpu()
    w = wl.WORKLOADS["heat2d_256"].with_(nx=24, ny=16, L=4, tol=1e-12, inner_tol=1e-13)
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    u, infos = p.solve_windows(4, tol=w.tol, max_iter=40)
    say("windows", [i["iterations"] for i in infos])
    op, Q, _ = _oracle(w, u0, None)
    ref = oracle.sequential_solve(op, Q, w.dt, u0[0], 4 * w.L, backend="spectral")
    assert rel_l2(host(u)[0], ref[-w.L:]) < 1e-10
    # the plan's own u0 is restored: a plain solve starts from it again
    u1, _ = p.solve(tol=w.tol, max_iter=40)
    assert rel_l2(host(u1)[0], ref[:w.L]) < 1e-10
