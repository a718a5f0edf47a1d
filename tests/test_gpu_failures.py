"""Inner-solve failures and stagnation reach the caller (Sec. 3.3, Alg. 2).

The error model of Alg. 2 rests on gamma = L (3 eps + tau) ||w||, which
assumes that every shifted system met its tolerance tau; and Sec. 3.3 notes
that the difference of consecutive iterates alone can take stagnation for
convergence.  The library therefore reports, per sweep, the shifted systems
that stopped at the iteration cap or broke down, refuses Alg. 2's model exit
after a sweep with such systems, and returns AAO_ESTAGNATE when the monitored
quantity stops contracting above tol.  The failures are forced from the host
(a small iteration cap, an unreachable tolerance): every kernel still ends
normally.
"""
import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import binding as bd
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu

HEAT = wl.WORKLOADS["heat2d_256"].with_(nx=32, ny=24, L=8)


def _oracle(w, u0):
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel, order=w.order)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(w.M))
    return oracle.sequential_solve(op, Q, w.dt, u0[0], w.L, backend="spectral")


@pytest.mark.parametrize("floor", ["off", "default"])
@pytest.mark.parametrize("inner,cap", [("cocg", 2), ("bicgstab", 2)])
def test_inner_iteration_cap_is_reported(inner, cap, floor):
    """Every shifted system is capped at two iterations.  Without the inner
    floor each sweep asks for tau relative to its residual, so some systems
    fail in every sweep; with the default floor the later sweeps' systems may
    meet it within the cap, but the first sweep's cannot."""
    need_gpu()
    say("inner cap", inner, cap, "floor", floor)
    w = HEAT.with_(inner=inner)
    p = plan_for(w, inner_maxit=cap)
    if floor == "off":
        p.set_inner_floor(0.0)
    p.set_u0(dev(wl.initial_batch(w)))
    u, info = p.solve(tol=1e-10, max_iter=12, raise_on_noconv=False)
    say("  status", info["status"], "sweeps", info["iterations"], "fails", info["inner_fail"],
        "dlast", ["%.1e" % d for d in info["dlast_inf"]])
    S = w.batch * (w.L // 2 + 1) * w.M
    assert all(0 <= f <= S for f in info["inner_fail"]) and info["inner_fail"][0] > 0
    if floor == "off":
        assert all(f > 0 for f in info["inner_fail"])
    assert info["inner_fail_total"] == sum(info["inner_fail"])
    assert all(m <= cap for m in info["inner_max"]) and info["inner_max"][0] == cap
    if floor == "off":
        assert all(m == cap for m in info["inner_max"])
    if info["status"] == "AAO_OK":
        # never Alg. 2's model exit after a sweep with failed systems: the stop rule held
        assert info["converged"] and info["dlast_inf"][-1] <= 1e-10
    else:
        assert info["status"] in ("AAO_ENOCONV", "AAO_ESTAGNATE") and not info["converged"]


def test_no_failures_reported_when_every_system_converges():
    need_gpu()
    w = HEAT
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    u, info = p.solve(tol=1e-12, max_iter=20)
    say("converging solve: fails", info["inner_fail"], "max iters", info["inner_max"])
    assert info["converged"] and info["inner_fail_total"] == 0 and not any(info["inner_fail"])
    assert rel_l2(host(u)[0], _oracle(w, u0)) < 1e-10


@pytest.mark.parametrize("stop", ["laststep", "residual"])
def test_unreachable_tolerance_stagnates(stop):
    """tol below FP64 round-off: the last-step differences (or residuals)
    settle at the round-off level and stop improving; the call returns
    AAO_ESTAGNATE well before max_iter, with a result as accurate as ever."""
    need_gpu()
    w = HEAT.with_(inner="fft", inner_tol=1e-15)
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    u, info = p.solve(tol=1e-300, stop=stop, max_iter=40, raise_on_noconv=False)
    mon = info["res_rel"] if stop == "residual" else info["dlast_inf"]
    say("unreachable tol", stop, info["status"], "sweeps", info["iterations"], ["%.1e" % v for v in mon])
    assert info["status"] == "AAO_ESTAGNATE" and not info["converged"]
    assert info["iterations"] < 40
    # the last four sweeps set no new best (none below 0.99 x the smallest before them)
    assert min(mon[-4:]) >= 0.99 * min(mon[:-4])
    assert rel_l2(host(u)[0], _oracle(w, u0)) < 1e-12
    with pytest.raises(bd.AAOError) as e:
        p.solve(tol=1e-300, stop=stop, max_iter=40)
    assert e.value.status == bd.AAO_ESTAGNATE


def test_adjoint_unreachable_tolerance_stagnates():
    need_gpu()
    w = wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=16, ny=12, L=8, batch=2, precision="fp64", inner="fft",
                                                 inner_tol=1e-15)
    p = plan_for(w)
    g = np.random.default_rng(3).standard_normal((w.batch, w.N))
    with pytest.raises(bd.AAOError) as e:
        p.adjoint_solve(dev(g), tol=1e-300, max_iter=40)
    say("adjoint unreachable tol:", str(e.value)[:120])
    assert e.value.status == bd.AAO_ESTAGNATE
