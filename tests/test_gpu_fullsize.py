"""Parity at the full workload sizes, in the configuration bench.py times.

The oracle's per-Fourier-mode back-end solves these sizes in seconds per
instance; for the batched adjoint workload two of the eight instances are
checked against it (sampled outputs), the others through invariants.
"""
import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say, torch

pytestmark = pytest.mark.gpu


def _oracle(w):
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(w.M))
    return op, Q


def _solve(w, **kw):
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    u, info = p.solve(tol=w.tol, stop=w.stop, max_iter=50, alphas=[w.alpha] if w.alpha > 0 else None, **kw)
    return p, u0, u, info


@pytest.mark.parametrize("name,tol", [("heat2d_256", 1e-10), ("adv1d_4096", 1e-10),
                                      ("heat2d_1024_mixed", 1e-8)])
def test_fullsize_solve(name, tol):
    need_gpu()
    w = wl.WORKLOADS[name]
    say("fullsize", name, "DOF", w.dof)
    p, u0, u, info = _solve(w)
    say("  sweeps", info["iterations"], "alphas", ["%.2e" % a for a in info["alpha"]],
        "inner mean", ["%.1f" % v for v in info["inner_mean"]], "max", info["inner_max"])
    assert info["converged"]
    op, Q = _oracle(w)
    uo = oracle.sequential_solve(op, Q, w.dt, u0[0], w.L, backend="spectral")
    e = rel_l2(host(u)[0], uo)
    say("  rel l2 vs oracle %.3e" % e)
    assert e <= tol


def test_fullsize_solve_heat2d_1024_fp64():
    """The 1024^2 workload on the FP64 path (COCG, tau = 1e-9, a scalar kernel
    between passes), as bench.py times it beside the mixed path."""
    need_gpu()
    w = wl.WORKLOADS["heat2d_1024_mixed"].with_(precision="fp64", inner_tol=1e-9)
    say("fullsize heat2d_1024 fp64 DOF", w.dof)
    p, u0, u, info = _solve(w)
    say("  sweeps", info["iterations"], "inner mean", ["%.1f" % v for v in info["inner_mean"]])
    assert info["converged"]
    op, Q = _oracle(w)
    uo = oracle.sequential_solve(op, Q, w.dt, u0[0], w.L, backend="spectral")
    e = rel_l2(host(u)[0], uo)
    say("  rel l2 vs oracle %.3e" % e)
    assert e <= 1e-8


def test_fullsize_adjoint_gradients():
    """Workload advdiff2d_512_adj (B = 8, complex64 inner solves): forward
    solve, adjoint solve and gradients; instances 0 and 7 against the oracle."""
    need_gpu()
    w = wl.WORKLOADS["advdiff2d_512_adj"]
    say("fullsize adjoint DOF", w.dof)
    p, u0, u, info = _solve(w)
    say("  forward sweeps", info["iterations"], "inner mean", ["%.1f" % v for v in info["inner_mean"]])
    assert info["converged"]
    us = wl.target_initial_batch(w)
    p.set_u0(dev(us))
    ut_gpu, _ = p.solve(tol=w.tol, stop=w.stop, max_iter=50)
    ut_gpu = ut_gpu[:, -1, -1, :].clone()
    p.set_u0(dev(u0))
    g = u[:, -1, -1, :] - ut_gpu
    lam, ainfo = p.adjoint_solve(g, tol=w.tol, max_iter=50)
    say("  adjoint sweeps", ainfo["iterations"], "inner mean", ["%.1f" % v for v in ainfo["inner_mean"]])
    gu0, gnu = p.grad(u, lam)
    uh, lh, gu0h, gnuh = host(u), host(lam), host(gu0), host(gnu)
    assert np.all(np.isfinite(gu0h)) and np.all(np.isfinite(gnuh))
    op, Q = _oracle(w)
    for b in (0, w.batch - 1):
        Uo = oracle.sequential_solve(op, Q, w.dt, u0[b], w.L, backend="spectral")
        eu = rel_l2(uh[b], Uo)
        uto = oracle.sequential_solve(op, Q, w.dt, us[b], w.L, backend="spectral")[-1, -1]
        lo = oracle.adjoint_solve(op, Q, w.dt, Uo[-1, -1] - uto, w.L, backend="spectral")
        el = rel_l2(lh[b], lo)
        g0, gn = oracle.gradients(op, Q, w.dt, Uo, lo)
        eg = rel_l2(gu0h[b], g0)
        say("  b=%d  u %.2e  lambda %.2e  dJ/du0 %.2e  dJ/dnu gpu %.10e oracle %.10e" % (b, eu, el, eg, gnuh[b], gn))
        # complex64 inner solves refined by the FP64 iteration: 1e-8 relative for every result
        assert eu <= 1e-8 and el <= 1e-8 and eg <= 1e-8
        assert abs(gnuh[b] - gn) <= 1e-8 * abs(gn)
