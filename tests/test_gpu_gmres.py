"""Outer flexible GMRES on C u = w with C_alpha as right preconditioner
(aao_solve_gmres) against the oracle's FGMRES (the same Krylov method, with
the preconditioner applied by a sparse direct solve) and against sequential
collocation.  Shapes span several tiles and ragged tails; B = 2 checks that
the instances keep separate Krylov spaces."""
import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import binding as bd
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say, torch

pytestmark = pytest.mark.gpu


def _setup(w):
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel, order=w.order)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(w.M))
    return p, u0, op, Q


@pytest.mark.parametrize("name,w,alphas", [
    ("heat2d_12x10_L8_fixed", wl.WORKLOADS["heat2d_256"].with_(nx=12, ny=10, L=8, inner_tol=1e-14), [0.05]),
    ("heat2d_12x10_L8_varying", wl.WORKLOADS["heat2d_256"].with_(nx=12, ny=10, L=8, inner_tol=1e-14),
     [0.2, 0.05, 0.3, 0.1, 0.25, 0.15]),
    ("advdiff_10x12_L4_fixed", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=10, ny=12, L=4, batch=1, precision="fp64",
                                                                        inner_tol=1e-14), [0.1]),
])
def test_gmres_steps_match_oracle_fgmres(name, w, alphas):
    """Least-squares residual of every step vs the oracle's FGMRES with the
    same alphas (while well above round-off)."""
    need_gpu()
    say("gmres steps", name)
    p, u0, op, Q = _setup(w)
    steps = len(alphas)
    _, info = p.solve_gmres(restart=10, alphas=alphas, tol=0.0, max_steps=steps, raise_on_noconv=False)
    _, hist = oracle.gmres_solve(op, Q, w.dt, u0[0], w.L, alphas, restart=10, tol=0.0, max_steps=steps)
    say("  gpu", ["%.3e" % v for v in info["res_est"]], "oracle", ["%.3e" % v for v in hist])
    assert info["steps"] == steps
    for g, o in zip(info["res_est"], hist):
        if o > 1e-9:
            assert abs(g - o) <= 1e-6 * o, (g, o)
        else:
            assert g <= 1e-8


@pytest.mark.parametrize("name,w,restart,alphas,tol", [
    ("heat2d_48x40_L8_M2_B2_cocg", wl.WORKLOADS["heat2d_256"].with_(nx=48, ny=40, L=8, M=2, batch=2,
                                                                    inner_tol=1e-13), 10, [0.05], 1e-10),
    ("heat2d_32_L16_default_alpha", wl.WORKLOADS["heat2d_256"].with_(nx=32, ny=32, L=16, inner_tol=1e-13),
     10, None, 1e-10),
    ("adv1d_130_L32_bicgstab_restart2", wl.WORKLOADS["adv1d_4096"].with_(nx=130, L=32, inner_tol=1e-13),
     2, [0.02], 1e-10),
    ("advdiff_32_L16_B2", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=32, ny=32, L=16, batch=2, precision="fp64",
                                                                  inner_tol=1e-13), 10, [0.1], 1e-10),
    ("heat2d_64_L8_mixed", wl.WORKLOADS["heat2d_1024_mixed"].with_(nx=64, ny=64, L=8), 10, None, 1e-8),
])
def test_gmres_solution_matches_sequential(name, w, restart, alphas, tol):
    need_gpu()
    say("gmres solve", name)
    p, u0, op, Q = _setup(w)
    u, info = p.solve_gmres(restart=restart, alphas=alphas, tol=1e-12 if w.precision == "fp64" else 1e-9,
                            max_steps=120)
    u = host(u)
    errs = [rel_l2(u[b], oracle.sequential_solve(op, Q, w.dt, u0[b], w.L, backend="spectral"))
            for b in range(w.batch)]
    say("  steps", info["steps"], "cycles", info["cycles"], "res", "%.2e" % info["res_rel"],
        "inner mean", ["%.1f" % v for v in info["inner_mean"]], "err", ["%.2e" % e for e in errs])
    assert info["converged"]
    assert max(errs) <= tol
    if restart < info["steps"]:
        assert info["cycles"] >= 2


def test_gmres_argument_errors():
    need_gpu()
    w = wl.WORKLOADS["heat2d_256"].with_(nx=16, ny=16, L=4)
    p, u0, _, _ = _setup(w)
    for bad in (0, 32):
        with pytest.raises(bd.AAOError, match="EINVAL"):
            p.solve_gmres(restart=bad)
    with pytest.raises(bd.AAOError, match="EINVAL"):
        p.solve_gmres(alphas=[1.5])
    u = torch.empty(p.shape, dtype=torch.float64, device="cuda")
    info = bd.aao_gmres_info()
    import ctypes as C
    s = bd.lib().aao_solve_gmres(p._h, bd._ptr(u), 4, None, 0, 1e-10, 10, C.c_void_p(p._ws.data_ptr() + 0), 256,
                                 C.byref(info))
    assert s in (bd.AAO_EWORKSPACE, bd.AAO_EINVAL)
    # ENOCONV with the history filled
    _, info = p.solve_gmres(restart=2, alphas=[0.45], tol=1e-14, max_steps=2, raise_on_noconv=False)
    assert not info["converged"] and info["steps"] == 2


def test_gmres_fullsize_heat2d_256():
    """The bench workload (2D heat 256^2, L = 64, M = 3, COCG) solved by GMRES."""
    need_gpu()
    w = wl.WORKLOADS["heat2d_256"]
    p, u0, op, Q = _setup(w)
    u, info = p.solve_gmres(restart=10, tol=1e-12, max_steps=40)
    ref = oracle.sequential_solve(op, Q, w.dt, u0[0], w.L, backend="spectral")
    e = rel_l2(host(u)[0], ref)
    say("gmres fullsize: steps", info["steps"], "alphas", ["%.2e" % a for a in info["alpha"]],
        "res_est", ["%.1e" % r for r in info["res_est"]], "err %.2e" % e)
    assert info["converged"] and e < 1e-10
