"""Adjoint sweep (transposed all-at-once system) and gradients vs the oracle."""
import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say, torch

pytestmark = pytest.mark.gpu


def _setup(w):
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(w.M))
    return op, Q


@pytest.mark.parametrize("name,w,tol", [
    ("advdiff_16x12_L8_B2_fp64", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=16, ny=12, L=8, batch=2,
                                                                           precision="fp64", inner_tol=1e-13,
                                                                           tol=1e-13), 1e-10),
    ("advdiff_32_L16_B2_mixed", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=32, ny=32, L=16, batch=2), 1e-8),
    ("heat2d_20x16_L4_M2_cocg", wl.WORKLOADS["heat2d_256"].with_(nx=20, ny=16, L=4, M=2, tol=1e-13), 1e-10),
    # BiCGStab beyond 4096 points: the matrix-vector phases on ragged 64 x 16 tiles with A^T
    ("advdiff_130x70_L8_fp64_tiled", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=130, ny=70, L=8, batch=1,
                                                                               precision="fp64", inner_tol=1e-13,
                                                                               tol=1e-13), 1e-10),
    ("advdiff_130x70_L8_B2_mixed_tiled", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=130, ny=70, L=8, batch=2),
     1e-8),
    # the spatial-FFT inner solve with the transposed stencil's symbol; it is
    # exact, so tau (which sets Alg. 2's gamma) is the FP64 round-off level
    ("advdiff_16x12_L8_B2_fp64_fft", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=16, ny=12, L=8, batch=2,
                                                                               precision="fp64", inner="fft",
                                                                               inner_tol=1e-15, tol=1e-13), 1e-10),
    ("advdiff_32_L16_B2_mixed_fft", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=32, ny=32, L=16, batch=2,
                                                                              inner="fft"), 1e-8),
    ("advdiff_12x10_L8_fp64_fft_bluestein", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=12, ny=10, L=8, batch=1,
                                                                                      precision="fp64", inner="fft",
                                                                                      inner_tol=1e-15, tol=1e-13),
     1e-10),
])
def test_adjoint_solve_parity(name, w, tol):
    need_gpu()
    say("adjoint", name)
    p = plan_for(w)
    g = np.random.default_rng(7).standard_normal((w.batch, w.N))
    lam, info = p.adjoint_solve(dev(g), tol=1e-12 if w.precision == "fp64" else 1e-9, max_iter=40)
    lam = host(lam)
    op, Q = _setup(w)
    for b in range(w.batch):
        lo = oracle.adjoint_solve(op, Q, w.dt, g[b], w.L)
        e = rel_l2(lam[b], lo)
        say("  b", b, "sweeps", info["iterations"], "err %.2e" % e)
        assert e < tol


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_gradients_vs_oracle_and_fd(prec, tol):
    """Workload advdiff2d_512_adj at 24 x 20, L = 8, B = 2."""
    need_gpu()
    from paper_2103_12571_amd.autograd import solve_uT
    w = wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=24, ny=20, L=8, batch=2, precision=prec,
                                                 inner_tol=1e-13 if prec == "fp64" else 1e-6,
                                                 tol=1e-12 if prec == "fp64" else 1e-9)
    say("gradients", prec)
    u0 = wl.initial_batch(w)
    us = wl.target_initial_batch(w)
    # u_target: the model's final value from u0* at the workload's nu, each side with its own solver
    pt = plan_for(w)
    pt.set_u0(dev(us))
    ut_gpu = pt.solve(tol=w.tol, max_iter=50)[0][:, -1, -1, :].clone()
    op, Q = _setup(w)
    ut = np.stack([oracle.sequential_solve(op, Q, w.dt, us[b], w.L)[-1, -1] for b in range(w.batch)])
    u0_t = dev(u0).requires_grad_(True)
    nu_t = torch.tensor(w.nu, dtype=torch.float64, device="cuda", requires_grad=True)
    uT = solve_uT(u0_t, nu_t, w, tol=w.tol, adj_tol=w.tol)
    loss = 0.5 * ((uT - ut_gpu) ** 2).sum()
    loss.backward()
    gu0 = host(u0_t.grad)
    gnu = float(nu_t.grad)
    gnu_o = 0.0
    for b in range(w.batch):
        U = oracle.sequential_solve(op, Q, w.dt, u0[b], w.L)
        lam = oracle.adjoint_solve(op, Q, w.dt, U[-1, -1] - ut[b], w.L)
        g0, gn = oracle.gradients(op, Q, w.dt, U, lam)
        e = rel_l2(gu0[b], g0)
        say("  b", b, "dJ/du0 err %.2e" % e)
        assert e < tol
        gnu_o += gn
    say("  dJ/dnu gpu %.12e oracle %.12e" % (gnu, gnu_o))
    assert abs(gnu - gnu_o) < tol * abs(gnu_o)
    # central finite difference of the oracle loss in nu
    def J(nu):
        o = oracle.stencil_for(w.kind, w.nx, w.ny, nu=nu, c=w.vel)
        return sum(0.5 * np.sum((oracle.sequential_solve(o, Q, w.dt, u0[b], w.L)[-1, -1] - ut[b]) ** 2)
                   for b in range(w.batch))
    h = 1e-6 * w.nu
    fd = (J(w.nu + h) - J(w.nu - h)) / (2 * h)
    say("  dJ/dnu finite difference %.12e" % fd)
    assert abs(gnu - fd) < 1e-5 * abs(fd)


def test_set_stencil_coef_matches_fresh_plan():
    """A plan moved to another nu by aao_set_stencil_coef solves like a plan
    set up at that nu (same launches, same weights) and matches the oracle."""
    need_gpu()
    from paper_2103_12571_amd.stencil import taps_for
    w0 = wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=32, ny=16, L=8, batch=2, precision="fp64",
                                                 inner_tol=1e-13, tol=1e-13)
    w1 = w0.with_(nu=2.5e-2)
    say("set_stencil_coef", w0.nu, "->", w1.nu)
    u0 = wl.initial_batch(w0)
    pa = plan_for(w0)
    _, _, c1, d1 = taps_for(w1.kind, w1.nx, w1.ny, nu=w1.nu, vel=w1.vel)
    pa.set_stencil_coef(c1, d1)
    pa.set_u0(dev(u0))
    ua, _ = pa.solve(tol=w1.tol, max_iter=40)
    pb = plan_for(w1)
    pb.set_u0(dev(u0))
    ub, _ = pb.solve(tol=w1.tol, max_iter=40)
    assert np.array_equal(host(ua), host(ub))
    op, Q = _setup(w1)
    for b in range(w1.batch):
        ref = oracle.sequential_solve(op, Q, w1.dt, u0[b], w1.L, backend="spectral")
        assert rel_l2(host(ua)[b], ref) < 1e-10
