"""Pins for the oracle's flexible GMRES on C u = w with right preconditioner
C_alpha (the Krylov alternative to Richardson): finite termination, the
minimal-residual property against an explicitly built Krylov basis, the closed
form of one GMRES(1) step, and agreement with the sequential collocation
solution."""
import numpy as np
import pytest

import oracle


def _tiny(kind="heat2d", L=2, M=2, nx=3, ny=2):
    op = oracle.stencil_for(kind, nx, ny, nu=0.2, c=(1.0, 0.5))
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(M))
    u0 = np.random.default_rng(7).standard_normal(op.N)
    return op, Q, 0.05, u0, L


def _dense(op, Q, dt, L, alpha):
    C = oracle.assemble_C(op, Q, dt, L).toarray()
    Ca = oracle.assemble_C_alpha(op, Q, dt, L, alpha).toarray()
    return C, Ca


@pytest.mark.parametrize("kind", ["heat2d", "advdiff2d"])
def test_finite_termination(kind):
    """GMRES without restart reaches the solution of an n x n system in at most
    n steps."""
    op, Q, dt, u0, L = _tiny(kind)
    n = L * Q.shape[0] * op.N
    U, hist = oracle.gmres_solve(op, Q, dt, u0, L, [0.3], restart=n, tol=1e-13, max_steps=n)
    ref = oracle.brute_force_solve(op, Q, dt, u0, L)
    assert len(hist) <= n
    assert np.max(np.abs(U - ref)) < 1e-11 * np.max(np.abs(ref))
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))  # monotone


def test_minimal_residual_over_explicit_krylov_basis():
    """After k steps from x0 the residual is min over y of ||r0 - A K_k y||,
    A = C C_alpha^{-1}, K_k = [r0, A r0, ..., A^{k-1} r0] (dense lstsq)."""
    op, Q, dt, u0, L = _tiny(L=4, nx=6, ny=5)  # C_alpha^{-1} C is I + a rank-N term: N = 30
    alpha = 0.2
    C, Ca = _dense(op, Q, dt, L, alpha)
    A = C @ np.linalg.inv(Ca)
    M = Q.shape[0]
    w = oracle.assemble_w(u0, L, M).reshape(-1)
    x0 = np.tile(u0, L * M)
    r0 = w - C @ x0
    _, hist = oracle.gmres_solve(op, Q, dt, u0, L, [alpha], restart=10, tol=0.0, max_steps=5)
    for k in range(1, 6):
        K = np.stack([np.linalg.matrix_power(A, i) @ r0 for i in range(k)], 1)
        y = np.linalg.lstsq(A @ K, r0, rcond=None)[0]
        best = np.linalg.norm(r0 - A @ K @ y) / np.linalg.norm(w)
        assert best > 1e-10  # well above round-off, where the two must agree
        # the monomial basis loses digits as k grows (its condition number
        # grows geometrically), so the reference itself is good to about 1e-7
        assert abs(hist[k - 1] - best) <= 1e-6 * best, (k, hist[k - 1], best)


def test_gmres1_step_closed_form():
    """GMRES(1): x1 = x0 + theta z, z = C_alpha^{-1} r0, theta = <C z, r0> / ||C z||^2."""
    op, Q, dt, u0, L = _tiny("advdiff2d", L=4, M=3, nx=4, ny=3)
    alpha = 0.1
    C, Ca = _dense(op, Q, dt, L, alpha)
    M = Q.shape[0]
    w = oracle.assemble_w(u0, L, M).reshape(-1)
    x0 = np.tile(u0, L * M)
    r0 = w - C @ x0
    z = np.linalg.solve(Ca, r0)
    Cz = C @ z
    x1 = x0 + (Cz @ r0) / (Cz @ Cz) * z
    U, hist = oracle.gmres_solve(op, Q, dt, u0, L, [alpha], restart=1, tol=0.0, max_steps=1)
    assert np.max(np.abs(U.reshape(-1) - x1)) < 1e-12 * np.max(np.abs(x1))
    assert abs(hist[0] - np.linalg.norm(w - C @ x1) / np.linalg.norm(w)) < 1e-12


def test_flexible_steps_minimise_over_the_preconditioned_vectors():
    """With a different alpha at every step the residual is the minimum over
    span{z_1, ..., z_k} of the vectors actually used."""
    op, Q, dt, u0, L = _tiny(L=4, nx=6, ny=5)
    M = Q.shape[0]
    C = oracle.assemble_C(op, Q, dt, L).toarray()
    w = oracle.assemble_w(u0, L, M).reshape(-1)
    x0 = np.tile(u0, L * M)
    alphas = [0.2, 0.05, 0.3, 0.1]

    def prec(v, k):
        return np.linalg.solve(oracle.assemble_C_alpha(op, Q, dt, L, alphas[k]).toarray(), v)

    x, hist, Z = oracle.fgmres(lambda v: C @ v, prec, w, x0, restart=4, tol=0.0, max_steps=4)
    Zm = np.array(Z).T
    r0 = w - C @ x0
    y = np.linalg.lstsq(C @ Zm, r0, rcond=None)[0]
    best = np.linalg.norm(r0 - C @ Zm @ y)
    assert best > 1e-10 * np.linalg.norm(w)
    assert abs(np.linalg.norm(w - C @ x) - best) <= 1e-9 * best
    assert abs(hist[-1] * np.linalg.norm(w) - best) <= 1e-9 * best


@pytest.mark.parametrize("restart", [3, 20])
def test_gmres_reaches_the_collocation_solution(restart):
    op = oracle.stencil_for("heat2d", 8, 6, nu=0.5)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(3))
    u0 = np.random.default_rng(1).standard_normal(op.N)
    L, dt = 8, 0.01
    U, hist = oracle.gmres_solve(op, Q, dt, u0, L, [0.05], restart=restart, tol=1e-13, max_steps=60)
    ref = oracle.sequential_solve(op, Q, dt, u0, L, backend="dense")
    assert hist[-1] <= 1e-13
    assert np.max(np.abs(U - ref)) < 1e-11 * np.max(np.abs(ref))
