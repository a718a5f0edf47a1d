"""Oracle pins for the source term b(t) and the operators of the two test
problems of Sec. 5 (eqs. (heat), (advection)): finite-difference weights
against textbook forms and their order of accuracy, Radau IIA collocation with
a source against exact ODE solutions (order 2M - 1 at step ends), and the two
PDEs against their exact solutions."""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def test_fd_weights_textbook_forms():
    # classical forms: (u_{j-1} - 2 u_j + u_{j+1}) / h^2, (u_j - u_{j-1}) / h,
    # (3 u_j - 4 u_{j-1} + u_{j-2}) / (2h)
    assert oracle.central_d2(2) == {-1: 1, 0: -2, 1: 1}
    assert oracle.upwind_d1(1) == {-1: -1, 0: 1}
    assert oracle.upwind_d1(2) == {-2: Fraction(1, 2), -1: -2, 0: Fraction(3, 2)}
    for k in (2, 4, 6):
        w = oracle.central_d2(k)
        assert all(w[o] == w[-o] for o in w)  # symmetric
    for k in range(1, 6):
        w = oracle.upwind_d1(k)
        assert sum(v for o, v in w.items() if o > 0) < sum(-v for o, v in w.items() if o < 0)  # upwind-heavy
        assert min(w) < 0 and len(w) == k + 1


@pytest.mark.parametrize("deriv,order,weights", [(2, k, oracle.central_d2(k)) for k in (2, 4, 6)]
                         + [(1, k, oracle.upwind_d1(k)) for k in range(1, 6)])
def test_fd_weights_order_of_accuracy(deriv, order, weights):
    """Error of the difference quotient on exp(sin x) at a fixed point falls
    like h^order."""
    x0 = 0.3
    f = lambda x: np.exp(np.sin(x))
    # exact derivatives of exp(sin x)
    d1 = np.cos(x0) * f(x0)
    d2 = (np.cos(x0) ** 2 - np.sin(x0)) * f(x0)
    exact = d1 if deriv == 1 else d2
    errs = []
    hs = [0.1 / 2 ** i for i in range(3)]
    for h in hs:
        approx = sum(float(w) * f(x0 + o * h) for o, w in weights.items()) / h ** deriv
        errs.append(abs(approx - exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > order - 0.3, (rates, errs)


def _scalar_op(lam):
    return oracle.PeriodicStencil(1, 1, {(0, 0): lam})


@pytest.mark.parametrize("M", [1, 2, 3])
def test_collocation_with_source_converges_at_order_2M_minus_1(M):
    """y' = lam y + f(t), f = cos t - lam sin t, y(0) = 1: y = sin t + e^{lam t}.
    The source enters as dT (Q (x) I) b_l with b at t_{l-1} + tau_m dT; a wrong
    node time or a missing factor breaks the superconvergence at step ends."""
    lam, T = -2.0, 1.0
    tau = oracle.radau_right_nodes(M)
    Q = oracle.collocation_matrix(tau)
    errs = []
    Ls = [8, 16, 32]
    for L in Ls:
        dt = T / L
        t = (np.arange(L)[:, None] + tau[None, :]) * dt
        b = (np.cos(t) - lam * np.sin(t))[:, :, None]
        U = oracle.sequential_solve(_scalar_op(lam), Q, dt, np.array([1.0]), L, backend="dense", forcing=b)
        errs.append(abs(U[-1, -1, 0] - (np.sin(T) + np.exp(lam * T))))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(rates) > 2 * M - 1 - 0.3, (rates, errs)


def test_forcing_backends_and_brute_force_agree():
    rng = np.random.default_rng(3)
    op = oracle.stencil_for("heat2d_central", 6, 5, nu=0.3, order=4)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(3))
    L, dt = 3, 0.02
    u0 = rng.standard_normal(op.N)
    b = rng.standard_normal((L, 3, op.N))
    ref = oracle.brute_force_solve(op, Q, dt, u0, L, forcing=b)
    for be in ("dense", "sparse", "spectral"):
        U = oracle.sequential_solve(op, Q, dt, u0, L, backend=be, forcing=b)
        assert np.max(np.abs(U - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(oracle.residual(op, Q, dt, u0, ref, forcing=b))) < 1e-11


def _heat_grid(n):
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x)
    return (np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)).reshape(-1)


def _heat_run(n, order, L, T, M=3):
    """eq. (heat) on [pi, pi + T]: u_t = Lap u + phi (8 pi^2 cos t - sin t)."""
    phi = _heat_grid(n)
    op = oracle.stencil_for("heat2d_central", n, n, nu=1.0, order=order)
    tau = oracle.radau_right_nodes(M)
    Q = oracle.collocation_matrix(tau)
    dt = T / L
    t = np.pi + (np.arange(L)[:, None] + tau[None, :]) * dt
    b = (8 * np.pi ** 2 * np.cos(t) - np.sin(t))[:, :, None] * phi[None, None, :]
    U = oracle.sequential_solve(op, Q, dt, np.cos(np.pi) * phi, L, backend="spectral", forcing=b)
    return U[-1, -1], phi


def test_heat_problem_exact_solution_reading():
    """The printed source gives u = cos(t) sin(2 pi x) sin(2 pi y) (u_t - Lap u
    = (-sin t + 8 pi^2 cos t) phi); the printed sin(t) phi does not solve the
    printed equation.  With cos(t) phi the error is the small spatial one."""
    T = 0.1
    uT, phi = _heat_run(32, 6, 16, T)
    e_cos = np.max(np.abs(uT - np.cos(np.pi + T) * phi))
    e_sin = np.max(np.abs(uT - np.sin(np.pi + T) * phi))
    assert e_cos < 1e-6
    assert e_sin > 0.5


@pytest.mark.parametrize("order", [2, 4, 6])
def test_heat_problem_spatial_order(order):
    T = 0.05
    errs = []
    for n in (8, 16):
        uT, phi = _heat_run(n, order, 8, T)
        errs.append(np.max(np.abs(uT - np.cos(np.pi + T) * phi)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.4, (rate, errs)


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_advection_problem_upwind_order(order):
    """eq. (advection): u_t + u_x + u_y = 0, exact sin(2 pi (x - t)) sin(2 pi (y - t))."""
    T, L, M = 0.02, 8, 3
    tau = oracle.radau_right_nodes(M)
    Q = oracle.collocation_matrix(tau)
    errs = []
    for n in (32, 64):
        x = np.arange(n) / n
        X, Y = np.meshgrid(x, x)
        u0 = (np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)).reshape(-1)
        exact = (np.sin(2 * np.pi * (X - T)) * np.sin(2 * np.pi * (Y - T))).reshape(-1)
        op = oracle.stencil_for("adv2d_upwind", n, n, c=(1.0, 1.0), order=order)
        U = oracle.sequential_solve(op, Q, T / L, u0, L, backend="spectral")
        errs.append(np.max(np.abs(U[-1, -1] - exact)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.4, (rate, errs)


def _adv_run(n, order, M, L, T):
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x)
    u0 = (np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)).reshape(-1)
    exact = (np.sin(2 * np.pi * (X - T)) * np.sin(2 * np.pi * (Y - T))).reshape(-1)
    op = oracle.stencil_for("adv2d_upwind", n, n, c=(1.0, 1.0), order=order)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(M))
    U = oracle.sequential_solve(op, Q, T / L, u0, L, backend="spectral")
    return np.max(np.abs(U[-1, -1] - exact))


@pytest.mark.slow
@pytest.mark.parametrize("eq,tol,N,order,M,L", [
    ("heat", 1e-5, 450, 2, 1, 32), ("heat", 1e-9, 400, 4, 2, 32), ("heat", 1e-12, 300, 6, 3, 16),
    ("adv", 1e-5, 350, 2, 2, 8), ("adv", 1e-9, 350, 4, 2, 16), ("adv", 1e-12, 600, 5, 3, 32)])
def test_table1_parameter_sets_reach_their_tolerance(eq, tol, N, order, M, L):
    """Table 1: with N points per dimension, the sequential collocation
    solution at T (heat T = 0.1 from t = pi, advection T = 1e-2) is within the
    stated tolerance of the exact solution."""
    if eq == "heat":
        uT, phi = _heat_run(N, order, L, 0.1, M)
        err = np.max(np.abs(uT - np.cos(np.pi + 0.1) * phi))
    else:
        err = _adv_run(N, order, M, L, 1e-2)
    assert err < tol, err
