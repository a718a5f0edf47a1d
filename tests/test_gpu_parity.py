"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Row a1: aao_residual vs the oracle's w - C u.  Rows a2-a4: aao_precond vs a
sparse direct solve of C_alpha (eq. (prec)).  Row a3: aao_shifted_solve vs a
sparse direct solve of I - c A.  Rows a1-a5 together: aao_solve vs sequential
collocation.  Shapes span several transform tiles and a ragged tail.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say, torch

pytestmark = pytest.mark.gpu

Q3 = None


def _oracle_op(w):
    return oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel, order=w.order)


def _Q(M):
    return oracle.collocation_matrix(oracle.radau_right_nodes(M))


CASES = [
    # name, workload, overrides (ragged N: 40 and 10x12 are not multiples of the tile)
    ("heat1d_N40_L8_M3", wl.WORKLOADS["heat1d_64"].with_(nx=40, L=8, nu=0.05), {}),
    ("heat1d_N200_L4_M2_B2", wl.WORKLOADS["heat1d_64"].with_(nx=200, L=4, M=2, batch=2), {}),
    ("heat2d_12x10_L16_M3", wl.WORKLOADS["heat2d_256"].with_(nx=12, ny=10, L=16), {}),
    ("heat2d_20x24_L1_M1", wl.WORKLOADS["heat2d_256"].with_(nx=20, ny=24, L=1, M=1), {}),
    ("adv1d_N130_L32_M3", wl.WORKLOADS["adv1d_4096"].with_(nx=130, L=32), {}),
    ("advdiff_10x12_L8_M3_B2", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=10, ny=12, L=8, batch=2,
                                                                         precision="fp64"), {}),
    ("heat2d_64x64_L2_M4", wl.WORKLOADS["heat2d_256"].with_(nx=64, ny=64, L=2, M=4), {}),
]


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("name,w,ov", CASES, ids=[c[0] for c in CASES])
def test_residual_parity(name, w, ov):
    need_gpu()
    say("residual", name)
    p = plan_for(w, inner_tol=1e-13)
    u0 = _rand((w.batch, w.N), 1)
    u = _rand((w.batch, w.L, w.M, w.N), 2)
    p.set_u0(dev(u0))
    r, nrm = p.residual(dev(u))
    r = host(r)
    op, Q = _oracle_op(w), _Q(w.M)
    for b in range(w.batch):
        ro = oracle.residual(op, Q, w.dt, u0[b], u[b])
        assert rel_l2(r[b], ro) < 1e-13
    w2 = w.M * np.sum(u0 ** 2)
    ro_all = np.stack([oracle.residual(op, Q, w.dt, u0[b], u[b]) for b in range(w.batch)])
    assert abs(nrm - np.linalg.norm(ro_all) / math.sqrt(w2)) < 1e-12 * nrm


@pytest.mark.parametrize("alpha", [1e-6, 1e-2, 0.3])
@pytest.mark.parametrize("name,w,ov", CASES, ids=[c[0] for c in CASES])
def test_precond_parity(name, w, ov, alpha):
    """delta = C_alpha^{-1} r through Alg. 1's diagonalised steps (rows a2-a4)."""
    need_gpu()
    say("precond", name, alpha)
    p = plan_for(w, inner_tol=1e-14, inner_maxit=4000)
    r = _rand((w.batch, w.L, w.M, w.N), 3)
    d = host(p.precond(dev(r), alpha))
    op, Q = _oracle_op(w), _Q(w.M)
    for b in range(w.batch):
        do = oracle.precond_solve(op, Q, w.dt, alpha, r[b])
        # round-off of the diagonalisation grows like L / alpha (Theorem 2)
        tol = 1e-12 * max(1.0, w.L / alpha) ** 0.5 * 10
        assert rel_l2(d[b], do) < max(tol, 1e-11), (b, rel_l2(d[b], do))


@pytest.mark.parametrize("inner,kind", [("cocg", "heat2d"), ("bicgstab", "advdiff2d"), ("bicgstab", "heat2d")])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_shifted_solve_parity(inner, kind, prec):
    """Row a3 alone: (I - c_s A) x_s = b_s for complex shifts c_s."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    need_gpu()
    say("shifted", inner, kind, prec)
    w = wl.Workload("t", kind, 24, 20, 8, 3, 1e-3, nu=1e-2, vel=(1.0, 0.5), inner=inner, precision=prec)
    tol = 1e-13 if prec == "fp64" else 1e-6
    p = plan_for(w, inner_tol=tol)
    S = 10
    rng = np.random.default_rng(4)
    shifts = (rng.uniform(0.0, 0.05, S) + 1j * rng.uniform(-0.05, 0.05, S))
    b = rng.standard_normal((S, w.N)) + 1j * rng.standard_normal((S, w.N))
    x, its = p.shifted_solve(shifts, torch.as_tensor(b, device="cuda"))
    x = x.cpu().numpy()
    A = _oracle_op(w).matrix()
    for s in range(S):
        xo = spla.spsolve((sp.identity(w.N) - shifts[s] * A).tocsc(), b[s])
        assert rel_l2(x[s], xo) < (1e-11 if prec == "fp64" else 5e-5)
    assert np.all(its > 0)


@pytest.mark.parametrize("kind,nx,ny,order", [("advdiff2d", 64, 64, 2), ("advdiff2d", 65, 64, 2),
                                              ("advdiff2d", 130, 70, 2), ("adv2d_upwind", 96, 80, 4),
                                              ("adv1d_c4", 4096, 1, 2), ("adv1d_c4", 4100, 1, 2)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_shifted_solve_bicgstab_both_paths(kind, nx, ny, order, prec):
    """Row a3 with BiCGStab on both sides of the 4096-point limit: smaller
    systems run every iteration in one workgroup per system (one launch),
    larger ones in the three-kernel form (2D grids: the matrix-vector phases
    on 64 x 16 tiles, here ragged in x, in y, and with a two-point reach;
    1D: flat chunks).  Shifts of |c| up to 10 / (Gershgorin bound of A),
    against a sparse direct solve."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    need_gpu()
    say("bicgstab paths", kind, nx, ny, order, prec)
    w = wl.Workload("t", kind, nx, ny, 8, 3, 1e-3, nu=1e-2, vel=(1.0, 0.5), inner="bicgstab", precision=prec,
                    order=order)
    p = plan_for(w, inner_tol=1e-13 if prec == "fp64" else 1e-6)
    A = _oracle_op(w).matrix()
    rho = abs(A).sum(axis=1).max()
    S = 6
    rng = np.random.default_rng(11)
    shifts = (rng.uniform(0.0, 7.0, S) + 1j * rng.uniform(-7.0, 7.0, S)) / rho
    b = rng.standard_normal((S, w.N)) + 1j * rng.standard_normal((S, w.N))
    p.reset_stats()
    x, its = p.shifted_solve(shifts, torch.as_tensor(b, device="cuda"))
    x = x.cpu().numpy()
    st = p.stats()
    assert ("bicgstab_wg" in st) == (w.N <= 4096), sorted(st)
    assert ("bicgstab_p_matvec" in st) == (w.N > 4096), sorted(st)
    for s in range(S):
        xo = spla.spsolve((sp.identity(w.N) - shifts[s] * A).tocsc(), b[s])
        assert rel_l2(x[s], xo) < (1e-11 if prec == "fp64" else 5e-5), (s, rel_l2(x[s], xo))
    assert np.all(its > 0)


@pytest.mark.parametrize("nx", [7, 4100])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_shifted_solve_bicgstab_edge_cases(nx, prec):
    """BiCGStab edge cases on both paths (7 points: one workgroup per system,
    most of its threads owning no point; 4100: the chunked form).  A zero
    right-hand side stops at the first test (one iteration) with x = 0
    exactly; the others match a sparse direct solve; with an unreachable
    tolerance every system stops at the iteration cap exactly."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    need_gpu()
    say("bicgstab edge cases", nx, prec)
    w = wl.Workload("t", "adv1d_c4", nx, 1, 8, 3, 1e-3, nu=1e-2, vel=(1.0, 0.5), inner="bicgstab", precision=prec)
    A = _oracle_op(w).matrix()
    rho = abs(A).sum(axis=1).max()
    assert rho > 0
    rng = np.random.default_rng(12)
    shifts = (np.array([0.5 + 1.0j, 2.0 - 1.0j, 1.0 + 0.0j]) / rho)
    b = rng.standard_normal((3, w.N)) + 1j * rng.standard_normal((3, w.N))
    b[1] = 0.0
    p = plan_for(w, inner_tol=1e-13 if prec == "fp64" else 1e-6)
    x, its = p.shifted_solve(shifts, torch.as_tensor(b, device="cuda"))
    x = x.cpu().numpy()
    assert its[1] == 1 and np.all(x[1] == 0), (its, np.abs(x[1]).max())
    for s in (0, 2):
        xo = spla.spsolve((sp.identity(w.N) - shifts[s] * A).tocsc(), b[s])
        assert rel_l2(x[s], xo) < (1e-11 if prec == "fp64" else 5e-5), (s, rel_l2(x[s], xo))
    b[1] = rng.standard_normal(w.N)
    pc = plan_for(w, inner_tol=1e-30, inner_maxit=3)
    xc, itc = pc.shifted_solve(shifts, torch.as_tensor(b, device="cuda"))
    assert np.all(itc == 3), itc
    assert np.all(np.isfinite(xc.cpu().numpy()))



@pytest.mark.parametrize("nx,ny", [(24, 20), (1024, 320)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_shifted_solve_cocg_exact_in_few_steps(prec, nx, ny):
    """A right-hand side made of m Fourier modes with distinct eigenvalues of
    the periodic 5-point Laplacian makes COCG exact after m iterations, so on
    24 x 20 (one fused reduction per system, 2 tiles) the systems stop after
    1 .. 5 iterations: odd and even last passes, the first one included, in
    one batch (x moves every other pass).  On 1024 x 320 (a scalar kernel
    between passes, 320 tiles) round-off spoils the exact steps beyond the
    first mode (|c A| reaches about 2000) and the systems stop after tens of
    iterations.  Each cosine mode is an eigenvector of A = nu Lap_h with
    eigenvalue -nu lam, so the exact solution is sum_j b_j / (1 + c nu lam_j);
    with Re c >= 0, ||(I - c A)^{-1}|| <= 1 bounds the error by the true
    residual, which a complex64 x cannot bring below about eps_32 |c A| here."""
    need_gpu()
    say("shifted exact", prec, nx, ny)
    w = wl.Workload("t", "heat2d", nx, ny, 8, 3, 1e-3, nu=1e-2, inner="cocg", precision=prec)
    small = w.N <= 1000
    tau = (1e-13 if small else 1e-10) if prec == "fp64" else 1e-6
    p = plan_for(w, inner_tol=tau)
    xg, yg = np.meshgrid(np.arange(w.nx), np.arange(w.ny))
    modes = [(1, 0), (2, 1), (0, 3), (3, 2), (4, 4)]  # distinct eigenvalues on both grids
    lam = [4.0 * nx * nx * np.sin(np.pi * kx / nx) ** 2 + 4.0 * ny * ny * np.sin(np.pi * ky / ny) ** 2
           for kx, ky in modes]
    assert min(abs(a - b) for i, a in enumerate(lam) for b in lam[i + 1:]) > 1e-6 * max(lam)
    shifts = np.array([0.02 + 0.01j, 0.03 - 0.02j, 0.01 + 0.04j, 0.05 + 0.0j, 0.02 - 0.03j])
    b = np.zeros((len(modes), w.N), dtype=np.complex128)
    xe = np.zeros_like(b)
    for s in range(len(modes)):  # system s: the first s + 1 modes
        for j, (kx, ky) in enumerate(modes[:s + 1]):
            e = (1.0 + 0.5j * j) * np.cos(2 * np.pi * (kx * xg / w.nx + ky * yg / w.ny)).reshape(-1)
            b[s] += e
            xe[s] += e / (1.0 + shifts[s] * w.nu * lam[j])
    p.reset_stats()
    x, its = p.shifted_solve(shifts, torch.as_tensor(b, device="cuda"))
    x = x.cpu().numpy()
    A = _oracle_op(w).matrix()
    say("  iterations", its.tolist())
    # algorithmic bytes the library reports for the passes: per element, pass
    # k reads r (and p_{k-1} after pass 0) and writes r, p; odd passes also
    # write x (and read it after pass 1); after an even last pass the pending
    # x update reads p (and x after pass 1) and writes x
    def words(ks):
        w_ = sum((3 if k == 0 else 4) + ((2 if k >= 3 else 1) if k % 2 else 0) for k in range(ks))
        return w_ + ((3 if ks >= 3 else 2) if ks % 2 else 0)
    st = p.stats()["cocg_pass"]
    csize = 16 if prec == "fp64" else 8
    assert st["bytes"] == w.N * csize * sum(words(int(k)) for k in its), (st, its)
    assert st["elements"] == w.N * int(np.sum(its))
    for s in range(len(modes)):
        res = np.linalg.norm(b[s] - (x[s] - shifts[s] * (A @ x[s]))) / np.linalg.norm(b[s])
        err = rel_l2(x[s], xe[s])
        say("  system %d: true residual %.2e, error %.2e" % (s, res, err))
        if prec == "fp64":
            assert res < (1e-12 if small else 2e-10) and err < (1e-12 if small else 1e-9), (s, res, err)
        else:
            assert err < (5e-6 if small else 1e-4), (s, res, err)
        if prec == "fp64" and small:
            assert its[s] == s + 1, its

def _solve_and_compare(w, tol_rel, **solve_kw):
    p = plan_for(w)
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    u, info = p.solve(**solve_kw)
    u = host(u)
    op, Q = _oracle_op(w), _Q(w.M)
    errs = []
    for b in range(w.batch):
        backend = "sparse" if w.N * w.M <= 20000 else "spectral"
        Uo = oracle.sequential_solve(op, Q, w.dt, u0[b], w.L, backend=backend)
        errs.append(rel_l2(u[b], Uo))
    say("  sweeps", info["iterations"], "alpha", ["%.2e" % a for a in info["alpha"]],
        "inner mean", ["%.1f" % v for v in info["inner_mean"]], "err", ["%.2e" % e for e in errs])
    assert max(errs) <= tol_rel, errs
    return info, errs



# the plan's limits: M <= 8 nodes, L <= 1024 steps, L * M <= 2048
LIMIT_CASES = [
    ("heat1d_N40_L16_M8", wl.WORKLOADS["heat1d_64"].with_(nx=40, L=16, M=8, nu=0.05)),
    ("heat2d_8x6_L256_M8", wl.WORKLOADS["heat2d_256"].with_(nx=8, ny=6, L=256, M=8)),
    ("heat1d_N16_L1024_M2", wl.WORKLOADS["heat1d_64"].with_(nx=16, L=1024, M=2, nu=0.05)),
]


@pytest.mark.parametrize("alpha", [1e-4, 0.1])
@pytest.mark.parametrize("name,w", LIMIT_CASES, ids=[c[0] for c in LIMIT_CASES])
def test_precond_parity_at_size_limits(name, w, alpha):
    """Rows a2-a4 at the largest M and L the plan accepts."""
    need_gpu()
    say("precond limits", name, alpha)
    p = plan_for(w, inner_tol=1e-14, inner_maxit=4000)
    r = _rand((w.batch, w.L, w.M, w.N), 5)
    d = host(p.precond(dev(r), alpha))
    op, Q = _oracle_op(w), _Q(w.M)
    do = oracle.precond_solve(op, Q, w.dt, alpha, r[0])
    tol = 1e-12 * max(1.0, w.L / alpha) ** 0.5 * 10  # round-off grows like L / alpha (Theorem 2)
    say("  rel l2 %.2e (bound %.1e)" % (rel_l2(d[0], do), max(tol, 1e-11)))
    assert rel_l2(d[0], do) < max(tol, 1e-11)


@pytest.mark.parametrize("name,w", LIMIT_CASES, ids=[c[0] for c in LIMIT_CASES])
def test_solve_at_size_limits(name, w):
    """Alg. 2 at the largest M and L against sequential collocation."""
    need_gpu()
    say("solve limits", name)
    info, _ = _solve_and_compare(w, 1e-9, tol=1e-12, max_iter=40)
    assert info["converged"]

def test_solve_heat1d_64_fixed_alpha_residual_stop():
    """Workload heat1d_64: fixed alpha = 1e-3, stop at relative residual 1e-12."""
    need_gpu()
    w = wl.WORKLOADS["heat1d_64"]
    say("solve", w.name)
    info, _ = _solve_and_compare(w, 1e-10, alphas=[w.alpha], tol=w.tol, stop="residual", max_iter=20)
    assert info["converged"]
    # closed form: u(T) = R(dT lam)^L sin(2 pi x) (Pade R of Radau IIA, M = 3)
    z = w.dt * w.nu * (2 * math.cos(2 * math.pi / w.nx) - 2) * w.nx ** 2
    R = (1 + 2 * z / 5 + z * z / 20) / (1 - 3 * z / 5 + 3 * z * z / 20 - z ** 3 / 60)
    assert abs(R ** 4 - 0.85403178) < 1e-8


def test_richardson_factor_matches_closed_form():
    """Per sweep the single-mode error shrinks by |alpha R^L / (1 - alpha R^L)|,
    derived from eq. (Riteration); Theorem 1 bounds it by alpha / (1 - alpha)."""
    need_gpu()
    w = wl.WORKLOADS["heat1d_64"]
    op, Q = _oracle_op(w), _Q(w.M)
    u0 = wl.initial_condition(w)
    Ustar = oracle.sequential_solve(op, Q, w.dt, u0, w.L)
    z = w.dt * w.nu * (2 * math.cos(2 * math.pi / w.nx) - 2) * w.nx ** 2
    RL = ((1 + 2 * z / 5 + z * z / 20) / (1 - 3 * z / 5 + 3 * z * z / 20 - z ** 3 / 60)) ** w.L
    for alpha in (0.05, 0.3):
        p = plan_for(w, inner_tol=1e-14)
        p.set_u0(dev(u0[None]))
        u = torch.as_tensor(np.tile(u0, (1, w.L, w.M, 1)), device="cuda").contiguous()
        errs = []
        for _ in range(3):
            p.sweep(u, alpha)
            errs.append(np.linalg.norm(host(u)[0] - Ustar))
        rho = abs(alpha * RL / (1 - alpha * RL))
        say("  alpha", alpha, "ratios", errs[1] / errs[0], errs[2] / errs[1], "closed form", rho)
        assert abs(errs[1] / errs[0] - rho) < 1e-6 * rho
        assert abs(errs[2] / errs[1] - rho) < 1e-5 * rho
        assert rho <= alpha / (1 - alpha)


@pytest.mark.parametrize("name,w,tol", [
    ("heat2d_32_L16_cocg_alg2", wl.WORKLOADS["heat2d_256"].with_(nx=32, ny=32, L=16), 1e-10),
    ("heat2d_48x40_L8_M2_B3", wl.WORKLOADS["heat2d_256"].with_(nx=48, ny=40, L=8, M=2, batch=3), 1e-10),
    ("adv1d_512_L32_bicgstab_alg2", wl.WORKLOADS["adv1d_4096"].with_(nx=512, L=32), 1e-10),
    ("advdiff_32_L16_B2_fp64", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=32, ny=32, L=16, batch=2,
                                                                         precision="fp64", inner_tol=1e-12), 1e-10),
    ("heat2d_64_L8_mixed", wl.WORKLOADS["heat2d_1024_mixed"].with_(nx=64, ny=64, L=8), 1e-8),
])
def test_solve_alg2_parity(name, w, tol):
    need_gpu()
    say("solve", name)
    info, _ = _solve_and_compare(w, tol, tol=w.tol, max_iter=40)
    assert info["converged"]


def test_solve_errors_and_edges():
    need_gpu()
    from paper_2103_12571_amd import binding as bd
    w = wl.WORKLOADS["heat1d_64"]
    p = plan_for(w)
    u = torch.zeros((1, w.L, w.M, w.N), dtype=torch.float64, device="cuda")
    with pytest.raises(bd.AAOError) as e:
        p.sweep(u, 0.1)  # before aao_set_u0
    assert e.value.status == bd.AAO_ESTATE
    u0 = wl.initial_batch(w)
    p.set_u0(dev(u0))
    for bad in (0.0, 1.0, 2.0):
        with pytest.raises(bd.AAOError) as e:
            p.sweep(u, bad)
        assert e.value.status == bd.AAO_EINVAL
    bad_u0 = u0.copy()
    bad_u0[0, 3] = np.nan
    with pytest.raises(bd.AAOError) as e:
        p.set_u0(dev(bad_u0))
    assert e.value.status == bd.AAO_ENAN
    p.set_u0(dev(u0))
    _, info = p.solve(alphas=[0.4], tol=1e-30, max_iter=2, raise_on_noconv=False)
    assert info["iterations"] == 2 and not info["converged"]
    with pytest.raises(bd.AAOError) as e:
        p.solve(alphas=[0.4], tol=1e-30, max_iter=2)
    assert e.value.status == bd.AAO_ENOCONV
    # zero initial value: converged at once, u stays zero
    p.set_u0(torch.zeros((1, w.N), dtype=torch.float64, device="cuda"))
    u, info = p.solve(alphas=[1e-3], tol=1e-12, stop="residual", max_iter=5)
    assert float(u.abs().max()) == 0.0


FFT_CASES = [
    ("heat1d_N64_L8_M3", wl.WORKLOADS["heat1d_64"].with_(L=8, inner="fft")),
    ("heat2d_32x16_L16_M3", wl.WORKLOADS["heat2d_256"].with_(nx=32, ny=16, L=16, inner="fft")),
    ("adv1d_N128_L32_M2", wl.WORKLOADS["adv1d_4096"].with_(nx=128, L=32, M=2, inner="fft")),
    ("advdiff_16x32_L8_B2", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=16, ny=32, L=8, batch=2, inner="fft",
                                                                      precision="fp64")),
    ("heat2d_8x8_L1_M1", wl.WORKLOADS["heat2d_256"].with_(nx=8, ny=8, L=1, M=1, inner="fft")),
    # lengths that are not powers of two go through Bluestein's chirp-z transform
    ("heat2d_12x10_L8_M3_bluestein", wl.WORKLOADS["heat2d_256"].with_(nx=12, ny=10, L=8, inner="fft")),
    ("heat2d_7x9_L4_M2_bluestein", wl.WORKLOADS["heat2d_256"].with_(nx=7, ny=9, L=4, M=2, inner="fft")),
    ("adv1d_N100_L16_M3_bluestein", wl.WORKLOADS["adv1d_4096"].with_(nx=100, L=16, inner="fft")),
    ("advdiff_24x32_L4_B2_bluestein_x", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=24, ny=32, L=4, batch=2,
                                                                                  inner="fft", precision="fp64")),
]


@pytest.mark.parametrize("alpha", [1e-6, 0.3])
@pytest.mark.parametrize("name,w", FFT_CASES, ids=[c[0] for c in FFT_CASES])
def test_precond_parity_fft_inner(name, w, alpha):
    """Rows a2-a4 with the spatial-FFT direct inner solve (exact)."""
    need_gpu()
    say("precond fft", name, alpha)
    p = plan_for(w)
    r = _rand((w.batch, w.L, w.M, w.N), 5)
    d = host(p.precond(dev(r), alpha))
    op, Q = _oracle_op(w), _Q(w.M)
    for b in range(w.batch):
        do = oracle.precond_solve(op, Q, w.dt, alpha, r[b])
        tol = 1e-12 * max(1.0, w.L / alpha) ** 0.5 * 10
        assert rel_l2(d[b], do) < max(tol, 1e-11), (b, rel_l2(d[b], do))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 2e-6)])
@pytest.mark.parametrize("kind,nx,ny", [("heat2d", 32, 64), ("advdiff2d", 64, 16), ("adv1d_c4", 256, 1),
                                        ("heat2d", 12, 10), ("advdiff2d", 40, 24), ("adv1d_c4", 100, 1),
                                        ("heat2d", 7, 128), ("advdiff2d", 64, 27), ("adv1d_c4", 2047, 1)])
def test_shifted_solve_fft(kind, nx, ny, prec, tol):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    need_gpu()
    w = wl.Workload("t", kind, nx, ny, 8, 3, 1e-3, nu=1e-2, vel=(1.0, 0.5), inner="fft", precision=prec)
    p = plan_for(w)
    S = 7
    rng = np.random.default_rng(9)
    shifts = rng.uniform(0.0, 0.05, S) + 1j * rng.uniform(-0.05, 0.05, S)
    b = rng.standard_normal((S, w.N)) + 1j * rng.standard_normal((S, w.N))
    x, its = p.shifted_solve(shifts, torch.as_tensor(b, device="cuda"))
    x = x.cpu().numpy()
    A = _oracle_op(w).matrix()
    # FP64: a backward-stable transform solve errs by about eps * cond(I - c A)
    # * log2(transform length); cond from the exact spectrum of the circulant A
    lam = np.linalg.eigvals(A.toarray()) if w.N <= 4096 else None
    line = max(n if n & (n - 1) == 0 else 1 << (2 * n - 2).bit_length() for n in (nx, ny))
    for s in range(S):
        xo = spla.spsolve((sp.identity(w.N) - shifts[s] * A).tocsc(), b[s])
        t = tol
        if prec == "fp64" and lam is not None:
            mag = np.abs(1 - shifts[s] * lam)
            t = max(tol, 2.2e-16 * (mag.max() / mag.min()) * np.log2(line))
        assert rel_l2(x[s], xo) < t, (s, rel_l2(x[s], xo), t)


@pytest.mark.parametrize("name,w,tol", [
    ("heat2d_64_L16_fft_alg2", wl.WORKLOADS["heat2d_256"].with_(nx=64, ny=64, L=16, inner="fft"), 1e-10),
    ("adv1d_512_L32_fft_alg2", wl.WORKLOADS["adv1d_4096"].with_(nx=512, L=32, inner="fft"), 1e-10),
    ("heat2d_64_L8_fft_mixed", wl.WORKLOADS["heat2d_1024_mixed"].with_(nx=64, ny=64, L=8, inner="fft"), 1e-8),
    ("heat2d_60x50_L16_fft_bluestein", wl.WORKLOADS["heat2d_256"].with_(nx=60, ny=50, L=16, inner="fft"), 1e-10),
    ("adv1d_300_L32_fft_bluestein", wl.WORKLOADS["adv1d_4096"].with_(nx=300, L=32, inner="fft"), 1e-10),
    ("heat2d_60x50_L8_fft_mixed_bluestein", wl.WORKLOADS["heat2d_1024_mixed"].with_(nx=60, ny=50, L=8, inner="fft"),
     1e-8),
])
def test_solve_fft_inner_parity(name, w, tol):
    need_gpu()
    say("solve", name)
    info, _ = _solve_and_compare(w, tol, tol=w.tol, max_iter=40)
    assert info["converged"]


def test_sweep_reports_of_consecutive_plans():
    """A sweep's reported residual is its own: each plan's report comes
    through pinned host memory with a tag that counts from 1, and a fresh plan
    may get pinned memory that a destroyed plan used (regression: the first
    sweep of such a plan read the old plan's report)."""
    need_gpu()
    H = wl.WORKLOADS["heat2d_256"]
    shapes = [H.with_(nx=128, ny=64, L=8, M=4), H.with_(nx=128, ny=64, L=32), H.with_(nx=48, ny=40, L=8, M=4),
              H.with_(nx=64, ny=64, L=2, M=4)]
    for rep in range(2):
        for w in shapes:
            for inner in ("cocg", "fft"):
                p = plan_for(w.with_(inner=inner))
                rng = np.random.default_rng(11 + rep)
                p.set_u0(dev(rng.standard_normal((w.batch, w.N))))
                u = dev(rng.standard_normal((w.batch, w.L, w.M, w.N)))
                _, nrm = p.residual(u)
                res, _ = p.sweep(u, 1e-3)
                say("  %dx%d L%d M%d %s: sweep %.12e residual %.12e" % (w.nx, w.ny, w.L, w.M, inner, res, nrm))
                assert abs(res - nrm) <= 1e-13 * nrm
                del p
