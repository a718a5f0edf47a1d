"""Seeded synthetic workloads shaped like the paper's test problems.

This module holds inputs only - grid sizes, PDE coefficients, step counts and
seeded initial data - and none of the method's arithmetic.  It is the one
module shared by the HIP path's callers (tests, bench) and the CPU oracle.

The paper's own problems are periodic heat and advection equations on the unit
square (Sec. 5, eqs. (heat), (advection)); the workloads below keep that
structure (periodic constant-coefficient stencils, Radau IIA with M = 3, L a
power of two) at the sizes used for measurement.
"""
from dataclasses import dataclass, field, replace
import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    kind: str            # heat1d | heat2d | adv1d_c4 | advdiff2d | heat2d_central | adv2d_upwind
    nx: int
    ny: int
    L: int
    M: int
    dt: float
    nu: float = 0.0
    vel: tuple = (0.0, 0.0)
    batch: int = 1
    init: str = "modes"  # sine | modes | gauss | heat_exact | adv_exact
    alpha: float = 0.0   # fixed alpha (0 -> adaptive rule of Alg. 2)
    stop: str = "laststep"   # laststep | residual
    tol: float = 1e-12
    inner: str = "cocg"      # cocg | bicgstab | fft
    inner_tol: float = 1e-12
    precision: str = "fp64"  # fp64 | mixed
    seed: int = 2103
    target_seed: int = 12103
    order: int = 2           # order of the differences (heat2d_central, adv2d_upwind)
    t0: float = 0.0          # initial time
    source: str = ""         # "" (b = 0) | heat (the source of eq. (heat))

    @property
    def N(self):
        return self.nx * self.ny

    @property
    def dof(self):
        return self.batch * self.L * self.M * self.N

    def with_(self, **kw):
        return replace(self, **kw)


WORKLOADS = {
    # 1D heat nu=0.1, N=64, L=4, dt=0.01, u0 = sin(2 pi x), fixed alpha 1e-3,
    # Richardson until the relative residual is 1e-12.
    "heat1d_64": Workload("heat1d_64", "heat1d", 64, 1, 4, 3, 0.01, nu=0.1, init="sine",
                          alpha=1e-3, stop="residual", tol=1e-12),
    # 2D heat nu=1e-2 on 256^2, L=64, dt=1e-3, 16 seeded Fourier modes, adaptive alpha, COCG.
    "heat2d_256": Workload("heat2d_256", "heat2d", 256, 256, 64, 3, 1e-3, nu=1e-2, init="modes",
                           tol=1e-12, inner="cocg"),
    # 1D advection c=1, N=4096, 4th-order central, L=128, dt=1e-3, Gaussian + noise.
    "adv1d_4096": Workload("adv1d_4096", "adv1d_c4", 4096, 1, 128, 3, 1e-3, vel=(1.0, 0.0),
                           init="gauss", tol=1e-11, inner="bicgstab"),
    # 2D heat nu=1e-2 on 1024^2, L=32, dt=1e-3; complex64 inner solves.
    "heat2d_1024_mixed": Workload("heat2d_1024_mixed", "heat2d", 1024, 1024, 32, 3, 1e-3, nu=1e-2,
                                  init="modes", tol=1e-8, inner="cocg", precision="mixed",
                                  inner_tol=1e-6),
    # The two problems of Sec. 5 with Table 1's middle column (tolerance 1e-9):
    # eq. (heat) on [pi, pi + 0.1], 400^2 points, 4th-order central, M = 2,
    # L = 32; eq. (advection) on [0, 1e-2], 350^2 points, 4th-order upwind,
    # M = 2, L = 16.  Inner tolerances are tighter than the sequential ones of
    # the table (the iteration's error floor scales with L tau / alpha).
    "heat2d_table1": Workload("heat2d_table1", "heat2d_central", 400, 400, 32, 2, 0.1 / 32, nu=1.0,
                              init="heat_exact", t0=np.pi, source="heat", order=4, tol=1e-11,
                              inner="cocg", inner_tol=1e-12),
    "adv2d_table1": Workload("adv2d_table1", "adv2d_upwind", 350, 350, 16, 2, 1e-2 / 16, vel=(1.0, 1.0),
                             init="adv_exact", order=4, tol=1e-11, inner="bicgstab", inner_tol=1e-13),
    # 2D advection-diffusion nu=5e-3, v=(1, 0.5) on 512^2, L=64, B=8; adjoint.
    "advdiff2d_512_adj": Workload("advdiff2d_512_adj", "advdiff2d", 512, 512, 64, 3, 1e-3, nu=5e-3,
                                  vel=(1.0, 0.5), batch=8, init="modes", tol=1e-10,
                                  inner="bicgstab", precision="mixed", inner_tol=1e-6),
}


# Sec. 5.1, Table 1: per problem and tolerance to reach, the points per
# dimension N, the order of the differences, the nodes M, the steps L and the
# sequential solver's tolerance tau.  Heat on [pi, pi + 0.1] (t0 = pi),
# advection on [0, 1e-2].
TABLE1 = {
    ("heat", 1e-5): dict(N=450, order=2, M=1, L=32, tau=1e-6),
    ("heat", 1e-9): dict(N=400, order=4, M=2, L=32, tau=1e-10),
    ("heat", 1e-12): dict(N=300, order=6, M=3, L=16, tau=1e-13),
    ("adv", 1e-5): dict(N=350, order=2, M=2, L=8, tau=1e-8),
    ("adv", 1e-9): dict(N=350, order=4, M=2, L=16, tau=1e-11),
    ("adv", 1e-12): dict(N=600, order=5, M=3, L=32, tau=1e-14),
}
TABLE1_T = {"heat": 0.1, "adv": 1e-2}

# Sec. 5.2, Table 2: the parameter sets of the moving window over 64 steps of
# dT = T64 / 64: N, order, M, T64, the sequential solver's tolerance tau and
# the inner tolerance of the parallel method (the table's tilde-tau).
TABLE2 = {
    ("heat", 1e-5): dict(N=350, order=2, M=1, T64=0.32, tau=1e-6, tau_par=1e-6),
    ("heat", 1e-9): dict(N=400, order=4, M=2, T64=0.16, tau=1e-10, tau_par=1e-10),
    ("heat", 1e-12): dict(N=350, order=6, M=3, T64=0.16, tau=1e-14, tau_par=1e-13),
    ("adv", 1e-5): dict(N=800, order=1, M=1, T64=0.00016, tau=1e-6, tau_par=1e-9),
    ("adv", 1e-9): dict(N=800, order=3, M=2, T64=0.00064, tau=1e-11, tau_par=1e-13),
    ("adv", 1e-12): dict(N=700, order=5, M=3, T64=0.0128, tau=1e-14, tau_par=1e-15),
}


def _problem_base(problem):
    return WORKLOADS["heat2d_table1"] if problem == "heat" else WORKLOADS["adv2d_table1"]


def table1_workload(problem, target, **kw):
    """The Sec. 5 problem at Table 1's parameters for the tolerance `target`
    (keyword overrides, e.g. inner solver and tolerances, go to the
    Workload)."""
    p = TABLE1[(problem, target)]
    w = _problem_base(problem).with_(name="%s_table1_%g" % (problem, target), nx=p["N"], ny=p["N"], order=p["order"],
                                     M=p["M"], L=p["L"], dt=TABLE1_T[problem] / p["L"])
    return w.with_(**kw)


def table2_workload(problem, target, L=16, **kw):
    """The Sec. 5 problem at Table 2's parameters for the tolerance `target`,
    as one window of L steps of dT = T64 / 64 (64 / L windows cover T64); the
    inner tolerance is the table's tilde-tau unless overridden."""
    p = TABLE2[(problem, target)]
    w = _problem_base(problem).with_(name="%s_table2_%g" % (problem, target), nx=p["N"], ny=p["N"], order=p["order"],
                                     M=p["M"], L=L, dt=p["T64"] / 64, inner_tol=p["tau_par"])
    return w.with_(**kw)


def grid(w):
    x = np.arange(w.nx) / w.nx
    y = np.arange(w.ny) / w.ny
    return x, y


def fourier_modes(nx, ny, seed, nmodes=16, kmax=8):
    """sum_j a_j cos(2 pi (kx_j x + ky_j y) + phi_j); per mode draw kx, ky, a, phi.

    (kx, ky) uniform integers in [-kmax, kmax]^2 without (0, 0) (redrawn),
    a ~ N(0, 1), phi ~ U[0, 2 pi), numpy default_rng(seed).  For ny = 1 the
    ky draw is kept (and ignored) so the stream layout does not depend on ny.
    """
    rng = np.random.default_rng(seed)
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)
    u = np.zeros((ny, nx))
    for _ in range(nmodes):
        while True:
            kx, ky = (int(v) for v in rng.integers(-kmax, kmax + 1, size=2))
            if ny == 1:
                ky = 0
            if kx != 0 or ky != 0:
                break
        a = rng.normal()
        phi = rng.uniform(0.0, 2.0 * np.pi)
        u += a * np.cos(2.0 * np.pi * (kx * X + ky * Y) + phi)
    return u.reshape(-1)


def initial_condition(w, b=0):
    """u0 for instance b (seed w.seed + b)."""
    x, _ = grid(w)
    if w.init == "sine":
        return np.sin(2.0 * np.pi * x).astype(np.float64)
    if w.init == "gauss":
        rng = np.random.default_rng(w.seed + b)
        return np.exp(-(x - 0.5) ** 2 / (2 * 0.05 ** 2)) + 1e-3 * rng.standard_normal(w.nx)
    if w.init == "modes":
        return fourier_modes(w.nx, w.ny, w.seed + b)
    if w.init in ("heat_exact", "adv_exact"):
        return exact_solution(w, w.t0)
    raise ValueError(w.init)


def _phi(w, shift=0.0):
    x, y = grid(w)
    X, Y = np.meshgrid(x, y)
    return (np.sin(2.0 * np.pi * (X - shift)) * np.sin(2.0 * np.pi * (Y - shift))).reshape(-1)


def exact_solution(w, t):
    """u(t) of the Sec. 5 problems on the grid: eq. (advection) gives
    sin(2 pi (x - t)) sin(2 pi (y - t)); the source printed in eq. (heat) is
    solved by cos(t) sin(2 pi x) sin(2 pi y)."""
    if w.init == "adv_exact":
        return _phi(w, t)
    if w.init == "heat_exact":
        return np.cos(t) * _phi(w)
    raise ValueError("no exact solution for %r" % w.init)


def source_values(w, times):
    """The source b(t, x) of the problem at the given absolute times
    (array [L, M]), as [B, L, M, N]; zeros when the problem has none.
    eq. (heat): b = sin(2 pi x) sin(2 pi y) (8 pi^2 cos t - sin t)."""
    times = np.asarray(times, dtype=np.float64)
    out = np.zeros((w.batch,) + times.shape + (w.N,))
    if w.source == "heat":
        out[:] = (8.0 * np.pi ** 2 * np.cos(times) - np.sin(times))[None, :, :, None] * _phi(w)[None, None, None, :]
    elif w.source:
        raise ValueError(w.source)
    return out


def initial_batch(w):
    return np.stack([initial_condition(w, b) for b in range(w.batch)])


def target_initial_batch(w):
    """u0* per instance (seeded Fourier modes, seed target_seed + b).  The
    adjoint loss's u_target is the final value of the same collocation
    problem started from u0* at the workload's nu (synthetic observations of
    the model); each side computes it with its own solver, and it is held
    fixed when nu varies."""
    return np.stack([fourier_modes(w.nx, w.ny, w.target_seed + b) for b in range(w.batch)])


def small(w, nx=None, ny=None, L=None, batch=None):
    """A reduced copy of a workload (same structure) for parity tests."""
    kw = {}
    if nx is not None:
        kw["nx"] = nx
    if ny is not None:
        kw["ny"] = ny
    if L is not None:
        kw["L"] = L
    if batch is not None:
        kw["batch"] = batch
    return replace(w, **kw)
