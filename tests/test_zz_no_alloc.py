"""The allocation-free residual (aao_residual_noalloc) against aao_residual.

aao_residual_noalloc keeps its partial sums in the library's fixed device
scratch instead of the plan's workspace; it runs the same kernels with the
same reduction order, so r and the relative norm must match aao_residual bit
for bit.  Two calls in a row (the second on a smaller problem, so the shared
scratch holds the first call's larger contents), one with a source term, and
one through a plan that was never given a workspace or u0.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2103_12571_amd import binding as bd
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for, taps_for
from tests.gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

HEAT = wl.WORKLOADS["heat2d_256"]
CASES = [HEAT.with_(nx=96, ny=80, L=16, batch=2), HEAT.with_(nx=40, ny=24, L=4, batch=1)]


def _both(p, u, u0):
    r1, n1 = p.residual(u)
    r2, n2 = p.residual_noalloc(u, u0)
    return host(r1), n1, host(r2), n2


def test_residual_noalloc_matches_residual_two_calls():
    need_gpu()
    rng = np.random.default_rng(11)
    for w in CASES:
        say("noalloc residual", w.nx, "x", w.ny, "L", w.L, "B", w.batch)
        p = plan_for(w)
        u0 = dev(wl.initial_batch(w))
        p.set_u0(u0)
        u = dev(rng.standard_normal(p.shape))
        r1, n1, r2, n2 = _both(p, u, u0)
        say("  norms %.17g %.17g" % (n1, n2))
        assert np.array_equal(r1, r2)
        assert n1 == n2


def test_residual_noalloc_with_source():
    need_gpu()
    w = wl.table1_workload("heat", 1e-9).with_(nx=48, ny=40, L=8)
    say("noalloc residual with source", w.nx, "x", w.ny, "L", w.L)
    p = plan_for(w)
    u0 = dev(wl.initial_batch(w))
    p.set_u0(u0)
    p.set_forcing(dev(wl.source_values(w, p.node_times(w.t0))))
    u = dev(np.random.default_rng(12).standard_normal(p.shape))
    r1, n1, r2, n2 = _both(p, u, u0)
    assert np.array_equal(r1, r2)
    assert n1 == n2


def test_residual_noalloc_without_workspace():
    """A plan from aao_setup alone (host-only: no workspace, no u0)."""
    need_gpu()
    import torch
    w = CASES[1]
    ref = plan_for(w)
    u0 = dev(wl.initial_batch(w))
    ref.set_u0(u0)
    u = dev(np.random.default_rng(13).standard_normal(ref.shape))
    r1, n1 = ref.residual(u)
    dx, dy, coef, _ = taps_for(w.kind, w.nx, w.ny, nu=w.nu, vel=w.vel, order=w.order)
    dx = np.ascontiguousarray(dx, dtype=np.int32)
    dy = np.ascontiguousarray(dy, dtype=np.int32)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    st = bd.aao_stencil(2, w.nx, w.ny, len(coef), dx.ctypes.data_as(C.POINTER(C.c_int32)),
                        dy.ctypes.data_as(C.POINTER(C.c_int32)), coef.ctypes.data_as(C.POINTER(C.c_double)), None)
    cfg = bd.aao_config(w.M, None, w.L, w.dt, w.batch, bd.AAO_FP64, bd.AAO_INNER_COCG, 1e-12, 100)
    h = C.c_void_p()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    bd.check(bd.lib().aao_setup(C.byref(st), C.byref(cfg), stream, C.byref(h)))
    try:
        r2 = torch.empty_like(u)
        n2 = C.c_double()
        bd.check(bd.lib().aao_residual_noalloc(h, C.c_void_p(u0.data_ptr()), C.c_void_p(u.data_ptr()),
                                               C.c_void_p(r2.data_ptr()), C.byref(n2)))
    finally:
        bd.lib().aao_destroy(h)
    assert np.array_equal(host(r1), host(r2))
    assert n1 == n2.value
