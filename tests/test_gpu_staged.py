"""The forward transform's fused residual on tiles staged in LDS with a halo.

aao_sweep forms r = w - C u inside the forward transform.  On grids of at
least 16384 transform tiles whose tiles lie inside one grid row it stages the
tile's u (and the points beside it) in LDS; otherwise it gathers every tap
from global memory.  Either way one sweep must equal u + C_alpha^{-1}(w - C u)
computed as aao_residual (its own kernel, checked against the oracle in
test_gpu_parity) followed by aao_precond: the same systems and the same
operations.  The staged shapes cover halos of one and two points, 1D and 2D,
tiles that are whole grid rows (periodic wrap inside the tile), M = 1, 2, 3, 4,
a source term and a batch; two small shapes keep the unstaged form.  Small dt
keeps the Krylov solves on the large 1D grids short (the identity only needs
the same systems on both sides).  The transposed residual (adjoint sweep) on
staged tiles is checked against the oracle's backward solve.
"""
import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import dev, host, need_gpu, rel_l2, say, torch

pytestmark = pytest.mark.gpu

H = wl.WORKLOADS["heat2d_256"]
SWEEP_CASES = [
    # name, workload, with a source; tiles per instance in the name's comment
    # 1024 x 512, L = 32: 32-point tiles, 16384 of them, halo 1
    ("heat2d_1024x512_L32_halo1_fft", H.with_(nx=1024, ny=512, L=32, inner="fft", inner_tol=1e-15), False),
    # 64 x 16384, L = 16: 64-point tiles = whole rows
    ("heat2d_64x16384_L16_whole_row", H.with_(nx=64, ny=16384, L=16, dt=1e-7), False),
    # 128 x 8192, L = 8, M = 4: 64-point tiles, halo 1
    ("heat2d_128x8192_L8_M4_halo1", H.with_(nx=128, ny=8192, L=8, M=4, dt=1e-7), False),
    # 64 x 16384, L = 16, M = 1: whole rows
    ("heat2d_64x16384_L16_M1_whole_row", H.with_(nx=64, ny=16384, L=16, M=1, dt=1e-7), False),
    # 256 x 2048, L = 32, M = 2, 4th-order stencil: 32-point tiles, halo 2, source of eq. (heat)
    ("heat2d_c4_256x2048_L32_M2_halo2_source",
     wl.WORKLOADS["heat2d_table1"].with_(nx=256, ny=2048, L=32, inner="fft", inner_tol=1e-15), True),
    # 1D, N = 2^20, L = 16, 4th-order central advection: 64-point tiles, halo 2
    ("adv1d_c4_1M_L16_halo2", wl.WORKLOADS["adv1d_4096"].with_(nx=1 << 20, L=16, dt=1e-9), False),
    # 256 x 256, L = 8, B = 16: 64-point tiles, 1024 per instance, 16384 in all
    ("advdiff_256_L8_B16_halo1", wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=256, ny=256, L=8, batch=16,
                                                                           precision="fp64", inner="fft",
                                                                           inner_tol=1e-15), False),
    # unstaged: tiles that cross grid rows, a ragged tail
    ("heat2d_48x40_L8_row_crossing", H.with_(nx=48, ny=40, L=8), False),
    ("heat1d_N40_L8_ragged", wl.WORKLOADS["heat1d_64"].with_(nx=40, L=8), False),
]


@pytest.mark.parametrize("name,w,src", SWEEP_CASES, ids=[c[0] for c in SWEEP_CASES])
def test_sweep_equals_residual_then_precond(name, w, src):
    need_gpu()
    say("staged sweep", name)
    p = plan_for(w)
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal((w.batch, w.N))
    p.set_u0(dev(u0))
    if src:
        p.set_forcing(dev(wl.source_values(w, p.node_times(w.t0))))
    u = dev(rng.standard_normal((w.batch, w.L, w.M, w.N)))
    alpha = 1e-3
    r, nrm = p.residual(u)
    d = p.precond(r, alpha)
    ref = u + d
    del r, d
    us = u.clone()
    res, _ = p.sweep(us, alpha)
    e = float(torch.linalg.vector_norm(us - ref) / torch.linalg.vector_norm(ref))
    say("  rel diff sweep vs residual + precond %.2e  residual norms %.6e %.6e" % (e, res, nrm))
    assert e <= 1e-14
    assert abs(res - nrm) <= 1e-13 * nrm


def test_adjoint_on_staged_tiles():
    """advdiff2d on 512 x 512, L = 32, B = 2 (8192 tiles of 32 points per
    instance, halo 1), FP64, spatial-FFT inner solve; lambda of instance 0
    against the oracle's backward solve (per-Fourier-mode back-end)."""
    need_gpu()
    w = wl.WORKLOADS["advdiff2d_512_adj"].with_(nx=512, ny=512, L=32, batch=2, precision="fp64", inner="fft",
                                               inner_tol=1e-15, tol=1e-13)
    say("staged adjoint 512x512 L32 B2")
    p = plan_for(w)
    g = np.random.default_rng(7).standard_normal((w.batch, w.N))
    lam, info = p.adjoint_solve(dev(g), tol=1e-12, max_iter=40)
    lam = host(lam)
    op = oracle.stencil_for(w.kind, w.nx, w.ny, nu=w.nu, c=w.vel)
    Q = oracle.collocation_matrix(oracle.radau_right_nodes(w.M))
    lo = oracle.adjoint_solve(op, Q, w.dt, g[0], w.L, backend="spectral")
    e = rel_l2(lam[0], lo)
    say("  sweeps", info["iterations"], "err %.2e" % e)
    assert e < 1e-10
