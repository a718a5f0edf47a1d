"""Bitwise reproducibility of a converged solve (fixed-order reductions
everywhere), also while another plan solves concurrently on another stream:
no result may depend on timing.  Regression test for a COCG early exit whose
flag could change under the workgroup within the pass that stops a system."""
import threading

import pytest

from paper_2103_12571_amd import workloads as wl
from paper_2103_12571_amd.stencil import plan_for
from tests.gpu_util import need_gpu, say, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,w", [
    ("heat2d_256_cocg", wl.WORKLOADS["heat2d_256"]),
    ("heat2d_96x64_L16_mixed", wl.WORKLOADS["heat2d_1024_mixed"].with_(nx=96, ny=64, L=16)),
    ("adv1d_512_L32_bicgstab", wl.WORKLOADS["adv1d_4096"].with_(nx=512, L=32)),
])
def test_solves_are_bitwise_reproducible_under_concurrency(name, w):
    need_gpu()
    say("determinism", name)
    u0 = torch.as_tensor(wl.initial_batch(w), device="cuda")
    plans = [plan_for(w), plan_for(w)]
    for p in plans:
        p.set_u0(u0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    us = [torch.empty(plans[0].shape, dtype=torch.float64, device="cuda") for _ in plans]
    with torch.cuda.stream(streams[0]):
        plans[0].solve(us[0], tol=w.tol, max_iter=50)
    streams[0].synchronize()
    ref = us[0].clone()
    torch.cuda.synchronize()  # the copy is read from the other streams below
    bad = []

    def run(i, n):
        try:
            with torch.cuda.stream(streams[i]):
                for r in range(n):
                    plans[i].solve(us[i], tol=w.tol, max_iter=50)
                    streams[i].synchronize()
                    if not torch.equal(us[i], ref):
                        bad.append((i, r, float((us[i] - ref).abs().max())))
        except Exception as e:  # surfaced by the assertion below
            bad.append((i, "raised", repr(e)))

    run(0, 2)  # alone
    th = [threading.Thread(target=run, args=(i, 4)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    say("  differing solves", bad)
    assert not bad
