"""C ABI checks that need no GPU: exported symbols, argument validation, and the
host-side collocation math of aao_setup / aao_tables pinned to the paper."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2103_12571_amd import binding as bd
from paper_2103_12571_amd.stencil import taps_for

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "aao.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aao_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert sorted(bd.EXPORTS) == _declared()


def test_kernel_classes_header_binding_and_names_agree():
    """The stats arrays' length in the header, the binding's copy of it, and
    aao_kernel_name: one distinct non-empty name per class, "" past the end."""
    src = open(os.path.join(ROOT, "include", "aao.h")).read()
    n = int(re.search(r"#define AAO_NUM_KERNELS (\d+)", src).group(1))
    assert n == bd.AAO_NUM_KERNELS
    names = [bd.lib().aao_kernel_name(i).decode() for i in range(n)]
    assert all(names) and len(set(names)) == n, names
    assert bd.lib().aao_kernel_name(n).decode() == ""
    assert bd.lib().aao_kernel_name(-1).decode() == ""
    assert "bicgstab_wg" in names and "cocg_pass" in names


def test_library_exports_every_declared_symbol():
    lib = bd.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def _c_layout(structs):
    """sizeof and offsetof of the named structs' fields, as the C compiler lays
    them out from include/aao.h (gcc, host ABI)."""
    import subprocess
    import tempfile
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "aao.h"', "int main(void) {"]
    for name, cls in structs:
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "lay.c"), os.path.join(d, "lay")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


def test_binding_struct_layouts_match_header():
    """Every struct the binding passes through the ABI has the C layout: same
    size and the same offset for every field."""
    structs = [("aao_stencil", bd.aao_stencil), ("aao_config", bd.aao_config),
               ("aao_solve_info", bd.aao_solve_info), ("aao_gmres_info", bd.aao_gmres_info),
               ("aao_kernel_stats", bd.aao_kernel_stats)]
    lay = _c_layout(structs)
    for name, cls in structs:
        assert lay[(name, "sizeof")] == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert lay[(name, f)] == getattr(cls, f).offset, (name, f)


def _setup(kind="heat1d", nx=16, ny=1, M=3, L=8, dt=0.01, inner=bd.AAO_INNER_COCG, batch=1, nodes=None,
           nu=0.1, vel=(1.0, 0.5), ntaps=None, prec=bd.AAO_FP64):
    dx, dy, c, d = taps_for(kind, nx, ny, nu=nu, vel=vel)
    keep = [np.ascontiguousarray(v) for v in (dx, dy, c)]
    st = bd.aao_stencil(1 if ny == 1 else 2, nx, ny, len(c) if ntaps is None else ntaps,
                        keep[0].ctypes.data_as(C.POINTER(C.c_int32)), keep[1].ctypes.data_as(C.POINTER(C.c_int32)),
                        keep[2].ctypes.data_as(C.POINTER(C.c_double)), None)
    nd = None if nodes is None else np.ascontiguousarray(nodes, dtype=np.float64)
    cfg = bd.aao_config(M, None if nd is None else nd.ctypes.data_as(C.POINTER(C.c_double)), L, dt, batch,
                        prec, inner, 1e-12, 100)
    h = C.c_void_p()
    s = bd.lib().aao_setup(C.byref(st), C.byref(cfg), None, C.byref(h))
    return s, h


def test_setup_is_host_only_and_destroy():
    s, h = _setup()
    assert s == bd.AAO_OK
    size = C.c_size_t()
    assert bd.lib().aao_workspace_size(h, C.byref(size)) == 0 and size.value > 0
    bd.lib().aao_destroy(h)
    bd.lib().aao_destroy(None)


@pytest.mark.parametrize("kw,expect", [
    (dict(L=6), bd.AAO_EINVAL),            # L not a power of two
    (dict(L=2048), bd.AAO_EINVAL),
    (dict(M=0), bd.AAO_EINVAL),
    (dict(M=9), bd.AAO_EINVAL),
    (dict(dt=-1.0), bd.AAO_EINVAL),
    (dict(batch=0), bd.AAO_EINVAL),
    (dict(ntaps=0), bd.AAO_EINVAL),
    (dict(kind="adv1d_c4", inner=bd.AAO_INNER_COCG), bd.AAO_EINVAL),  # COCG needs A = A^T
    (dict(kind="adv1d_c4", inner=bd.AAO_INNER_BICGSTAB), bd.AAO_OK),
    (dict(nodes=[0.3, 0.8, 0.9]), bd.AAO_EINVAL),  # last node must be 1
    (dict(nodes=[0.5, 0.2, 1.0]), bd.AAO_EINVAL),
    (dict(inner=bd.AAO_INNER_FFT), bd.AAO_OK),                     # nx = 16: power of two
    (dict(inner=bd.AAO_INNER_FFT, nx=12), bd.AAO_OK),               # Bluestein: P = 32
    (dict(inner=bd.AAO_INNER_FFT, nx=2048), bd.AAO_OK),             # 2048 x 16 B = 32 KiB
    (dict(inner=bd.AAO_INNER_FFT, nx=2049), bd.AAO_EINVAL),         # Bluestein P = 8192: 128 KiB of LDS
    (dict(inner=bd.AAO_INNER_FFT, nx=8192), bd.AAO_EINVAL),         # row exceeds 64 KiB of LDS
    (dict(prec=7), bd.AAO_EINVAL),
])
def test_setup_argument_checks(kw, expect):
    s, h = _setup(**kw)
    assert s == expect, bd.lib().aao_last_error()
    if s == bd.AAO_OK:
        bd.lib().aao_destroy(h)
    else:
        assert bd.lib().aao_last_error()


def test_null_arguments():
    lib = bd.lib()
    assert lib.aao_setup(None, None, None, None) == bd.AAO_EINVAL
    assert lib.aao_sweep(None, None, 0.1, None, None) == bd.AAO_EINVAL
    assert lib.aao_workspace_size(None, None) == bd.AAO_EINVAL


def test_inner_floor_setter_checks_arguments():
    """aao_set_inner_floor is host-only: a null plan or a non-finite tau_w is
    EINVAL, any finite value (negative: the default) is taken."""
    lib = bd.lib()
    assert lib.aao_set_inner_floor(None, 1e-14) == bd.AAO_EINVAL
    s, h = _setup()
    assert s == 0
    for v in (float("nan"), float("inf"), -float("inf")):
        assert lib.aao_set_inner_floor(h, v) == bd.AAO_EINVAL
    for v in (-1.0, 0.0, 1e-14, 0.3):
        assert lib.aao_set_inner_floor(h, v) == 0
    lib.aao_destroy(h)


def test_calls_before_workspace_report_state():
    s, h = _setup()
    lib = bd.lib()
    assert lib.aao_sweep(h, C.c_void_p(256), 0.1, None, None) == bd.AAO_EWORKSPACE
    assert lib.aao_set_workspace(h, C.c_void_p(255), 1 << 30) == bd.AAO_EINVAL  # misaligned
    assert lib.aao_set_workspace(h, C.c_void_p(256), 16) == bd.AAO_EWORKSPACE   # too small
    lib.aao_destroy(h)


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8])
def test_host_nodes_and_Q_match_oracle(M):
    s, h = _setup(M=M)
    assert s == 0
    t = np.zeros(M)
    Q = np.zeros((M, M))
    bd.check(bd.lib().aao_collocation(h, t.ctypes.data_as(C.POINTER(C.c_double)), Q.ctypes.data_as(C.POINTER(C.c_double))))
    bd.lib().aao_destroy(h)
    assert np.allclose(t, oracle.radau_right_nodes(M), atol=2e-16, rtol=0)
    # the Vandermonde solve of the oracle loses digits as M grows (cond ~ 1e4 at M = 8)
    assert np.allclose(Q, oracle.collocation_matrix(oracle.radau_right_nodes(M)), atol=5e-15 if M <= 5 else 1e-12, rtol=0)


def _tables(h, alpha, L, M):
    Lh = L // 2 + 1
    d, r, djm, cond = np.zeros(2 * Lh), np.zeros(2 * Lh), np.zeros(2 * Lh * M), C.c_double()
    P = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    s = bd.lib().aao_tables(h, alpha, P(d), P(r), P(djm), C.byref(cond))
    cp = lambda v: v[0::2] + 1j * v[1::2]
    return s, cp(d), cp(r), cp(djm).reshape(Lh, M), cond.value


@pytest.mark.parametrize("M,L,alpha", [(1, 4, 0.1), (2, 8, 1e-3), (3, 64, 1e-6), (3, 16, 0.4), (4, 32, 0.05)])
def test_tables_lemma1_and_eigenvalues(M, L, alpha):
    """d_j of Lemma 1, r_j of eq. (QGL), and d_jm = eig(Q - r_j D_t H_M)."""
    s, h = _setup(M=M, L=L)
    st, d, r, djm, cond = _tables(h, alpha, L, M)
    bd.lib().aao_destroy(h)
    assert st == 0
    j = np.arange(L // 2 + 1)
    assert np.allclose(d, -alpha ** (1.0 / L) * np.exp(-2j * np.pi * j / L), atol=1e-15)
    assert np.allclose(r, d / (1 + d), atol=1e-14)
    t = oracle.radau_right_nodes(M)
    Q = oracle.collocation_matrix(t)
    H = np.zeros((M, M))
    H[:, -1] = 1
    for jj in j:
        ev = np.linalg.eigvals(Q - r[jj] * np.diag(t) @ H)
        got = list(djm[jj])
        for e in ev:
            k = int(np.argmin([abs(e - g) for g in got]))
            assert abs(e - got.pop(k)) < 1e-12 * max(1.0, abs(e))
    assert 1.0 <= cond < 1e4


def test_tables_alpha_range():
    s, h = _setup()
    for a in (0.0, 1.0, -0.5, 1.5, float("nan")):
        assert _tables(h, a, 8, 3)[0] == bd.AAO_EINVAL
    bd.lib().aao_destroy(h)


def test_nondiagonalisable_alpha_is_rejected():
    """Example 1 (M = 2) read with eq. (QGL)'s sign: Q - r D_t H_M is defective at
    r_* = (1 - sqrt 3)/3, reached at frequency 0 when d_0 = -alpha^{1/L} equals
    r_*/(1 - r_*), i.e. alpha_* = |r_*/(1 - r_*)|^L."""
    L = 4
    rs = (1 - math.sqrt(3)) / 3
    a_star = abs(rs / (1 - rs)) ** L
    s, h = _setup(M=2, L=L)
    assert _tables(h, a_star, L, 2)[0] == bd.AAO_ENODIAG
    assert "diagonalisable" in bd.lib().aao_last_error().decode()
    assert _tables(h, a_star * 1.2, L, 2)[0] == bd.AAO_OK
    bd.lib().aao_destroy(h)


def test_set_stencil_coef_checks():
    lib = bd.lib()
    s, h = _setup(kind="heat1d", nx=16, nu=0.1)
    assert s == bd.AAO_OK
    _, _, c2, d2 = taps_for("heat1d", 16, nu=0.3)
    cp = np.ascontiguousarray(c2).ctypes.data_as(C.POINTER(C.c_double))
    assert lib.aao_set_stencil_coef(h, cp, None) == bd.AAO_OK            # host-only, no GPU needed
    assert lib.aao_set_stencil_coef(None, cp, None) == bd.AAO_EINVAL
    assert lib.aao_set_stencil_coef(h, None, None) == bd.AAO_EINVAL
    bad = np.array([1.0, float("nan"), 1.0])
    assert lib.aao_set_stencil_coef(h, bad.ctypes.data_as(C.POINTER(C.c_double)), None) == bd.AAO_EINVAL
    skew = np.array([1.0, 0.0, -1.0])                                     # A != A^T: refused under COCG
    assert lib.aao_set_stencil_coef(h, skew.ctypes.data_as(C.POINTER(C.c_double)), None) == bd.AAO_EINVAL
    assert "symmetric" in lib.aao_last_error().decode()
    lib.aao_destroy(h)
    s, h = _setup(kind="heat1d", nx=16, nu=0.1, inner=bd.AAO_INNER_BICGSTAB)
    assert lib.aao_set_stencil_coef(h, skew.ctypes.data_as(C.POINTER(C.c_double)), None) == bd.AAO_OK
    lib.aao_destroy(h)


@pytest.mark.parametrize("kind,order", [("heat2d_central", k) for k in (2, 4, 6)]
                         + [("adv2d_upwind", k) for k in range(1, 6)])
def test_test_problem_stencils_match_oracle(kind, order):
    """The product's stencil taps of the Sec. 5 problems equal the oracle's
    operators (weights derived independently from the moment conditions)."""
    nx, ny = 12, 9
    dx, dy, c, _ = taps_for(kind, nx, ny, nu=0.7, vel=(1.0, 1.0), order=order)
    op = oracle.stencil_for(kind, nx, ny, nu=0.7, c=(1.0, 1.0), order=order)
    mine = {(int(a), int(b)): v for a, b, v in zip(dx, dy, c)}
    assert set(mine) == set(op.weights)
    for k, v in op.weights.items():
        assert abs(mine[k] - v) <= 1e-13 * max(1.0, abs(v)), (k, mine[k], v)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asking for more exits with a message (and
    touches no GPU on the way)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
