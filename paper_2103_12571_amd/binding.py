"""ctypes binding of libaao.so (include/aao.h): argument marshalling only.

Every step of the sweep runs in the HIP library; PyTorch provides device
memory (the caller's tensors and the plan workspace) and the stream.  There is
no CPU fallback: if the library is missing, ``lib()`` raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaao.so")

AAO_OK, AAO_EINVAL, AAO_EHIP, AAO_ENODIAG, AAO_ENOCONV = 0, -1, -2, -3, -4
AAO_ESTAGNATE, AAO_EWORKSPACE, AAO_ENAN, AAO_ESTATE = -5, -6, -7, -8
AAO_FP64, AAO_MIXED = 0, 1
AAO_INNER_COCG, AAO_INNER_BICGSTAB, AAO_INNER_FFT = 0, 1, 2
AAO_STOP_LASTSTEP, AAO_STOP_RESIDUAL = 0, 1
AAO_MAX_HIST = 64
AAO_NUM_KERNELS = 14

STATUS_NAMES = {0: "AAO_OK", -1: "AAO_EINVAL", -2: "AAO_EHIP", -3: "AAO_ENODIAG", -4: "AAO_ENOCONV",
                -5: "AAO_ESTAGNATE", -6: "AAO_EWORKSPACE", -7: "AAO_ENAN", -8: "AAO_ESTATE"}

EXPORTS = ["aao_setup", "aao_set_stream", "aao_set_inner_floor", "aao_workspace_size", "aao_set_workspace", "aao_set_u0",
           "aao_set_stencil_coef", "aao_set_forcing", "aao_solve_windows", "aao_gmres_workspace_size",
           "aao_solve_gmres",
           "aao_residual", "aao_residual_noalloc", "aao_precond", "aao_sweep", "aao_solve", "aao_adjoint_solve", "aao_grad",
           "aao_shifted_solve", "aao_set_timing", "aao_get_stats", "aao_reset_stats", "aao_kernel_name",
           "aao_tables", "aao_collocation", "aao_last_error", "aao_destroy"]


class AAOError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class aao_stencil(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nx", C.c_int64), ("ny", C.c_int64), ("ntaps", C.c_int),
                ("dx", C.POINTER(C.c_int32)), ("dy", C.POINTER(C.c_int32)),
                ("coef", C.POINTER(C.c_double)), ("dcoef_dnu", C.POINTER(C.c_double))]


class aao_config(C.Structure):
    _fields_ = [("M", C.c_int), ("nodes", C.POINTER(C.c_double)), ("L", C.c_int), ("dt", C.c_double),
                ("batch", C.c_int), ("precision", C.c_int), ("inner", C.c_int),
                ("inner_tol", C.c_double), ("inner_maxit", C.c_int)]


class aao_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("gamma", C.c_double), ("m0", C.c_double),
                ("alpha", C.c_double * AAO_MAX_HIST), ("m", C.c_double * AAO_MAX_HIST),
                ("res_rel", C.c_double * AAO_MAX_HIST), ("dlast_inf", C.c_double * AAO_MAX_HIST),
                ("inner_mean", C.c_double * AAO_MAX_HIST), ("inner_max", C.c_int * AAO_MAX_HIST),
                ("inner_fail", C.c_int * AAO_MAX_HIST), ("inner_fail_total", C.c_int)]

    def as_dict(self):
        k = min(self.iterations, AAO_MAX_HIST)
        return {"iterations": self.iterations, "converged": bool(self.converged), "gamma": self.gamma,
                "m0": self.m0, "alpha": list(self.alpha[:k]), "m": list(self.m[:k]),
                "res_rel": list(self.res_rel[:k]), "dlast_inf": list(self.dlast_inf[:k]),
                "inner_mean": list(self.inner_mean[:k]), "inner_max": list(self.inner_max[:k]),
                "inner_fail": list(self.inner_fail[:k]), "inner_fail_total": self.inner_fail_total}


class aao_gmres_info(C.Structure):
    _fields_ = [("steps", C.c_int), ("cycles", C.c_int), ("converged", C.c_int), ("res_rel", C.c_double),
                ("alpha", C.c_double * AAO_MAX_HIST), ("res_est", C.c_double * AAO_MAX_HIST),
                ("inner_mean", C.c_double * AAO_MAX_HIST), ("inner_max", C.c_int * AAO_MAX_HIST)]

    def as_dict(self):
        k = min(self.steps, AAO_MAX_HIST)
        return {"steps": self.steps, "cycles": self.cycles, "converged": bool(self.converged),
                "res_rel": self.res_rel, "alpha": list(self.alpha[:k]), "res_est": list(self.res_est[:k]),
                "inner_mean": list(self.inner_mean[:k]), "inner_max": list(self.inner_max[:k])}


class aao_kernel_stats(C.Structure):
    _fields_ = [("launches", C.c_int64 * AAO_NUM_KERNELS), ("elements", C.c_double * AAO_NUM_KERNELS),
                ("bytes", C.c_double * AAO_NUM_KERNELS), ("ms", C.c_double * AAO_NUM_KERNELS)]


_LIB = None


def lib():
    """Load libaao.so (built by paper_2103_12571_amd.build); raise if absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libaao.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    sig = {
        "aao_setup": [C.POINTER(aao_stencil), C.POINTER(aao_config), P, C.POINTER(P)],
        "aao_set_stream": [P, P],
        "aao_set_inner_floor": [P, C.c_double],
        "aao_workspace_size": [P, C.POINTER(C.c_size_t)],
        "aao_set_workspace": [P, P, C.c_size_t],
        "aao_set_u0": [P, P],
        "aao_set_stencil_coef": [P, D, D],
        "aao_set_forcing": [P, P],
        "aao_solve_windows": [P, P, C.c_int, P, D, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int,
                              C.POINTER(aao_solve_info)],
        "aao_gmres_workspace_size": [P, C.c_int, C.POINTER(C.c_size_t)],
        "aao_solve_gmres": [P, P, C.c_int, D, C.c_int, C.c_double, C.c_int, P, C.c_size_t,
                            C.POINTER(aao_gmres_info)],
        "aao_residual": [P, P, P, D],
        "aao_residual_noalloc": [P, P, P, P, D],
        "aao_precond": [P, P, P, C.c_double],
        "aao_sweep": [P, P, C.c_double, D, D],
        "aao_solve": [P, P, D, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.POINTER(aao_solve_info)],
        "aao_adjoint_solve": [P, P, P, D, C.c_int, C.c_double, C.c_double, C.c_int, C.POINTER(aao_solve_info)],
        "aao_grad": [P, P, P, P, P],
        "aao_shifted_solve": [P, C.c_int, D, P, P, C.POINTER(C.c_int)],
        "aao_set_timing": [P, C.c_int],
        "aao_get_stats": [P, C.POINTER(aao_kernel_stats)],
        "aao_reset_stats": [P],
        "aao_tables": [P, C.c_double, D, D, D, D],
        "aao_collocation": [P, D, D],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.aao_last_error.restype = C.c_char_p
    L.aao_last_error.argtypes = []
    L.aao_kernel_name.restype = C.c_char_p
    L.aao_kernel_name.argtypes = [C.c_int]
    L.aao_destroy.restype = None
    L.aao_destroy.argtypes = [P]
    _LIB = L
    return L


def check(status):
    if status != AAO_OK:
        raise AAOError(status, lib().aao_last_error().decode())
    return status


def kernel_name(i):
    return lib().aao_kernel_name(i).decode()


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Plan:
    """An aao plan bound to torch's current stream, with a torch-owned workspace."""

    def __init__(self, taps, nx, ny, M, L, dt, batch=1, precision="fp64", inner="cocg",
                 inner_tol=1e-12, inner_maxit=2000, nodes=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        dx, dy, coef, dcoef = taps
        self.ndim = 1 if ny == 1 else 2
        self.nx, self.ny, self.N = int(nx), int(ny), int(nx) * int(ny)
        self.M, self.L, self.B, self.dt = int(M), int(L), int(batch), float(dt)
        self._dx = np.ascontiguousarray(dx, dtype=np.int32)
        self._dy = np.ascontiguousarray(dy, dtype=np.int32)
        self._c = np.ascontiguousarray(coef, dtype=np.float64)
        self._dc = None if dcoef is None else np.ascontiguousarray(dcoef, dtype=np.float64)
        st = aao_stencil(self.ndim, self.nx, self.ny, len(self._c),
                         self._dx.ctypes.data_as(C.POINTER(C.c_int32)),
                         self._dy.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(self._c),
                         _dptr(self._dc) if self._dc is not None else None)
        self._nodes = None if nodes is None else np.ascontiguousarray(nodes, dtype=np.float64)
        prec = {"fp64": AAO_FP64, "mixed": AAO_MIXED}[precision]
        inn = {"cocg": AAO_INNER_COCG, "bicgstab": AAO_INNER_BICGSTAB, "fft": AAO_INNER_FFT}[inner]
        cfg = aao_config(self.M, _dptr(self._nodes) if self._nodes is not None else None, self.L,
                         self.dt, self.B, prec, inn, float(inner_tol), int(inner_maxit))
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(lib().aao_setup(C.byref(st), C.byref(cfg), C.c_void_p(stream), C.byref(self._h)))
            size = C.c_size_t()
            check(lib().aao_workspace_size(self._h, C.byref(size)))
            self.workspace_bytes = size.value
            self._ws = torch.empty(max(size.value, 256) + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            off = (-base) % 256
            check(lib().aao_set_workspace(self._h, C.c_void_p(base + off), size.value))
        self._u0 = None
        self._frc = None
        self._gmres_ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.aao_destroy(h)
            self._h = None

    # -- helpers
    def _f64(self, t, shape):
        t = t.to(device=self.device, dtype=self.torch.float64).contiguous()
        if tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t

    def _sync_stream(self):
        check(lib().aao_set_stream(self._h, C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)))

    @property
    def shape(self):
        return (self.B, self.L, self.M, self.N)

    def collocation(self):
        t = np.zeros(self.M)
        Q = np.zeros((self.M, self.M))
        check(lib().aao_collocation(self._h, _dptr(t), _dptr(Q)))
        return t, Q

    def tables(self, alpha):
        Lh = self.L // 2 + 1
        d = np.zeros(2 * Lh)
        r = np.zeros(2 * Lh)
        djm = np.zeros(2 * Lh * self.M)
        cond = C.c_double()
        check(lib().aao_tables(self._h, float(alpha), _dptr(d), _dptr(r), _dptr(djm), C.byref(cond)))
        cplx = lambda v: v[0::2] + 1j * v[1::2]
        return cplx(d), cplx(r), cplx(djm).reshape(Lh, self.M), cond.value

    # -- C-ABI calls
    def set_inner_floor(self, tau_w):
        """Absolute floor of the inner stop in solve / solve_windows /
        adjoint_solve (aao_set_inner_floor): 0 off, < 0 the default."""
        check(lib().aao_set_inner_floor(self._h, float(tau_w)))

    def set_stencil_coef(self, coef, dcoef=None):
        """New stencil weights (same offsets), e.g. another nu, without re-planning."""
        c = np.ascontiguousarray(coef, dtype=np.float64)
        if c.shape != self._c.shape:
            raise ValueError("expected %d weights" % self._c.size)
        d = None if dcoef is None else np.ascontiguousarray(dcoef, dtype=np.float64)
        if d is not None and d.shape != c.shape:
            raise ValueError("dcoef must match coef")
        self._sync_stream()
        check(lib().aao_set_stencil_coef(self._h, _dptr(c), _dptr(d) if d is not None else None))
        self._c = c
        if d is not None:
            self._dc = d

    def set_forcing(self, b):
        """Source b at the collocation times, [B, L, M, N] (None removes it)."""
        if b is None:
            self._frc = None
            self._sync_stream()
            check(lib().aao_set_forcing(self._h, None))
            return
        frc = self._f64(self.torch.as_tensor(b), (self.B, self.L, self.M, self.N))
        self._sync_stream()
        check(lib().aao_set_forcing(self._h, _ptr(frc)))
        self._frc = frc  # keep the device buffer alive while the plan uses it

    def node_times(self, t0=0.0):
        """Absolute collocation times t0 + (l + tau_m) dT, array [L, M]."""
        tau, _ = self.collocation()
        return t0 + (np.arange(self.L)[:, None] + np.asarray(tau)[None, :]) * self.dt

    def set_u0(self, u0):
        self._u0 = self._f64(u0, (self.B, self.N))
        self._sync_stream()
        check(lib().aao_set_u0(self._h, _ptr(self._u0)))

    def residual(self, u):
        u = self._f64(u, self.shape)
        r = self.torch.empty_like(u)
        nrm = C.c_double()
        self._sync_stream()
        check(lib().aao_residual(self._h, _ptr(u), _ptr(r), C.byref(nrm)))
        return r, nrm.value

    def residual_noalloc(self, u, u0=None):
        """aao_residual_noalloc: the residual with the library's fixed device
        scratch (no workspace); u0 defaults to the plan's own."""
        u = self._f64(u, self.shape)
        u0 = self._u0 if u0 is None else self._f64(u0, (self.B, self.N))
        r = self.torch.empty_like(u)
        nrm = C.c_double()
        self._sync_stream()
        check(lib().aao_residual_noalloc(self._h, _ptr(u0), _ptr(u), _ptr(r), C.byref(nrm)))
        return r, nrm.value

    def precond(self, r, alpha):
        r = self._f64(r, self.shape)
        d = self.torch.empty_like(r)
        self._sync_stream()
        check(lib().aao_precond(self._h, _ptr(r), _ptr(d), float(alpha)))
        return d

    def sweep(self, u, alpha):
        assert u.dtype == self.torch.float64 and u.is_contiguous() and tuple(u.shape) == self.shape
        res = C.c_double()
        dl = C.c_double()
        self._sync_stream()
        check(lib().aao_sweep(self._h, _ptr(u), float(alpha), C.byref(res), C.byref(dl)))
        return res.value, dl.value

    def solve(self, u=None, alphas=None, m0=0.0, tol=1e-12, stop="laststep", max_iter=50, raise_on_noconv=True):
        """aao_solve.  AAO_ENOCONV and AAO_ESTAGNATE raise (with the sweep
        history) unless raise_on_noconv is False; then info["status"] tells."""
        if u is None:
            u = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        info = aao_solve_info()
        al = None if alphas is None else np.ascontiguousarray(alphas, dtype=np.float64)
        self._sync_stream()
        s = lib().aao_solve(self._h, _ptr(u), _dptr(al) if al is not None else None,
                            0 if al is None else len(al), float(m0), float(tol),
                            {"laststep": AAO_STOP_LASTSTEP, "residual": AAO_STOP_RESIDUAL}[stop],
                            int(max_iter), C.byref(info))
        noconv = s in (AAO_ENOCONV, AAO_ESTAGNATE)
        if s != AAO_OK and (raise_on_noconv or not noconv):
            if noconv:
                raise AAOError(s, "%s; history %s" % (lib().aao_last_error().decode(), info.as_dict()))
            check(s)
        out = info.as_dict()
        out["status"] = STATUS_NAMES.get(s, s)
        return u, out

    def solve_windows(self, n_windows, sources=None, u=None, alphas=None, m0=0.0, tol=1e-12, stop="laststep",
                      max_iter=50):
        """Moving window: n_windows blocks of L steps from the plan's u0;
        sources [W, B, L, M, N] or None.  Returns (u of the last window, infos)."""
        if u is None:
            u = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        frc = None
        if sources is not None:
            frc = self.torch.as_tensor(sources).to(device=self.device, dtype=self.torch.float64).contiguous()
            if tuple(frc.shape) != (n_windows,) + tuple(self.shape):
                raise ValueError("sources must be [W, B, L, M, N]")
        infos = (aao_solve_info * n_windows)()
        al = None if alphas is None else np.ascontiguousarray(alphas, dtype=np.float64)
        self._sync_stream()
        s = lib().aao_solve_windows(self._h, _ptr(u), int(n_windows), _ptr(frc) if frc is not None else None,
                                    _dptr(al) if al is not None else None, 0 if al is None else len(al),
                                    float(m0), float(tol),
                                    {"laststep": AAO_STOP_LASTSTEP, "residual": AAO_STOP_RESIDUAL}[stop],
                                    int(max_iter), infos)
        out = [infos[k].as_dict() for k in range(n_windows)]
        if s != AAO_OK:
            raise AAOError(s, "%s; histories %s" % (lib().aao_last_error().decode(), out))
        return u, out

    def solve_gmres(self, u=None, restart=20, alphas=None, tol=1e-12, max_steps=200, raise_on_noconv=True):
        """Flexible GMRES(restart) on C u = w with C_alpha as right preconditioner
        (aao_solve_gmres); the scratch is a torch allocation kept per restart.
        Returns (u, info)."""
        if u is None:
            u = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        need = C.c_size_t()
        check(lib().aao_gmres_workspace_size(self._h, int(restart), C.byref(need)))
        ws = self._gmres_ws.get(int(restart))
        if ws is None or ws.numel() < need.value + 256:
            ws = self.torch.empty(need.value + 256, dtype=self.torch.uint8, device=self.device)
            self._gmres_ws = {int(restart): ws}
        base = ws.data_ptr() + (-ws.data_ptr()) % 256
        info = aao_gmres_info()
        al = None if alphas is None else np.ascontiguousarray(alphas, dtype=np.float64)
        self._sync_stream()
        s = lib().aao_solve_gmres(self._h, _ptr(u), int(restart), _dptr(al) if al is not None else None,
                                  0 if al is None else len(al), float(tol), int(max_steps), C.c_void_p(base),
                                  need.value, C.byref(info))
        if s != AAO_OK and (raise_on_noconv or s != AAO_ENOCONV):
            raise AAOError(s, "%s; history %s" % (lib().aao_last_error().decode(), info.as_dict()))
        return u, info.as_dict()

    def adjoint_solve(self, g_last, alphas=None, m0=0.0, tol=1e-12, max_iter=50):
        g = self._f64(g_last, (self.B, self.N))
        lam = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        info = aao_solve_info()
        al = None if alphas is None else np.ascontiguousarray(alphas, dtype=np.float64)
        self._sync_stream()
        s = lib().aao_adjoint_solve(self._h, _ptr(g), _ptr(lam), _dptr(al) if al is not None else None,
                                    0 if al is None else len(al), float(m0), float(tol), int(max_iter),
                                    C.byref(info))
        if s in (AAO_ENOCONV, AAO_ESTAGNATE):
            raise AAOError(s, "%s; history %s" % (lib().aao_last_error().decode(), info.as_dict()))
        check(s)
        return lam, info.as_dict()

    def grad(self, u, lam):
        u = self._f64(u, self.shape)
        lam = self._f64(lam, self.shape)
        gu0 = self.torch.empty((self.B, self.N), dtype=self.torch.float64, device=self.device)
        gnu = self.torch.empty((self.B,), dtype=self.torch.float64, device=self.device)
        self._sync_stream()
        check(lib().aao_grad(self._h, _ptr(u), _ptr(lam), _ptr(gu0), _ptr(gnu)))
        return gu0, gnu

    def shifted_solve(self, shifts, b):
        """Solve (I - shift_s A) x_s = b_s; b complex128 [S, N]."""
        S = b.shape[0]
        bb = b.to(device=self.device, dtype=self.torch.complex128).contiguous()
        x = self.torch.empty_like(bb)
        sh = np.ascontiguousarray(np.stack([np.real(shifts), np.imag(shifts)], 1).reshape(-1), dtype=np.float64)
        its = (C.c_int * S)()
        self._sync_stream()
        check(lib().aao_shifted_solve(self._h, S, _dptr(sh), _ptr(bb), _ptr(x), its))
        return x, np.array(its[:], dtype=np.int64)

    def set_timing(self, on):
        check(lib().aao_set_timing(self._h, 1 if on else 0))

    def reset_stats(self):
        check(lib().aao_reset_stats(self._h))

    def stats(self):
        s = aao_kernel_stats()
        check(lib().aao_get_stats(self._h, C.byref(s)))
        out = {}
        for i in range(AAO_NUM_KERNELS):
            if s.launches[i]:
                out[kernel_name(i)] = {"launches": int(s.launches[i]), "elements": s.elements[i],
                                       "bytes": s.bytes[i], "ms": s.ms[i]}
        return out
