"""Python binding of liblowrank.so (argument marshalling only).

Tensors are passed by device pointer together with torch's current HIP stream;
every computation happens in the library's GPU kernels.  There is no CPU or
PyTorch fallback: if the shared library is missing this module raises on
import of any entry point.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblowrank.so")

LR_OK, LR_EINVAL, LR_ENOMEM, LR_ENOGAP, LR_ENOCONV, LR_ESHIFT, LR_ENOTSPD, LR_EDEVICE, LR_EBUSY = \
    range(9)
LR_MAX_P = 64
LR_MAX_SHIFT_ROUNDS = 64
LR_MAX_SLOTS = 16
LR_F64, LR_F32, LR_BF16 = 0, 1, 2
LR_PREC_F64, LR_PREC_BF16_STEPS, LR_PREC_F32_STEPS, LR_PREC_MC_PASS, LR_PREC_MC = 0, 1, 2, 3, 4


class lr_matrix(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int64), ("n", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("values", ctypes.c_void_p), ("col_ptr", ctypes.c_void_p),
                ("row_idx", ctypes.c_void_p)]


class lr_schedule(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("mu_hat", ctypes.c_double),
                ("delta_hat", ctypes.c_double), ("eta", ctypes.c_double), ("tau", ctypes.c_double),
                ("eps_stop", ctypes.c_double), ("m", ctypes.c_int64), ("b", ctypes.c_int64),
                ("first_solve", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("n_epochs", ctypes.c_int32), ("epochs", ctypes.POINTER(ctypes.c_int32))]


class lr_options(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("shift_mode", ctypes.c_int32),
                ("est_iters", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("max_epochs", ctypes.c_int32), ("max_shift_rounds", ctypes.c_int32),
                ("polish", ctypes.c_int32), ("batch", ctypes.c_int64),
                ("eta_scale", ctypes.c_double), ("tau_shift", ctypes.c_double),
                ("replay", ctypes.POINTER(lr_schedule)), ("timing", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("adaptive", ctypes.c_int32),
                ("norm", ctypes.c_int32), ("accel", ctypes.c_int32),
                ("fill_workspace", ctypes.c_int32), ("shift_start", ctypes.c_double)]


class lr_report(ctypes.Structure):
    _fields_ = [("theta_est", ctypes.c_double * LR_MAX_P), ("res_est", ctypes.c_double * LR_MAX_P),
                ("fro2", ctypes.c_double), ("mu_F", ctypes.c_double),
                ("shift_rounds", ctypes.c_int32),
                ("shift_lambda", ctypes.c_double * LR_MAX_SHIFT_ROUNDS),
                ("shift_gap", ctypes.c_double * LR_MAX_SHIFT_ROUNDS),
                ("outer", ctypes.c_int32), ("total_epochs", ctypes.c_int64),
                ("passes", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("last_change", ctypes.c_double), ("ms_pass_total", ctypes.c_double),
                ("ms_steps_total", ctypes.c_double), ("timed_passes", ctypes.c_int64),
                ("timed_steps", ctypes.c_int64), ("ms_sample_dot_probe", ctypes.c_double),
                ("ms_update_probe", ctypes.c_double), ("probes", ctypes.c_int64),
                ("n_intervals", ctypes.c_int32),
                ("interval_s", ctypes.c_int32 * LR_MAX_P), ("interval_q", ctypes.c_int32 * LR_MAX_P),
                ("interval_branch", ctypes.c_int32 * LR_MAX_P),
                ("interval_cols", ctypes.c_int32 * LR_MAX_P),
                ("interval_iters", ctypes.c_int32 * LR_MAX_P),
                ("accel_kappa", ctypes.c_double), ("accel_beta", ctypes.c_double),
                ("mc_passes", ctypes.c_int64)]


class lr_ticket_info(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("slot", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("workspace_bytes", ctypes.c_uint64)]


class lr_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("budget_bytes", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("slots", ctypes.c_int32),
                ("peak_running", ctypes.c_int32), ("elapsed", ctypes.c_double)]


# name -> (restype, argtypes); the full exported surface of include/lowrank.h
_P = ctypes.c_void_p
SIGNATURES = {
    "lowrank_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lowrank_last_error": (ctypes.c_char_p, []),
    "lowrank_options_default": (None, [ctypes.POINTER(lr_options)]),
    "lowrank_plan": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(lr_matrix), ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, ctypes.POINTER(lr_options), _P]),
    "lowrank_solve": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(lr_report)]),
    "lowrank_get_schedule": (ctypes.c_int, [_P, ctypes.POINTER(lr_schedule)]),
    "lowrank_destroy": (None, [_P]),
    "lowrank_plan_bytes": (ctypes.c_int, [ctypes.POINTER(lr_matrix), ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(lr_options),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "lowrank_solve_noalloc": (ctypes.c_int, [ctypes.POINTER(lr_matrix), ctypes.c_int,
                                             ctypes.c_int, ctypes.c_double,
                                             ctypes.POINTER(lr_options), _P, _P,
                                             ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(lr_report)]),
    "lowrank_op_apply_A": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "lowrank_op_prepare": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "lowrank_op_sample": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, _P, _P]),
    "lowrank_op_gaussian": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, _P]),
    "lowrank_op_cholqr2": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "lowrank_op_eigh": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P]),
    "lowrank_op_estimate": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), _P]),
    "lowrank_op_power": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double)]),
    "lowrank_op_svrg_solve": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_double)]),
    "lowrank_op_acc_svrg_solve": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                                 ctypes.c_int32, _P,
                                                 ctypes.POINTER(ctypes.c_double)]),
    "lowrank_server_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_size_t, ctypes.c_int]),
    "lowrank_submit": (ctypes.c_int, [_P, ctypes.POINTER(lr_matrix), ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.POINTER(lr_options), _P,
                                      ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_uint64)]),
    "lowrank_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(lr_report),
                                    ctypes.POINTER(lr_ticket_info)]),
    "lowrank_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(lr_report),
                                    ctypes.POINTER(lr_ticket_info)]),
    "lowrank_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(lr_server_stats)]),
    "lowrank_server_destroy": (None, [_P]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load liblowrank.so and declare every entry point.  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liblowrank.so not built: run __graft_entry__.build() "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LowRankError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_status_name(code), code, msg))
        self.code = code


def _status_name(code):
    lib = load_library()
    return lib.lowrank_status_string(code).decode()


def _check(code):
    if code != LR_OK:
        lib = load_library()
        raise LowRankError(code, lib.lowrank_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    import torch
    m = {torch.float64: LR_F64, torch.float32: LR_F32, torch.bfloat16: LR_BF16}
    if t.dtype not in m:
        raise ValueError("X must be float64, float32 or bfloat16")
    return m[t.dtype]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Schedule:
    """Host copy of lr_schedule; usable as a replay schedule."""

    def __init__(self, lam, mu_hat, eta, m, b, first_solve, outer, epochs, delta_hat=0.0,
                 tau=0.0, eps_stop=0.0):
        self.lam, self.mu_hat, self.eta, self.m, self.b = lam, mu_hat, eta, int(m), int(b)
        self.first_solve, self.outer, self.epochs = int(first_solve), int(outer), list(epochs)
        self.delta_hat, self.tau, self.eps_stop = delta_hat, tau, eps_stop

    def to_c(self):
        arr = (ctypes.c_int32 * max(1, len(self.epochs)))(*self.epochs)
        s = lr_schedule(lam=self.lam, mu_hat=self.mu_hat, delta_hat=self.delta_hat,
                        eta=self.eta, tau=self.tau, eps_stop=self.eps_stop, m=self.m, b=self.b,
                        first_solve=self.first_solve, outer=self.outer,
                        n_epochs=len(self.epochs), epochs=arr)
        return s, arr


class CscMatrix:
    """Compressed-column X (d x n) on the device: col_ptr (int32, n + 1),
    row_idx (int32, nnz; increasing within each column) and values (float64,
    float32 or bfloat16, nnz)."""

    def __init__(self, d, n, col_ptr, row_idx, values):
        import torch
        for t in (col_ptr, row_idx, values):
            if not t.is_cuda or t.dim() != 1 or not t.is_contiguous():
                raise ValueError("CSC arrays must be contiguous 1-D device tensors")
        if col_ptr.dtype != torch.int32 or row_idx.dtype != torch.int32:
            raise ValueError("col_ptr and row_idx must be int32")
        if col_ptr.numel() != n + 1 or row_idx.numel() != values.numel():
            raise ValueError("CSC array sizes do not match")
        self.d, self.n = int(d), int(n)
        self.col_ptr, self.row_idx, self.values = col_ptr, row_idx, values
        self.nnz = values.numel()
        self.device = values.device
        self.shape = (self.n, self.d)     # as the (n, d) view of dense X

    @classmethod
    def from_arrays(cls, d, n, col_ptr, row_idx, values, device="cuda"):
        """From host arrays (values as float64/float32, or uint16 BF16 bits)."""
        import torch
        if values.dtype == np.uint16:
            v = torch.from_numpy(np.ascontiguousarray(values).view(np.int16)).to(device)
            v = v.view(torch.bfloat16)
        else:
            v = torch.from_numpy(np.ascontiguousarray(values)).to(device)
        return cls(d, n, torch.from_numpy(np.ascontiguousarray(col_ptr, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(row_idx, np.int32)).to(device), v)


def _matrix(Xt):
    if isinstance(Xt, CscMatrix):
        return lr_matrix(d=Xt.d, n=Xt.n, ld=Xt.d, nnz=Xt.nnz, dtype=_dtype_code(Xt.values),
                         layout=1, values=Xt.values.data_ptr(), col_ptr=Xt.col_ptr.data_ptr(),
                         row_idx=Xt.row_idx.data_ptr())
    if not Xt.is_cuda or Xt.dim() != 2 or not Xt.is_contiguous():
        raise ValueError("X must be a contiguous 2-D device tensor of shape (n, d)")
    n, d = Xt.shape
    return lr_matrix(d=d, n=n, ld=d, nnz=0, dtype=_dtype_code(Xt), layout=0,
                     values=Xt.data_ptr(), col_ptr=None, row_idx=None)


def make_options(seed=0, shift_mode=0, est_iters=4, max_outer=2000, max_epochs=60,
                 max_shift_rounds=30, polish=0, batch=0, eta_scale=1.0, tau_shift=1e-2,
                 replay=None, timing=0, precision=0, adaptive=0, norm=0, accel=0,
                 fill_workspace=0, shift_start=0.0):
    """lr_options plus the host objects it points to (kept alive by the caller)."""
    lib = load_library()
    opt = lr_options()
    lib.lowrank_options_default(ctypes.byref(opt))
    opt.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    opt.shift_mode, opt.est_iters, opt.max_outer = shift_mode, est_iters, max_outer
    opt.max_epochs, opt.max_shift_rounds, opt.polish = max_epochs, max_shift_rounds, polish
    opt.batch, opt.eta_scale, opt.tau_shift, opt.timing = batch, eta_scale, tau_shift, timing
    opt.precision = precision
    opt.adaptive = adaptive
    opt.norm = norm
    opt.accel = accel
    opt.fill_workspace = fill_workspace
    opt.shift_start = float(shift_start)
    keep = None
    if replay is not None:
        sc, arr = replay.to_c()
        keep = (sc, arr)
        opt.replay = ctypes.pointer(sc)
    return opt, keep


def plan_bytes(Xt, k, p, **kw):
    """Device workspace bytes of a plan (or server request) for this problem."""
    lib = load_library()
    mat = _matrix(Xt)
    opt, _keep = make_options(**kw)
    out = ctypes.c_size_t()
    _check(lib.lowrank_plan_bytes(ctypes.byref(mat), k, p, ctypes.byref(opt), ctypes.byref(out)))
    return out.value


NOALLOC_MAX_BYTES = 64 * 1024 * 1024


def solve_noalloc(Xt, k, p, eps, out=None, **kw):
    """One solve through lowrank_solve_noalloc (no device allocation by the
    library: its workspace is the library's fixed device array).  Dense X only.
    Returns (status, U (d x k float64 device tensor), theta (numpy k), report)."""
    import torch
    lib = load_library()
    mat = _matrix(Xt)
    n, d = Xt.shape
    opt, _keep = make_options(**kw)
    U = out if out is not None else torch.empty((k, d), dtype=torch.float64, device=Xt.device)
    theta = (ctypes.c_double * k)()
    rep = lr_report()
    with torch.cuda.device(Xt.device):
        st = lib.lowrank_solve_noalloc(ctypes.byref(mat), k, p, float(eps), ctypes.byref(opt),
                                       _stream(), _ptr(U), theta, ctypes.byref(rep))
    if st != LR_OK and st != LR_ENOCONV:
        _check(st)
    return st, U.T, np.array(theta[:]), report_dict(rep, p)


class Plan:
    """A plan over a device matrix X given as an (n, d) C-contiguous tensor, i.e.
    X (d x n) in column-major order (each row of the tensor is a data point), or
    as a CscMatrix."""

    def __init__(self, Xt, k, p, eps, seed=0, shift_mode=0, est_iters=4, max_outer=2000,
                 max_epochs=60, max_shift_rounds=30, polish=0, batch=0, eta_scale=1.0,
                 tau_shift=1e-2, replay=None, timing=0, precision=0, adaptive=0, norm=0,
                 accel=0, fill_workspace=0, shift_start=0.0):
        import torch
        self.lib = load_library()
        self._mat = _matrix(Xt)
        self.Xt = Xt
        n, d = Xt.shape
        self.d, self.n, self.k, self.p = d, n, k, p
        self.device = Xt.device
        opt, self._replay_keep = make_options(
            seed=seed, shift_mode=shift_mode, est_iters=est_iters, max_outer=max_outer,
            max_epochs=max_epochs, max_shift_rounds=max_shift_rounds, polish=polish, batch=batch,
            eta_scale=eta_scale, tau_shift=tau_shift, replay=replay, timing=timing,
            precision=precision, adaptive=adaptive, norm=norm, accel=accel,
            fill_workspace=fill_workspace, shift_start=shift_start)
        self._opt = opt
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.lowrank_plan(ctypes.byref(h), ctypes.byref(self._mat), k, p,
                                         float(eps), ctypes.byref(opt), _stream()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.lowrank_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, out=None, raise_on_noconv=False):
        """Returns (status, U (d x k float64 device tensor), theta (numpy k), report)."""
        import torch
        U = out if out is not None else torch.empty((self.k, self.d), dtype=torch.float64,
                                                     device=self.device)
        theta = (ctypes.c_double * self.k)()
        rep = lr_report()
        with torch.cuda.device(self.device):
            st = self.lib.lowrank_solve(self._h, _ptr(U), theta, ctypes.byref(rep))
        if st != LR_OK and (st != LR_ENOCONV or raise_on_noconv):
            _check(st)
        # U is d x k column-major == a (k, d) row-major tensor; hand back d x k view
        return st, U.T, np.array(theta[:]), report_dict(rep, self.p)

    def schedule(self, cap=100000):
        arr = (ctypes.c_int32 * cap)()
        s = lr_schedule(epochs=arr, n_epochs=cap)
        _check(self.lib.lowrank_get_schedule(self._h, ctypes.byref(s)))
        return Schedule(s.lam, s.mu_hat, s.eta, s.m, s.b, s.first_solve, s.outer,
                        list(arr[:min(cap, s.outer)]), s.delta_hat, s.tau, s.eps_stop)

    # ---- single steps ----
    def apply_A(self, W):
        import torch
        Wc = W.T.contiguous() if W.shape[0] == self.d else W.contiguous()  # stored (ncols, d)
        Y = torch.empty_like(Wc)
        _check(self.lib.lowrank_op_apply_A(self._h, _ptr(Wc), _ptr(Y), Wc.shape[0]))
        return Y.T

    def prepare(self):
        import torch
        w = torch.empty(self.n, dtype=torch.float64, device=self.device)
        cdf = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        fro2 = ctypes.c_double()
        _check(self.lib.lowrank_op_prepare(self._h, _ptr(w), _ptr(cdf), ctypes.byref(fro2)))
        return w, cdf, fro2.value

    def sample(self, solve, epoch, step, b):
        import torch
        idx = torch.empty(b, dtype=torch.int32, device=self.device)
        sc = torch.empty(b, dtype=torch.float64, device=self.device)
        _check(self.lib.lowrank_op_sample(self._h, solve, epoch, step, b, _ptr(idx), _ptr(sc)))
        return idx, sc

    def gaussian(self, tag, solve, ncols):
        import torch
        S = torch.empty((ncols, self.d), dtype=torch.float64, device=self.device)
        _check(self.lib.lowrank_op_gaussian(self._h, tag, solve, ncols, _ptr(S)))
        return S.T

    def cholqr2(self, W):
        import torch
        Wc = W.T.contiguous()
        S = torch.empty_like(Wc)
        _check(self.lib.lowrank_op_cholqr2(self._h, _ptr(Wc), _ptr(S), Wc.shape[0]))
        return S.T

    def eigh(self, H):
        import torch
        m = H.shape[0]
        Hc = H.T.contiguous()
        vals = torch.empty(m, dtype=torch.float64, device=self.device)
        vecs = torch.empty((m, m), dtype=torch.float64, device=self.device)
        _check(self.lib.lowrank_op_eigh(self._h, _ptr(Hc), m, _ptr(vals), _ptr(vecs)))
        return vals, vecs.T

    def estimate(self, ncols, iters=4, stream_index=0):
        """Algorithm musco on A with ncols columns: (theta, residual norms, V d x ncols)."""
        import torch
        th = (ctypes.c_double * ncols)()
        rs = (ctypes.c_double * ncols)()
        V = torch.empty((ncols, self.d), dtype=torch.float64, device=self.device)
        _check(self.lib.lowrank_op_estimate(self._h, ncols, iters, stream_index, th, rs, _ptr(V)))
        return np.array(th[:]), np.array(rs[:]), V.T

    def power(self, S, max_iters, tol=0.0):
        """Plain subspace iteration on A from S (d x ncols): (S_out, iters, change)."""
        import torch
        Sc = S.T.contiguous()
        out = torch.empty_like(Sc)
        it = ctypes.c_int32()
        ch = ctypes.c_double()
        _check(self.lib.lowrank_op_power(self._h, _ptr(Sc), Sc.shape[0], int(max_iters),
                                         float(tol), _ptr(out), ctypes.byref(it),
                                         ctypes.byref(ch)))
        return out.T, it.value, ch.value

    def svrg_solve(self, S, lam, eta, m, b, solve, epochs):
        import torch
        Sc = S.T.contiguous()
        W = torch.empty_like(Sc)
        res = (ctypes.c_double * (epochs + 1))()
        _check(self.lib.lowrank_op_svrg_solve(self._h, _ptr(Sc), float(lam), float(eta), int(m),
                                              int(b), int(solve), int(epochs), _ptr(W), res))
        return W.T, np.array(res[:])

    def acc_svrg_solve(self, S, lam, kappa, beta, eta, m, b, solve, epochs):
        import torch
        Sc = S.T.contiguous()
        W = torch.empty_like(Sc)
        res = (ctypes.c_double * (epochs + 1))()
        _check(self.lib.lowrank_op_acc_svrg_solve(self._h, _ptr(Sc), float(lam), float(kappa),
                                                  float(beta), float(eta), int(m), int(b),
                                                  int(solve), int(epochs), _ptr(W), res))
        return W.T, np.array(res[:])


class Server:
    """Request server over the library's continuous-batching loop.

    submit() queues one problem (X as for Plan) and returns a ticket; wait() or
    poll() hand back (status, U d x k, theta, report, info) once it finished.
    The binding keeps X and the output buffers of every pending request alive.
    """

    def __init__(self, budget_bytes, slots=4, device=None):
        import torch
        self.lib = load_library()
        self.device = torch.device(device) if device is not None else \
            torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.lowrank_server_create(ctypes.byref(h), int(budget_bytes), int(slots)))
        self._h = h
        self._pending = {}

    def submit(self, Xt, k, p, eps, sync=True, **kw):
        import torch
        mat = _matrix(Xt)
        opt, keep = make_options(**kw)
        d = Xt.shape[1]
        U = torch.empty((k, d), dtype=torch.float64, device=Xt.device)
        theta = (ctypes.c_double * k)()
        if sync:   # the server's streams do not wait on torch's
            torch.cuda.current_stream(Xt.device).synchronize()
        t = ctypes.c_uint64()
        _check(self.lib.lowrank_submit(self._h, ctypes.byref(mat), k, p, float(eps),
                                       ctypes.byref(opt), _ptr(U), theta, ctypes.byref(t)))
        self._pending[t.value] = (Xt, U, theta, keep, k, p)
        return t.value

    def _finish(self, ticket, st, rep, info):
        Xt, U, theta, _keep, k, p = self._pending.pop(ticket)
        inf = {"t_submit": info.t_submit, "t_admit": info.t_admit, "t_done": info.t_done,
               "slot": info.slot, "workspace_bytes": info.workspace_bytes}
        return st, U.T, np.array(theta[:]), report_dict(rep, p), inf

    def poll(self, ticket):
        """None while pending, else (status, U, theta, report, info)."""
        rep, info = lr_report(), lr_ticket_info()
        st = self.lib.lowrank_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(rep),
                                   ctypes.byref(info))
        if st == LR_EBUSY:
            return None
        if st == LR_EINVAL and ticket not in self._pending:
            _check(st)
        return self._finish(ticket, st, rep, info)

    def wait(self, ticket):
        rep, info = lr_report(), lr_ticket_info()
        st = self.lib.lowrank_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(rep),
                                   ctypes.byref(info))
        if st == LR_EINVAL and ticket not in self._pending:
            _check(st)
        return self._finish(ticket, st, rep, info)

    def error(self):
        return self.lib.lowrank_last_error().decode()

    def stats(self):
        s = lr_server_stats()
        _check(self.lib.lowrank_server_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in lr_server_stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self.lib.lowrank_server_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def report_dict(rep, p):
    r = rep.shift_rounds
    return {
        "theta_est": np.array(rep.theta_est[:p]), "res_est": np.array(rep.res_est[:p]),
        "fro2": rep.fro2, "mu_F": rep.mu_F, "shift_rounds": r,
        "shift_lambda": list(rep.shift_lambda[:r]), "shift_gap": list(rep.shift_gap[:r]),
        "outer": rep.outer, "total_epochs": rep.total_epochs, "passes": rep.passes,
        "steps": rep.steps, "last_change": rep.last_change,
        "ms_pass_total": rep.ms_pass_total, "ms_steps_total": rep.ms_steps_total,
        "timed_passes": rep.timed_passes, "timed_steps": rep.timed_steps,
        "ms_sample_dot_probe": rep.ms_sample_dot_probe, "ms_update_probe": rep.ms_update_probe,
        "probes": rep.probes,
        "intervals": [{"s": rep.interval_s[i], "q": rep.interval_q[i],
                       "branch": "power" if rep.interval_branch[i] == 0 else "shift-invert",
                       "cols": rep.interval_cols[i], "iters": rep.interval_iters[i]}
                      for i in range(min(rep.n_intervals, LR_MAX_P))],
        "accel_kappa": rep.accel_kappa, "accel_beta": rep.accel_beta,
        "mc_passes": rep.mc_passes,
    }
