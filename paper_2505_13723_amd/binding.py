"""Thin ctypes binding of libadasap.so (the C ABI declared in include/adasap.h and
include/adasap_warm.h).

Only argument marshalling lives here: torch tensors are passed as device pointers
with torch's current HIP stream; every step of the computation runs in the
library's HIP kernels.  Loading fails loudly when the library is missing.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadasap.so")

RBF, MATERN12, MATERN32, MATERN52 = 0, 1, 2, 3
KERNELS = {"rbf": RBF, "matern12": MATERN12, "matern32": MATERN32, "matern52": MATERN52}
FP64, FP32, MIXED = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "mixed": MIXED}
PRECOND_NYSTROM, PRECOND_IDENTITY, PRECOND_EXACT = 0, 1, 2
PRECONDS = {"nystrom": PRECOND_NYSTROM, "identity": PRECOND_IDENTITY, "exact": PRECOND_EXACT}
DTYPE_F32, DTYPE_F64 = 0, 1
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "device error",
          4: "Nystrom core not positive definite", 5: "non-finite values", 6: "unsupported",
          7: "not converged"}
NOT_CONVERGED = 7

# purposes of the random streams (second Philox key word)
PURPOSE_B, PURPOSE_OMEGA, PURPOSE_POW, PURPOSE_SWEEP_STRIDE = 5, 6, 7, 16


class AdasapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("kernel", ctypes.c_int32),
        ("lengthscale", ctypes.c_double), ("lam", ctypes.c_double),
        ("block_size", ctypes.c_int64), ("rank", ctypes.c_int32), ("rho_rule", ctypes.c_int32),
        ("rho", ctypes.c_double), ("mu", ctypes.c_double), ("nu", ctypes.c_double),
        ("power_iters", ctypes.c_int32), ("max_iters", ctypes.c_int64), ("tol", ctypes.c_double),
        ("check_every", ctypes.c_int64), ("refine_sweeps", ctypes.c_int32),
        ("precond", ctypes.c_int32), ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("accel", ctypes.c_int32), ("grad_at_z", ctypes.c_int32),
        ("z_uses_v_next", ctypes.c_int32), ("tail_average", ctypes.c_int32),
        ("n_lengthscale", ctypes.c_int32), ("lengthscales", ctypes.POINTER(ctypes.c_double)),
        ("outputscale", ctypes.c_double), ("check_rows", ctypes.c_int64),
    ]


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("k", ctypes.c_int32),
                ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("lengthscale", ctypes.c_double)]


class Report(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int64), ("relres", ctypes.c_double), ("relres_maxcol", ctypes.c_double),
        ("solve_ms", ctypes.c_double), ("check_ms", ctypes.c_double),
        ("eta_last", ctypes.c_double), ("rho_last", ctypes.c_double),
        ("lambda_hat_last", ctypes.c_double), ("delta_last", ctypes.c_double),
        ("refine_done", ctypes.c_int32), ("not_pd_events", ctypes.c_int32), ("status", ctypes.c_int32),
        ("step1_kernel_ms", ctypes.c_double), ("step1_launches", ctypes.c_int64),
        ("jacobi_sweeps_max", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("tuned_rows_per_wg", ctypes.c_int32), ("tuned_wg_per_cu", ctypes.c_int32),
        ("tuned_from_cache", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class WsConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("d", ctypes.c_int32), ("D", ctypes.c_int32),
                ("hidden", ctypes.c_int32), ("lam", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("adam_eps", ctypes.c_double)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_U64 = ctypes.c_uint64
_D = ctypes.c_double

_SIGNATURES = {
    "adasap_config_default": (_I32, [ctypes.POINTER(Config)]),
    "adasap_create": (_I32, [ctypes.POINTER(Config), _I64, _I32, _I32, _P, _P, _I32, _P, ctypes.POINTER(_P)]),
    "adasap_workspace_bytes": (_I64, [ctypes.POINTER(Config), _I64, _I32, _I32]),
    "adasap_solve": (_I32, [_P, _P, ctypes.POINTER(Report)]),
    "adasap_solve_more": (_I32, [_P, _P, _I64, ctypes.POINTER(Report)]),
    "adasap_predict": (_I32, [_P, _P, _I64, _P, _P]),
    "adasap_posterior_samples": (_I32, [_P, _P, _I64, _P, _P, _P]),
    "adasap_column_argmax": (_I32, [_I64, _I32, _I64, _P, _I32, _P, _P]),
    "adasap_probe_rates": (_I32, [_P, ctypes.POINTER(ctypes.c_double)]),
    "adasap_predictive_metrics": (_I32, [_I64, _I32, _P, _P, _D, _I32, _P, ctypes.POINTER(_D),
                                         ctypes.POINTER(_D)]),
    "adasap_residual": (_I32, [_P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "adasap_get_trace": (_I32, [_P, _P, _P, _P, _I64]),
    "adasap_block_gradient": (_I32, [_P, _I64, _P, _P, _P]),
    "adasap_residual_rows": (_I32, [_P, _P, _I64, _U64, ctypes.POINTER(_D), ctypes.POINTER(_D), _P]),
    "adasap_residual_rows_f64": (_I32, [_P, _P, _I64, _U64, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                        ctypes.POINTER(_D), _P]),
    "adasap_destroy": (None, [_P]),
    "adasap_sample_block": (_I32, [_U64, _U64, _U64, _I64, _I64, _P]),
    "adasap_normals": (_I32, [_U64, _U64, _U64, _I64, _P, _P]),
    "adasap_kblock_matmul": (_I32, [_I32, _D, _I32, _I64, _I64, _I32, _I32, _P, _P, _P, _P, _I32, _P]),
    "adasap_kblock_matmul_noalloc": (_I32, [_I32, _D, _I32, _I64, _I64, _I32, _I32, _P, _P, _P, _P,
                                            _I32, _P]),
    "adasap_nystrom": (_I32, [_I64, _I32, _P, _P, _D, _P, _P, _P, _P]),
    "adasap_precond_apply": (_I32, [_I64, _I32, _I32, _P, _P, _D, _I32, _P, _P, _P]),
    "adasap_solve_batch": (_I32, [ctypes.POINTER(Problem), _I32, ctypes.POINTER(Config), _I32, _P,
                                  ctypes.POINTER(Report)]),
    "adasap_ws_config_default": (_I32, [ctypes.POINTER(WsConfig)]),
    "adasap_ws_param_count": (_I64, [ctypes.POINTER(WsConfig)]),
    "adasap_ws_create": (_I32, [ctypes.POINTER(WsConfig), _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "adasap_ws_add_problem": (_I32, [_P, _I64, _P, _P, _P]),
    "adasap_ws_train_rows": (_I64, [_P]),
    "adasap_ws_train": (_I32, [_P, _I32, _I32, _D, _U64, _P]),
    "adasap_ws_features": (_I32, [_P, _I64, _P, _P, _P, _P]),
    "adasap_ws_loss_grad": (_I32, [_P, _I64, _P, _P, ctypes.POINTER(_D), _P]),
    "adasap_ws_predict_mean": (_I32, [_P, _I64, _P, _P, _P]),
    "adasap_ws_initial_iterate": (_I32, [_P, _I64, _P, _P, _P]),
    "adasap_ws_get_params": (_I32, [_P, _P]),
    "adasap_ws_set_params": (_I32, [_P, _P]),
    "adasap_ws_destroy": (None, [_P]),
    "adasap_last_error": (ctypes.c_char_p, []),
    "adasap_status_string": (ctypes.c_char_p, [_I32]),
}

EXPORTED = tuple(_SIGNATURES)


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return DTYPE_F64
    if t.dtype == torch.float32:
        return DTYPE_F32
    raise TypeError("tensors must be float32 or float64, got %s" % t.dtype)


def _check_dev(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("expected a device tensor")
        if not t.is_contiguous():
            raise ValueError("expected a contiguous tensor")


class Library:
    def __init__(self, path=LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError("HIP library %s is missing: run __graft_entry__.build() or "
                               "python -m paper_2505_13723_amd.build" % path)
        self.path = path
        # torch first: the library then binds to the HIP runtime torch already loaded, so that
        # both share one runtime (one device context, one allocator view)
        _torch()
        self.cdll = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(self.cdll, name)
            fn.restype = res
            fn.argtypes = args

    # -- errors ----------------------------------------------------------------------------
    def last_error(self):
        return self.cdll.adasap_last_error().decode()

    def check(self, status):
        if status != 0:
            raise AdasapError(status, self.last_error())

    # -- configuration -----------------------------------------------------------------------
    def config(self, **kw):
        cfg = Config()
        self.check(self.cdll.adasap_config_default(ctypes.byref(cfg)))
        for key, val in kw.items():
            if key == "kernel" and isinstance(val, str):
                val = KERNELS[val]
            if key == "precision" and isinstance(val, str):
                val = PRECISIONS[val]
            if key == "precond" and isinstance(val, str):
                val = PRECONDS[val]
            if key == "lambda":
                key = "lam"
            if key == "lengthscales":
                # one lengthscale per coordinate: the array is kept with the config until
                # adasap_create copies it
                arr = (ctypes.c_double * len(val))(*[float(v) for v in val])
                cfg._ell_keep = arr
                cfg.n_lengthscale = len(val)
                val = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
            if not hasattr(cfg, key):
                raise KeyError(key)
            setattr(cfg, key, val)
        return cfg

    def ws_config(self, **kw):
        cfg = WsConfig()
        self.check(self.cdll.adasap_ws_config_default(ctypes.byref(cfg)))
        for key, val in kw.items():
            if key == "lambda":
                key = "lam"
            if not hasattr(cfg, key):
                raise KeyError(key)
            setattr(cfg, key, val)
        return cfg

    def warm_start(self, cfg, freqs, phases, params):
        return WarmStart(self, cfg, freqs, phases, params)

    def workspace_bytes(self, cfg, n, d, k):
        return self.cdll.adasap_workspace_bytes(ctypes.byref(cfg), n, d, k)

    def create(self, cfg, X, Y):
        _check_dev(X, Y)
        if X.dtype != Y.dtype:
            raise TypeError("X and Y must have the same dtype")
        Y2 = Y if Y.dim() == 2 else Y.view(-1, 1)
        h = ctypes.c_void_p()
        self.check(self.cdll.adasap_create(ctypes.byref(cfg), X.shape[0], X.shape[1], Y2.shape[1],
                                           _ptr(X), _ptr(Y2), _dtype_code(X), _stream(),
                                           ctypes.byref(h)))
        return Handle(self, h, X, Y2, cfg)

    # -- single steps ------------------------------------------------------------------------
    def sample_block(self, seed, purpose, t, n, b):
        out = np.zeros(b, dtype=np.int64)
        self.check(self.cdll.adasap_sample_block(seed, purpose, t, n, b,
                                                 out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def normals(self, seed, purpose, t, count, device="cuda"):
        torch = _torch()
        out = torch.empty(count, dtype=torch.float64, device=device)
        self.check(self.cdll.adasap_normals(seed, purpose, t, count, _ptr(out), _stream()))
        return out

    def kblock_matmul(self, kernel, ell, precision, Xr, Xc, R):
        torch = _torch()
        _check_dev(Xr, Xc, R)
        R2 = R if R.dim() == 2 else R.view(-1, 1)
        out = torch.empty((Xr.shape[0], R2.shape[1]), dtype=Xr.dtype, device=Xr.device)
        kernel = KERNELS.get(kernel, kernel)
        precision = PRECISIONS.get(precision, precision)
        self.check(self.cdll.adasap_kblock_matmul(kernel, ell, precision, Xr.shape[0], Xc.shape[0],
                                                  Xr.shape[1], R2.shape[1], _ptr(Xr), _ptr(Xc),
                                                  _ptr(R2), _ptr(out), _dtype_code(Xr), _stream()))
        return out if R.dim() == 2 else out[:, 0]

    def kblock_matmul_noalloc(self, kernel, ell, precision, Xr, Xc, R, out):
        """The kernel-block product with no allocation, into the caller's `out` (enqueued on
        torch's current stream, not synchronised)."""
        _check_dev(Xr, Xc, R, out)
        R2 = R if R.dim() == 2 else R.view(-1, 1)
        kernel = KERNELS.get(kernel, kernel)
        precision = PRECISIONS.get(precision, precision)
        self.check(self.cdll.adasap_kblock_matmul_noalloc(kernel, ell, precision, Xr.shape[0],
                                                          Xc.shape[0], Xr.shape[1], R2.shape[1],
                                                          _ptr(Xr), _ptr(Xc), _ptr(R2), _ptr(out),
                                                          _dtype_code(Xr), _stream()))
        return out

    def predictive_metrics(self, samples, ystar, lam):
        """(test RMSE, mean NLL) of [posterior mean | samples] against ystar."""
        _check_dev(samples, ystar)
        a, b = ctypes.c_double(), ctypes.c_double()
        self.check(self.cdll.adasap_predictive_metrics(samples.shape[0], samples.shape[1],
                                                       _ptr(samples), _ptr(ystar), float(lam),
                                                       _dtype_code(samples), _stream(),
                                                       ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def column_argmax(self, a):
        """Row index of the largest entry of every column of a (m x k device matrix, any row
        stride), as a device int64 tensor."""
        torch = _torch()
        if not a.is_cuda or a.dim() != 2 or a.stride(1) != 1:
            raise ValueError("expected a device matrix with contiguous rows")
        out = torch.empty(a.shape[1], dtype=torch.int64, device=a.device)
        self.check(self.cdll.adasap_column_argmax(a.shape[0], a.shape[1], a.stride(0), _ptr(a),
                                                  _dtype_code(a), _stream(), _ptr(out)))
        return out

    def probe_rates(self):
        """Measured instruction rates of the device: ns per v_exp_f32 and per v_fma_f32 wave
        instruction per SIMD, and TFLOP/s of float16 32x32x16 MFMAs."""
        out = (ctypes.c_double * 3)()
        self.check(self.cdll.adasap_probe_rates(_stream(), out))
        return {"exp_ns": out[0], "valu_ns": out[1], "mfma32_f16_tflops": out[2]}

    def nystrom(self, Ysk, Omega, eps):
        torch = _torch()
        _check_dev(Ysk, Omega)
        b, r = Omega.shape
        U = torch.empty((b, r), dtype=torch.float64, device=Omega.device)
        S = torch.empty(r, dtype=torch.float64, device=Omega.device)
        delta = torch.empty(1, dtype=torch.float64, device=Omega.device)
        self.check(self.cdll.adasap_nystrom(b, r, _ptr(Ysk), _ptr(Omega), eps, _ptr(U), _ptr(S),
                                            _ptr(delta), _stream()))
        return U, S, float(delta.item())

    def precond_apply(self, U, S, rho, G, power):
        torch = _torch()
        _check_dev(U, S, G)
        G2 = G if G.dim() == 2 else G.view(-1, 1)
        out = torch.empty_like(G2)
        self.check(self.cdll.adasap_precond_apply(U.shape[0], U.shape[1], G2.shape[1], _ptr(U),
                                                  _ptr(S), rho, power, _ptr(G2), _ptr(out),
                                                  _stream()))
        return out if G.dim() == 2 else out[:, 0]


    def solve_batch(self, cfg, Xs, Ys, Ws, lengthscales):
        """Solve len(Xs) independent problems together; W tensors are updated in place."""
        P = len(Xs)
        probs = (Problem * P)()
        dtype = None
        for p in range(P):
            X, Y, W = Xs[p], Ys[p], Ws[p]
            _check_dev(X, Y, W)
            dtype = _dtype_code(X) if dtype is None else dtype
            if _dtype_code(Y) != dtype or _dtype_code(W) != dtype or _dtype_code(X) != dtype:
                raise TypeError("every array of a batch must have the same dtype")
            probs[p].n, probs[p].d = X.shape[0], X.shape[1]
            probs[p].k = 1 if Y.dim() == 1 else Y.shape[1]
            probs[p].X, probs[p].Y, probs[p].W = X.data_ptr(), Y.data_ptr(), W.data_ptr()
            probs[p].lengthscale = float(lengthscales[p])
        reps = (Report * P)()
        self.check(self.cdll.adasap_solve_batch(probs, P, ctypes.byref(cfg), dtype, _stream(), reps))
        return [r.as_dict() for r in reps]


class WarmStart:
    """Learned warm start: a network trained on solved problems predicts the posterior mean
    m^ of a new problem, giving W0 = (y - m^) / lambda.  All tensors float32 on the device."""

    def __init__(self, lib, cfg, freqs, phases, params):
        torch = _torch()
        self.lib, self.cfg = lib, cfg
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()
        self._keep = [f32(freqs), f32(phases), f32(params)]
        h = ctypes.c_void_p()
        lib.check(lib.cdll.adasap_ws_create(ctypes.byref(cfg), _ptr(self._keep[0]), _ptr(self._keep[1]),
                                            _ptr(self._keep[2]), _stream(), ctypes.byref(h)))
        self.h = h
        self.np = lib.cdll.adasap_ws_param_count(ctypes.byref(cfg))

    def add_problem(self, X, y, W):
        _check_dev(X, y, W)
        self.lib.check(self.lib.cdll.adasap_ws_add_problem(self.h, X.shape[0], _ptr(X), _ptr(y), _ptr(W)))

    def train_rows(self):
        return self.lib.cdll.adasap_ws_train_rows(self.h)

    def train(self, epochs, batch, lr, seed):
        loss = np.zeros(max(1, epochs))
        self.lib.check(self.lib.cdll.adasap_ws_train(self.h, epochs, batch, lr, seed,
                                                     loss.ctypes.data_as(ctypes.c_void_p)))
        return loss[:epochs]

    def features(self, X, y):
        torch = _torch()
        _check_dev(X, y)
        out = torch.empty((X.shape[0], self.cfg.D + 2), dtype=torch.float32, device=X.device)
        theta = torch.empty(self.cfg.D, dtype=torch.float64, device=X.device)
        self.lib.check(self.lib.cdll.adasap_ws_features(self.h, X.shape[0], _ptr(X), _ptr(y), _ptr(out),
                                                        _ptr(theta)))
        return out, theta

    def loss_grad(self, A, t):
        torch = _torch()
        _check_dev(A, t)
        g = torch.empty(self.np, dtype=torch.float32, device=A.device)
        loss = ctypes.c_double()
        self.lib.check(self.lib.cdll.adasap_ws_loss_grad(self.h, A.shape[0], _ptr(A), _ptr(t),
                                                         ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def predict_mean(self, X, y):
        torch = _torch()
        _check_dev(X, y)
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        self.lib.check(self.lib.cdll.adasap_ws_predict_mean(self.h, X.shape[0], _ptr(X), _ptr(y), _ptr(out)))
        return out

    def initial_iterate(self, X, y):
        torch = _torch()
        _check_dev(X, y)
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        self.lib.check(self.lib.cdll.adasap_ws_initial_iterate(self.h, X.shape[0], _ptr(X), _ptr(y),
                                                               _ptr(out)))
        return out

    def params(self):
        torch = _torch()
        out = torch.empty(self.np, dtype=torch.float32, device="cuda")
        self.lib.check(self.lib.cdll.adasap_ws_get_params(self.h, _ptr(out)))
        return out

    def set_params(self, p):
        _check_dev(p)
        self.lib.check(self.lib.cdll.adasap_ws_set_params(self.h, _ptr(p)))

    def close(self):
        if self.h:
            self.lib.cdll.adasap_ws_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Handle:
    def __init__(self, lib, h, X, Y, cfg):
        self.lib, self.h, self.X, self.Y, self.cfg = lib, h, X, Y, cfg

    def solve(self, W):
        """Run the solve in place on W; returns the report.  A solve that ends above its
        tolerance (status "not converged") returns its report too: report["status"] says so."""
        _check_dev(W)
        rep = Report()
        st = self.lib.cdll.adasap_solve(self.h, _ptr(W), ctypes.byref(rep))
        if st != NOT_CONVERGED:
            self.lib.check(st)
        return rep.as_dict()

    def solve_more(self, W, iters):
        """Continue the last solve for `iters` iterations (same random streams and state)."""
        _check_dev(W)
        rep = Report()
        st = self.lib.cdll.adasap_solve_more(self.h, _ptr(W), int(iters), ctypes.byref(rep))
        if st != NOT_CONVERGED:
            self.lib.check(st)
        return rep.as_dict()

    def predict(self, W, Xstar):
        torch = _torch()
        _check_dev(W, Xstar)
        out = torch.empty((Xstar.shape[0], self.Y.shape[1]), dtype=self.X.dtype, device=self.X.device)
        self.lib.check(self.lib.cdll.adasap_predict(self.h, _ptr(W), Xstar.shape[0], _ptr(Xstar),
                                                    _ptr(out)))
        return out

    def posterior_samples(self, W, Xstar, prior_star):
        """[posterior mean | k - 1 pathwise samples] at Xstar (m x k) from the solutions W."""
        torch = _torch()
        _check_dev(W, Xstar, prior_star)
        out = torch.empty((Xstar.shape[0], self.Y.shape[1]), dtype=self.X.dtype, device=self.X.device)
        self.lib.check(self.lib.cdll.adasap_posterior_samples(self.h, _ptr(W), Xstar.shape[0],
                                                              _ptr(Xstar), _ptr(prior_star), _ptr(out)))
        return out

    def residual(self, W):
        a, m = ctypes.c_double(), ctypes.c_double()
        self.lib.check(self.lib.cdll.adasap_residual(self.h, _ptr(W), ctypes.byref(a), ctypes.byref(m)))
        return a.value, m.value

    def residual_rows(self, W, m, seed, rows=False):
        """Row-subsampled relative residual (estimate, worst column); with rows=True also the
        sampled row indices (device int64 tensor)."""
        torch = _torch()
        _check_dev(W)
        a, mx = ctypes.c_double(), ctypes.c_double()
        R = torch.empty(m, dtype=torch.int64, device=W.device) if rows else None
        self.lib.check(self.lib.cdll.adasap_residual_rows(self.h, _ptr(W), int(m), int(seed),
                                                          ctypes.byref(a), ctypes.byref(mx), _ptr(R)))
        return (a.value, mx.value, R) if rows else (a.value, mx.value)

    def residual_rows_f64(self, W, m, seed):
        """Row-subsampled relative residual with float64 kernel values and products:
        (estimate, worst column, relative standard error)."""
        _check_dev(W)
        a, mx, se = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self.lib.check(self.lib.cdll.adasap_residual_rows_f64(self.h, _ptr(W), int(m), int(seed),
                                                              ctypes.byref(a), ctypes.byref(mx),
                                                              ctypes.byref(se), None))
        return a.value, mx.value, se.value

    def block_gradient(self, t, Z):
        """(B_t, G) of Step I at iterate Z, through the solver's own Step-I launch."""
        torch = _torch()
        _check_dev(Z)
        b = self.cfg.block_size
        B = torch.empty(b, dtype=torch.int64, device=self.X.device)
        G = torch.empty((b, self.Y.shape[1]), dtype=torch.float64, device=self.X.device)
        self.lib.check(self.lib.cdll.adasap_block_gradient(self.h, int(t), _ptr(Z), _ptr(B), _ptr(G)))
        return B, G

    def trace(self, count):
        eta, rho, lh = (np.full(count, np.nan) for _ in range(3))
        self.lib.check(self.lib.cdll.adasap_get_trace(
            self.h, eta.ctypes.data_as(ctypes.c_void_p), rho.ctypes.data_as(ctypes.c_void_p),
            lh.ctypes.data_as(ctypes.c_void_p), count))
        return {"eta": eta, "rho": rho, "lambda_hat": lh}

    def close(self):
        if self.h:
            self.lib.cdll.adasap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_LIB = None


def load():
    global _LIB
    if _LIB is None:
        _LIB = Library()
    return _LIB
