"""ctypes binding of libgmf (include/gmf.h).

The functions here only marshal arguments: every step of the computation runs
in the HIP kernels of libgmf.so.  PyTorch provides device memory and the
stream.  Importing this module raises if the shared library is missing; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmf.so")

GMF_OK, GMF_EINVAL, GMF_EWORKSPACE, GMF_EDEVICE, GMF_ENUMERIC, GMF_ENOTCONV = 0, -1, -2, -3, -4, -5
GMF_POISSON, GMF_NEGBIN, GMF_GAUSSIAN, GMF_GAMMA, GMF_BERNOULLI, GMF_INVGAUSS = 0, 1, 2, 3, 4, 5
GMF_LINK_LOG, GMF_LINK_IDENTITY, GMF_LINK_LOGIT = 0, 1, 2
GMF_PREC_FP32, GMF_PREC_BF16, GMF_PREC_BF16X3 = 0, 1, 2
GMF_Y_INT32, GMF_Y_FLOAT32 = 0, 1

FAMILY_CODES = {"poisson": GMF_POISSON, "negbin": GMF_NEGBIN, "gaussian": GMF_GAUSSIAN,
                "gamma": GMF_GAMMA, "bernoulli": GMF_BERNOULLI, "invgauss": GMF_INVGAUSS}
LINK_CODES = {"log": GMF_LINK_LOG, "identity": GMF_LINK_IDENTITY, "logit": GMF_LINK_LOGIT}
PREC_CODES = {"fp32": GMF_PREC_FP32, "bf16": GMF_PREC_BF16, "bf16x3": GMF_PREC_BF16X3}


class gmf_config(C.Structure):
    _fields_ = [
        ("family", C.c_int32), ("link", C.c_int32), ("precision", C.c_int32),
        ("bias_mode", C.c_int32),
        ("n", C.c_int64), ("m", C.c_int64),
        ("d", C.c_int32), ("p", C.c_int32), ("q", C.c_int32),
        ("R", C.c_int32), ("S", C.c_int32),
        ("phi", C.c_double), ("nb_alpha", C.c_double),
        ("lambda_", C.c_double * 4),
        ("rate0", C.c_double), ("decay", C.c_double), ("tau", C.c_double),
        ("alpha1", C.c_double), ("alpha2", C.c_double),
        ("damping", C.c_double), ("eps", C.c_double), ("eta_max", C.c_double),
        ("seed", C.c_uint64),
        ("tile_rows", C.c_int32), ("skip_block_deviance", C.c_int32),
        ("panel_stride", C.c_int32), ("tile_waves", C.c_int32), ("eval_overlap", C.c_int32),
        ("allow_missing", C.c_int32), ("estimate_phi", C.c_int32), ("estimate_alpha", C.c_int32),
        ("compact_counts", C.c_int32),
    ]


class gmf_mlp_config(C.Structure):
    _fields_ = [("m", C.c_int32), ("hidden", C.c_int32), ("d", C.c_int32), ("batch", C.c_int32),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("weight_decay", C.c_double)]


class GMFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libgmf error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgmf.so (raises if it has not been built).  torch is imported
    first, so that the library binds to the HIP runtime torch has loaded (the
    same soname): loaded the other way round, the process would hold two HIP
    runtimes, and the library's would see no device."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libgmf.so not found at {path}: build it with "
                          f"`python -m paper_2412_20509_amd.build`")
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, i32, i64, f64p = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    cfgp = C.POINTER(gmf_config)
    sig = {
        "gmf_config_default": (None, [cfgp]),
        "gmf_workspace_bytes": (C.c_size_t, [cfgp, i32]),
        "gmf_init": (C.c_int, [C.POINTER(vp), cfgp, vp, C.c_size_t, vp, vp, i32, vp, vp,
                               vp, vp, vp, vp, vp]),
        "gmf_step": (C.c_int, [vp, i64]),
        "gmf_fit": (C.c_int, [vp, i32, C.c_double, i32, f64p, C.POINTER(i32)]),
        "gmf_deviance": (C.c_int, [vp, f64p, f64p]),
        "gmf_run": (C.c_int, [vp, i32, i32, f64p, f64p]),
        "gmf_set_precision": (C.c_int, [vp, i32]),
        "gmf_compact_counts": (C.c_int, [vp]),
        "gmf_row_deviance": (C.c_int, [vp, vp]),
        "gmf_block_deviance": (C.c_int, [vp, f64p, i64]),
        "gmf_get_params": (C.c_int, [vp, vp, vp, vp, vp, i32]),
        "gmf_set_params": (C.c_int, [vp, vp, vp, vp, vp]),
        "gmf_get_moments": (C.c_int, [vp, vp, vp, vp, vp]),
        "gmf_get_schedule": (C.c_int, [vp, C.POINTER(i32), C.POINTER(i32), i64, i64,
                                       C.POINTER(i32)]),
        "gmf_schedule_host": (C.c_int, [C.c_uint64, i64, i64, i32, i64, i64, C.POINTER(i32),
                                        C.POINTER(i32), C.POINTER(i32)]),
        "gmf_initialize_workspace_bytes": (C.c_size_t, [vp, i32]),
        "gmf_initialize": (C.c_int, [vp, vp, C.c_size_t, vp, i32, i32, i32, C.c_double]),
        "gmf_set_column_alpha": (C.c_int, [vp, vp]),
        "gmf_init_spectrum": (C.c_int, [vp, f64p, i32]),
        "gmf_rank_eigengap": (C.c_int, [f64p, i32, i32, C.POINTER(i32)]),
        "gmf_rank_select_cv": (C.c_int, [f64p, i32, i32, C.POINTER(i32)]),
        "gmf_get_dispersion": (C.c_int, [vp, f64p, f64p]),
        "gmf_heldout_metrics": (C.c_int, [vp, vp, i32, f64p]),
        "gmf_state_bytes": (C.c_size_t, [vp]),
        "gmf_save_state": (C.c_int, [vp, vp, C.c_size_t]),
        "gmf_load_state": (C.c_int, [vp, vp, C.c_size_t]),
        "gmf_project_workspace_bytes": (C.c_size_t, [vp, i64]),
        "gmf_project": (C.c_int, [vp, vp, C.c_size_t, vp, i32, i64, vp, vp, vp, i32, i32, vp, vp,
                                  f64p]),
        "gmf_project_warm": (C.c_int, [vp, vp, C.c_size_t, vp, i32, i64, vp, vp, i32, i32, vp,
                                       vp, f64p, f64p, C.POINTER(i64)]),
        "gmf_project_noalloc": (C.c_int, [vp, vp, i32, i64, vp, vp, vp, i32, i32, vp, vp, f64p]),
        "gmf_batch_workspace_bytes": (C.c_size_t, [C.POINTER(vp), i32, i32]),
        "gmf_batch_init": (C.c_int, [C.POINTER(vp), C.POINTER(vp), i32, vp, C.c_size_t, i32,
                                     i32]),
        "gmf_batch_run": (C.c_int, [vp, i32, i32, f64p]),
        "gmf_batch_destroy": (None, [vp]),
        "gmf_tune": (C.c_int, [cfgp, vp, C.c_size_t, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                               C.POINTER(i32), i32, i32, C.POINTER(i32), f64p]),
        "gmf_tune_lookup": (i32, [cfgp]),
        "gmf_tune_table_clear": (None, []),
        "gmf_tune_table_save": (C.c_int, [C.c_char_p]),
        "gmf_tune_table_load": (C.c_int, [C.c_char_p]),
        "gmf_mlp_config_default": (None, [C.POINTER(gmf_mlp_config)]),
        "gmf_encoder_workspace_bytes": (C.c_size_t, [C.POINTER(gmf_mlp_config)]),
        "gmf_encoder_init": (C.c_int, [C.POINTER(vp), C.POINTER(gmf_mlp_config), vp, C.c_size_t,
                                       vp, vp, vp, vp, vp, vp, vp]),
        "gmf_encoder_train": (C.c_int, [vp, vp, i32, vp, i64, i32, f64p]),
        "gmf_encoder_forward": (C.c_int, [vp, vp, i32, i64, vp, i32]),
        "gmf_encoder_loss_grad": (C.c_int, [vp, vp, i32, vp, i64, f64p, vp]),
        "gmf_encoder_get_weights": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "gmf_encoder_destroy": (None, [vp]),
        "gmf_encoder_last_error": (C.c_char_p, []),
        "gmf_set_trace": (C.c_int, [vp, vp, i64]),
        "gmf_set_timing": (C.c_int, [vp, i32]),
        "gmf_get_timing": (C.c_int, [vp, f64p, f64p, C.POINTER(i64)]),
        "gmf_get_timing_by_kind": (C.c_int, [vp, f64p, f64p]),
        "gmf_steps_done": (i64, [vp]),
        "gmf_sync": (C.c_int, [vp]),
        "gmf_destroy": (None, [vp]),
        "gmf_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != GMF_OK:
        raise GMFError(rc, load_library().gmf_last_error().decode())
    return rc


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# --------------------------------------------------------------- C ABI ----

def gmf_config_default() -> gmf_config:
    cfg = gmf_config()
    load_library().gmf_config_default(C.byref(cfg))
    return cfg


def gmf_workspace_bytes(cfg: gmf_config, with_weights: bool = False) -> int:
    return load_library().gmf_workspace_bytes(C.byref(cfg), int(with_weights))


def gmf_init(cfg, workspace, stream, Y, y_dtype, X, Z, W, B0, A0, U0, V0):
    ctx = C.c_void_p()
    _check(load_library().gmf_init(C.byref(ctx), C.byref(cfg), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), stream,
                                   _ptr(Y), y_dtype, _ptr(X), _ptr(Z), _ptr(W), _ptr(B0),
                                   _ptr(A0), _ptr(U0), _ptr(V0)))
    return ctx


def gmf_step(ctx, nsteps: int):
    return _check(load_library().gmf_step(ctx, int(nsteps)))


def gmf_fit(ctx, max_epochs: int, tol: float = 0.0, eval_every: int = 1):
    n_eval = max(1, max_epochs // eval_every)
    trace = (C.c_double * n_eval)()
    done = C.c_int32(0)
    rc = load_library().gmf_fit(ctx, int(max_epochs), float(tol), int(eval_every), trace,
                                C.byref(done))
    if rc not in (GMF_OK, GMF_ENOTCONV):
        _check(rc)
    k = done.value // eval_every
    return rc, list(trace)[:k], done.value


def gmf_run(ctx, epochs: int, eval_every: int = 1, trace: bool = True):
    """(deviance trace, device completion ms of each evaluation) or (None, None)."""
    nev = epochs // eval_every if trace else 0
    tr = (C.c_double * max(nev, 1))() if trace else None
    ms = (C.c_double * max(nev, 1))() if trace else None
    _check(load_library().gmf_run(ctx, int(epochs), int(eval_every), tr, ms))
    if not trace:
        return None, None
    return list(tr)[:nev], list(ms)[:nev]


def gmf_deviance(ctx):
    tot, pen = C.c_double(), C.c_double()
    _check(load_library().gmf_deviance(ctx, C.byref(tot), C.byref(pen)))
    return tot.value, pen.value


def gmf_block_deviance(ctx, count: int):
    out = (C.c_double * count)()
    _check(load_library().gmf_block_deviance(ctx, out, int(count)))
    return np.array(list(out))


def gmf_get_params(ctx, B, A, U, V, postprocess: int = 0):
    return _check(load_library().gmf_get_params(ctx, _ptr(B), _ptr(A), _ptr(U), _ptr(V),
                                                 int(postprocess)))


def gmf_set_params(ctx, B, A, U, V):
    return _check(load_library().gmf_set_params(ctx, _ptr(B), _ptr(A), _ptr(U), _ptr(V)))


def gmf_get_moments(ctx, Grow, Hrow, Gcol, Hcol):
    return _check(load_library().gmf_get_moments(ctx, _ptr(Grow), _ptr(Hrow), _ptr(Gcol),
                                                  _ptr(Hcol)))


def gmf_get_schedule(ctx, n: int, m: int, t_first: int = 1, count: int = 0):
    rp = (C.c_int32 * n)()
    cp = (C.c_int32 * m)()
    rr = (C.c_int32 * max(count, 1))()
    _check(load_library().gmf_get_schedule(ctx, rp, cp, int(t_first), int(count), rr))
    return np.array(rp), np.array(cp), np.array(rr)[:count]


def gmf_schedule_host(seed: int, n: int, m: int, R: int, t_first: int = 1, count: int = 0):
    rp = (C.c_int32 * max(n, 1))()
    cp = (C.c_int32 * max(m, 1))()
    rr = (C.c_int32 * max(count, 1))()
    _check(load_library().gmf_schedule_host(seed, n, m, R, t_first, count, rp, cp, rr))
    return np.array(rp)[:n], np.array(cp)[:m], np.array(rr)[:count]


def gmf_project_workspace_bytes(ctx, n_new: int) -> int:
    return load_library().gmf_project_workspace_bytes(ctx, int(n_new))


def gmf_project(ctx, workspace, Ynew, y_dtype, n_new, Xnew, A0, U0, epochs, frozen, A_out,
                U_out, trace: bool = False):
    tr = (C.c_double * (epochs + 1))() if trace else None
    _check(load_library().gmf_project(ctx, _ptr(workspace),
                                      workspace.numel() * workspace.element_size(), _ptr(Ynew),
                                      y_dtype, int(n_new), _ptr(Xnew), _ptr(A0), _ptr(U0),
                                      int(epochs), int(frozen), _ptr(A_out), _ptr(U_out), tr))
    return None if tr is None else list(tr)


def gmf_project_noalloc(ctx, Ynew, y_dtype, n_new, Xnew, A0, U0, epochs, frozen, A_out, U_out,
                        trace: bool = False):
    tr = (C.c_double * (epochs + 1))() if trace else None
    _check(load_library().gmf_project_noalloc(ctx, _ptr(Ynew), y_dtype, int(n_new), _ptr(Xnew),
                                              _ptr(A0), _ptr(U0), int(epochs), int(frozen),
                                              _ptr(A_out), _ptr(U_out), tr))
    return None if tr is None else list(tr)


def gmf_project_warm(ctx, workspace, Ynew, y_dtype, n_new, Xnew, U_cand, epochs, frozen, A_out,
                     U_out, trace: bool = False):
    """Returns (deviance trace or None, wall ms per trace point or None, fallback rows)."""
    tr = (C.c_double * (epochs + 1))() if trace else None
    ms = (C.c_double * (epochs + 1))() if trace else None
    fb = C.c_int64(-1)
    _check(load_library().gmf_project_warm(ctx, _ptr(workspace),
                                           workspace.numel() * workspace.element_size(), _ptr(Ynew),
                                           y_dtype, int(n_new), _ptr(Xnew), _ptr(U_cand),
                                           int(epochs), int(frozen), _ptr(A_out), _ptr(U_out), tr,
                                           ms, C.byref(fb)))
    return (None if tr is None else list(tr)), (None if ms is None else list(ms)), fb.value


def gmf_set_trace(ctx, buffer, records: int):
    return _check(load_library().gmf_set_trace(ctx, _ptr(buffer), int(records)))


def gmf_set_timing(ctx, enable: bool):
    return _check(load_library().gmf_set_timing(ctx, int(bool(enable))))


def gmf_get_timing(ctx):
    """(summed step-launch ms, launches, steps) since the last call."""
    a, b, k = C.c_double(), C.c_double(), C.c_int64()
    _check(load_library().gmf_get_timing(ctx, C.byref(a), C.byref(b), C.byref(k)))
    return a.value, b.value, k.value


def gmf_get_timing_by_kind(ctx):
    """((tile-launch ms, tile launches), (update-launch ms, update launches))
    of the current timing window (not reset)."""
    ms, n = (C.c_double * 2)(), (C.c_double * 2)()
    _check(load_library().gmf_get_timing_by_kind(ctx, ms, n))
    return (ms[0], n[0]), (ms[1], n[1])


def gmf_steps_done(ctx) -> int:
    return load_library().gmf_steps_done(ctx)


def gmf_sync(ctx):
    return _check(load_library().gmf_sync(ctx))


def gmf_destroy(ctx):
    load_library().gmf_destroy(ctx)


# ---------------------------------------------------- torch convenience ----

@dataclass
class FitConfig:
    family: str = "poisson"
    link: str = "log"
    precision: str = "fp32"
    d: int = 1
    R: int = 10
    S: int = 5
    phi: float = 1.0
    nb_alpha: float = 5.0
    lam: tuple = (0.0, 0.0, 1.0, 1.0)
    rate0: float = 0.05
    decay: float = 0.05
    tau: float = 0.75
    alpha1: float = 0.1
    alpha2: float = 0.01
    damping: float = 1e-3
    eps: float = 1e-8
    eta_max: float = 30.0
    bias_mode: int = 0
    seed: int = 0
    tile_rows: int = 0
    skip_block_deviance: int = 0
    panel_stride: int = 0
    tile_waves: int = 0
    eval_overlap: int = 0
    allow_missing: int = 0
    estimate_phi: int = 0
    estimate_alpha: int = 0
    compact_counts: int = 1

    def to_c(self, n, m, p, q) -> gmf_config:
        c = gmf_config_default()
        c.family = FAMILY_CODES[self.family]
        c.link = LINK_CODES[self.link]
        c.precision = PREC_CODES[self.precision]
        c.bias_mode = self.bias_mode
        c.n, c.m, c.d, c.p, c.q = n, m, self.d, p, q
        c.R, c.S = self.R, self.S
        c.phi, c.nb_alpha = self.phi, self.nb_alpha
        for i in range(4):
            c.lambda_[i] = self.lam[i]
        c.rate0, c.decay, c.tau = self.rate0, self.decay, self.tau
        c.alpha1, c.alpha2 = self.alpha1, self.alpha2
        c.damping, c.eps, c.eta_max = self.damping, self.eps, self.eta_max
        c.seed = self.seed
        c.tile_rows = self.tile_rows
        c.skip_block_deviance = self.skip_block_deviance
        c.panel_stride = self.panel_stride
        c.tile_waves = self.tile_waves
        c.eval_overlap = self.eval_overlap
        c.allow_missing = self.allow_missing
        c.estimate_phi = self.estimate_phi
        c.estimate_alpha = self.estimate_alpha
        c.compact_counts = self.compact_counts
        return c


class GMF:
    """Owns a libgmf context, its workspace tensor and the device inputs."""

    def __init__(self, fc: FitConfig, Y, X, Z, B0, A0, U0, V0, W=None, device="cuda:0",
                 stream=None):
        import torch
        self.torch = torch
        dev = torch.device(device)
        self.device = dev
        n, m = Y.shape
        p = X.shape[1] if X is not None else 0
        q = Z.shape[1] if Z is not None else 0
        self.n, self.m, self.p, self.q, self.d = n, m, p, q, fc.d
        self.cfg = fc.to_c(n, m, p, q)
        nbytes = gmf_workspace_bytes(self.cfg, W is not None)
        if nbytes == 0:
            raise GMFError(GMF_EINVAL, "invalid configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)

        def f32(a, shape):
            if a is None or (hasattr(a, "size") and np.size(a) == 0):
                return None
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32).reshape(shape),
                                   device=dev)

        if np.issubdtype(np.asarray(Y).dtype, np.integer):
            Yt = torch.as_tensor(np.ascontiguousarray(Y, dtype=np.int32), device=dev)
            ydt = GMF_Y_INT32
        else:
            Yt = torch.as_tensor(np.ascontiguousarray(Y, dtype=np.float32), device=dev)
            ydt = GMF_Y_FLOAT32
        Xt, Zt = f32(X, (n, p)), f32(Z, (m, q))
        Wt = f32(W, (n, m))
        B0t, A0t = f32(B0, (m, p)), f32(A0, (n, q))
        U0t, V0t = f32(U0, (n, fc.d)), f32(V0, (m, fc.d))
        self.ctx = gmf_init(self.cfg, self._ws, self.stream.cuda_stream, Yt, ydt, Xt, Zt, Wt,
                            B0t, A0t, U0t, V0t)

    # thin forwards -------------------------------------------------------
    def step(self, nsteps=1):
        gmf_step(self.ctx, nsteps)

    def fit(self, max_epochs, tol=0.0, eval_every=1):
        return gmf_fit(self.ctx, max_epochs, tol, eval_every)

    def set_precision(self, precision):
        """gmf_set_precision: 'fp32', 'bf16' or 'bf16x3' for the following steps
        and projections."""
        _check(load_library().gmf_set_precision(self.ctx, PREC_CODES[precision]))

    @property
    def compact_counts(self):
        """gmf_compact_counts: True when the step tiles and the full deviance
        read the 16-bit copy of the counts."""
        rc = load_library().gmf_compact_counts(self.ctx)
        if rc < 0:
            _check(rc)
        return rc == 1

    def run(self, epochs, eval_every=1, trace=True):
        """gmf_run: epochs with the deviance overlapped every eval_every epochs."""
        out = gmf_run(self.ctx, epochs, eval_every, trace)
        self.stream.synchronize()
        return out

    def deviance(self):
        return gmf_deviance(self.ctx)

    def row_deviance(self):
        """gmf_row_deviance: the deviance of every row (float64, n, caller's order)."""
        t = self.torch
        out = t.empty(self.n, dtype=t.float64, device=self.device)
        _check(load_library().gmf_row_deviance(self.ctx, C.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        return out.cpu().numpy()

    def block_deviance(self, count):
        return gmf_block_deviance(self.ctx, count)

    def params(self, postprocess=0):
        t = self.torch
        mk = lambda r, c: t.empty((r, c), dtype=t.float32, device=self.device) if c > 0 else None
        B, A, U, V = mk(self.m, self.p), mk(self.n, self.q), mk(self.n, self.d), mk(self.m, self.d)
        gmf_get_params(self.ctx, B, A, U, V, postprocess)
        self.stream.synchronize()
        cv = lambda x, r: np.zeros((r, 0)) if x is None else x.double().cpu().numpy()
        return cv(B, self.m), cv(A, self.n), cv(U, self.n), cv(V, self.m)

    def moments(self):
        t = self.torch
        ku, kv = self.q + self.d, self.p + self.d
        out = [t.empty((r, c), dtype=t.float64, device=self.device)
               for r, c in ((self.n, ku), (self.n, ku), (self.m, kv), (self.m, kv))]
        gmf_get_moments(self.ctx, *out)
        self.stream.synchronize()
        return [o.cpu().numpy() for o in out]

    def set_params(self, B, A, U, V):
        t = self.torch
        conv = lambda a, r, c: (t.as_tensor(np.ascontiguousarray(a, np.float32).reshape(r, c),
                                            device=self.device) if c > 0 else None)
        gmf_set_params(self.ctx, conv(B, self.m, self.p), conv(A, self.n, self.q),
                       conv(U, self.n, self.d), conv(V, self.m, self.d))

    def initialize(self, Omega, power_iters=2, residual="pearson", y_offset=-1.0):
        """gmf_initialize: the least-squares initialization (Section 4.1) into the
        context's iterate, from the m x k test matrix Omega (caller's column
        order)."""
        t = self.torch
        lib = load_library()
        if isinstance(Omega, t.Tensor):
            Om = Omega.to(self.device).float().contiguous()
        else:
            Om = t.as_tensor(np.ascontiguousarray(Omega, np.float32), device=self.device)
        k = Om.shape[1]
        nbytes = lib.gmf_initialize_workspace_bytes(self.ctx, k)
        if nbytes == 0:
            raise GMFError(GMF_EINVAL, "k must be in [d, 64]")
        ws = t.empty(nbytes + 256, dtype=t.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        _check(lib.gmf_initialize(self.ctx, _ptr(ws[off:off + nbytes]), nbytes, _ptr(Om), k,
                                  int(power_iters), {"pearson": 0, "deviance": 1}[residual],
                                  float(y_offset)))
        self.stream.synchronize()

    def set_column_alpha(self, alpha):
        """gmf_set_column_alpha: one NB shape per column (caller's column order)."""
        t = self.torch
        a = t.as_tensor(np.ascontiguousarray(alpha, np.float32), device=self.device)
        _check(load_library().gmf_set_column_alpha(self.ctx, _ptr(a)))
        self.stream.synchronize()

    def init_spectrum(self, count):
        """gmf_init_spectrum: leading singular values of the last initialization's
        residual matrix."""
        out = (C.c_double * count)()
        _check(load_library().gmf_init_spectrum(self.ctx, out, int(count)))
        return list(out)

    def dispersion(self):
        """gmf_get_dispersion: (phi, NB shape) in use."""
        phi, alpha = C.c_double(), C.c_double()
        _check(load_library().gmf_get_dispersion(self.ctx, C.byref(phi), C.byref(alpha)))
        return phi.value, alpha.value

    def heldout_metrics(self, Ytest):
        """gmf_heldout_metrics: Ytest (n x m) holds the held-out values and NaN
        (or a negative int) elsewhere.  Returns (relative squared log error,
        relative Poisson deviance, relative family deviance, held-out count,
        training mean, training count)."""
        t = self.torch
        if np.issubdtype(np.asarray(Ytest).dtype, np.integer):
            Yt = t.as_tensor(np.ascontiguousarray(Ytest, np.int32), device=self.device)
            ydt = GMF_Y_INT32
        else:
            Yt = t.as_tensor(np.ascontiguousarray(Ytest, np.float32), device=self.device)
            ydt = GMF_Y_FLOAT32
        out = (C.c_double * 6)()
        _check(load_library().gmf_heldout_metrics(self.ctx, _ptr(Yt), ydt, out))
        return tuple(out)

    def save_state(self) -> bytes:
        """gmf_save_state: the fit's state as bytes (host memory)."""
        lib = load_library()
        nbytes = lib.gmf_state_bytes(self.ctx)
        buf = C.create_string_buffer(nbytes)
        _check(lib.gmf_save_state(self.ctx, C.cast(buf, C.c_void_p), nbytes))
        return buf.raw

    def load_state(self, state: bytes):
        """gmf_load_state: resume from bytes written by save_state."""
        buf = C.create_string_buffer(state, len(state))
        _check(load_library().gmf_load_state(self.ctx, C.cast(buf, C.c_void_p), len(state)))

    def schedule(self, t_first=1, count=0):
        return gmf_get_schedule(self.ctx, self.n, self.m, t_first, count)

    def _project_inputs(self, Ynew):
        t = self.torch
        n_new = Ynew.shape[0]
        nbytes = gmf_project_workspace_bytes(self.ctx, n_new)
        if nbytes == 0:
            raise GMFError(GMF_EINVAL, "bad n_new")
        ws = t.empty(nbytes + 256, dtype=t.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        wsv = ws[off:off + nbytes]
        if isinstance(Ynew, t.Tensor):
            Yt = Ynew.to(self.device).contiguous()
            ydt = GMF_Y_INT32 if Yt.dtype == t.int32 else GMF_Y_FLOAT32
        elif np.issubdtype(np.asarray(Ynew).dtype, np.integer):
            Yt = t.as_tensor(np.ascontiguousarray(Ynew, dtype=np.int32), device=self.device)
            ydt = GMF_Y_INT32
        else:
            Yt = t.as_tensor(np.ascontiguousarray(Ynew, dtype=np.float32), device=self.device)
            ydt = GMF_Y_FLOAT32
        return n_new, ws, wsv, Yt, ydt

    def _dev_f32(self, a, n_new, c):
        t = self.torch
        if c == 0 or a is None:
            return None
        if isinstance(a, t.Tensor):
            return a.to(self.device).float().contiguous()
        return t.as_tensor(np.ascontiguousarray(a, np.float32).reshape(n_new, c), device=self.device)

    def project(self, Ynew, Xnew, A0, U0, epochs, frozen=0, trace=False):
        """Row-side fit of new rows with the column side frozen (gmf_project)."""
        t = self.torch
        n_new, ws, wsv, Yt, ydt = self._project_inputs(Ynew)
        Xt = self._dev_f32(Xnew, n_new, self.p)
        At = self._dev_f32(A0, n_new, self.q)
        Ut = self._dev_f32(U0, n_new, self.d)
        Ao = t.empty((n_new, self.q), dtype=t.float32, device=self.device) if self.q else None
        Uo = t.empty((n_new, self.d), dtype=t.float32, device=self.device)
        tr = gmf_project(self.ctx, wsv, Yt, ydt, n_new, Xt, At, Ut, epochs, frozen, Ao, Uo, trace)
        self.stream.synchronize()
        return Ao, Uo, tr

    def project_noalloc(self, Ynew, Xnew, A0, U0, epochs, frozen=0, trace=False):
        """gmf_project_noalloc: as project(), with the library's resident scratch
        instead of a workspace (inputs and outputs still come from the caller)."""
        t = self.torch
        n_new = Ynew.shape[0]
        if isinstance(Ynew, t.Tensor):
            Yt = Ynew.to(self.device).contiguous()
            ydt = GMF_Y_INT32 if Yt.dtype == t.int32 else GMF_Y_FLOAT32
        elif np.issubdtype(np.asarray(Ynew).dtype, np.integer):
            Yt = t.as_tensor(np.ascontiguousarray(Ynew, dtype=np.int32), device=self.device)
            ydt = GMF_Y_INT32
        else:
            Yt = t.as_tensor(np.ascontiguousarray(Ynew, dtype=np.float32), device=self.device)
            ydt = GMF_Y_FLOAT32
        Xt = self._dev_f32(Xnew, n_new, self.p)
        At = self._dev_f32(A0, n_new, self.q)
        Ut = self._dev_f32(U0, n_new, self.d)
        Ao = t.empty((n_new, self.q), dtype=t.float32, device=self.device) if self.q else None
        Uo = t.empty((n_new, self.d), dtype=t.float32, device=self.device)
        tr = gmf_project_noalloc(self.ctx, Yt, ydt, n_new, Xt, At, Ut, epochs, frozen, Ao, Uo,
                                 trace)
        self.stream.synchronize()
        return Ao, Uo, tr

    def project_warm(self, Ynew, Xnew, U_cand, epochs, frozen=1, trace=False):
        """gmf_project_warm: starting values built on the device (row intercept;
        U_cand per row where it lowers the row deviance, else 0; U_cand None =
        cold start).  Returns (A, U, deviance trace, wall ms trace, fallback rows)."""
        t = self.torch
        n_new, ws, wsv, Yt, ydt = self._project_inputs(Ynew)
        Xt = self._dev_f32(Xnew, n_new, self.p)
        Uc = self._dev_f32(U_cand, n_new, self.d)
        Ao = t.empty((n_new, self.q), dtype=t.float32, device=self.device) if self.q else None
        Uo = t.empty((n_new, self.d), dtype=t.float32, device=self.device)
        tr, ms, fb = gmf_project_warm(self.ctx, wsv, Yt, ydt, n_new, Xt, Uc, epochs, frozen, Ao,
                                      Uo, trace)
        self.stream.synchronize()
        return Ao, Uo, tr, ms, fb

    def set_trace(self, buffer, records):
        gmf_set_trace(self.ctx, buffer, records)

    def set_timing(self, enable):
        gmf_set_timing(self.ctx, enable)

    def get_timing(self):
        return gmf_get_timing(self.ctx)

    def get_timing_by_kind(self):
        return gmf_get_timing_by_kind(self.ctx)

    def steps_done(self):
        return gmf_steps_done(self.ctx)

    def sync(self):
        gmf_sync(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            gmf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ encoder ----

def _echeck(rc):
    if rc != GMF_OK:
        raise GMFError(rc, load_library().gmf_encoder_last_error().decode())
    return rc


class Encoder:
    """Warm-start MLP encoder (gmf_encoder_*): weights in a torch workspace."""

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, m, d, weights, hidden=256, batch=256, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, weight_decay=0.0, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        lib = load_library()
        cfg = gmf_mlp_config()
        lib.gmf_mlp_config_default(C.byref(cfg))
        cfg.m, cfg.hidden, cfg.d, cfg.batch = m, hidden, d, batch
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, cfg.weight_decay = lr, beta1, beta2, eps, weight_decay
        self.cfg = cfg
        self.m, self.d, self.hidden = m, d, hidden
        nbytes = lib.gmf_encoder_workspace_bytes(C.byref(cfg))
        if nbytes == 0:
            raise GMFError(GMF_EINVAL, "invalid encoder configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        ws = self.workspace[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        w = [torch.as_tensor(np.ascontiguousarray(weights[k], np.float32), device=self.device)
             for k in self.NAMES]
        self.enc = C.c_void_p()
        _echeck(lib.gmf_encoder_init(C.byref(self.enc), C.byref(cfg), ws.data_ptr(), nbytes,
                                     self.stream.cuda_stream, *[t.data_ptr() for t in w]))
        self.nparam = (hidden * m + hidden + hidden * hidden + hidden + d * hidden + d)

    def _y(self, Y):
        t = self.torch
        if isinstance(Y, t.Tensor):
            Yt = Y.to(self.device).contiguous()
            return Yt, (GMF_Y_INT32 if Yt.dtype == t.int32 else GMF_Y_FLOAT32)
        if np.issubdtype(np.asarray(Y).dtype, np.integer):
            return t.as_tensor(np.ascontiguousarray(Y, np.int32), device=self.device), GMF_Y_INT32
        return t.as_tensor(np.ascontiguousarray(Y, np.float32), device=self.device), GMF_Y_FLOAT32

    def _u(self, U):
        t = self.torch
        if isinstance(U, t.Tensor):
            return U.to(self.device).float().contiguous()
        return t.as_tensor(np.ascontiguousarray(U, np.float32), device=self.device)

    def train(self, Y, U, epochs, trace=True):
        Yt, ydt = self._y(Y)
        Ut = self._u(U)
        tr = (C.c_double * max(epochs, 1))() if trace else None
        _echeck(load_library().gmf_encoder_train(self.enc, Yt.data_ptr(), ydt, Ut.data_ptr(),
                                                 Yt.shape[0], int(epochs), tr))
        self.stream.synchronize()
        return list(tr)[:epochs] if trace else None

    def forward(self, Y, bf16=True, fused=True):
        """Encoder output; bf16 with fused=False runs the layer-by-layer kernels."""
        t = self.torch
        Yt, ydt = self._y(Y)
        out = t.empty((Yt.shape[0], self.d), dtype=t.float32, device=self.device)
        mode = 0 if not bf16 else (1 if fused else 2)
        _echeck(load_library().gmf_encoder_forward(self.enc, Yt.data_ptr(), ydt, Yt.shape[0],
                                                   out.data_ptr(), mode))
        self.stream.synchronize()
        return out

    def loss_grad(self, Y, U):
        t = self.torch
        Yt, ydt = self._y(Y)
        Ut = self._u(U)
        g = t.empty(self.nparam, dtype=t.float32, device=self.device)
        loss = C.c_double()
        _echeck(load_library().gmf_encoder_loss_grad(self.enc, Yt.data_ptr(), ydt, Ut.data_ptr(),
                                                     Yt.shape[0], C.byref(loss), g.data_ptr()))
        gn = g.cpu().numpy().astype(np.float64)
        H, m, d = self.hidden, self.m, self.d
        out, o = {}, 0
        for k, shp in (("W1", (H, m)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                       ("W3", (d, H)), ("b3", (d,))):
            sz = int(np.prod(shp))
            out[k] = gn[o:o + sz].reshape(shp)
            o += sz
        return loss.value, out

    def weights(self):
        t = self.torch
        H, m, d = self.hidden, self.m, self.d
        shapes = {"W1": (H, m), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (d, H), "b3": (d,)}
        ts = {k: t.empty(s, dtype=t.float32, device=self.device) for k, s in shapes.items()}
        _echeck(load_library().gmf_encoder_get_weights(self.enc, *[ts[k].data_ptr()
                                                                   for k in self.NAMES]))
        return {k: v.cpu().numpy().astype(np.float64) for k, v in ts.items()}

    def close(self):
        if getattr(self, "enc", None) is not None and self.enc.value:
            load_library().gmf_encoder_destroy(self.enc)
            self.enc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ batched fits --

class Batch:
    """Several GMF contexts advanced together (gmf_batch_*)."""

    def __init__(self, gmfs, table_epochs=4, use_graph=True, mode=None):
        """mode: 0 fixed launch sequence, 1 its recorded HIP graph, 2 level
        placement (gmf_batch_init); None: 1 if use_graph else 0."""
        import torch
        self.torch = torch
        self.gmfs = list(gmfs)
        lib = load_library()
        n = len(self.gmfs)
        self._ctxs = (C.c_void_p * n)(*[g.ctx.value for g in self.gmfs])
        nbytes = lib.gmf_batch_workspace_bytes(self._ctxs, n, int(table_epochs))
        if nbytes == 0:
            raise GMFError(GMF_EINVAL, "invalid batch")
        dev = self.gmfs[0].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.batch = C.c_void_p()
        if mode is None:
            mode = 1 if use_graph else 0
        _check(lib.gmf_batch_init(C.byref(self.batch), self._ctxs, n,
                                  self.workspace.data_ptr() + off, nbytes, int(table_epochs),
                                  int(mode)))

    def run(self, epochs, eval_every=1, trace=True):
        """Run `epochs` epochs; returns the deviance trace (nfits x evaluations) or None."""
        n = len(self.gmfs)
        nev = epochs // eval_every
        tr = (C.c_double * max(1, n * nev))() if trace else None
        _check(load_library().gmf_batch_run(self.batch, int(epochs), int(eval_every), tr))
        if not trace:
            return None
        return np.array(list(tr)[:n * nev]).reshape(n, nev)

    def close(self):
        if getattr(self, "batch", None) is not None and self.batch.value:
            load_library().gmf_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ tuning --

def tune_table_load(path):
    _check(load_library().gmf_tune_table_load(str(path).encode()))


def tune_table_save(path):
    _check(load_library().gmf_tune_table_save(str(path).encode()))


def tune_table_clear():
    load_library().gmf_tune_table_clear()


def tune_lookup(cfg: gmf_config) -> int:
    return int(load_library().gmf_tune_lookup(C.byref(cfg)))


def tune(fc: FitConfig, Y, X, Z, B0, A0, U0, V0, candidates=(32, 64, 128, 256, 512),
         steps=50, device="cuda:0", stream=None):
    """gmf_tune on the given problem: returns (best tile_rows, {candidate: us per step});
    the best value is recorded in the library's table for this shape class."""
    import torch
    dev = torch.device(device)
    Y = np.asarray(Y)
    n, m = Y.shape
    p = 0 if X is None else np.asarray(X).reshape(n, -1).shape[1]
    q = 0 if Z is None else np.asarray(Z).reshape(m, -1).shape[1]
    cfg = fc.to_c(n, m, p, q)
    need = 0
    for cand in candidates:
        ci = fc.to_c(n, m, p, q)
        ci.tile_rows = int(cand)
        nb = gmf_workspace_bytes(ci, False)
        if nb == 0:
            raise GMFError(GMF_EINVAL, f"bad candidate {cand}")
        need = max(need, nb)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    f32 = lambda a: None if a is None else torch.as_tensor(np.ascontiguousarray(a, np.float32),
                                                          device=dev)
    if np.issubdtype(Y.dtype, np.integer):
        Yt, ydt = torch.as_tensor(np.ascontiguousarray(Y, np.int32), device=dev), GMF_Y_INT32
    else:
        Yt, ydt = f32(Y), GMF_Y_FLOAT32
    Xt, Zt = f32(None if p == 0 else X), f32(None if q == 0 else Z)
    Bt, At = f32(None if p == 0 else B0), f32(None if q == 0 else A0)
    Ut, Vt = f32(U0), f32(V0)
    cands = (C.c_int32 * len(candidates))(*[int(c) for c in candidates])
    us = (C.c_double * len(candidates))()
    best = C.c_int32(0)
    _check(load_library().gmf_tune(C.byref(cfg), ws.data_ptr() + off, need, st.cuda_stream,
                                   _ptr(Yt), ydt, _ptr(Xt), _ptr(Zt), None, _ptr(Bt), _ptr(At),
                                   _ptr(Ut), _ptr(Vt), cands, len(candidates), int(steps),
                                   C.byref(best), us))
    return best.value, {int(c): float(u) for c, u in zip(candidates, us)}


# ------------------------------------------------------------ rank selection --

def rank_eigengap(eigenvalues, rmax):
    """gmf_rank_eigengap (Onatski's edge-distribution estimator) on host values."""
    ev = np.ascontiguousarray(eigenvalues, dtype=np.float64)
    r = C.c_int32()
    _check(load_library().gmf_rank_eigengap(ev.ctypes.data_as(C.POINTER(C.c_double)), len(ev),
                                            int(rmax), C.byref(r)))
    return r.value


def rank_select_cv(dev_table):
    """gmf_rank_select_cv: index of the candidate with the smallest mean held-out
    deviance; dev_table is candidates x folds."""
    t = np.ascontiguousarray(dev_table, dtype=np.float64)
    best = C.c_int32()
    _check(load_library().gmf_rank_select_cv(t.ctypes.data_as(C.POINTER(C.c_double)), t.shape[0],
                                             t.shape[1], C.byref(best)))
    return best.value


def cv_rank_table(fc: FitConfig, Y, X, Z, B0, A0, starts, folds, epochs, metric=2,
                  device="cuda:0", mode=2):
    """Out-of-sample rank selection (Section 4.2) on the batched engine: for
    every candidate rank d (starts: {d: (U0, V0)}) and fold (a boolean mask of
    held-out entries), a fit of Y with the fold's entries missing; all fits
    advance together in one batch (gmf_batch_*) for `epochs` epochs, then
    gmf_heldout_metrics scores each on its held-out entries.  Returns
    (ranks, table[rank][fold] = metric `metric` of gmf_heldout_metrics, best
    rank by gmf_rank_select_cv)."""
    import dataclasses
    ranks = sorted(starts)
    p = X.shape[1] if X is not None else 0
    q = Z.shape[1] if Z is not None else 0
    stride = max(((p + q + d + 15) // 16) * 16 for d in ranks)
    Yf = np.asarray(Y, dtype=np.float64)
    fits = []
    for d in ranks:
        for mask in folds:
            f = dataclasses.replace(fc, d=d, allow_missing=1, panel_stride=stride,
                                    skip_block_deviance=1)
            Ytr = np.where(mask, np.nan, Yf).astype(np.float32)
            U0, V0 = starts[d]
            fits.append(GMF(f, Ytr, X, Z, B0, A0, U0, V0, device=device))
    b = Batch(fits, table_epochs=max(epochs, 1), mode=mode)
    b.run(epochs, trace=False)
    b.close()
    table = np.zeros((len(ranks), len(folds)))
    k = 0
    for i, _ in enumerate(ranks):
        for j, mask in enumerate(folds):
            Ytest = np.where(mask, Yf, np.nan).astype(np.float32)
            table[i, j] = fits[k].heldout_metrics(Ytest)[metric]
            fits[k].close()
            k += 1
    return ranks, table, ranks[rank_select_cv(table)]

