"""MI355X (gfx950) per-event LO integrand: thin Python binding of ``libmf.so``.

Argument marshalling only: every step of the event pipeline runs in the HIP
kernels of the library (``include/mf.h`` documents each entry point).  torch
supplies device memory and streams.  The library must have been built
(``python -m paper_2105_10529_amd.build_lib`` or ``__graft_entry__.build()``);
there is no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf.so")

MF_OK, MF_EINVAL, MF_ERANGE, MF_ENOMEM, MF_EDEVICE, MF_ENOTSUP = range(6)
PROCESSES = {"gg>ttx": 0, "uux>ttx": 1, "ddx>ttx": 2, "gg>ttxg": 3, "gg>ttxgg": 4, "gg>ttxggg": 5,
             "uux>ttxg": 6, "ddx>ttxg": 7, "qg>ttxq": 8}
PRECISIONS = {"fp64": 0, "fp32": 1}
NOALLOC_MAX_POINTS = 1 << 22  # MF_NOALLOC_MAX_POINTS of include/mf.h
DEFAULT_PDF = (1.6, -0.2, -0.05, 5.0, 0.3,   # g
               2.2, 0.5, -0.02, 3.0, 0.2,    # u
               1.1, 0.5, -0.02, 4.0, 0.2,    # d
               0.2, -0.2, -0.05, 7.0, 0.3)   # u~ (= d~)


class MFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mf status {status}: {msg}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [
        ("process", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("sqrt_s", ctypes.c_double),
        ("m_t", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("alpha_s", ctypes.c_double),
        ("pt_min", ctypes.c_double),
        ("eta_max", ctypes.c_double),
        ("dr_min", ctypes.c_double),
        ("pdf_params", ctypes.c_double * 20),
        ("n_bins", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("helicity", ctypes.c_int32),
        ("dynamic_scale", ctypes.c_int32),
        ("colour_form", ctypes.c_int32),
    ]


class _IntegrateOpts(ctypes.Structure):
    _fields_ = [
        ("n_iter", ctypes.c_int32),
        ("n_events", ctypes.c_int64),
        ("target_rel_err", ctypes.c_double),
        ("warmup_iters_discarded", ctypes.c_int32),
        ("adapt", ctypes.c_int32),
        ("iter_offset", ctypes.c_uint64),
        ("edges_in", ctypes.c_void_p),
        ("edges_out", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("flow", ctypes.c_void_p),
        ("flow_mix", ctypes.c_double),
        ("prior", ctypes.c_void_p),
        ("obs", ctypes.c_void_p),
        ("fallback_rel_var", ctypes.c_double),
    ]


N_OBS = 3
OBSERVABLES = ("pt_top", "m_ttbar", "pt_gluon_max")


class _Observables(ctypes.Structure):
    _fields_ = [
        ("nbins", ctypes.c_int32),
        ("lo", ctypes.c_double * N_OBS),
        ("hi", ctypes.c_double * N_OBS),
        ("sums", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p),
    ]


class _FlowConfig(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n_layers", ctypes.c_int32),
        ("hidden", ctypes.c_int32),
        ("bins", ctypes.c_int32),
        ("max_batch", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
    ]


class _FlowTrainOpts(ctypes.Structure):
    _fields_ = [
        ("epochs", ctypes.c_int32),
        ("batch", ctypes.c_int64),
        ("lr", ctypes.c_double),
        ("lr_final", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("loss", ctypes.c_int32),
    ]


class _FlowOnlineOpts(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int32),
        ("batch", ctypes.c_int64),
        ("lr", ctypes.c_double),
        ("lr_final", ctypes.c_double),
        ("loss", ctypes.c_int32),
        ("flow_mix", ctypes.c_double),
        ("iter_offset", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
        ("group_steps", ctypes.c_int32),
        ("target_rel_err", ctypes.c_double),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("integral", ctypes.c_double),
        ("error", ctypes.c_double),
        ("chi2_dof", ctypes.c_double),
        ("n_iter_done", ctypes.c_int32),
        ("n_events_total", ctypes.c_int64),
        ("n_nonzero", ctypes.c_int64),
        ("n_nonfinite", ctypes.c_int64),
        ("seconds", ctypes.c_double),
        ("time_to_target", ctypes.c_double),
        ("kernel_seconds", ctypes.c_double),
        ("iter_integral", ctypes.c_void_p),
        ("iter_error", ctypes.c_void_p),
        ("fallback_iter", ctypes.c_int32),
        ("flow_rel_var", ctypes.c_double),
        ("iter_seconds", ctypes.c_void_p),
    ]


EXPORTS = ("mf_process_create", "mf_process_destroy", "mf_process_ndim", "mf_last_error", "mf_integrand",
           "mf_integrand_grad", "mf_vegas_refine", "mf_integrate", "mf_grad", "mf_weights", "mf_weight_stats",
           "mf_flow_create", "mf_flow_destroy", "mf_flow_ndim", "mf_flow_param_count", "mf_flow_masks",
           "mf_flow_set_params", "mf_flow_get_params", "mf_flow_forward", "mf_flow_inverse", "mf_flow_loss_grad",
           "mf_flow_adam_step", "mf_flow_train", "mf_flow_train_online", "mf_vjp", "mf_integrand_noalloc",
           "mf_vjp_workspace", "mf_weight_stats_workspace")

_lib = None


def lib():
    """Load libmf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.mf_process_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(P)]
        L.mf_process_create.restype = i32
        L.mf_process_destroy.argtypes = [P]
        L.mf_process_destroy.restype = None
        L.mf_process_ndim.argtypes = [P]
        L.mf_process_ndim.restype = ctypes.c_int
        L.mf_last_error.argtypes = []
        L.mf_last_error.restype = ctypes.c_char_p
        L.mf_integrand.argtypes = [P, P, i64, P, P]
        L.mf_integrand.restype = i32
        L.mf_integrand_noalloc.argtypes = [P, P, i64, P, P]
        L.mf_integrand_noalloc.restype = i32
        L.mf_integrand_grad.argtypes = [P, P, i64, P, P, P]
        L.mf_integrand_grad.restype = i32
        L.mf_vegas_refine.argtypes = [P, P, ctypes.c_int, ctypes.c_int, d, P, P]
        L.mf_vegas_refine.restype = i32
        L.mf_integrate.argtypes = [P, ctypes.POINTER(_IntegrateOpts), ctypes.POINTER(_Result)]
        L.mf_integrate.restype = i32
        L.mf_grad.argtypes = [P, ctypes.POINTER(_IntegrateOpts), P, P]
        L.mf_grad.restype = i32
        L.mf_weights.argtypes = [P, P, d, ctypes.c_uint64, i64, P, P, P]
        L.mf_weights.restype = i32
        L.mf_weight_stats.argtypes = [P, i64, d, P, P, i64, P]
        L.mf_weight_stats.restype = i32
        L.mf_weight_stats_workspace.argtypes = [i64]
        L.mf_weight_stats_workspace.restype = i64
        L.mf_vjp.argtypes = [P, i32, P, i64, P, P, i64, P]
        L.mf_vjp.restype = i32
        L.mf_vjp_workspace.argtypes = [i32, i64]
        L.mf_vjp_workspace.restype = i64
        L.mf_flow_create.argtypes = [ctypes.POINTER(_FlowConfig), ctypes.POINTER(P)]
        L.mf_flow_create.restype = i32
        L.mf_flow_destroy.argtypes = [P]
        L.mf_flow_destroy.restype = None
        L.mf_flow_ndim.argtypes = [P]
        L.mf_flow_ndim.restype = ctypes.c_int
        L.mf_flow_param_count.argtypes = [P]
        L.mf_flow_param_count.restype = i64
        L.mf_flow_masks.argtypes = [P, P]
        L.mf_flow_masks.restype = i32
        L.mf_flow_set_params.argtypes = [P, P, i64]
        L.mf_flow_set_params.restype = i32
        L.mf_flow_get_params.argtypes = [P, P, i64]
        L.mf_flow_get_params.restype = i32
        L.mf_flow_forward.argtypes = [P, P, i64, P, P, P]
        L.mf_flow_forward.restype = i32
        L.mf_flow_inverse.argtypes = [P, P, i64, P, P, P]
        L.mf_flow_inverse.restype = i32
        L.mf_flow_loss_grad.argtypes = [P, P, P, i64, i32, P, ctypes.POINTER(d), P]
        L.mf_flow_loss_grad.restype = i32
        L.mf_flow_adam_step.argtypes = [P, d, P]
        L.mf_flow_adam_step.restype = i32
        L.mf_flow_train.argtypes = [P, P, P, i64, ctypes.POINTER(_FlowTrainOpts), P]
        L.mf_flow_train.restype = i32
        L.mf_flow_train_online.argtypes = [P, P, ctypes.POINTER(_FlowOnlineOpts), P, ctypes.POINTER(_Result)]
        L.mf_flow_train_online.restype = i32
        _lib = L
    return _lib


def _check(status: int):
    if status != MF_OK:
        raise MFError(status, lib().mf_last_error().decode())


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_ptr(t, dtype_name="float64") -> int:
    import torch

    assert t.is_cuda, "device tensor expected"
    assert t.dtype == getattr(torch, dtype_name), f"{dtype_name} tensor expected"
    assert t.is_contiguous(), "contiguous tensor expected"
    return t.data_ptr()


@dataclass
class Config:
    process: str = "gg>ttx"
    precision: str = "fp64"
    sqrt_s: float = 13000.0
    m_t: float = 173.0
    mu: float = -1.0
    alpha_s: float = 0.118
    pt_min: float = 20.0
    eta_max: float = 2.5
    dr_min: float = 0.0
    pdf_params: tuple = DEFAULT_PDF
    n_bins: int = 50
    alpha: float = 1.5
    seed: int = 2105105290
    helicity: int = 0  # g g -> t t~ g g g: 0 sum, 1 one sampled state (x64), 2 + k only state k
    dynamic_scale: bool = False  # True: mu = H_T / 2 per event
    colour_form: int = 0  # g g -> t t~ g g: 0 default, 1 vector ALUs in registers, 2 matrix cores

    def _c(self) -> _Config:
        c = _Config()
        c.process = PROCESSES[self.process]
        c.precision = PRECISIONS[self.precision]
        c.sqrt_s, c.m_t, c.mu, c.alpha_s = self.sqrt_s, self.m_t, self.mu, self.alpha_s
        c.pt_min, c.eta_max, c.dr_min = self.pt_min, self.eta_max, self.dr_min
        for k in range(20):
            c.pdf_params[k] = float(self.pdf_params[k])
        c.n_bins, c.alpha, c.seed = self.n_bins, self.alpha, self.seed
        c.helicity = self.helicity
        c.dynamic_scale = int(self.dynamic_scale)
        c.colour_form = self.colour_form
        return c


@dataclass
class IntegrationResult:
    integral: float
    error: float
    chi2_dof: float
    n_iter_done: int
    n_events_total: int
    n_nonzero: int
    n_nonfinite: int
    seconds: float
    time_to_target: float
    kernel_seconds: float
    iter_integral: np.ndarray = field(default_factory=lambda: np.zeros(0))
    iter_error: np.ndarray = field(default_factory=lambda: np.zeros(0))
    observables: dict | None = None  # see Process.integrate(observables=...)
    fallback_iter: int = -1          # first iteration that sampled VEGAS after a flow fallback, -1 none
    flow_rel_var: float = -1.0       # per-event relative variance of the flow's first iteration (fallback test)
    iter_seconds: np.ndarray = field(default_factory=lambda: np.zeros(0))  # wall time at each iteration's end


class Process:
    """An integrand on the current HIP device (mf_process_create)."""

    def __init__(self, cfg: Config | None = None, **kw):
        self.cfg = cfg if cfg is not None else Config(**kw)
        h = ctypes.c_void_p()
        c = self.cfg._c()
        _check(lib().mf_process_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mf_process_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ndim(self) -> int:
        return lib().mf_process_ndim(self._h)

    @property
    def nbins(self) -> int:
        return self.cfg.n_bins

    def integrand(self, u, w=None, stream=None):
        """w[n] = integrand at u ([ndim][n] float64 cuda tensor, SoA) -- mf_integrand."""
        import torch

        n = u.shape[1] if u.dim() == 2 else 0
        assert u.dim() == 2 and u.shape[0] == self.ndim
        if w is None:
            w = torch.empty(n, dtype=torch.float64, device=u.device)
        _check(lib().mf_integrand(self._h, _dev_ptr(u), n, _dev_ptr(w), _stream_ptr(stream)))
        return w

    def integrand_noalloc(self, u, w, stream=None):
        """w[n] = integrand at u into a caller-allocated w, with no device allocation -- mf_integrand_noalloc."""
        assert u.dim() == 2 and u.shape[0] == self.ndim and w.dim() == 1 and w.shape[0] == u.shape[1]
        _check(lib().mf_integrand_noalloc(self._h, _dev_ptr(u), u.shape[1], _dev_ptr(w), _stream_ptr(stream)))
        return w

    def integrand_grad(self, u, stream=None):
        """(w[n], dw[9][n]) -- mf_integrand_grad."""
        import torch

        n = u.shape[1]
        w = torch.empty(n, dtype=torch.float64, device=u.device)
        dw = torch.empty((9, n), dtype=torch.float64, device=u.device)
        _check(lib().mf_integrand_grad(self._h, _dev_ptr(u), n, _dev_ptr(w), _dev_ptr(dw), _stream_ptr(stream)))
        return w, dw

    def integrate(self, n_iter: int, n_events: int, target_rel_err: float = 0.0, warmup: int = 0, adapt: bool = True,
                  iter_offset: int = 0, edges_in=None, edges_out=None, stream=None,
                  flow: "Flow | None" = None, flow_mix: float = 0.0,
                  prior: "IntegrationResult | None" = None, observables: dict | None = None,
                  fallback_rel_var: float = 0.0) -> IntegrationResult:
        """VEGAS integration entirely on the device -- mf_integrate (flow: learned proposal, frozen grid;
        fallback_rel_var: with a flow, the VEGAS proposal's per-event relative variance on that grid, above
        which the flow's first iteration switches the rest to VEGAS; prior: an earlier estimate combined
        with the new iterations; observables: {"nbins": n, "lo": (3,), "hi": (3,)} fills histograms of
        OBSERVABLES, returned as result.observables with the raw per-bin sums of w and w^2
        ([3][nbins][2]), the bin edges, and the library's per-bin cross sections (pb) and Monte Carlo
        errors over the counted iterations)."""
        o = _IntegrateOpts()
        ob = sums = sig = None
        if observables is not None:
            nb = int(observables["nbins"])
            sums = np.zeros((N_OBS, nb, 2))
            sig = np.zeros((N_OBS, nb, 2))
            ob = _Observables()
            ob.nbins = nb
            for q in range(N_OBS):
                ob.lo[q] = float(observables["lo"][q])
                ob.hi[q] = float(observables["hi"][q])
            ob.sums = sums.ctypes.data
            ob.sigma = sig.ctypes.data
            o.obs = ctypes.addressof(ob)
        o.fallback_rel_var = fallback_rel_var
        o.flow = flow._h.value if flow is not None else None
        o.flow_mix = flow_mix
        pr = None
        if prior is not None:
            pr = _Result()
            pr.integral, pr.error = prior.integral, prior.error
            o.prior = ctypes.addressof(pr)
        o.n_iter, o.n_events, o.target_rel_err = n_iter, n_events, target_rel_err
        o.warmup_iters_discarded, o.adapt, o.iter_offset = warmup, int(adapt), iter_offset
        o.edges_in = _dev_ptr(edges_in) if edges_in is not None else None
        o.edges_out = _dev_ptr(edges_out) if edges_out is not None else None
        o.stream = _stream_ptr(stream)
        r = _Result()
        Ii = np.zeros(n_iter)
        Ie = np.zeros(n_iter)
        Is = np.zeros(n_iter)
        r.iter_integral = Ii.ctypes.data
        r.iter_error = Ie.ctypes.data
        r.iter_seconds = Is.ctypes.data
        _check(lib().mf_integrate(self._h, ctypes.byref(o), ctypes.byref(r)))
        k = r.n_iter_done
        res = IntegrationResult(r.integral, r.error, r.chi2_dof, k, r.n_events_total, r.n_nonzero, r.n_nonfinite,
                                r.seconds, r.time_to_target, r.kernel_seconds, Ii[:k].copy(), Ie[:k].copy())
        res.fallback_iter = r.fallback_iter
        res.flow_rel_var = r.flow_rel_var
        res.iter_seconds = Is[:k].copy()
        if sums is not None:
            res.observables = {
                "names": OBSERVABLES, "sums": sums, "events": float(n_events) * max(k - warmup, 0),
                "edges": [np.linspace(observables["lo"][q], observables["hi"][q], sums.shape[1] + 1)
                          for q in range(N_OBS)],
                "sigma_pb": sig[:, :, 0].copy(), "error_pb": sig[:, :, 1].copy()}
        return res

    def weights(self, it: int, n: int, flow: "Flow | None" = None, want_y: bool = False, stream=None,
                flow_mix: float = 0.0):
        """(w[n] float64, y[ndim][n] float32 or None) of one frozen-grid sample -- mf_weights."""
        import torch

        w = torch.empty(n, dtype=torch.float64, device="cuda")
        y = torch.empty((self.ndim, n), dtype=torch.float32, device="cuda") if want_y else None
        _check(lib().mf_weights(self._h, flow._h.value if flow is not None else None, flow_mix, it, n,
                                _dev_ptr(y, "float32") if y is not None else None, _dev_ptr(w),
                                _stream_ptr(stream)))
        return w, y

    def train_flow_online(self, flow: "Flow", steps: int, batch: int = 16384, lr: float = 1e-3,
                          lr_final: float = 1e-5, loss: str = "variance", flow_mix: float = 0.1,
                          iter_offset: int = 1 << 20, stream=None, group_steps: int = 0, target_rel_err: float = 0.0,
                          with_estimate: bool = False):
        """On-policy training of the flow on this integrand -- mf_flow_train_online.

        Returns the relative variance per event of each step's batch, and with
        with_estimate also the combined estimate of the integral from the
        training batches (IntegrationResult)."""
        o = _FlowOnlineOpts(steps, batch, lr, lr_final, Flow.LOSSES[loss], flow_mix, iter_offset, _stream_ptr(stream),
                            group_steps, target_rel_err)
        out = np.zeros(steps)
        r = _Result()
        ng = -(-steps // (group_steps if group_steps > 0 else steps))
        Ii, Ie = np.zeros(ng), np.zeros(ng)
        r.iter_integral, r.iter_error = Ii.ctypes.data, Ie.ctypes.data
        _check(lib().mf_flow_train_online(self._h, flow._h, ctypes.byref(o), out.ctypes.data, ctypes.byref(r)))
        if not with_estimate:
            return out
        k = r.n_iter_done
        est = IntegrationResult(r.integral, r.error, r.chi2_dof, k, r.n_events_total, r.n_nonzero, r.n_nonfinite,
                                r.seconds, r.time_to_target, r.kernel_seconds, Ii[:k].copy(), Ie[:k].copy())
        return out, est

    def grad(self, n_events: int, iter_offset: int = 0, edges_in=None, stream=None):
        """(values[10], errors[10]): sigma, d sigma/d m_t, d sigma/d theta_0..7 -- mf_grad."""
        o = _IntegrateOpts()
        o.n_iter, o.n_events, o.iter_offset = 1, n_events, iter_offset
        o.edges_in = _dev_ptr(edges_in) if edges_in is not None else None
        o.stream = _stream_ptr(stream)
        out = np.zeros(10)
        err = np.zeros(10)
        _check(lib().mf_grad(self._h, ctypes.byref(o), out.ctypes.data, err.ctypes.data))
        return out, err


def vjp(dw, g, stream=None):
    """out[j] = sum_e dw[j][e] g[e] on the device -- mf_vjp."""
    import torch

    k, n = dw.shape
    out = torch.empty(k, dtype=torch.float64, device=dw.device)
    nbytes = lib().mf_vjp_workspace(k, n)
    work = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dw.device)
    _check(lib().mf_vjp(_dev_ptr(dw), k, _dev_ptr(g), n, _dev_ptr(out), _dev_ptr(work), 8 * work.numel(),
                        _stream_ptr(stream)))
    return out


def weight_stats(w, q: float = 0.999, stream=None) -> dict:
    """mean, max, q-quantile, non-zero count and relative variance per event of device weights -- mf_weight_stats."""
    import torch

    out = np.zeros(5)
    nbytes = lib().mf_weight_stats_workspace(w.numel())
    work = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=w.device)
    _check(lib().mf_weight_stats(_dev_ptr(w), w.numel(), q, out.ctypes.data, _dev_ptr(work), 8 * work.numel(),
                                 _stream_ptr(stream)))
    return {"mean": out[0], "max": out[1], "quantile": out[2], "nonzero": int(out[3]), "relvar": out[4]}


class Flow:
    """Coupling normalising flow on the device (include/mf_flow.h)."""

    HIDDEN = 256
    BINS = 32

    def __init__(self, ndim: int, n_layers: int = 6, max_batch: int = 16384, seed: int = 2105105290):
        c = _FlowConfig(ndim, n_layers, self.HIDDEN, self.BINS, max_batch, seed)
        h = ctypes.c_void_p()
        _check(lib().mf_flow_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        self.ndim, self.n_layers, self.max_batch = ndim, n_layers, max_batch

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mf_flow_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return lib().mf_flow_param_count(self._h)

    def masks(self) -> np.ndarray:
        out = np.zeros((self.n_layers, self.ndim), dtype=np.uint8)
        _check(lib().mf_flow_masks(self._h, out.ctypes.data))
        return out.astype(bool)

    def set_params(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().mf_flow_set_params(self._h, flat.ctypes.data, flat.size))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.param_count, dtype=np.float32)
        _check(lib().mf_flow_get_params(self._h, out.ctypes.data, out.size))
        return out

    @staticmethod
    def flatten(layers) -> np.ndarray:
        """Concatenate per-layer dicts (W1, b1, W2, b2, W3, b3; [in][out]) in the library's layout."""
        return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel()
                               for p in layers for k in ("W1", "b1", "W2", "b2", "W3", "b3")])

    def unflatten(self, flat: np.ndarray):
        """Inverse of flatten for this flow's masks."""
        out, off = [], 0
        H, NO = self.HIDDEN, 2 * self.BINS + 1
        for m in self.masks():
            dA, dB = int((~m).sum()), int(m.sum())
            shapes = [("W1", (dA, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, dB * NO)),
                      ("b3", (dB * NO,))]
            p = {}
            for k, shp in shapes:
                size = int(np.prod(shp))
                p[k] = np.asarray(flat[off:off + size], dtype=np.float64).reshape(shp)
                off += size
            out.append(p)
        return out

    def _run(self, fn, x, stream):
        import torch

        n = x.shape[1]
        out = torch.empty_like(x)
        lq = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(fn(self._h, _dev_ptr(x, "float32"), n, _dev_ptr(out, "float32"), _dev_ptr(lq, "float32"),
                  _stream_ptr(stream)))
        return out, lq

    def forward(self, y, stream=None):
        """(z, log q(y)) for y [ndim][n] float32 -- mf_flow_forward."""
        return self._run(lib().mf_flow_forward, y, stream)

    def inverse(self, z, stream=None):
        """(y, log q(y)) for z [ndim][n] float32 -- mf_flow_inverse."""
        return self._run(lib().mf_flow_inverse, z, stream)

    LOSSES = {"kl": 0, "variance": 1}

    def loss_grad(self, y, w, loss: str = "kl", stream=None):
        """(loss value, gradient [param_count] float32 device tensor) of one batch -- mf_flow_loss_grad."""
        import torch

        g = torch.empty(self.param_count, dtype=torch.float32, device=y.device)
        val = ctypes.c_double()
        _check(lib().mf_flow_loss_grad(self._h, _dev_ptr(y, "float32"), _dev_ptr(w, "float32"), y.shape[1],
                                       self.LOSSES[loss], _dev_ptr(g, "float32"), ctypes.byref(val),
                                       _stream_ptr(stream)))
        return val.value, g

    def adam_step(self, lr: float, stream=None):
        _check(lib().mf_flow_adam_step(self._h, lr, _stream_ptr(stream)))

    def train(self, y, w, epochs: int, batch: int = 16384, lr: float = 1e-3, lr_final: float = 1e-5,
              loss: str = "kl", stream=None) -> np.ndarray:
        """Mean batch loss value per epoch -- mf_flow_train."""
        o = _FlowTrainOpts(epochs, batch, lr, lr_final, _stream_ptr(stream), self.LOSSES[loss])
        out = np.zeros(epochs)
        _check(lib().mf_flow_train(self._h, _dev_ptr(y, "float32"), _dev_ptr(w, "float32"), y.shape[1],
                                   ctypes.byref(o), out.ctypes.data))
        return out


def vegas_refine(edges, hist, alpha: float = 1.5, stream=None):
    """In-place refinement of a device grid [ndim][nbins+1] from a device histogram -- mf_vegas_refine."""
    import torch

    d, nb1 = edges.shape
    status = torch.empty(1, dtype=torch.int32, device=edges.device)
    _check(lib().mf_vegas_refine(_dev_ptr(edges), _dev_ptr(hist), d, nb1 - 1, alpha, _dev_ptr(status, "int32"),
                                 _stream_ptr(stream)))
    return edges


def make_autograd_integrand(process: "Process"):
    """torch.autograd.Function over mf_integrand_grad for one process.

    forward(u, m_t, theta) -> w[n]: u is the [ndim][n] device tensor of points,
    m_t a 0-d tensor and theta the 8 PDF parameters (A_g, a_g, b_g, c_g, d_g,
    A_u, A_d, A_u~); their values must equal the process configuration (the
    kernels read the configured ones) -- they are inputs so that autograd can
    route d sigma/d m_t and d sigma/d theta.  backward contracts the upstream
    gradient with the per-event derivatives from the same kernel launch.
    """
    import torch

    cfg = process.cfg
    theta_cfg = [cfg.pdf_params[i] for i in (0, 1, 2, 3, 4, 5, 10, 15)]

    class MfIntegrand(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u, m_t, theta):
            if abs(float(m_t) - cfg.m_t) > 1e-12 * cfg.m_t:
                raise ValueError("m_t differs from the process configuration")
            th = theta.detach().cpu().double().numpy()
            if np.max(np.abs(th - np.array(theta_cfg))) > 1e-12 * np.max(np.abs(theta_cfg)):
                raise ValueError("theta differs from the process configuration")
            w, dw = process.integrand_grad(u.detach())
            ctx.save_for_backward(dw)
            ctx.devices = (m_t.device, theta.device)
            return w

        @staticmethod
        def backward(ctx, g):
            (dw,) = ctx.saved_tensors
            gd = vjp(dw, g.to(dw.dtype).contiguous())  # [9], mf_vjp
            return None, gd[0].to(ctx.devices[0], torch.float64), gd[1:].to(ctx.devices[1], torch.float64)

    return MfIntegrand
