"""Plain FP64 CPU oracle for the per-event LO integrand (arXiv:2105.10529).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``; never by the product package, with which it
shares no code.  The arithmetic lives in ``oracle.cpp`` (Philox, VEGAS, PDF
interpolation, phase space, cuts, matrix elements, dual-number gradients),
``colour.py`` (colour matrices from explicit Gell-Mann matrices and an
explicit-colour amplitude for cross-checks), ``quad.py`` (closed-form partonic
cross sections and a deterministic quadrature of the hadronic one) and
``flow.py`` (the coupling normalising flow in numpy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")


def build(force: bool = True) -> str:
    """Compile the oracle shared object with g++ (-O2, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
        )
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        d, i, i64, u64 = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        P = ctypes.c_void_p
        L.or_philox4x64_10.argtypes = [P, P, P]
        L.or_max_threads.restype = ctypes.c_int
        L.or_event_uniforms.argtypes = [u64, u64, u64, u64, u64, i, P]
        L.or_vegas_map.argtypes = [P, i, i, P, P, P]
        L.or_vegas_map.restype = d
        L.or_vegas_refine.argtypes = [P, P, i, i, d]
        L.or_set_colour.argtypes = [i, i, P]
        L.or_set_colour_qq.argtypes = [P, P]
        L.or_me_qq.argtypes = [i, P, d, i]
        L.or_me_qq.restype = d
        L.or_state_create.argtypes = [P]
        L.or_state_create.restype = i
        L.or_state_destroy.argtypes = [i]
        L.or_pass_cuts.argtypes = [i, i, P, d, d]
        L.or_pass_cuts.restype = i
        L.or_pdf_table.argtypes = [i, i, P]
        L.or_pdf.argtypes = [i, i, i, P, P, i, P]
        L.or_hermite2d.argtypes = [P, i, P, P, P]
        L.or_phase_space.argtypes = [i, i, P, d, d, P, P]
        L.or_me_gg.argtypes = [i, P, d, P]
        L.or_me_gg.restype = d
        L.or_partial_amps.argtypes = [i, P, P, P, P, d, i, i, P]
        L.or_wavefunction.argtypes = [i, P, d, i, P]
        L.or_gamma.argtypes = [P, P]
        L.or_me_qqbar.argtypes = [P, d]
        L.or_me_qqbar.restype = d
        L.or_integrand.argtypes = [i, i64, P, P, P, i]
        L.or_integrand_grad.argtypes = [i, i64, P, i, P, P, i]
        L.or_integrand_mom.argtypes = [i, i64, P, P, P]
        L.or_vegas_iteration.argtypes = [i, P, i, u64, i64, i64, u64, u64, P, P, P, i]
        L.or_vegas_iteration_gauss.argtypes = [i, d, P, i, u64, i64, u64, u64, P, P]
        _lib = L
        _install_colour()
        _install_colour_qq()
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


_installed = set()


def _install_colour(ms=(2, 3, 4)):
    from . import colour

    for m in ms:
        if m in _installed:
            continue
        C = _c(colour.colour_matrix(m))
        _lib.or_set_colour(m, C.shape[0], _ptr(C))
        _installed.add(m)


def _install_colour_qq():
    from . import colour

    CC = colour.two_line_colour_matrix()
    re_ = _c(CC.real)
    im_ = _c(CC.imag)
    _lib.or_set_colour_qq(_ptr(re_), _ptr(im_))


# ------------------------------------------------------------------ constants
ALPHA_S = 0.118
GEV2_TO_PB = 3.893793721e8
PDF_PARAMS = {
    # (A, a, b, c, d) of x f = A x^(a + b L) (1 - x)^(c + d L), L = ln(Q / 1.65 GeV)
    "g": (1.6, -0.2, -0.05, 5.0, 0.3),
    "u": (2.2, 0.5, -0.02, 3.0, 0.2),
    "d": (1.1, 0.5, -0.02, 4.0, 0.2),
    "ubar": (0.2, -0.2, -0.05, 7.0, 0.3),
}
FLAVOURS = ("g", "u", "d", "ubar")
# gg; u u~ and d d~ (both beam assignments); q g = q g -> t t~ q and
# q~ g -> t t~ q~ for q = u, d (both beam assignments; needs n_g = 1)
CHANNELS = {"gg": 0, "uu~": 1, "dd~": 2, "qg": 3}


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_g", ctypes.c_int),
        ("channel", ctypes.c_int),
        ("sqrt_s", ctypes.c_double),
        ("m_t", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("alpha_s", ctypes.c_double),
        ("pt_min", ctypes.c_double),
        ("eta_max", ctypes.c_double),
        ("dr_min", ctypes.c_double),
        ("pdf", ctypes.c_double * 20),
        ("dyn_scale", ctypes.c_int),
    ]


def default_pdf() -> np.ndarray:
    return np.array([v for f in FLAVOURS for v in PDF_PARAMS[f]], dtype=np.float64)


@dataclass
class Config:
    n_g: int = 0
    channel: str = "gg"
    sqrt_s: float = 13000.0
    m_t: float = 173.0
    mu: float = -1.0          # <= 0: mu = m_t
    alpha_s: float = ALPHA_S
    pt_min: float = 20.0
    eta_max: float = 2.5
    dr_min: float = 0.0
    pdf: np.ndarray = field(default_factory=default_pdf)
    dyn_scale: bool = False   # True: mu = H_T / 2 per event (half the final-state transverse masses)

    @property
    def ndim(self) -> int:
        return 3 * (self.n_g + 2) - 2


class Oracle:
    """One configured integrand (owns the oracle's PDF tables)."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        c = _Cfg()
        c.n_g = cfg.n_g
        c.channel = CHANNELS[cfg.channel]
        c.sqrt_s, c.m_t, c.mu, c.alpha_s = cfg.sqrt_s, cfg.m_t, cfg.mu, cfg.alpha_s
        c.pt_min, c.eta_max, c.dr_min = cfg.pt_min, cfg.eta_max, cfg.dr_min
        for k in range(20):
            c.pdf[k] = float(cfg.pdf[k])
        c.dyn_scale = int(cfg.dyn_scale)
        if cfg.channel == "gg":
            lib()
            _install_colour((cfg.n_g + 2,))
        self._h = lib().or_state_create(ctypes.byref(c))

    def __del__(self):
        try:
            if _lib is not None:
                _lib.or_state_destroy(self._h)
        except Exception:
            pass

    @property
    def ndim(self) -> int:
        return self.cfg.ndim

    def integrand(self, x: np.ndarray, nthreads: int = 0, return_pass: bool = False):
        x = _c(x)
        n = x.shape[0]
        assert x.shape[1] == self.ndim
        w = np.zeros(n)
        p = np.zeros(n, dtype=np.int32)
        lib().or_integrand(self._h, n, _ptr(x), _ptr(w), _ptr(p), nthreads)
        return (w, p.astype(bool)) if return_pass else w

    def integrand_grad(self, x: np.ndarray, direction: int, nthreads: int = 0):
        """(w, dw/dparam) with direction 1 = m_t, 2..9 = theta (A_g, a_g, b_g, c_g, d_g, A_u, A_d, A_ubar)."""
        x = _c(x)
        n = x.shape[0]
        w = np.zeros(n)
        dw = np.zeros(n)
        lib().or_integrand_grad(self._h, n, _ptr(x), direction, _ptr(w), _ptr(dw), nthreads)
        return w, dw

    def integrand_momenta(self, x: np.ndarray):
        x = _c(x)
        n = x.shape[0]
        ng = self.cfg.n_g
        w = np.zeros(n)
        mom = np.zeros((n, ng + 4, 4))
        lib().or_integrand_mom(self._h, n, _ptr(x), _ptr(w), _ptr(mom))
        return w, mom

    def pass_cuts(self, gluons: np.ndarray, x1: float, x2: float) -> bool:
        """The cut decision for partonic-frame gluon momenta gluons[ng][4] at momentum fractions x1, x2."""
        g = _c(np.atleast_2d(gluons))
        return bool(lib().or_pass_cuts(self._h, g.shape[0], _ptr(g), float(x1), float(x2)))

    def pdf(self, flavour: str, x, Q, analytic: bool = False):
        x = _c(np.atleast_1d(x))
        Q = _c(np.broadcast_to(np.atleast_1d(Q), x.shape))
        out = np.zeros(x.shape[0])
        lib().or_pdf(self._h, FLAVOURS.index(flavour), x.shape[0], _ptr(x), _ptr(Q), int(analytic), _ptr(out))
        return out

    def pdf_table(self, flavour: str) -> np.ndarray:
        out = np.zeros((50, 196))
        lib().or_pdf_table(self._h, FLAVOURS.index(flavour), _ptr(out))
        return out

    def vegas_iteration(self, edges: np.ndarray, iteration: int, n: int, seed: int, purpose: int = 0,
                        ev0: int = 0, nthreads: int = 0):
        """One VEGAS iteration with Philox uniforms; returns (S1, S2, hist[d][nb], n_nonzero, n_bad)."""
        edges = _c(edges)
        d, nb1 = edges.shape
        out = np.zeros(2)
        hist = np.zeros((d, nb1 - 1))
        cnt = np.zeros(2, dtype=np.int64)
        lib().or_vegas_iteration(self._h, _ptr(edges), nb1 - 1, iteration, ev0, n, seed, purpose, _ptr(out),
                                 _ptr(hist), _ptr(cnt), nthreads)
        return out[0], out[1], hist, int(cnt[0]), int(cnt[1])


# ------------------------------------------------------------- free functions
def philox4x64_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint64)
    k = _c(key, np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def event_uniforms(n: int, d: int, iteration: int, seed: int, purpose: int = 0, ev0: int = 0) -> np.ndarray:
    u = np.zeros((n, d))
    lib().or_event_uniforms(n, ev0, iteration, seed, purpose, d, _ptr(u))
    return u


def vegas_map(edges: np.ndarray, y: np.ndarray):
    edges = _c(edges)
    d, nb1 = edges.shape
    y = _c(y)
    x = np.zeros(d)
    bins = np.zeros(d, dtype=np.int32)
    jac = lib().or_vegas_map(_ptr(edges), d, nb1 - 1, _ptr(y), _ptr(x), _ptr(bins))
    return x, jac, bins


def vegas_refine(edges: np.ndarray, hist: np.ndarray, alpha: float = 1.5) -> np.ndarray:
    e = _c(edges).copy()
    h = _c(hist)
    d, nb1 = e.shape
    lib().or_vegas_refine(_ptr(e), _ptr(h), d, nb1 - 1, alpha)
    return e


def max_threads() -> int:
    return lib().or_max_threads()


def uniform_edges(d: int, nb: int = 50) -> np.ndarray:
    return np.tile(np.linspace(0.0, 1.0, nb + 1), (d, 1))


def combine(I: np.ndarray, sig: np.ndarray):
    """Inverse-variance weighted mean, its error and chi^2/dof of iteration estimates."""
    I = np.asarray(I, dtype=np.float64)
    sig = np.asarray(sig, dtype=np.float64)
    wts = 1.0 / sig**2
    mean = np.sum(I * wts) / np.sum(wts)
    err = np.sum(wts) ** -0.5
    chi2 = np.sum((I - mean) ** 2 * wts) / max(len(I) - 1, 1)
    return mean, err, chi2


def iteration_estimate(S1: float, S2: float, n: int):
    I = S1 / n
    var = (S2 / n - I * I) / (n - 1)
    return I, np.sqrt(max(var, 0.0))


def vegas_run(orc: Oracle, n_iter: int, n: int, seed: int, purpose: int = 2, alpha: float = 1.5, nb: int = 50,
              nthreads: int = 0):
    """Full VEGAS integration with the oracle; returns (mean, err, chi2, per-iteration, final edges)."""
    edges = uniform_edges(orc.ndim, nb)
    Is, sigs = [], []
    for it in range(n_iter):
        S1, S2, hist, _, _ = orc.vegas_iteration(edges, it, n, seed, purpose, nthreads=nthreads)
        I, s = iteration_estimate(S1, S2, n)
        Is.append(I)
        sigs.append(s)
        edges = vegas_refine(edges, hist, alpha)
    mean, err, chi2 = combine(Is, sigs)
    return mean, err, chi2, (np.array(Is), np.array(sigs)), edges


def vegas_iteration_gauss(d: int, sig: float, edges: np.ndarray, iteration: int, n: int, seed: int,
                          purpose: int = 2):
    """One VEGAS iteration on the analytic Gaussian-product test integrand."""
    edges = _c(edges)
    out = np.zeros(2)
    hist = np.zeros((d, edges.shape[1] - 1))
    lib().or_vegas_iteration_gauss(d, sig, _ptr(edges), edges.shape[1] - 1, iteration, n, seed, purpose,
                                   _ptr(out), _ptr(hist))
    return out[0], out[1], hist


def phase_space(n_g: int, x: np.ndarray, sqrt_shat: float, m_t: float):
    x = _c(np.atleast_2d(x))
    n = x.shape[0]
    mom = np.zeros((n, n_g + 4, 4))
    wt = np.zeros(n)
    lib().or_phase_space(n_g, n, _ptr(x), sqrt_shat, m_t, _ptr(mom), _ptr(wt))
    return mom, wt


def me_gg(m: int, mom: np.ndarray, m_t: float, per_helicity: bool = False):
    """Colour/helicity-summed |M|^2 with g = 1 for g g -> t t~ + (m-2) g; mom = (p1,p2,t,tb,g...)."""
    mom = _c(mom)
    lib()
    _install_colour((m,))
    ph = np.zeros(1 << (m + 2))
    v = lib().or_me_gg(m, _ptr(mom), m_t, _ptr(ph))
    return (v, ph) if per_helicity else v


def me_qqbar(mom: np.ndarray, m_t: float) -> float:
    return lib().or_me_qqbar(_ptr(_c(mom)), m_t)


def me_qq(kind: str, mom: np.ndarray, m_t: float, ward: bool = False) -> float:
    """Colour/helicity-summed |M|^2 (g = 1) with two quark lines: kind "qqg" =
    q(p1) q~(p2) -> t(p3) t~(p4) g(p5), "qgq" = q(p1) g(p2) -> t(p3) t~(p4) q(p5);
    mom = (p1, ..., p5); ward: the gluon's polarisation replaced by its momentum."""
    return lib().or_me_qq({"qqg": 0, "qgq": 1}[kind], _ptr(_c(mom)), m_t, int(ward))


def partial_amplitudes(m: int, k: np.ndarray, incoming, pt, ptb, m_t: float, hel: int, ward: int = -1):
    k = _c(k)
    inc = _c(incoming, np.int32)
    out = np.zeros(2 * int(np.prod(range(1, m + 1))))
    lib().or_partial_amps(m, _ptr(k), _ptr(inc), _ptr(_c(pt)), _ptr(_c(ptb)), m_t, hel, ward, _ptr(out))
    return out[0::2] + 1j * out[1::2]


def wavefunction(kind: str, p, m: float, lam: int) -> np.ndarray:
    kinds = {"u": 0, "v": 1, "ubar": 2, "vbar": 3, "eps": 4, "eps*": 5}
    out = np.zeros(8)
    lib().or_wavefunction(kinds[kind], _ptr(_c(p)), m, lam, _ptr(out))
    return out[0::2] + 1j * out[1::2]


def gamma_matrices() -> np.ndarray:
    re = np.zeros((4, 4, 4))
    im = np.zeros((4, 4, 4))
    lib().or_gamma(_ptr(re), _ptr(im))
    return re + 1j * im


def hermite2d(table: np.ndarray, x, Q) -> np.ndarray:
    t = _c(table)
    assert t.shape == (50, 196)
    x = _c(np.atleast_1d(x))
    Q = _c(np.broadcast_to(np.atleast_1d(Q), x.shape))
    out = np.zeros(x.shape[0])
    lib().or_hermite2d(_ptr(t), x.shape[0], _ptr(x), _ptr(Q), _ptr(out))
    return out


def x_knots() -> np.ndarray:
    return 10.0 ** (-9.0 + 9.0 * np.arange(196) / 195.0)


def q_knots() -> np.ndarray:
    return 1.65 * (1e5 / 1.65) ** (np.arange(50) / 49.0)
