"""Closed-form partonic cross sections and a deterministic hadronic quadrature.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Textbook LO heavy-quark pair production (Combridge 1979; Gluck-Owens-Reya
1978; Ellis-Stirling-Webber, "QCD and Collider Physics", ch. 10), with
rho = 4 m^2 / s, beta = sqrt(1 - rho):
  sigma_gg = (pi as^2 / 3s) [ (1 + rho + rho^2/16) ln((1+beta)/(1-beta)) - beta (7/4 + 31 rho/16) ]
  sigma_qq = (8 pi as^2 / 27 s) beta (1 + rho/2)
and the spin/colour-averaged squared matrix elements
  gg: g^4 [1/(6 t1 t2) - 3/8] [t1^2 + t2^2 + rho - rho^2/(4 t1 t2)]
  qq: g^4 (4/9) (t1^2 + t2^2 + rho/2),  t1 = 2 p1.p3/s, t2 = 2 p2.p3/s.
The hadronic cross section sigma = int dx1 dx2 f(x1) f(x2) sigma_hat(x1 x2 S)
is integrated deterministically: tau = x1 x2 by adaptive quadrature, the
rapidity y = ln(x1/x2)/2 by 4-point Gauss-Legendre on every interval between
the PDF grid knots, where the interpolated x f is a cubic polynomial in ln x
(so the inner rule is exact up to rounding).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate

from . import GEV2_TO_PB, Oracle, x_knots


def me_gg_closed(s, t1, t2, mt, alpha_s=0.118):
    g4 = (4 * np.pi * alpha_s) ** 2
    rho = 4 * mt * mt / s
    return g4 * (1 / (6 * t1 * t2) - 3 / 8) * (t1**2 + t2**2 + rho - rho**2 / (4 * t1 * t2))


def me_qq_closed(s, t1, t2, mt, alpha_s=0.118):
    g4 = (4 * np.pi * alpha_s) ** 2
    rho = 4 * mt * mt / s
    return g4 * (4 / 9) * (t1**2 + t2**2 + rho / 2)


def sigma_hat_gg(s, mt, alpha_s=0.118):
    s = np.asarray(s, dtype=np.float64)
    rho = 4 * mt * mt / s
    out = np.zeros_like(s)
    ok = rho < 1
    r = rho[ok]
    b = np.sqrt(1 - r)
    out[ok] = (np.pi * alpha_s**2 / (3 * s[ok])) * (
        (1 + r + r * r / 16) * np.log((1 + b) / (1 - b)) - b * (7 / 4 + 31 * r / 16))
    return out


def sigma_hat_qq(s, mt, alpha_s=0.118):
    s = np.asarray(s, dtype=np.float64)
    rho = 4 * mt * mt / s
    out = np.zeros_like(s)
    ok = rho < 1
    r = rho[ok]
    out[ok] = (8 * np.pi * alpha_s**2 / (27 * s[ok])) * np.sqrt(1 - r) * (1 + r / 2)
    return out


_GL_X, _GL_W = np.polynomial.legendre.leggauss(4)


def _rapidity_nodes(tau: float):
    """Gauss-Legendre nodes/weights in y over [ln(tau)/2, -ln(tau)/2], split at PDF knots."""
    lt = np.log(tau)
    lk = np.log(x_knots())
    ymax = -0.5 * lt
    cuts = np.concatenate([lk - 0.5 * lt, 0.5 * lt - lk])
    cuts = cuts[(cuts > -ymax) & (cuts < ymax)]
    b = np.unique(np.concatenate([[-ymax, ymax], cuts]))
    a0, a1 = b[:-1], b[1:]
    mid = 0.5 * (a0 + a1)
    half = 0.5 * (a1 - a0)
    y = (mid[:, None] + half[:, None] * _GL_X[None, :]).ravel()
    w = (half[:, None] * _GL_W[None, :]).ravel()
    return y, w


def hadronic_sigma(orc: Oracle, channel: str = "gg", analytic_pdf: bool = False, epsrel: float = 1e-10,
                   mt: float | None = None, mu: float | None = None) -> float:
    """sigma in pb for g g -> t t~ ("gg") or q q~ -> t t~ summed over u u~, d d~ and both beam orders ("qq")."""
    cfg = orc.cfg
    mt = cfg.m_t if mt is None else mt
    mu = (cfg.mu if cfg.mu > 0 else mt) if mu is None else mu
    S = cfg.sqrt_s**2
    tau0 = 4 * mt * mt / S

    def lum(tau):
        y, w = _rapidity_nodes(tau)
        r = np.sqrt(tau)
        x1 = r * np.exp(y)
        x2 = r * np.exp(-y)
        x1 = np.minimum(x1, 1.0)
        x2 = np.minimum(x2, 1.0)
        f = lambda fl, x: orc.pdf(fl, x, mu, analytic=analytic_pdf)
        if channel == "gg":
            prod = f("g", x1) * f("g", x2)
        else:
            ub1, ub2 = f("ubar", x1), f("ubar", x2)
            prod = (f("u", x1) * ub2 + ub1 * f("u", x2) + f("d", x1) * ub2 + ub1 * f("d", x2))
        return np.sum(w * prod) / tau  # f = xf / x and x1 x2 = tau

    sh = sigma_hat_gg if channel == "gg" else sigma_hat_qq

    # tau = tau0 + (1 - tau0) u^2 removes the square-root threshold behaviour.
    def integrand(u):
        tau = tau0 + (1 - tau0) * u * u
        if tau >= 1.0:
            return 0.0
        return float(sh(np.array([tau * S]), mt, cfg.alpha_s)[0]) * lum(tau) * 2 * (1 - tau0) * u

    val, err = integrate.quad(integrand, 0.0, 1.0, epsrel=epsrel, epsabs=0.0, limit=400)
    return val * GEV2_TO_PB
