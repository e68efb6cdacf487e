"""Riemannian preconditioned conjugate gradient, Algorithm 1 (PCG-ATKM), Sec. 2.3.

Steps per iteration n (paper notation):
  Phi_n = Phi[|phi_n|^2]                                   (ATKM)
  r_n = H phi_n - mu_n phi_n,  mu_n = <H phi_n, phi_n>
  P = P_V^{1/2} P_Lap P_V^{1/2}, P_Lap = (alpha - [[Lap]]/2)^{-1},
      P_V = (alpha + V + beta|phi|^2 + |lambda| (1 + sign Phi) Phi / 2)^{-1},
      alpha = <-1/2 Lap phi + V phi + beta |phi|^2 phi, phi> + |lambda <Phi phi, phi>|
  J(f) = f - <f, phi> phi
  p_n = J(-P r_n) + beta_cg J(p_{n-1}), beta_cg = max(beta_PR, 0),
      beta_PR = <r_n - J(r_{n-1}), J(P r_n)> / <r_{n-1}, J_{phi_{n-1}}(P r_{n-1})>
  if <H phi_n, p_n> >= 0: p_n = J(-P r_n)                  (PSD reset)
  c2 = <H_phi p, p> + <g, p> - mu ||p||^2,  g = 2 phi (beta Re(conj(phi) p) + lambda Phi[Re(conj(phi) p)])
  t = -<H phi, p> / c2 if c2 > 0 else 0.3
  phi_t = cos(t||p||) phi + sin(t||p||) p / ||p||          (retraction)
  halve t until E(phi_t) decreases.

Readings where the paper is silent:
 * alpha is recomputed every iteration at phi_n and excludes the rotation term.
 * (1 + sign Phi) Phi / 2 = max(Phi, 0); the |lambda| factor is kept for lambda < 0.
 * U * Re(conj(phi) p) in g means the dipolar operator Phi[.] (with its -rho term):
   that is what the second variation of lambda/2 <Phi[rho], rho> gives.
 * The PR denominator is the previous iteration's <r, J(P r)>, stored also on PSD-reset
   iterations. After a forced accept the next beta_cg is 0.
 * The CG direction is kept iff <H phi, p> < 0; t_app is used iff c2 > 0.
 * "until the energy decreases" is tested as E(phi_t) < E_n + tau_E with
   tau_E = tau_ulps * eps64 * (|E_kin| + |E_pot| + |E_int| + |E_dip| + |E_rot|): near the
   stopping tolerance the true decrease is below FP64 resolution of E and a strict test
   stalls. At most max_halvings halvings, then the last trial is accepted anyway
   (forced accept) and CG restarts.
 * Stop when ||r_n||_inf <= tol_res (unweighted max over grid points); the paper's
   ||phi_{n+1} - phi_n||_inf <= eps is available as tol_step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import spectral
from .energy import ip, norm, Energies

EPS64 = 2.0 ** -52


@dataclass
class PCGResult:
    phi: np.ndarray
    status: str
    iters: int
    halvings: int
    resets: int
    forced: int
    res_inf: float
    step_inf: float
    energies: Energies
    trace: list = field(default_factory=list)


def preconditioner(model, phi, Phi, r, alpha):
    """P r = P_V^{1/2} ifftn( fftn(P_V^{1/2} r) / (alpha + |nu|^2 / 2) ) P_V^{1/2}."""
    g = model.grid
    rho = np.abs(phi) ** 2
    PV = 1.0 / (alpha + model.V + model.beta * rho + abs(model.lam) * np.maximum(Phi, 0.0))
    sq = np.sqrt(PV)
    NX, NY, NZ = g.nu_mesh()
    lap = alpha + 0.5 * (NX * NX + NY * NY + NZ * NZ)
    return sq * spectral.ifftn(spectral.fftn(sq * r) / lap)


def shift_alpha(model, phi, Phi):
    g = model.grid
    rho = np.abs(phi) ** 2
    a = ip(g, model.kinetic(phi) + model.V * phi + model.beta * rho * phi, phi)
    return a + abs(model.lam * ip(g, Phi * phi, phi))


def pcg(model, phi0, tol_res=1e-8, tol_step=0.0, max_iter=20000, max_halvings=30,
        t_default=0.3, tau_ulps=64.0, trace=False, debug=None, on_iter=None):
    """Run Algorithm 1 from phi0 (normalised). `on_iter(n)`, if given, is called after each
    completed iteration (timing only; it sees no state). `debug` may hold:
    'force_t' (first trial step every iteration), 'force_c2' (override c2),
    'nan_at' (iteration at which a NaN is injected into the trial)."""
    debug = debug or {}
    g = model.grid
    J = lambda f, ph: f - ip(g, f, ph) * ph
    phi = np.array(phi0, dtype=np.complex128, copy=True)
    n = 0
    halv_total = resets = forced = 0
    r_prev = p_prev = None
    den_prev = None
    restart = True
    terms = model.terms(phi)
    E_n = sum(terms)
    step_inf = math.inf
    log = []
    status = "ok"
    while True:
        rho = np.abs(phi) ** 2
        Phi = model.Phi(rho)
        Hphi = model.H(phi, Phi=Phi)
        mu = ip(g, Hphi, phi)
        r = Hphi - mu * phi
        res = float(np.max(np.abs(r)))
        if res <= tol_res or (tol_step > 0 and step_inf <= tol_step):
            break
        if n >= max_iter:
            status = "notconv"
            break
        alpha = shift_alpha(model, phi, Phi)
        Pr = preconditioner(model, phi, Phi, r, alpha)
        q = J(Pr, phi)
        den = ip(g, r, q)
        if restart:
            beta_cg = 0.0
        else:
            beta_cg = max(ip(g, r - J(r_prev, phi), q) / den_prev, 0.0)
        p = -q + beta_cg * J(p_prev, phi) if beta_cg != 0.0 else -q
        d1 = ip(g, Hphi, p)
        reset = False
        if d1 >= 0.0:
            p = -q
            d1 = ip(g, Hphi, p)
            reset = True
            resets += 1
        rho1 = np.real(np.conj(phi) * p)
        gp = 2.0 * g.h3 * float(np.sum((model.beta * rho1 + model.lam * model.Phi(rho1)) * rho1))
        pn = norm(g, p)
        c2 = ip(g, model.H(phi, u=p, Phi=Phi), p) + gp - mu * pn * pn
        if "force_c2" in debug:
            c2 = debug["force_c2"]
        t = -d1 / c2 if c2 > 0.0 else t_default
        if "force_t" in debug:
            t = debug["force_t"]
        tau = tau_ulps * EPS64 * sum(abs(v) for v in terms)
        accepted = False
        halv = 0
        while True:
            phi_t = math.cos(t * pn) * phi + math.sin(t * pn) * p / pn
            if debug.get("nan_at") == n:
                phi_t = phi_t.copy()
                phi_t.flat[0] = np.nan
            terms_t = model.terms(phi_t)
            E_t = sum(terms_t)
            if not np.isfinite(E_t):
                status = "numeric"
                break
            if E_t < E_n + tau:
                accepted = True
                break
            if halv == max_halvings:
                break
            t *= 0.5
            halv += 1
        if status == "numeric":
            break
        halv_total += halv
        if not accepted:
            forced += 1
        step_inf = float(np.max(np.abs(phi_t - phi)))
        if trace:
            log.append(dict(n=n, E=E_n, mu=mu, res=res, t=t, beta_cg=beta_cg if not reset else 0.0,
                            reset=reset, halvings=halv, forced=not accepted, c2=c2, d1=d1, alpha=alpha))
        r_prev, p_prev, den_prev = r, p, den
        restart = not accepted
        phi, E_n, terms = phi_t, E_t, terms_t
        n += 1
        if on_iter is not None:
            on_iter(n)
    e = model.energies(phi)
    return PCGResult(phi, status, n, halv_total, resets, forced, res, step_inf, e, log)
