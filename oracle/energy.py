"""Discrete energy, Hamiltonian apply and chemical potential (Sec. 2.3).

 <U, V> = Re( h_x h_y h_z sum_j U_j conj(V_j) )                 (eq. "innerPro")
 E(phi) = < -1/2 [[Lap]] phi + V phi + beta/2 |phi|^2 phi + lambda/2 Phi phi
            - Omega [[L_z]] phi, phi >                              (discrete energy)
 H_phi u = -1/2 [[Lap]] u + (V + beta |phi|^2 + lambda Phi[|phi|^2]) u - Omega [[L_z]] u
 mu_phi = < H_phi phi, phi >
Energy parts (Sec. 3, virial identity and energy study):
 E_kin = <-1/2 Lap phi, phi>, E_pot = <V phi, phi>, E_int = beta/2 h^3 sum |phi|^4,
 E_dip = lambda/2 h^3 sum Phi |phi|^2, E_rot = -Omega <L_z phi, phi>;
 virial I = 2 E_kin - 2 E_pot + 3 E_int + 3 E_dip (eq. "vir_iden").
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import spectral, dipolar
from .grid import Grid


def ip(grid, u, v):
    """<u, v> = Re(h^3 sum u conj(v))."""
    return float(np.real(grid.h3 * np.vdot(v.ravel(), u.ravel())))


def norm(grid, u):
    return float(np.sqrt(ip(grid, u, u)))


@dataclass
class Energies:
    E: float
    Ekin: float
    Epot: float
    Eint: float
    Edip: float
    Erot: float
    mu: float
    mass: float

    @property
    def virial(self):
        return 2 * self.Ekin - 2 * self.Epot + 3 * self.Eint + 3 * self.Edip

    def as_dict(self):
        d = dict(self.__dict__)
        d["virial"] = self.virial
        return d


class Model:
    """One problem instance: grid + parameters + precomputed V and S."""

    def __init__(self, n, a, gamma, beta, lam, ndip, omega, uhat_full=None):
        self.grid = Grid(n, a)
        self.gamma = tuple(float(g) for g in gamma)
        self.beta = float(beta)
        self.lam = float(lam)
        self.ndip = dipolar.normalize_axis(ndip)
        self.omega = float(omega)
        self.V = spectral.trap(self.grid, self.gamma)
        self.S = dipolar.dipolar_symbol(self.grid, self.ndip, uhat_full) if self.lam != 0.0 else None

    @classmethod
    def from_workload(cls, w, n=None, uhat_full=None):
        return cls(n or w.n, w.a, w.gamma, w.beta, w.lam, w.ndip, w.omega, uhat_full)

    # --- pieces ---------------------------------------------------------
    def Phi(self, rho):
        if self.S is None:
            return np.zeros(self.grid.n)
        return dipolar.potential(self.grid, self.S, rho)

    def kinetic(self, u):
        return spectral.neg_half_laplacian(self.grid, u)

    def Lz(self, u):
        return spectral.Lz(self.grid, u)

    def H(self, phi, u=None, Phi=None):
        """H_phi u (u defaults to phi); Phi = Phi[|phi|^2] may be passed in."""
        if u is None:
            u = phi
        rho = np.abs(phi) ** 2
        if Phi is None:
            Phi = self.Phi(rho)
        return (self.kinetic(u) + (self.V + self.beta * rho + self.lam * Phi) * u
                - self.omega * self.Lz(u))

    def terms(self, phi, Phi=None):
        """(E_kin, E_pot, E_int, E_dip, E_rot) of phi."""
        g = self.grid
        rho = np.abs(phi) ** 2
        if Phi is None:
            Phi = self.Phi(rho)
        Ekin = ip(g, self.kinetic(phi), phi)
        Epot = g.h3 * float(np.sum(self.V * rho))
        Eint = 0.5 * self.beta * g.h3 * float(np.sum(rho * rho))
        Edip = 0.5 * self.lam * g.h3 * float(np.sum(Phi * rho))
        Erot = -self.omega * ip(g, self.Lz(phi), phi)
        return Ekin, Epot, Eint, Edip, Erot

    def energies(self, phi, Phi=None):
        g = self.grid
        rho = np.abs(phi) ** 2
        if Phi is None:
            Phi = self.Phi(rho)
        Ekin, Epot, Eint, Edip, Erot = self.terms(phi, Phi)
        E = Ekin + Epot + Eint + Edip + Erot
        Hphi = self.H(phi, Phi=Phi)
        mu = ip(g, Hphi, phi)
        mass = g.h3 * float(np.sum(rho))
        return Energies(E, Ekin, Epot, Eint, Edip, Erot, mu, mass)

    def energy(self, phi):
        """E(phi) as the discrete energy functional."""
        g = self.grid
        rho = np.abs(phi) ** 2
        Phi = self.Phi(rho)
        lin = self.kinetic(phi) + self.V * phi - self.omega * self.Lz(phi)
        return (ip(g, lin, phi) + 0.5 * self.beta * g.h3 * float(np.sum(rho * rho))
                + 0.5 * self.lam * g.h3 * float(np.sum(Phi * rho)))
