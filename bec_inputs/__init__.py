"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module holds workload descriptions (box, grid, physical parameters) and the
initial wave functions the solver starts from. It contains none of the method's
arithmetic: no spectral operator, no dipolar kernel, no energy, no solver step.
Everything is FP64 NumPy on the host; both sides receive the same arrays.

Initial guesses follow the list of starting states in Section 3 of the paper
(Gaussian (a), vortex (b), mixes (c)/(d)/(e), conjugates, Thomas-Fermi (f)).
The configured workloads use a trap-matched Gaussian
G = prod_a (gamma_a/pi)^{1/4} exp(-gamma_a x_a^2 / 2) in place of the isotropic
(a) because the isotropic one is far too wide for thin boxes (e.g. z in [-2,2]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "grid_axes", "normalize", "gaussian_trap",
    "vortex", "guess_c", "guess_d", "guess_e", "guess_isotropic_a",
    "guess_thomas_fermi", "random_phase", "initial_guess", "batched_sweep",
    "mlp_param_draw", "mlp_init", "paper_guesses", "PAPER_GUESS_NAMES",
]


@dataclass
class Workload:
    name: str
    n: tuple            # (Nx, Ny, Nz), even
    a: tuple            # box half-widths: box = prod [-a, a)
    gamma: tuple        # trap frequencies
    beta: float
    lam: float
    ndip: tuple         # dipole axis, unit vector
    omega: float
    guess: str = "c"    # 'c' | 'd' | 'd_phase' | 'a' | 'tf' | 'gauss'
    seed: int = 0
    tol_res: float = 1e-8

    def params(self) -> dict:
        return dict(gamma=tuple(self.gamma), beta=self.beta, lam=self.lam,
                    ndip=tuple(self.ndip), omega=self.omega)

    def to_dict(self) -> dict:
        return asdict(self)

    def with_grid(self, n) -> "Workload":
        d = asdict(self)
        d["n"] = tuple(n)
        return Workload(**d)


_S30, _C30 = 0.5, math.sqrt(3.0) / 2.0

WORKLOADS = {
    # small full-solve case: 32^3 on [-8,8]^2 x [-4,4]
    "small_32": Workload("small_32", (32, 32, 32), (8.0, 8.0, 4.0), (1.0, 1.0, 4.0),
                         200.0, 50.0, (0.0, 0.0, 1.0), 0.5, guess="c"),
    # pancake trap, many vortices: 256x256x64 on [-16,16]^2 x [-2,2]
    "pancake_256": Workload("pancake_256", (256, 256, 64), (16.0, 16.0, 2.0), (1.0, 1.0, 20.0),
                            2000.0, 600.0, (_S30, 0.0, _C30), 0.9, guess="d_phase", seed=0),
    # cigar trap: 128x128x256 on [-4,4]^2 x [-24,24]
    "cigar_128": Workload("cigar_128", (128, 128, 256), (4.0, 4.0, 24.0), (10.0, 10.0, 1.0),
                          1000.0, 300.0, (1.0, 0.0, 0.0), 0.8, guess="d"),
}


def grid_axes(n, a):
    """Grid points x_j = -a + j h, h = 2a/N, j = 0..N-1 (Section 2.1)."""
    return [(-a[d] + np.arange(n[d]) * (2.0 * a[d] / n[d])) for d in range(3)]


def _mesh(n, a):
    x, y, z = grid_axes(n, a)
    return np.meshgrid(x, y, z, indexing="ij")


def normalize(f, n, a):
    """f / ||f|| with ||f||^2 = h_x h_y h_z sum |f|^2."""
    h3 = np.prod([2.0 * a[d] / n[d] for d in range(3)])
    return f / math.sqrt(h3 * float(np.sum(np.abs(f) ** 2)))


def gaussian_trap(n, a, gamma):
    X, Y, Z = _mesh(n, a)
    g = 1.0
    for d, C in enumerate((X, Y, Z)):
        g = g * (gamma[d] / math.pi) ** 0.25 * np.exp(-gamma[d] * C * C / 2.0)
    return g.astype(np.complex128)


def vortex(n, a, base):
    X, Y, _ = _mesh(n, a)
    return normalize((X + 1j * Y) * base, n, a)


def guess_c(n, a, gamma):
    g = gaussian_trap(n, a, gamma)
    return normalize(normalize(g, n, a) + vortex(n, a, g), n, a)


def guess_d(n, a, gamma, omega):
    g = normalize(gaussian_trap(n, a, gamma), n, a)
    return normalize((1.0 - omega) * g + omega * vortex(n, a, g), n, a)


def guess_e(n, a, gamma, omega):
    g = normalize(gaussian_trap(n, a, gamma), n, a)
    return normalize(omega * g + (1.0 - omega) * vortex(n, a, g), n, a)


def guess_isotropic_a(n, a):
    X, Y, Z = _mesh(n, a)
    return (math.pi ** -0.75 * np.exp(-(X * X + Y * Y + Z * Z) / 2.0)).astype(np.complex128)


def guess_thomas_fermi(n, a, gamma, beta):
    X, Y, Z = _mesh(n, a)
    V = 0.5 * (gamma[0] ** 2 * X * X + gamma[1] ** 2 * Y * Y + gamma[2] ** 2 * Z * Z)
    mu = 0.5 * (15.0 * beta * gamma[0] * gamma[1] * gamma[2] / (4.0 * math.pi)) ** 0.4
    f = np.sqrt(np.maximum(mu - V, 0.0) / beta)
    return normalize(f.astype(np.complex128), n, a)


def random_phase(n, a, seed, modes=16):
    """theta_s(x,y) = sum_m A_m cos(q_m (x cos psi_m + y sin psi_m) + c_m),
    A ~ U(0, pi/4), q ~ U(0.1, 1), psi, c ~ U(0, 2 pi); PCG64 stream of `seed`."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.0, math.pi / 4.0, modes)
    q = rng.uniform(0.1, 1.0, modes)
    psi = rng.uniform(0.0, 2.0 * math.pi, modes)
    c = rng.uniform(0.0, 2.0 * math.pi, modes)
    X, Y, _ = _mesh(n, a)
    th = np.zeros(X.shape)
    for m in range(modes):
        th += A[m] * np.cos(q[m] * (X * math.cos(psi[m]) + Y * math.sin(psi[m])) + c[m])
    return np.exp(1j * th)


def initial_guess(w: Workload, n=None) -> np.ndarray:
    """Normalised complex128 array [Nx][Ny][Nz] (z fastest) for workload `w`."""
    n = tuple(n or w.n)
    if w.guess == "c":
        return guess_c(n, w.a, w.gamma)
    if w.guess == "d":
        return guess_d(n, w.a, w.gamma, w.omega)
    if w.guess == "e":
        return guess_e(n, w.a, w.gamma, w.omega)
    if w.guess == "d_phase":
        return normalize(guess_d(n, w.a, w.gamma, w.omega) * random_phase(n, w.a, w.seed), n, w.a)
    if w.guess == "a":
        return normalize(guess_isotropic_a(n, w.a), n, w.a)
    if w.guess == "tf":
        return guess_thomas_fermi(n, w.a, w.gamma, w.beta)
    if w.guess == "gauss":
        return normalize(gaussian_trap(n, w.a, w.gamma), n, w.a)
    raise ValueError(f"unknown guess {w.guess!r}")


def random_field(n, seed, scale=1.0):
    """Smooth-ish random complex field for operator tests (not normalised)."""
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n))


def batched_sweep(quick=False):
    """Omega x lambda/beta sweep at beta = 1000, gamma = (1,1,10), n = z.

    Omega in linspace(0.1, 0.95, 16), lambda/beta in {0.1, 0.3, 0.5, 0.7};
    the transverse grid grows with Omega (96, 128, 160, 192 by quartile), Nz = 48
    for N_perp <= 128 else 64, box [-16,16]^2 x [-2,2].
    """
    omegas = np.linspace(0.1, 0.95, 16)
    ratios = (0.1, 0.3, 0.5, 0.7)
    out = []
    for r in ratios:
        for i, om in enumerate(omegas):
            nperp = (96, 128, 160, 192)[i // 4]
            nz = 48 if nperp <= 128 else 64
            if quick:
                nperp, nz = nperp // 4, 16
            out.append(Workload(f"sweep_l{r}_o{om:.3f}", (nperp, nperp, nz), (16.0, 16.0, 2.0),
                                (1.0, 1.0, 10.0), 1000.0, 1000.0 * r, (0.0, 0.0, 1.0), float(om),
                                guess="d"))
    return out


def mlp_param_draw(seed):
    """One draw of (beta, lambda/beta, Omega, gamma_z, theta_n, phi_n), uniform on
    [200,3000] x [0,0.8] x [0,0.95] x [4,40] x [0,pi/2] x [0,pi)."""
    rng = np.random.default_rng(seed)
    beta = rng.uniform(200.0, 3000.0)
    ratio = rng.uniform(0.0, 0.8)
    omega = rng.uniform(0.0, 0.95)
    gz = rng.uniform(4.0, 40.0)
    th = rng.uniform(0.0, math.pi / 2.0)
    ph = rng.uniform(0.0, math.pi)
    return np.array([beta, ratio, omega, gz, th, ph])


def mlp_init(dims, seed):
    """Seeded initial weights of the d_in -> d_h -> d_h -> d_out network, packed
    [W1 b1 W2 b2 W3 b3] as FP32: W uniform on +-sqrt(6/(fan_in + fan_out)) (Glorot and
    Bengio's uniform scaling), biases zero."""
    d_in, d_h, d_out = dims
    rng = np.random.default_rng(seed)
    parts = []
    for fo, fi in ((d_h, d_in), (d_h, d_h), (d_out, d_h)):
        lim = math.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-lim, lim, fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


PAPER_GUESS_NAMES = ("a", "b", "b_bar", "c", "c_bar", "d", "d_bar", "e", "e_bar", "f")


def paper_guesses(n, a, gamma, beta, omega):
    """The ten starting states listed in Sec. 3, in order (a), (b), conj(b), (c), conj(c), (d),
    conj(d), (e), conj(e), (f): phi_a is the isotropic Gaussian pi^(-3/4) exp(-|x|^2/2),
    phi_b = N[(x + i y) phi_a], (c) = N[phi_a + phi_b], (d) = N[(1-Omega) phi_a + Omega phi_b],
    (e) = N[Omega phi_a + (1-Omega) phi_b], (f) the normalised Thomas-Fermi profile; N[.]
    normalises on the grid. Returns a complex128 array [10][Nx][Ny][Nz]."""
    n = tuple(n)
    pa = normalize(guess_isotropic_a(n, a), n, a)
    pb = vortex(n, a, pa)
    pc = normalize(pa + pb, n, a)
    pd = normalize((1.0 - omega) * pa + omega * pb, n, a)
    pe = normalize(omega * pa + (1.0 - omega) * pb, n, a)
    pf = guess_thomas_fermi(n, a, gamma, beta)
    return np.stack([pa, pb, np.conj(pb), pc, np.conj(pc), pd, np.conj(pd), pe, np.conj(pe), pf])
