"""Pins of the oracle's Algorithm 1 pieces that do not change the ground state, only the path:
the preconditioner P = P_V^{1/2} (alpha - Lap/2)^{-1} P_V^{1/2}, the shift alpha, and the
Polak-Ribiere coefficient with its resets (Sec. 2.3, the preconditioner and conjugate-direction
paragraphs; Algorithm 1).

 * The preconditioner is compared with a dense linear solve: alpha - Lap/2 is assembled entry by
   entry from the Fourier basis (tests/pins.dft_matrices), P_V from its definition on the grid
   points, and P r = D solve(A, D r) with D = diag(P_V^{1/2}).
 * alpha at a trap-matched Gaussian has a closed form: E_kin + E_pot = sum gamma / 2,
   beta int |phi|^4 = beta sqrt(gx gy gz) / (2 pi)^{3/2}, and <Phi phi, phi> = J from a 1-D
   quadrature (tests/pins.gaussian_dipolar_J).
 * beta_PR: with zero steps the iterate does not move, r_n = r_{n-1}, and the Polak-Ribiere
   numerator <r_n - J(r_{n-1}), J(P r_n)> vanishes, so beta_cg = 0 (a Fletcher-Reeves ratio
   would give 1); after a forced accept the next beta_cg is 0; every kept direction is a descent
   direction (d1 < 0, the PSD reset) and beta_cg >= 0.
Each pin is also run on mutants of the oracle function written out below (the mistakes a reader
could make in the formula), which it must reject."""
import math

import numpy as np
import pytest

import bec_inputs as bi
from oracle import symbol, dipolar
from oracle.energy import Model, ip
from oracle.grid import Grid
from oracle.pcg import pcg, preconditioner, shift_alpha
from oracle import spectral
from tests import pins


# ---------------------------------------------------------------- preconditioner vs dense solve
PN, PA, PG = (6, 4, 6), (3.0, 2.0, 2.5), (1.0, 1.4, 2.2)


def _dense_minus_half_laplacian(n, a):
    """-Lap/2 as a dense matrix on the C-order flattening, from the 1-D basis matrices."""
    ops = []
    for d in range(3):
        F, B, nu, _ = pins.dft_matrices(n[d], a[d])
        ops.append(B @ np.diag(-(nu ** 2)) @ F)      # d^2/dx^2 on the Fourier interpolant
    eye = [np.eye(v) for v in n]
    lap = (np.kron(np.kron(ops[0], eye[1]), eye[2]) + np.kron(np.kron(eye[0], ops[1]), eye[2])
           + np.kron(np.kron(eye[0], eye[1]), ops[2]))
    return -0.5 * lap


def _prec_case(lam=-20.0, beta=30.0, seed=11):
    rng = np.random.default_rng(seed)
    m = Model(PN, PA, PG, beta, lam, (0.6, 0.0, 0.8), 0.4)
    phi = (rng.standard_normal(PN) + 1j * rng.standard_normal(PN)) * 0.3
    Phi = 0.02 * rng.standard_normal(PN)             # both signs, so max(Phi, 0) matters
    r = rng.standard_normal(PN) + 1j * rng.standard_normal(PN)
    alpha = 1.7
    return m, phi, Phi, r, alpha


def _prec_reference(m, phi, Phi, r, alpha):
    xs = [pins.dft_matrices(PN[d], PA[d])[3] for d in range(3)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    V = 0.5 * (PG[0] ** 2 * X * X + PG[1] ** 2 * Y * Y + PG[2] ** 2 * Z * Z)
    PV = 1.0 / (alpha + V + m.beta * np.abs(phi) ** 2 + abs(m.lam) * np.where(Phi > 0, Phi, 0.0))
    D = np.sqrt(PV).reshape(-1)
    A = alpha * np.eye(D.size) + _dense_minus_half_laplacian(PN, PA)
    y = np.linalg.solve(A, D * r.reshape(-1))
    return (D * y).reshape(PN)


def _prec_error(fn, **kw):
    m, phi, Phi, r, alpha = _prec_case(**kw)
    ref = _prec_reference(m, phi, Phi, r, alpha)
    got = fn(m, phi, Phi, r, alpha)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


# mutants of oracle.pcg.preconditioner, each with one plausible mistake
def _mut_signed_lambda(model, phi, Phi, r, alpha):
    g = model.grid
    PV = 1.0 / (alpha + model.V + model.beta * np.abs(phi) ** 2 + model.lam * np.maximum(Phi, 0.0))
    sq = np.sqrt(PV)
    NX, NY, NZ = g.nu_mesh()
    return sq * spectral.ifftn(spectral.fftn(sq * r) / (alpha + 0.5 * (NX * NX + NY * NY + NZ * NZ)))


def _mut_no_max(model, phi, Phi, r, alpha):
    g = model.grid
    PV = 1.0 / (alpha + model.V + model.beta * np.abs(phi) ** 2 + abs(model.lam) * Phi)
    sq = np.sqrt(PV)
    NX, NY, NZ = g.nu_mesh()
    return sq * spectral.ifftn(spectral.fftn(sq * r) / (alpha + 0.5 * (NX * NX + NY * NY + NZ * NZ)))


def _mut_one_sided(model, phi, Phi, r, alpha):
    g = model.grid
    PV = 1.0 / (alpha + model.V + model.beta * np.abs(phi) ** 2 + abs(model.lam) * np.maximum(Phi, 0.0))
    NX, NY, NZ = g.nu_mesh()
    return PV * spectral.ifftn(spectral.fftn(r) / (alpha + 0.5 * (NX * NX + NY * NY + NZ * NZ)))


def _mut_no_shift(model, phi, Phi, r, alpha):
    g = model.grid
    PV = 1.0 / (alpha + model.V + model.beta * np.abs(phi) ** 2 + abs(model.lam) * np.maximum(Phi, 0.0))
    sq = np.sqrt(PV)
    NX, NY, NZ = g.nu_mesh()
    lap = 0.5 * (NX * NX + NY * NY + NZ * NZ)
    lap[0, 0, 0] = 1.0
    return sq * spectral.ifftn(spectral.fftn(sq * r) / lap)


def test_preconditioner_equals_dense_solve():
    """P r = P_V^{1/2} (alpha - Lap/2)^{-1} P_V^{1/2} r with the Laplacian built from the Fourier basis."""
    assert _prec_error(preconditioner) < 1e-12
    assert _prec_error(preconditioner, lam=35.0, seed=4) < 1e-12


@pytest.mark.parametrize("mutant", [_mut_signed_lambda, _mut_no_max, _mut_one_sided, _mut_no_shift])
def test_preconditioner_pin_rejects_mutants(mutant):
    assert _prec_error(mutant) > 1e-3


# ---------------------------------------------------------------- shift alpha at a Gaussian
AG_N, AG_A, AG_G = (48, 48, 48), (6.0, 6.0, 6.0), (1.0, 1.5, 2.0)
AG_ND = (0.6, 0.0, 0.8)


@pytest.fixture(scope="module")
def alpha_case():
    sig = tuple(1.0 / math.sqrt(2.0 * gm) for gm in AG_G)       # |G|^2 is a Gaussian of these widths
    J = pins.gaussian_dipolar_J(sig, AG_ND)
    lam = -40.0 * math.copysign(1.0, J)                          # lambda J < 0: |lambda J| != lambda J
    beta = 75.0
    m = Model(AG_N, AG_A, AG_G, beta, lam, AG_ND, 0.3)
    G = bi.normalize(bi.gaussian_trap(AG_N, AG_A, AG_G), AG_N, AG_A).astype(np.complex128)
    Phi = m.Phi(np.abs(G) ** 2)
    ref = sum(AG_G) / 2 + beta * math.sqrt(np.prod(AG_G)) / (2 * math.pi) ** 1.5 + abs(lam * J)
    return m, G, Phi, ref, lam * J


def _mut_alpha_no_abs(model, phi, Phi):
    g = model.grid
    rho = np.abs(phi) ** 2
    a = ip(g, model.kinetic(phi) + model.V * phi + model.beta * rho * phi, phi)
    return a + model.lam * ip(g, Phi * phi, phi)


def _mut_alpha_no_dip(model, phi, Phi):
    g = model.grid
    rho = np.abs(phi) ** 2
    return ip(g, model.kinetic(phi) + model.V * phi + model.beta * rho * phi, phi)


def _mut_alpha_half_beta(model, phi, Phi):
    g = model.grid
    rho = np.abs(phi) ** 2
    a = ip(g, model.kinetic(phi) + model.V * phi + 0.5 * model.beta * rho * phi, phi)
    return a + abs(model.lam * ip(g, Phi * phi, phi))


def test_shift_alpha_gaussian_closed_form(alpha_case):
    m, G, Phi, ref, lamJ = alpha_case
    assert lamJ < -0.05                       # the dipolar term is well above the tolerance
    assert abs(shift_alpha(m, G, Phi) - ref) < 1e-10 * ref


@pytest.mark.parametrize("mutant", [_mut_alpha_no_abs, _mut_alpha_no_dip, _mut_alpha_half_beta])
def test_shift_alpha_pin_rejects_mutants(alpha_case, mutant):
    m, G, Phi, ref, _ = alpha_case
    assert abs(mutant(m, G, Phi) - ref) > 1e-3


# ---------------------------------------------------------------- Polak-Ribiere coefficient and resets
@pytest.fixture(scope="module")
def small12():
    w = bi.WORKLOADS["small_32"]
    n = (12, 12, 12)
    return Model.from_workload(w, n=n), bi.initial_guess(w, n)


def test_beta_pr_vanishes_for_zero_steps(small12):
    """t = 0 leaves phi unchanged, so r_n = r_{n-1} and the PR numerator is exactly a difference
    of equal vectors (up to the rounding of <r_{n-1}, phi> = 0): beta_cg = 0, not the
    Fletcher-Reeves value 1."""
    m, phi0 = small12
    r = pcg(m, phi0, max_iter=4, debug={"force_t": 0.0}, trace=True)
    assert len(r.trace) == 4
    for t in r.trace[1:]:
        assert abs(t["beta_cg"]) < 1e-10, t["beta_cg"]


def test_beta_after_forced_accept_is_zero(small12):
    m, phi0 = small12
    r = pcg(m, phi0, max_iter=8, max_halvings=1, debug={"force_t": 1e5}, trace=True)
    forced = [t["forced"] for t in r.trace]
    assert any(forced)
    for prev, t in zip(r.trace, r.trace[1:]):
        if prev["forced"]:
            assert t["beta_cg"] == 0.0


def test_directions_descend_and_beta_nonnegative(small12):
    """beta_cg = max(beta_PR, 0): with fixed steps (t = 1) the raw Polak-Ribiere ratio is negative
    on every iteration of this case, so a missing max(., 0) shows as beta < 0; the plain run uses
    the conjugate direction."""
    m, phi0 = small12
    r = pcg(m, phi0, max_iter=60, trace=True)
    betas = [t["beta_cg"] for t in r.trace]
    assert all(b >= 0.0 for b in betas)
    assert sum(b > 0.0 for b in betas) > 10          # the conjugate direction is in use
    assert all(t["d1"] < 0.0 for t in r.trace)
    r = pcg(m, phi0, max_iter=20, trace=True, debug={"force_t": 1.0})
    assert all(t["beta_cg"] >= 0.0 for t in r.trace)


def test_psd_reset_keeps_descent(small12):
    """From a state near the minimum, forced long steps (t = 37, halved until the energy drops)
    overshoot along p, so the next Polak-Ribiere direction points uphill (<H phi, p> >= 0) on
    several iterations; the reset to -J(P r) must leave every direction a descent direction."""
    m, phi0 = small12
    r0 = pcg(m, phi0, tol_res=1e-4)
    r = pcg(m, r0.phi, max_iter=30, trace=True, debug={"force_t": 37.0})
    assert r.resets >= 3
    assert all(t["d1"] < 0.0 for t in r.trace)
