"""CPU pins of the oracle's network and interpolation functions against facts that do not come
from the oracle's own arithmetic: bit-level BF16 rounding, finite differences, closed forms of
Adam and of degenerate networks, trigonometric polynomials sampled exactly."""
import math

import numpy as np
import pytest

from oracle import interp as oi
from oracle import mlp as om
from oracle.grid import Grid


# ------------------------------------------------------------------ BF16 rounding
def bf16_bitwise(x32):
    """Nearest BF16 by enumerating the two BF16 neighbours of an FP32 value bit-wise."""
    bits = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lo = (bits & 0xFFFF0000).astype(np.uint32)
    hi = (lo.astype(np.uint64) + 0x10000).astype(np.uint32)
    flo = lo.view(np.float32).astype(np.float64)
    fhi = hi.view(np.float32).astype(np.float64)
    x = np.asarray(x32, dtype=np.float32).astype(np.float64)
    dlo, dhi = np.abs(x - flo), np.abs(fhi - x)
    lo_even = ((lo >> 16) & 1) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & lo_even)
    return np.where(pick_lo, flo, fhi)


def test_bf16_round_matches_bitwise_neighbours():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.uniform(-1, 1, 20000)]).astype(np.float32)
    assert np.array_equal(om.bf16_round(x.astype(np.float64)), bf16_bitwise(x))


def test_bf16_round_ties_to_even():
    one = 1.0
    assert om.bf16_round(one + 2.0 ** -8) == 1.0                       # tie, even mantissa below
    assert om.bf16_round(one + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6       # tie, even mantissa above
    assert om.bf16_round(-(one + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)
    assert om.bf16_round(0.0) == 0.0
    assert om.bf16_round(3.0) == 3.0


# ------------------------------------------------------------------ network gradient
DIMS = (6, 16, 24)


def small_problem(seed=0, B=5):
    rng = np.random.default_rng(seed)
    P = 16 * 6 + 16 + 16 * 16 + 16 + 24 * 16 + 24
    params = rng.standard_normal(P) * 0.5
    x = rng.uniform(-1, 1, (B, 6))
    t = rng.standard_normal((B, 24))
    return params, x, t


def test_gradient_matches_central_differences():
    params, x, t = small_problem()
    loss, g, _ = om.loss_grad(params, x, t, DIMS, bf16=False)
    rng = np.random.default_rng(7)
    offs = np.cumsum([0, 96, 16, 256, 16, 384, 24])
    eps = 1e-5
    for blk in range(6):
        for i in rng.integers(offs[blk], offs[blk + 1], 4):
            e = np.zeros_like(params)
            e[i] = eps
            lp = om.loss_grad(params + e, x, t, DIMS, bf16=False)[0]
            lm = om.loss_grad(params - e, x, t, DIMS, bf16=False)[0]
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (blk, i, fd, g[i])
    # directional derivative along a random direction
    d = rng.standard_normal(params.size)
    fd = (om.loss_grad(params + 1e-6 * d, x, t, DIMS, bf16=False)[0]
          - om.loss_grad(params - 1e-6 * d, x, t, DIMS, bf16=False)[0]) / 2e-6
    assert abs(fd - g @ d) <= 1e-6 * abs(g @ d)


def test_bf16_network_close_to_fp64_network():
    params, x, t = small_problem(3)
    l0, g0, y0 = om.loss_grad(params, x, t, DIMS, bf16=False)
    l1, g1, y1 = om.loss_grad(params, x, t, DIMS, bf16=True)
    assert np.linalg.norm(y1 - y0) <= 2e-2 * np.linalg.norm(y0)
    assert np.linalg.norm(g1 - g0) <= 5e-2 * np.linalg.norm(g0)
    assert l1 != l0


def test_degenerate_network_closed_form():
    """W1 = W2 = W3 = 0: h1 = tanh(b1), h2 = tanh(b2), y = b3, so
    dL/db3 = 2/(BD) sum_b (b3 - T_b), dL/dW3[o][i] = 2/(BD) sum_b (b3 - T_b)[o] tanh(b2)[i] (before the
    BF16 rounding of dL/dy and h2), every other gradient zero. Values are chosen BF16-exact."""
    B, (din, dh, dout) = 4, DIMS
    b1 = np.full(dh, 0.5)
    b2 = np.linspace(-1, 1, dh)
    b3 = np.linspace(-2, 2, dout)
    params = np.concatenate([np.zeros(dh * din), b1, np.zeros(dh * dh), b2, np.zeros(dout * dh), b3])
    T = np.tile(np.arange(dout) / 8.0, (B, 1)) + np.arange(B)[:, None]
    loss, g, y = om.loss_grad(params, np.ones((B, din)), T, DIMS, bf16=False)
    assert np.array_equal(y, np.tile(b3, (B, 1)))
    r = b3[None, :] - T
    assert loss == pytest.approx(np.mean(r * r), rel=1e-15)
    G = om.unpack(g, *DIMS)
    assert np.allclose(G["b3"], 2.0 / (B * dout) * r.sum(0), rtol=1e-14, atol=0)
    assert np.allclose(G["W3"], 2.0 / (B * dout) * np.outer(r.sum(0), np.tanh(b2)), rtol=1e-14, atol=1e-17)
    for k in ("W1", "b1", "W2", "b2"):
        assert not np.any(G[k])


# ------------------------------------------------------------------ Adam
def test_adam_first_step_and_constant_gradient_closed_form():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(1000)
    g = rng.standard_normal(1000)
    lr, eps = 1e-3, 1e-8
    p, m, v = om.adam_step(p0, g, np.zeros(1000), np.zeros(1000), 1, lr, eps=eps)
    assert np.allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    for t in range(2, 6):
        p, m, v = om.adam_step(p, g, m, v, t, lr, eps=eps)
    assert np.allclose(p, p0 - 5 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


# ------------------------------------------------------------------ interpolation
def trig_poly(grid, modes):
    """sum_m c_m exp(i (kx nu_x (x + a) + ...)) evaluated at the grid points (closed form)."""
    X, Y, Z = grid.mesh()
    u = np.zeros(grid.n, dtype=np.complex128)
    for (kx, ky, kz), c in modes:
        ph = (kx * math.pi / grid.a[0] * (X + grid.a[0]) + ky * math.pi / grid.a[1] * (Y + grid.a[1])
              + kz * math.pi / grid.a[2] * (Z + grid.a[2]))
        u += c * np.exp(1j * ph)
    return u


MODES = [((0, 0, 0), 0.7), ((3, -2, 1), 0.2 - 0.1j), ((-7, 5, -3), 0.05j), ((2, 7, 3), -0.3), ((-1, -7, -2), 0.11)]


def test_resample_upsamples_trig_polynomial_exactly():
    a = (4.0, 3.0, 2.0)
    gc, gf = Grid((16, 16, 8), a), Grid((40, 32, 24), a)
    u = oi.resample(trig_poly(gc, MODES), gf.n)
    assert np.max(np.abs(u - trig_poly(gf, MODES))) <= 1e-13


def test_resample_truncates_to_common_modes():
    a = (4.0, 3.0, 2.0)
    gf, gc = Grid((32, 32, 16), a), Grid((16, 12, 8), a)
    keep = [m for m in MODES if abs(m[0][0]) < 8 and abs(m[0][1]) < 6 and abs(m[0][2]) < 4]
    assert len(keep) < len(MODES)
    u = oi.resample(trig_poly(gf, MODES), gc.n)
    assert np.max(np.abs(u - trig_poly(gc, keep))) <= 1e-13


def test_resample_drops_nyquist_mode():
    g = Grid((8, 8, 8), (1.0, 1.0, 1.0))
    u = np.ones(g.n) * ((-1.0) ** np.arange(8))[:, None, None]
    assert np.max(np.abs(oi.resample(u, (16, 8, 8)))) <= 1e-15


def test_normalize_and_gauge_fix_properties():
    g = Grid((8, 10, 6), (2.0, 2.5, 1.5))
    rng = np.random.default_rng(2)
    u = rng.standard_normal(g.n) + 1j * rng.standard_normal(g.n)
    v = oi.normalize(u, g.h3)
    assert g.h3 * np.sum(np.abs(v) ** 2) == pytest.approx(1.0, abs=1e-14)
    w = oi.gauge_fix(u * np.exp(0.9j), g, (1.0, 2.0, 3.0))
    X, Y, Z = g.mesh()
    s = np.sum(w * np.exp(-0.5 * (X ** 2 + 2 * Y ** 2 + 3 * Z ** 2)))
    assert abs(s.imag) <= 1e-13 * abs(s) and s.real > 0
    assert np.allclose(np.abs(w), np.abs(u), rtol=1e-14)
