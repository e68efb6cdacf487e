"""Host logic of the learned initial guess and of the multigrid cascade: gamma_z bands and
boxes, input features, the dipole axis, and the grid levels."""
import math

import numpy as np
import pytest

import bec_inputs as bi
from paper_2603_05194_amd import learned as L
from paper_2603_05194_amd import multigrid as MG


def test_bands_cover_the_sampling_range_and_share_boxes():
    assert L.box_for(20.0) == (16.0, 16.0, 2.0)
    assert L.gz_band(4.0) == -7 and L.gz_band(40.0) == 3
    for gz in np.linspace(4.0, 40.0, 200):
        k = L.gz_band(gz)
        lo = 20.0 * 2.0 ** (k / 3.0)
        assert lo <= gz * (1 + 1e-12) and gz < 20.0 * 2.0 ** ((k + 1) / 3.0) * (1 + 1e-12)
        a = L.box_for(gz)
        assert a[:2] == (16.0, 16.0)
        assert a[2] == pytest.approx(2.0 * math.sqrt(20.0 / lo), rel=1e-14)
        assert a[2] >= 2.0 * math.sqrt(20.0 / gz) * (1 - 1e-12)   # never smaller than the rule at gz


def test_features_map_sampling_ranges_to_unit_interval():
    lo = L.features([200.0, 0.0, 0.0, 4.0, 0.0, 0.0])
    hi = L.features([3000.0, 0.8, 0.95, 40.0, math.pi / 2, math.pi])
    assert np.allclose(lo, -1.0, atol=1e-6) and np.allclose(hi, 1.0, atol=1e-6)
    for s in range(20):
        f = L.features(bi.mlp_param_draw(s))
        assert f.dtype == np.float32 and np.all(np.abs(f) <= 1.0 + 1e-6)


def test_physical_parameters_of_a_draw():
    d = bi.mlp_param_draw(3)
    p = L.physical(d)
    assert p["gamma"] == (1.0, 1.0, d[3])
    assert p["lam"] == pytest.approx(d[0] * d[1])
    assert np.linalg.norm(p["ndip"]) == pytest.approx(1.0, abs=1e-15)
    assert p["ndip"][2] == pytest.approx(math.cos(d[4]))


def test_multigrid_levels():
    assert MG.levels((256, 256, 64)) == [(64, 64, 16), (128, 128, 32), (256, 256, 64)]
    assert MG.levels((96, 96, 48), count=2) == [(48, 48, 24), (96, 96, 48)]
    with pytest.raises(ValueError):
        MG.levels((96, 96, 12))          # 12/4 = 3 is odd
    with pytest.raises(ValueError):
        MG.levels((16, 16, 8))           # 8/4 = 2 < 4


def test_mlp_init_is_seeded_and_glorot_scaled():
    a, b = bi.mlp_init((6, 16, 24), 1), bi.mlp_init((6, 16, 24), 1)
    assert np.array_equal(a, b) and a.dtype == np.float32
    W1 = a[:96]
    assert np.max(np.abs(W1)) <= math.sqrt(6.0 / 22.0)
    assert not np.any(a[96:112])   # b1 = 0


def test_paper_guesses_follow_the_listed_combinations():
    import bec_inputs as bi
    n, a = (12, 10, 8), (4.0, 5.0, 6.0)
    g = bi.paper_guesses(n, a, (1.0, 2.0, 0.5), 300.0, 0.3)
    assert g.shape == (10,) + n
    h3 = np.prod([2 * a[i] / n[i] for i in range(3)])
    for k in range(10):
        assert h3 * np.sum(np.abs(g[k]) ** 2) == pytest.approx(1.0, abs=1e-13)
    names = dict(zip(bi.PAPER_GUESS_NAMES, g))
    X, Y, Z = np.meshgrid(*[-a[i] + np.arange(n[i]) * 2 * a[i] / n[i] for i in range(3)], indexing="ij")
    ga = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 2)
    assert np.allclose(names["a"], ga / np.sqrt(h3 * np.sum(ga ** 2)), rtol=1e-13, atol=0)
    vb = (X + 1j * Y) * ga
    assert np.allclose(names["b"], vb / np.sqrt(h3 * np.sum(np.abs(vb) ** 2)), rtol=1e-12, atol=1e-15)
    for k in ("b", "c", "d", "e"):
        assert np.array_equal(names[k + "_bar"], np.conj(names[k]))
    mix = 0.7 * names["a"] + 0.3 * names["b"]
    assert np.allclose(names["d"], mix / np.sqrt(h3 * np.sum(np.abs(mix) ** 2)), rtol=1e-12, atol=1e-15)
    assert np.all(names["f"].imag == 0) and np.all(names["f"].real >= 0)
