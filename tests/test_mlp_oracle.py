"""Pins of the warm-start MLP oracle: features against the clamped-window
definition written as loops, gradients against central finite differences,
the first Adam step against its closed form, SplitMix64 against its
published outputs.  CPU only."""
import json
import os

import numpy as np

from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_features_match_clamped_window_loops():
    rng = np.random.default_rng(0)
    m = 6
    R = rng.normal(0, 0.1, m ** 3)
    states = [0, 5, 36, 107, m ** 3 - 1, 77]
    X = mlp.features(R, m, 0.97, 0.12, states)
    for row, s in zip(X, states):
        i = (s // (m * m), (s // m) % m, s % m)
        ref = [c / (m - 1) for c in i]
        for d0 in range(-2, 3):
            for d1 in range(-2, 3):
                for d2 in range(-2, 3):
                    j = [min(max(c + d, 0), m - 1) for c, d in zip(i, (d0, d1, d2))]
                    ref.append(10.0 * R[(j[0] * m + j[1]) * m + j[2]])
        ref += [(0.97 - 0.945) / 0.026, (0.12 - 0.175) / 0.072]
        np.testing.assert_allclose(row, ref, rtol=0, atol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = rng.normal(0, 0.1, mlp.N_PARAMS)
    X = rng.normal(0, 1, (12, mlp.F))
    t = rng.normal(0, 1, 12)
    L, g = mlp.loss_grad(p, X, t)
    assert abs(L - mlp.loss(p, X, t)) < 1e-14
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False),
                          [mlp.N_PARAMS - 1, mlp.F * mlp.H, mlp.F * mlp.H + 3]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[k] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m1, v1 = mlp.adam(p, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # bias-corrected moments equal g and g^2 at step 1
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_splitmix64_published_outputs():
    gold = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    inc = int(gold["state_increment"], 16)
    state = 0
    for out in gold["outputs_from_state_0"]:
        assert mlp.splitmix64(state) == int(out, 16)
        state = (state + inc) & ((1 << 64) - 1)


def test_pack_roundtrip_and_count():
    assert mlp.N_PARAMS == 99585
    p = np.arange(mlp.N_PARAMS, dtype=np.float64)
    np.testing.assert_array_equal(mlp.pack(mlp.unpack(p)), p)
