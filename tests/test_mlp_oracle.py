"""Pins of the warm-start network oracle (CPU only)."""
import numpy as np

from oracle import mlp_oracle as mo


def _setup(seed=0, F=8, W=32, O=32, n=5, n_cols=6):
    rng = np.random.default_rng(seed)
    n_par = W * F + W + W * W + W + O * W + O
    p = rng.standard_normal(n_par) * 0.3
    phi = mo.features(rng.uniform(0, 2, n), F // 2, 2.0)
    tgt = rng.standard_normal((n, O))
    return p, phi, tgt, F, W, O, n_cols


def test_backward_matches_central_differences():
    p, phi, tgt, F, W, O, nc = _setup()
    loss, g = mo.loss_grad(p, phi, tgt, nc, F, W, O)
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        num = (mo.loss_grad(p + e, phi, tgt, nc, F, W, O)[0] - mo.loss_grad(p - e, phi, tgt, nc, F, W, O)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-7 * max(1.0, abs(num)), (i, num, g[i])


def test_loss_is_mean_squared_error_of_counted_columns():
    p, phi, tgt, F, W, O, nc = _setup(seed=2)
    _, _, out = mo.forward(p, phi, F, W, O)
    loss, _ = mo.loss_grad(p, phi, tgt, nc, F, W, O)
    assert abs(loss - np.mean((out[:, :nc] - tgt[:, :nc]) ** 2)) < 1e-14
    # columns beyond n_cols carry no gradient into the output bias
    _, g = mo.loss_grad(p, phi, tgt, nc, F, W, O)
    assert np.all(g[-O + nc:] == 0.0)


def test_features_closed_form():
    phi = mo.features([0.0, 0.5], 3, 2.0)
    assert np.allclose(phi[0], [0, 1, 0, 1, 0, 1])
    k = np.array([1, 2, 3])
    assert np.allclose(phi[1, 0::2], np.sin(k * np.pi * 0.25))
    assert np.allclose(phi[1, 1::2], np.cos(k * np.pi * 0.25))


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.14159, 0.0])
    r = mo.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0            # tie to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6                 # tie to even (up)
    assert abs(r[4] + 3.14159) <= 2 ** -8 * 3.15
    assert r[5] == 0.0
