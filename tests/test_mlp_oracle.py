"""Pins of the CPU cost-model reference: finite differences and closed forms."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    w = mlp.random_weights(3)
    x = rng.normal(0, 2, (20, mlp.NF))
    t = rng.normal(10, 3, 20)
    loss, g = mlp.loss_and_grad(w, x, t)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 300, replace=False), [mlp.OFF_B3, mlp.OFF_B1, mlp.OFF_W3]])
    eps = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += eps
        wm = w.copy(); wm[i] -= eps
        fd = (mlp.loss_and_grad(wp, x, t)[0] - mlp.loss_and_grad(wm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_linear_special_case():
    """With all hidden units active and W2 = I, the network is affine: y = W3 (W1 x + b1) + ..."""
    w = np.zeros(mlp.NTOTAL)
    w[mlp.NPARAM + mlp.NF:] = 1.0                    # std 1, mean 0
    W1 = np.zeros((mlp.H, mlp.NF)); W1[:mlp.NF, :] = np.eye(mlp.NF)
    w[mlp.OFF_W1:mlp.OFF_B1] = W1.ravel()
    w[mlp.OFF_B1:mlp.OFF_W2] = 100.0                 # keeps every unit active
    w[mlp.OFF_W2:mlp.OFF_B2] = np.eye(mlp.H).ravel()
    w[mlp.OFF_W3:mlp.OFF_W3 + mlp.NF] = np.arange(1, mlp.NF + 1)
    x = np.random.default_rng(0).normal(0, 1, (5, mlp.NF))
    y, _ = mlp.forward(w, x)
    expect = (x + 100.0) @ np.arange(1, mlp.NF + 1) + 100.0 * 0  # units beyond NF carry W3 = 0
    np.testing.assert_allclose(y, expect, rtol=1e-12)
