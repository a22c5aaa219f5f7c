"""CPU reference of the subtask cost model (test infrastructure only): a 12-64-64-1 ReLU
network on standardised features, mean squared error on log2 cycles, in float64.

Parameter layout (flat): W1[64][12] b1[64] W2[64][64] b2[64] W3[64] b3, then the feature
mean[12] and standard deviation[12]; forward and backward follow the chain rule written
out layer by layer.
"""
import numpy as np

H, NF = 64, 12
OFF_W1 = 0
OFF_B1 = H * NF
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
NPARAM = OFF_B3 + 1
NTOTAL = NPARAM + 2 * NF


def unpack(w):
    w = np.asarray(w, np.float64)
    return dict(W1=w[OFF_W1:OFF_B1].reshape(H, NF), b1=w[OFF_B1:OFF_W2], W2=w[OFF_W2:OFF_B2].reshape(H, H),
                b2=w[OFF_B2:OFF_W3], W3=w[OFF_W3:OFF_B3], b3=w[OFF_B3], mean=w[NPARAM:NPARAM + NF],
                std=w[NPARAM + NF:NTOTAL])


def normalise(w, xraw):
    p = unpack(w)
    return (np.asarray(xraw, np.float64) - p["mean"]) / p["std"]


def forward(w, xraw):
    p = unpack(w)
    x = normalise(w, xraw)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0)
    y = h2 @ p["W3"] + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(w, xraw, t):
    """Mean squared error and its gradient with respect to the NPARAM parameters."""
    p = unpack(w)
    y, (x, z1, h1, z2, h2) = forward(w, xraw)
    nb = len(t)
    r = y - np.asarray(t, np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / nb
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = h2.T @ dy
    g[OFF_B3] = dy.sum()
    dz2 = np.outer(dy, p["W3"]) * (z2 > 0)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)
    g[OFF_W1:OFF_B1] = (dz1.T @ x).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(0)
    return loss, g


def random_weights(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    w = np.zeros(NTOTAL)
    w[OFF_W1:OFF_B1] = rng.uniform(-1, 1, H * NF) * np.sqrt(6 / NF) * scale
    w[OFF_B1:OFF_W2] = rng.uniform(-0.1, 0.1, H)
    w[OFF_W2:OFF_B2] = rng.uniform(-1, 1, H * H) * np.sqrt(6 / H) * scale
    w[OFF_B2:OFF_W3] = rng.uniform(-0.1, 0.1, H)
    w[OFF_W3:OFF_B3] = rng.uniform(-1, 1, H) * np.sqrt(6 / H) * scale
    w[OFF_B3] = 0.3
    w[NPARAM:NPARAM + NF] = rng.normal(0, 1, NF)
    w[NPARAM + NF:] = rng.uniform(0.5, 2.0, NF)
    return w
