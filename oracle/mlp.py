"""Reference perceptron for the near-field surrogate (test infrastructure).

Plain numpy in FP64: layers 12 -> H -> H -> H -> 12 with ReLU on the hidden
layers, loss = mean over the batch and the 12 outputs of (y - t)^2, and its
gradient by the chain rule written out layer by layer.  The parameter vector
uses the same packing as the library: W1 [12][H], b1 [H], W2 [H][H], b2,
W3 [H][H], b3, W4 [H][12], b4 [12], where W[k][n] maps input k to output n.

Surrogate targets for a tet seen from a target x: inputs s_i = (v_i - x) /
|x - centroid| (corner i, in the library's corner order), outputs
y_j = 16 pi C_j rho^2 / (V / d^3) with d the tet diameter (longest edge),
rho = |x - centroid| / d and C_j = u_T(x) / d for the unit nodal field j
(component j % 3 at corner j // 3).
"""
import numpy as np

N_IN = 12
N_OUT = 12


def layout(H):
    K = [N_IN, H, H, H]
    N = [H, H, H, N_OUT]
    out, o = [], 0
    for k, n in zip(K, N):
        out.append((o, k, n, o + k * n))
        o += k * n + n
    return out, o


def unpack(params, H):
    lay, n = layout(H)
    params = np.asarray(params, dtype=np.float64)
    assert params.size == n
    return [(params[w:w + k * nn].reshape(k, nn), params[b:b + nn]) for w, k, nn, b in lay]


def forward(params, H, X):
    """Returns the output [B, 12] and the hidden activations."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(params, H)
    for i, (W, b) in enumerate(layers):
        z = acts[-1] @ W + b
        acts.append(np.maximum(z, 0.0) if i < 3 else z)
    return acts[-1], acts


def loss_and_grad(params, H, X, T):
    Y, acts = forward(params, H, X)
    n = Y.size
    loss = float(np.sum((Y - T) ** 2) / n)
    d = 2.0 * (Y - T) / n
    layers = unpack(params, H)
    grads = [None] * 4
    for i in range(3, -1, -1):
        W, _ = layers[i]
        a = acts[i]
        grads[i] = (a.T @ d, d.sum(axis=0))
        if i > 0:
            d = (d @ W.T) * (acts[i] > 0.0)
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads])
    return loss, flat


def surrogate_target(s, tet_potential):
    """Targets y [12] for the inputs s [4, 3] (target at the origin, unit
    distance to the centroid), from an exact pair integral tet_potential(x, v, M)."""
    s = np.asarray(s, dtype=np.float64)
    d = max(np.linalg.norm(s[a] - s[b]) for a in range(4) for b in range(a + 1, 4))
    vh = abs(np.linalg.det(np.stack([s[1] - s[0], s[2] - s[0], s[3] - s[0]]))) / 6.0 / d ** 3
    rho = np.linalg.norm(s.mean(axis=0)) / d
    y = np.zeros(12)
    for j in range(12):
        M = np.zeros((4, 3))
        M[j // 3, j % 3] = 1.0
        y[j] = 16.0 * np.pi * tet_potential(np.zeros(3), s, M) / d * rho ** 2 / vh
    return y
