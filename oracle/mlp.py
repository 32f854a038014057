"""Reference perceptron for the near-field surrogate (test infrastructure).

Plain numpy in FP64: layers 16 -> H -> H -> H -> 12 with ReLU on the hidden
layers, loss = mean over the batch and the 12 outputs of (y - t)^2, and its
gradient by the chain rule written out layer by layer.  The parameter vector
uses the same packing as the library: W1 [16][H], b1 [H], W2 [H][H], b2,
W3 [H][H], b3, W4 [H][12], b4 [12], where W[k][n] maps input k to output n.

Surrogate targets for a tet seen from a target x (the network predicts the
part of the pair integral of Sec. 2.1 that the tet's own quadrupole
expansion misses).  The tet is given by its corners in the target's frame,
s_i = (v_i - x) / |x - centroid| (corner i, in the library's corner order);
the network's 16 inputs are the same geometry as scale-free O(1) numbers:
the unit direction (x - c)/|x - c|, the corners about the centroid in units
of the diameter (v_i - c)/d, and 1/rho.  Outputs
    y_j = Y_SCALE (C_j - Cq_j) rho^4 / Vh
with d the tet diameter (longest edge), rho = |x - centroid| / d,
Vh = V / d^3, C_j = u_T(x) / d for the unit nodal field j (component j % 3
at corner j // 3) and Cq_j the same for the expansion of the tet about its
centroid truncated at |n| <= 2 (dipole and quadrupole terms of the Taylor
expansion of Sec. 2.2).  The pair then is u_T = d sum_j (Cq_j + y_j Vh /
(Y_SCALE rho^4)) M_j; rho^4 makes y O(1) over the band 2 <= rho < 6
(the residual falls like rho^-4).
"""
import numpy as np

N_IN = 16
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


Y_SCALE = 2048.0


def quadrupole_potential(x, v, M, p2m_tet, taylor_coeffs):
    """u of the tet's multipole expansion about its centroid truncated at
    |n| <= 2: (1/4 pi) sum_n a_n(x - c) Q_n with the oracle's P2M and Taylor
    coefficients (Sec. 2.2)."""
    c = np.asarray(v, dtype=np.float64).mean(axis=0)
    Q = p2m_tet(v, M, c, 2)
    a = taylor_coeffs(np.asarray(x, dtype=np.float64) - c, 2)
    return float(a @ Q) / (4.0 * np.pi)


def surrogate_features(s):
    """The 16 network inputs of the scaled corners s [4, 3] (target at the
    origin, unit distance to the centroid)."""
    s = np.asarray(s, dtype=np.float64)
    c = s.mean(axis=0)
    d = max(np.linalg.norm(s[a] - s[b]) for a in range(4) for b in range(a + 1, 4))
    dist = np.linalg.norm(c)
    return np.concatenate([-c / dist, ((s - c) / d).ravel(), [d / dist]])


def corners_from_features(f):
    """Inverse of surrogate_features: the scaled corners [4, 3]."""
    f = np.asarray(f, dtype=np.float64)
    c = -f[:3] / np.linalg.norm(f[:3])
    return c + f[3:15].reshape(4, 3) * f[15]


def surrogate_target(s, tet_potential, p2m_tet, taylor_coeffs):
    """Targets y [12] for the inputs s [4, 3] (target at the origin, unit
    distance to the centroid), from an exact pair integral tet_potential(x,
    v, M) and the oracle's P2M / Taylor coefficients for the quadrupole part."""
    s = np.asarray(s, dtype=np.float64)
    d = max(np.linalg.norm(s[a] - s[b]) for a in range(4) for b in range(a + 1, 4))
    vh = abs(np.linalg.det(np.stack([s[1] - s[0], s[2] - s[0], s[3] - s[0]]))) / 6.0 / d ** 3
    rho = np.linalg.norm(s.mean(axis=0)) / d
    x = np.zeros(3)
    y = np.zeros(12)
    for j in range(12):
        M = np.zeros((4, 3))
        M[j // 3, j % 3] = 1.0
        res = tet_potential(x, s, M) - quadrupole_potential(x, s, M, p2m_tet, taylor_coeffs)
        y[j] = Y_SCALE * res / d * rho ** 4 / vh
    return y


def pair_from_target(s, y, M, dist, p2m_tet, taylor_coeffs):
    """u_T at the target from the network's outputs y [12] (or the exact
    targets), the inputs s [4, 3], the nodal field M [4, 3] and the distance
    |x - centroid| of the unscaled pair (u is homogeneous of degree 1 in
    length, so u = dist * u(scaled))."""
    s = np.asarray(s, dtype=np.float64)
    d = max(np.linalg.norm(s[a] - s[b]) for a in range(4) for b in range(a + 1, 4))
    vh = abs(np.linalg.det(np.stack([s[1] - s[0], s[2] - s[0], s[3] - s[0]]))) / 6.0 / d ** 3
    rho = np.linalg.norm(s.mean(axis=0)) / d
    uq = quadrupole_potential(np.zeros(3), s, M, p2m_tet, taylor_coeffs)
    ures = d * float(np.dot(np.asarray(y).ravel(), np.asarray(M, dtype=np.float64).ravel())) * vh / (Y_SCALE * rho ** 4)
    return dist * (uq + ures)
