"""FP64 CPU reference of the message-passing surrogate (forward, loss, backward).

TEST INFRASTRUCTURE ONLY: it judges the gradients of the GPU training kernels
and is itself checked against central finite differences.

The surrogate jumps the enthalpy state `horizon` explicit steps ahead.  Given
two consecutive plain states H0 = H^n and H1 = H^{n+1} it predicts

    H^{n+horizon} ~ H1 + (horizon - 1) (H1 - H0) + c_i * DH_SCALE * y_i,

a linear extrapolation in time corrected by the network output y_i of node i.
Per-node input features (8):

    x0 = (T(H1) - T_REF) / T_SCALE          temperature
    x1 = fs(H1)                             fraction solid
    x2 = 1 if the node's material has latent heat else 0
    x3 = b_i dt / (m_i c_i)                 Robin strength per step
    x4 = 2 sum_j w_ij dt / (m_i c_i)        interface strength per step
    x5 = sum_j |K_ij| dt / (m_i c_i)        conduction strength per step
    x6 = horizon (H1 - H0) / (c_i T_SCALE)  extrapolated change over the horizon
    x7 = 1

Network (width W, L message-passing layers, ReLU):

    h_0 = relu(X W_in + b_in)
    a_l = A h_{l-1}                         A: mean over mesh neighbours
    h_l = h_{l-1} + relu([h_{l-1}, a_l] W_l + b_l)      l = 1..L
    y   = h_L w_out + b_out

Loss over the nodes of one sample: mean_i (y_i - t_i)^2 with the target
t_i = (H_true_i - base_i) / (c_i DH_SCALE).
"""
import numpy as np

T_REF = 25.0
T_SCALE = 700.0
DH_SCALE = 10.0   # K of sensible heat per unit of network output
N_FEAT = 8


def graph_mean_operator(conn, n_nodes):
    """Rows of A: 1/deg_i on the mesh neighbours of i (nodes sharing an element), as CSR."""
    nen = conn.shape[1]
    pairs = []
    for a in range(nen):
        for b in range(nen):
            if a != b:
                pairs.append(np.stack([conn[:, a], conn[:, b]], axis=1))
    p = np.unique(np.concatenate(pairs, axis=0), axis=0)
    ptr = np.zeros(n_nodes + 1, np.int64)
    np.add.at(ptr, p[:, 0] + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr, p[:, 1].astype(np.int64)


def apply_mean(ptr, col, h):
    out = np.zeros_like(h)
    deg = np.diff(ptr)
    rows = np.repeat(np.arange(ptr.size - 1), deg)
    np.add.at(out, rows, h[col])
    return out / deg[:, None]


def apply_mean_T(ptr, col, g):
    """Transpose of apply_mean."""
    deg = np.diff(ptr)
    rows = np.repeat(np.arange(ptr.size - 1), deg)
    out = np.zeros_like(g)
    np.add.at(out, col, g[rows] / deg[rows][:, None])
    return out


def init_params(width, layers, seed):
    rng = np.random.default_rng(seed)
    p = {"W_in": rng.normal(0, np.sqrt(2.0 / N_FEAT), (N_FEAT, width)), "b_in": np.zeros(width)}
    for l in range(layers):
        p["W%d" % l] = rng.normal(0, np.sqrt(1.0 / (2 * width)), (2 * width, width))
        p["b%d" % l] = np.zeros(width)
    p["w_out"] = rng.normal(0, 0.01, width)
    p["b_out"] = np.zeros(1)
    return p


def forward(p, X, ptr, col, layers):
    cache = {}
    z = X @ p["W_in"] + p["b_in"]
    h = np.maximum(z, 0.0)
    cache["z_in"] = z
    hs = [h]
    for l in range(layers):
        a = apply_mean(ptr, col, h)
        u = np.concatenate([h, a], axis=1)
        z = u @ p["W%d" % l] + p["b%d" % l]
        cache["u%d" % l], cache["z%d" % l] = u, z
        h = h + np.maximum(z, 0.0)
        hs.append(h)
    y = h @ p["w_out"] + p["b_out"][0]
    cache["hs"] = hs
    return y, cache


def loss_and_grad(p, X, t, ptr, col, layers):
    y, c = forward(p, X, ptr, col, layers)
    n = y.size
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / n
    g = {"w_out": c["hs"][-1].T @ dy, "b_out": np.array([dy.sum()])}
    dh = np.outer(dy, p["w_out"])
    width = p["b_in"].size
    for l in reversed(range(layers)):
        z = c["z%d" % l]
        dz = dh * (z > 0)
        g["W%d" % l] = c["u%d" % l].T @ dz
        g["b%d" % l] = dz.sum(axis=0)
        du = dz @ p["W%d" % l].T
        dh = dh + du[:, :width] + apply_mean_T(ptr, col, du[:, width:])
    dz = dh * (c["z_in"] > 0)
    g["W_in"] = X.T @ dz
    g["b_in"] = dz.sum(axis=0)
    return loss, g, y
