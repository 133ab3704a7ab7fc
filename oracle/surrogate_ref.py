"""FP64 CPU reference of the message-passing surrogate (forward, loss, backward).

TEST INFRASTRUCTURE ONLY: it is the reference for the gradients of the GPU training kernels
and is itself checked against central finite differences.

The surrogate jumps the enthalpy state `horizon` explicit steps ahead.  Given
three consecutive plain states H0 = H^n, H1 = H^{n+1}, H2 = H^{n+2}, with
m = horizon - 2, q = m (m + 1) / 2, r = H2 - H1 and a = (H2 - H1) - (H1 - H0),
it predicts

    H^{n+horizon} ~ base_i + mu_i s_i y'_i,   base = H2 + m r  [+ q a],

the linear (or quadratic) extrapolation in time, corrected by the network
output where the extrapolation is known to fail: near the kinks of the
enthalpy relation.  s_i = |m r_i| + |q a_i| + c_i EPS_T is the node's
activity over the window (enthalpy units), and the mask mu_i is 1 at a free
phase-change node whose enthalpy lies within REACH activities of the solidus
or liquidus enthalpy (c T_sol, c T_liq + L), else 0.  Elsewhere the jump is
the extrapolation itself.  y' is the network output made energy-neutral over
the masked nodes of the scenario: y' = y - sum_j w_j y_j with
w_j = m_j mu_j s_j / sum_k m_k mu_k s_k, so that sum_i m_i mu_i s_i y'_i = 0.

Per-node input features (12):

    x0  = (T(H2) - T_REF) / T_SCALE         temperature
    x1  = fs(H2)                            fraction solid
    x2  = 1 if the node's material has latent heat else 0
    x3  = b_i dt / (m_i c_i)                Robin strength per step
    x4  = 2 sum_j w_ij dt / (m_i c_i)       interface strength per step
    x5  = sum_j |K_ij| dt / (m_i c_i)       conduction strength per step
    x6  = m r / s                           rate over the window, relative
    x7  = q a / s                           curvature over the window, relative
    x8  = 1
    x9  = ln(s / (c * 1 K)) / 8             activity in kelvin, logarithmic
    x10 = clip((H2 - H_liq) / s, -4, 4) / 4 distance to the liquidus (0 without latent heat)
    x11 = clip((H2 - H_sol) / s, -4, 4) / 4 distance to the solidus (0 without latent heat)

Network (width W, L message-passing layers, ReLU):

    h_0 = relu(X W_in + b_in)
    a_l = A h_{l-1}                         A: mean over mesh neighbours
    h_l = h_{l-1} + relu([h_{l-1}, a_l] W_l + b_l)      l = 1..L
    y   = h_L w_out + b_out

Loss over the rows of one sample, a mean over all rows of the masked terms:
in enthalpy, mu_i (y'_i - t_i)^2 with t_i = (H_true_i - base_i) / s_i (or its
Huber form), or in temperature, ((T(H_pred_i) - T(H_true_i)) / DT_SCALE)^2.
"""
import numpy as np

from . import oracle as orc

T_REF = 25.0
T_SCALE = 700.0
DT_SCALE = 10.0   # K per unit of the temperature loss
EPS_T = 0.01      # K: activity floor of the correction scale
REACH = 2.0       # a kink within REACH activities of H2 enables the correction
N_FEAT = 12


def _tri_area(x):
    return 0.5 * np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)


def _face_area(x):
    """Triangle area, or for a quad half the norm of the cross product of its diagonals."""
    if x.shape[1] == 3:
        return _tri_area(x)
    return 0.5 * np.linalg.norm(np.cross(x[:, 2] - x[:, 0], x[:, 3] - x[:, 1]), axis=1)


def node_strengths(prob):
    """Per node (input numbering): m_i c_i, the Robin coefficient b_i = sum over
    flux faces at i of (A_f / nodes per face) h_f, the interface weight sum
    sum_j w_ij = sum over contact pairs at i of h A / 3, and sum_j |K_ij| of the
    assembled conduction matrix (element matrices from the oracle)."""
    P = orc.Problem(prob)
    N = P.n_nodes
    xyz = np.asarray(prob["xyz"], np.float64)
    conn = np.asarray(prob["conn"], np.int64)
    mats = np.asarray(prob["materials"], np.float64).reshape(-1, 6)
    nmat = orc.node_material(P)
    mc = orc.lumped_mass(P) * mats[nmat, 2]
    b = np.zeros(N)
    ff = np.asarray(prob.get("flux_faces", np.zeros((0, 3))), np.int64)
    if ff.size:
        A = _face_area(xyz[ff])
        np.add.at(b, ff, (A * np.asarray(prob["flux_h"], np.float64) / ff.shape[1])[:, None] * np.ones(ff.shape[1]))
    w = np.zeros(N)
    fa = np.asarray(prob.get("if_a", np.zeros((0, 3))), np.int64)
    if fa.size:
        fb = np.asarray(prob["if_b"], np.int64)
        g = np.asarray(prob["if_h"], np.float64) * _tri_area(xyz[fa]) / 3.0
        np.add.at(w, fa, g[:, None] * np.ones(3))
        np.add.at(w, fb, g[:, None] * np.ones(3))
    ke = orc.tet_ke if conn.shape[1] == 4 else orc.hex_ke
    emat = np.asarray(prob["elem_mat"], np.int64)
    rows, cols, vals = [], [], []
    for e in range(conn.shape[0]):
        K, _ = ke(xyz[conn[e]], mats[emat[e], 0])
        rows.append(np.repeat(conn[e], conn.shape[1]))
        cols.append(np.tile(conn[e], conn.shape[1]))
        vals.append(K.ravel())
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    key = rows * N + cols
    uk, inv = np.unique(key, return_inverse=True)
    assembled = np.zeros(uk.size)
    np.add.at(assembled, inv, vals)
    kabs = np.zeros(N)
    np.add.at(kabs, uk // N, np.abs(assembled))
    return dict(mc=mc, robin_b=b, iface_w=w, kabs=kabs, node_mat=nmat)


def _materials(prob, strengths):
    mats = np.asarray(prob["materials"], np.float64).reshape(-1, 6)
    return mats[strengths["node_mat"]]


def activity(prob, H0, H1, H2, horizon=16, strengths=None):
    """Per node: the activity s, the mask mu (bool) and the kink enthalpies (H_sol, H_liq)."""
    st = node_strengths(prob) if strengths is None else strengths
    m_ = _materials(prob, st)
    c, Ts, Tl, L = m_[:, 2], m_[:, 3], m_[:, 4], m_[:, 5]
    H0, H1, H2 = (np.asarray(a, np.float64) for a in (H0, H1, H2))
    m = horizon - 2
    q = 0.5 * m * (m + 1)
    r = H2 - H1
    a = (H2 - H1) - (H1 - H0)
    span = np.abs(m * r) + np.abs(q * a)
    s = span + c * EPS_T
    H_sol, H_liq = c * Ts, c * Tl + L
    free = np.ones(H2.size, bool)
    free[np.asarray(prob.get("dirichlet_nodes", np.zeros(0, np.int64)), np.int64)] = False
    near = (np.abs(H2 - H_liq) < REACH * span) | (np.abs(H2 - H_sol) < REACH * span)
    mu = free & (L > 0) & near
    return s, mu, H_sol, H_liq


def features(prob, H0, H1, H2, dt, horizon=16, strengths=None):
    """The node features of the module docstring for one triple of states (FP64)."""
    st = node_strengths(prob) if strengths is None else strengths
    m_ = _materials(prob, st)
    c, L = m_[:, 2], m_[:, 5]
    H0, H1, H2 = (np.asarray(a, np.float64) for a in (H0, H1, H2))
    s, _, H_sol, H_liq = activity(prob, H0, H1, H2, horizon, st)
    T2, fs2 = orc.state_T(orc.Problem(prob), H2)
    m = horizon - 2
    q = 0.5 * m * (m + 1)
    lat = L > 0
    X = np.empty((H2.size, N_FEAT))
    X[:, 0] = (T2 - T_REF) / T_SCALE
    X[:, 1] = fs2
    X[:, 2] = lat.astype(np.float64)
    X[:, 3] = st["robin_b"] * dt / st["mc"]
    X[:, 4] = 2.0 * st["iface_w"] * dt / st["mc"]
    X[:, 5] = st["kabs"] * dt / st["mc"]
    X[:, 6] = m * (H2 - H1) / s
    X[:, 7] = q * ((H2 - H1) - (H1 - H0)) / s
    X[:, 8] = 1.0
    X[:, 9] = np.log(s / c) / 8.0
    X[:, 10] = np.where(lat, np.clip((H2 - H_liq) / s, -4.0, 4.0) / 4.0, 0.0)
    X[:, 11] = np.where(lat, np.clip((H2 - H_sol) / s, -4.0, 4.0) / 4.0, 0.0)
    return X


def base_and_target(prob, H0, H1, H2, Ht, horizon=16, quadratic=False, strengths=None):
    """Extrapolation to step `horizon` (linear through H1, H2, or quadratic through H0, H1, H2),
    the target (Ht - base) / s, and the correction scale mu s."""
    H0, H1, H2, Ht = (np.asarray(a, np.float64) for a in (H0, H1, H2, Ht))
    m = horizon - 2
    base = H2 + m * (H2 - H1)
    if quadratic:
        base = base + 0.5 * m * (m + 1) * ((H2 - H1) - (H1 - H0))
    s, mu, _, _ = activity(prob, H0, H1, H2, horizon, strengths)
    return base, (Ht - base) / s, np.where(mu, s, 0.0)


def flatten_params(p, layers):
    """Parameter dict -> one vector in the order W_in, b_in, (W_l, b_l)..., w_out, b_out."""
    parts = [p["W_in"].ravel(), p["b_in"]]
    for l in range(layers):
        parts += [p["W%d" % l].ravel(), p["b%d" % l]]
    parts += [p["w_out"], p["b_out"]]
    return np.concatenate(parts)


def unflatten_params(v, width, layers):
    v = np.asarray(v, np.float64)
    p, o = {}, 0

    def take(name, shape):
        nonlocal o
        n = int(np.prod(shape))
        p[name] = v[o:o + n].reshape(shape)
        o += n
    take("W_in", (N_FEAT, width))
    take("b_in", (width,))
    for l in range(layers):
        take("W%d" % l, (2 * width, width))
        take("b%d" % l, (width,))
    take("w_out", (width,))
    take("b_out", (1,))
    assert o == v.size
    return p


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


def bf16_round(x):
    """Round to the nearest BF16 value (8 significant bits, ties to even), returned as float64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _identity(x):
    return x


def projection_weights(prob, scale, strengths=None):
    """w_i = m_i scale_i / sum_j m_j scale_j (m the lumped mass, scale = mu s); all zero when
    no node is masked."""
    st = node_strengths(prob) if strengths is None else strengths
    c = _materials(prob, st)[:, 2]
    w = st["mc"] / c * np.asarray(scale, np.float64)
    tot = w.sum()
    return w / tot if tot > 0 else np.zeros_like(w)


def forward(p, X, ptr, col, layers, bf16=False, proj_w=None):
    """Forward pass.  With bf16=True the operands the GPU keeps in BF16 (features, weight
    matrices, pre-activations, hidden states, aggregated states) are rounded to BF16 where
    the GPU rounds them; sums stay exact.  With proj_w the output is made energy-neutral:
    y - sum_j w_j y_j, so that sum_i w_i y_i = 0 (w sums to 1)."""
    r = bf16_round if bf16 else _identity
    W = {k: (r(v) if k.startswith("W") else v) for k, v in p.items()}
    cache = {"r": r, "W": W}
    X = r(X)
    z = X @ W["W_in"] + p["b_in"]
    h = r(np.maximum(z, 0.0))
    cache["X"], cache["z_in"] = X, r(z)
    hs = [h]
    for l in range(layers):
        a = r(apply_mean(ptr, col, h))
        u = np.concatenate([h, a], axis=1)
        z = u @ W["W%d" % l] + p["b%d" % l]
        cache["u%d" % l], cache["z%d" % l] = u, r(z)
        h = r(h + np.maximum(z, 0.0))
        hs.append(h)
    y = h @ p["w_out"] + p["b_out"][0]
    if proj_w is not None:
        y = y - np.dot(proj_w, y)
    cache["hs"] = hs
    return y, cache


def h_loss(t, mask=None):
    """Enthalpy loss mean(mu (y - t)^2) over all rows and its derivative in y."""
    mu = np.ones_like(t) if mask is None else np.asarray(mask, np.float64)

    def f(y):
        return float(np.mean(mu * (y - t) ** 2)), 2.0 * mu * (y - t) / y.size
    return f


HUBER_DELTA = 0.1


def huber_loss(t, mask=None, delta=HUBER_DELTA):
    """mean of mu (e^2 (|e| <= delta) or delta (2|e| - delta)), e = y - t, and its derivative."""
    mu = np.ones_like(t) if mask is None else np.asarray(mask, np.float64)

    def f(y):
        e = y - t
        a = np.abs(e)
        L = np.where(a <= delta, e * e, delta * (2.0 * a - delta))
        return float(np.mean(mu * L)), 2.0 * mu * np.clip(e, -delta, delta) / y.size
    return f


def t_loss(prob, base, H_true, scale):
    """Temperature loss mean ((T(base + scale y) - T(H_true)) / DT_SCALE)^2 and its
    derivative in y, through the slope of the branch of T(H) the prediction lies on
    (1/c outside the mushy range, (T_liq - T_sol) / (c (T_liq - T_sol) + L) inside)."""
    P = orc.Problem(prob)
    mats = np.asarray(prob["materials"], np.float64).reshape(-1, 6)
    m = mats[orc.node_material(P)]
    c, Ts, Tl, L = m[:, 2], m[:, 3], m[:, 4], m[:, 5]
    mushy_slope = np.where(L > 0, (Tl - Ts) / (c * (Tl - Ts) + L), 0.0)
    T_true, _ = orc.state_T(P, H_true)
    scale = np.asarray(scale, np.float64)

    def f(y):
        Hp = base + scale * y
        Tp, fs = orc.state_T(P, Hp)
        slope = np.where((L > 0) & (fs > 0) & (fs < 1), mushy_slope, 1.0 / c)
        e = (Tp - T_true) / DT_SCALE
        return float(np.mean(e ** 2)), 2.0 * e / y.size * slope * scale / DT_SCALE
    return f


def loss_and_grad(p, X, t, ptr, col, layers, bf16=False, proj_w=None):
    """Loss and parameter gradient; t is the H-loss target array or a loss callable y -> (loss, dL/dy).
    bf16=True also rounds the backward operands the GPU keeps in BF16 (the pre-activation
    gradients dz); proj_w as in forward."""
    y, c = forward(p, X, ptr, col, layers, bf16, proj_w)
    r, W = c["r"], c["W"]
    loss, dy = (t if callable(t) else h_loss(t))(y)
    if proj_w is not None:
        dy = dy - proj_w * dy.sum()
    g = {"w_out": c["hs"][-1].T @ dy, "b_out": np.array([dy.sum()])}
    dh = np.outer(dy, p["w_out"])
    width = p["b_in"].size
    for l in reversed(range(layers)):
        z = c["z%d" % l]
        dz = r(dh * (z > 0))
        g["W%d" % l] = c["u%d" % l].T @ dz
        g["b%d" % l] = dz.sum(axis=0)
        du = dz @ W["W%d" % l].T
        dh = dh + du[:, :width] + apply_mean_T(ptr, col, du[:, width:])
    dz = r(dh * (c["z_in"] > 0))
    g["W_in"] = c["X"].T @ dz
    g["b_in"] = dz.sum(axis=0)
    return loss, g, y


# BF16 unit roundoff: 8 significant bits, round to nearest
BF16_U = 2.0 ** -8


def bf16_rounding_points(layers):
    """Roundings on the longest chain from an input to a gradient entry: features,
    W_in, z_in and h_0; per layer W_l, the aggregated and the hidden states, z_l and
    the backward dz_l; and the backward dz_in."""
    return 4 + 5 * layers + 1


def gradient_error_bound(p, X, t, ptr, col, layers, proj_w=None):
    """First-order forward error bound of the gradient computed with BF16 operands
    (rounded at the kernels' points) against the exact one.  Every rounded operand
    carries a relative error below u = 2^-8, and through k roundings a product of
    them is off by at most gamma_k = k u / (1 - k u) of itself (Higham, Accuracy and
    Stability of Numerical Algorithms, Sec. 3.1), so each entry of a block is off
    by at most gamma_k times the same sum taken over absolute values: the backward
    pass below with |W|, |activations|, |dy| and the masks of the exact pass.
    Returns (per-block bound arrays, loss bound)."""
    y, c = forward(p, X, ptr, col, layers, False, proj_w)
    k = bf16_rounding_points(layers)
    gam = k * BF16_U / (1.0 - k * BF16_U)
    W = c["W"]
    # |y| as built from absolute values, and |dL/dy| from the loss derivative
    ha = [np.abs(h) for h in c["hs"]]
    ya = ha[-1] @ np.abs(p["w_out"]) + abs(p["b_out"][0])
    if proj_w is not None:
        ya = ya + np.dot(proj_w, ya)
    loss, dy = (t if callable(t) else h_loss(t))(y)
    dya = np.abs(dy)
    if proj_w is not None:
        dya = dya + proj_w * dya.sum()
    # the loss: |d loss| <= sum |dL/dy| |dy| with |dy| <= gamma |y|
    loss_bound = gam * float(np.dot(dya, ya))
    g = {"w_out": ha[-1].T @ dya, "b_out": np.array([dya.sum()])}
    dh = np.outer(dya, np.abs(p["w_out"]))
    width = p["b_in"].size
    for l in reversed(range(layers)):
        dz = dh * (c["z%d" % l] > 0)
        g["W%d" % l] = np.abs(c["u%d" % l]).T @ dz
        g["b%d" % l] = dz.sum(axis=0)
        du = dz @ np.abs(W["W%d" % l]).T
        dh = dh + du[:, :width] + apply_mean_T(ptr, col, du[:, width:])
    dz = dh * (c["z_in"] > 0)
    g["W_in"] = np.abs(c["X"]).T @ dz
    g["b_in"] = dz.sum(axis=0)
    return {key: gam * v for key, v in g.items()}, loss_bound
