"""The FP64 reference surrogate (the reference for the GPU training kernels) checked
against central finite differences of its own loss."""
import numpy as np
import pytest

from castgen import configs
from oracle import surrogate_ref as S


def small_case(seed=0, layers=3, width=8):
    p = configs.hex_cube(n=3, noise_amp=0.0, dirichlet_x0=None)
    N = p["xyz"].shape[0]
    ptr, col = S.graph_mean_operator(p["conn"], N)
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (N, S.N_FEAT))
    t = rng.normal(0, 1, N)
    params = S.init_params(width, layers, seed)
    for k in params:                         # non-zero biases exercise every term
        params[k] = params[k] + rng.normal(0, 0.1, params[k].shape)
    return params, X, t, ptr, col, layers


def test_mean_operator_and_transpose():
    params, X, t, ptr, col, layers = small_case()
    N = ptr.size - 1
    assert np.all(np.diff(ptr) == np.diff(ptr))
    deg = np.diff(ptr)
    assert deg.min() == 7 and deg.max() == 26           # corner and interior nodes of a 3^3 hex grid
    h = np.random.default_rng(1).normal(size=(N, 4))
    g = np.random.default_rng(2).normal(size=(N, 4))
    # <A h, g> = <h, A^T g>
    assert np.sum(S.apply_mean(ptr, col, h) * g) == pytest.approx(np.sum(h * S.apply_mean_T(ptr, col, g)), rel=1e-13)
    ones = np.ones((N, 1))
    assert np.allclose(S.apply_mean(ptr, col, ones), 1.0)


@pytest.mark.parametrize("layers,project", [(1, False), (3, False), (3, True)])
def test_gradients_match_central_differences(layers, project):
    params, X, t, ptr, col, layers = small_case(layers=layers)
    w, f = None, None
    if project:
        # the projection over a masked subset, and the loss over the same subset
        rng = np.random.default_rng(9)
        mask = rng.uniform(size=t.size) < 0.6
        w = np.where(mask, rng.uniform(0.5, 1.5, t.size), 0.0)
        w /= w.sum()
        f = S.h_loss(t, mask)
    loss, g, y = S.loss_and_grad(params, X, t if f is None else f, ptr, col, layers, proj_w=w)
    if project:
        assert abs(np.dot(w, y)) <= 1e-14 * np.abs(y).max()
    rng = np.random.default_rng(3)
    eps = 1e-6

    def L():
        return S.loss_and_grad(params, X, t if f is None else f, ptr, col, layers, proj_w=w)[0]
    for name, val in params.items():
        idx = [tuple(rng.integers(0, s) for s in val.shape) for _ in range(4)]
        for ix in idx:
            old = val[ix]
            val[ix] = old + eps
            lp = L()
            val[ix] = old - eps
            lm = L()
            val[ix] = old
            fd = (lp - lm) / (2 * eps)
            assert g[name][ix] == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, ix)


def test_masked_loss_ignores_unmasked_rows():
    params, X, t, ptr, col, layers = small_case(layers=2)
    mask = np.arange(t.size) % 3 == 0
    f = S.h_loss(t, mask)
    loss, _, y = S.loss_and_grad(params, X, f, ptr, col, layers)
    assert loss == pytest.approx(np.sum((y - t)[mask] ** 2) / t.size, rel=1e-13)
    t2 = np.where(mask, t, t + 100.0)                # unmasked targets do not matter
    assert S.loss_and_grad(params, X, S.h_loss(t2, mask), ptr, col, layers)[0] == pytest.approx(loss, rel=1e-13)


def test_parameter_vector_layout():
    p = S.init_params(64, 3, 0)
    v = S.flatten_params(p, 3)
    assert v.size == 12 * 64 + 64 + 3 * (128 * 64 + 64) + 64 + 1
    q = S.unflatten_params(v, 64, 3)
    for k in p:
        assert np.array_equal(p[k], q[k])


def test_conduction_strength_of_an_interior_hex_node():
    # trilinear cube of side h: K_ii = kh/3, face diagonals and body diagonal -kh/12,
    # edge neighbours 0; an interior node of a uniform grid gathers 8 elements, so
    # sum_j |K_ij| = kh (8/3 + 12/6 + 8/12) = 16 kh / 3 and m_i = rho h^3
    n, L = 4, 0.1
    p = configs.hex_cube(n=n, length=L, noise_amp=0.0, dirichlet_x0=None)
    st = S.node_strengths(p)
    k, rho, c = configs.ALLOY[:3]
    h = L / n
    xyz = p["xyz"]
    interior = np.all((xyz > 1e-9) & (xyz < L - 1e-9), axis=1)
    dt = 0.1
    H = np.full(xyz.shape[0], 900.0 * 700.0)
    X = S.features(p, H, H, H, dt, strengths=st)
    assert np.allclose(X[interior, 5], 16.0 / 3.0 * k * dt / (rho * c * h * h), rtol=1e-12)
    assert np.allclose(st["kabs"][interior], 16.0 / 3.0 * k * h, rtol=1e-12)
    # a corner node sits in one element: sum_j |K_ij| = kh (1/3 + 4/12)
    corner = np.all(np.isclose(xyz, 0.0), axis=1)
    assert st["kabs"][corner][0] == pytest.approx(2.0 / 3.0 * k * h, rel=1e-12)
    assert np.all(X[:, 3] == 0) and np.all(X[:, 4] == 0)


def test_robin_strength_on_the_chill_face():
    # interior node of the x = 0 face: four quads of area h^2 each give h^2 h_c / 4,
    # and the lumped weight of a face node is rho h^3 / 2
    n, L, hc = 4, 0.1, 1234.0
    p = configs.hex_cube(n=n, length=L, noise_amp=0.0, dirichlet_x0=None, robin_x0=(hc, 25.0))
    st = S.node_strengths(p)
    rho, c = configs.ALLOY[1:3]
    h = L / n
    xyz = p["xyz"]
    face = np.isclose(xyz[:, 0], 0.0) & np.all((xyz[:, 1:] > 1e-9) & (xyz[:, 1:] < L - 1e-9), axis=1)
    dt = 0.2
    H = np.full(xyz.shape[0], 900.0 * 700.0)
    X = S.features(p, H, H, H, dt, strengths=st)
    assert np.allclose(X[face, 3], 2.0 * hc * dt / (rho * c * h), rtol=1e-12)
    assert np.all(X[~np.isclose(xyz[:, 0], 0.0), 3] == 0)


def test_interface_strength_sums_to_h_times_area():
    # unjittered cube region [0.2, 0.8]^3 of the 0.1 m domain: area 6 (0.06)^2 per side
    hi = 800.0
    p = configs.tet_casting(n=5, jitter=0, region="cube", h_interface=hi, permute=False)
    st = S.node_strengths(p)
    nm = st["node_mat"]
    area = 6 * 0.06 ** 2
    assert st["iface_w"][nm == 0].sum() == pytest.approx(hi * area, rel=1e-12)
    assert st["iface_w"][nm == 1].sum() == pytest.approx(hi * area, rel=1e-12)


def test_temperature_and_rate_features():
    p = configs.hex_cube(n=2, noise_amp=0.0, dirichlet_x0=None)
    mat = configs.ALLOY
    c, Ts, Tl, L = mat[2], mat[3], mat[4], mat[5]
    Hs, Hl = c * Ts, c * Tl + L
    N = p["xyz"].shape[0]
    H2 = np.full(N, Hs + 0.25 * (Hl - Hs))                        # a quarter of the way through the mushy zone
    H1 = H2 + 160.0
    H0 = H1 + 170.0                                                # the cooling slows down by 10 J/kg per step
    X = S.features(p, H0, H1, H2, 0.1, horizon=16)
    assert np.allclose(X[:, 0], (Ts + 0.25 * (Tl - Ts) - S.T_REF) / S.T_SCALE, rtol=1e-12)
    assert np.allclose(X[:, 1], 0.75, rtol=1e-12)
    assert np.all(X[:, 2] == 1) and np.all(X[:, 8] == 1)
    # activity over the window: |14 r| + |105 a| + c EPS_T with r = -160, a = 10
    s = 14 * 160.0 + 105 * 10.0 + c * S.EPS_T
    assert np.allclose(X[:, 6], 14 * (-160.0) / s, rtol=1e-12)
    assert np.allclose(X[:, 7], 105 * 10.0 / s, rtol=1e-12)
    assert np.allclose(X[:, 9], np.log(s / c) / 8, rtol=1e-12)
    assert np.allclose(X[:, 10], -1.0) and np.allclose(X[:, 11], 1.0)    # both kinks beyond 4 activities
    # the quadratic through (0, H0), (1, H1), (2, H2) at 16: Lagrange weights 105, -224, 120
    base, t, scale = S.base_and_target(p, H0, H1, H2, H2, horizon=16, quadratic=True)
    assert np.allclose(base, 105 * H0 - 224 * H1 + 120 * H2, rtol=1e-13)
    lin, t, scale = S.base_and_target(p, H0, H1, H2, H2, horizon=16)
    assert np.allclose(lin, 15 * H2 - 14 * H1, rtol=1e-13)
    assert np.allclose(t * s, H2 - lin)
    assert np.all(scale == 0)                      # no kink within reach: the jump is the extrapolation
    # 1000 J/kg above the liquidus, the same history: the liquidus is within reach
    d = Hl + 1000.0 - H2
    X = S.features(p, H0 + d, H1 + d, H2 + d, 0.1, horizon=16)
    assert np.allclose(X[:, 10], 1000.0 / s / 4, rtol=1e-12) and np.allclose(X[:, 11], 1.0)
    _, _, scale = S.base_and_target(p, H0 + d, H1 + d, H2 + d, H2 + d, horizon=16)
    assert np.allclose(scale, s, rtol=1e-13)
    # an exactly quadratic history is reproduced by the quadratic base, a linear one by both
    k = np.arange(17.0)
    hist = 6e5 - 150.0 * k + 2.5 * k ** 2
    h = [np.full(N, hist[j]) for j in (0, 1, 2, 16)]
    b2, _, _ = S.base_and_target(p, *h, quadratic=True)
    assert np.allclose(b2, hist[16], rtol=1e-14)
    line = 6e5 - 150.0 * k
    h = [np.full(N, line[j]) for j in (0, 1, 2, 16)]
    assert np.allclose(S.base_and_target(p, *h)[0], line[16], rtol=1e-14)


def test_mask_of_a_cube_in_a_mould():
    # alloy cube in sand: only free alloy nodes near a kink carry a correction
    p = configs.tet_casting(n=5, jitter=0, region="cube", h_interface=800.0, permute=False)
    st = S.node_strengths(p)
    mats = np.asarray(p["materials"], np.float64).reshape(-1, 6)[st["node_mat"]]
    c, Ts, Tl, L = mats[:, 2], mats[:, 3], mats[:, 4], mats[:, 5]
    N = c.size
    H2 = c * Tl + L + 50.0                                      # 50 J/kg above the liquidus
    H1 = H2 + 30.0
    H0 = H1 + 30.0                                              # activity 14 * 30 + c EPS_T
    s, mu, H_sol, H_liq = S.activity(p, H0, H1, H2, 16, st)
    assert np.allclose(s, 14 * 30.0 + c * S.EPS_T, rtol=1e-13)
    assert np.array_equal(mu, L > 0)                           # the mould has no kink
    assert np.allclose(H_liq[L > 0], H2[L > 0] - 50.0)
    # far above the liquidus nothing is masked
    s2, mu2, _, _ = S.activity(p, H0 + 1e5, H1 + 1e5, H2 + 1e5, 16, st)
    assert not mu2.any()


def test_temperature_loss_gradient_matches_central_differences(orc):
    # states away from the kinks of T(H): the loss is smooth there
    p = configs.hex_cube(n=3, noise_amp=0.0, dirichlet_x0=None)
    N = p["xyz"].shape[0]
    ptr, col = S.graph_mean_operator(p["conn"], N)
    rng = np.random.default_rng(5)
    c, Ts, Tl, L = configs.ALLOY[2:]
    Hs, Hl = c * Ts, c * Tl + L
    kind = rng.integers(0, 3, N)                        # solid, mushy, liquid nodes
    base = np.where(kind == 0, c * rng.uniform(300, 590, N),
                    np.where(kind == 1, rng.uniform(Hs + 2e4, Hl - 2e4, N), rng.uniform(Hl + 2e4, Hl + 5e4, N)))
    H_true = base + rng.normal(0, 2000, N)
    X = rng.normal(0, 1, (N, S.N_FEAT))
    layers = 2
    params = S.init_params(8, layers, 1)
    params["w_out"] = rng.normal(0, 0.05, 8)
    scale = rng.uniform(5e3, 1.5e4, N)
    f = S.t_loss(p, base, H_true, scale)
    loss, g, y = S.loss_and_grad(params, X, f, ptr, col, layers)
    assert np.max(np.abs(y * scale)) < 1.5e4            # predictions stay on their branch
    eps = 1e-6
    for name in ("W_in", "W1", "w_out", "b_out"):
        val = params[name]
        for ix in [tuple(rng.integers(0, s) for s in val.shape) for _ in range(3)]:
            old = val[ix]
            val[ix] = old + eps
            lp = S.loss_and_grad(params, X, f, ptr, col, layers)[0]
            val[ix] = old - eps
            lm = S.loss_and_grad(params, X, f, ptr, col, layers)[0]
            val[ix] = old
            assert g[name][ix] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-10), (name, ix)
    # the loss is the mean squared temperature error in units of DT_SCALE
    T_pred, _ = orc.state_T(p, base + scale * y)
    T_true, _ = orc.state_T(p, H_true)
    assert loss == pytest.approx(np.mean(((T_pred - T_true) / S.DT_SCALE) ** 2), rel=1e-12)


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -7), 1.0 + 2.0 ** -8 + 2.0 ** -20, 3.0e38, 0.0])
    got = S.bf16_round(x)
    want = [1.0, 1.0 + 2.0 ** -6, -(1.0 + 2.0 ** -7), 1.0 + 2.0 ** -7, np.float32(3.0e38), 0.0]
    assert got[:4].tolist() == want[:4] and got[5] == 0.0
    assert abs(got[4] - 3.0e38) <= 3.0e38 * 2.0 ** -8


def test_bf16_reference_stays_close_to_exact():
    params, X, t, ptr, col, layers = small_case(width=64)
    _, g, _ = S.loss_and_grad(params, X, t, ptr, col, layers)
    _, gb, _ = S.loss_and_grad(params, X, t, ptr, col, layers, bf16=True)
    for k in g:
        assert np.linalg.norm(gb[k] - g[k]) <= 0.05 * np.linalg.norm(g[k]) + 1e-12, k


def test_projection_weights_of_the_chill_cube():
    # uniform hex grid, one material: the lumped mass is rho h^3 times 1, 1/2, 1/4 or 1/8
    p = configs.hex_cube(n=4, noise_amp=0.0, dirichlet_x0=25.0)
    N = p["xyz"].shape[0]
    free = np.setdiff1d(np.arange(N), p["dirichlet_nodes"])
    scale = np.zeros(N)
    scale[free] = 7.0
    w = S.projection_weights(p, scale)
    assert w.sum() == pytest.approx(1.0, rel=1e-14)
    assert np.all(w[p["dirichlet_nodes"]] == 0)
    ratio = w[free] / w[free].max()
    assert set(np.round(ratio, 12)) <= {1.0, 0.5, 0.25, 0.125}
    # a masked subset with different scales: w proportional to m scale on it, 0 elsewhere
    sc = np.zeros(N)
    sc[free[::2]] = np.linspace(1.0, 3.0, free[::2].size)
    w = S.projection_weights(p, sc)
    assert w.sum() == pytest.approx(1.0, rel=1e-14) and np.all(w[sc == 0] == 0)
    m = S.node_strengths(p)["mc"]
    assert np.allclose(w[sc > 0] / (m[sc > 0] * sc[sc > 0]), w[free[0]] / (m[free[0]] * sc[free[0]]), rtol=1e-12)
    assert np.all(S.projection_weights(p, np.zeros(N)) == 0)


def test_huber_loss_gradient_matches_central_differences():
    params, X, t, ptr, col, layers = small_case(layers=2)
    t = 3.0 * t                                  # both branches of the Huber loss occur
    f = S.huber_loss(t)
    loss, g, y = S.loss_and_grad(params, X, f, ptr, col, layers)
    e = np.abs(y - t)
    assert np.any(e < S.HUBER_DELTA) and np.any(e > S.HUBER_DELTA)
    rng = np.random.default_rng(4)
    eps = 1e-6
    for name in ("W_in", "W0", "w_out", "b_out"):
        val = params[name]
        for ix in [tuple(rng.integers(0, s) for s in val.shape) for _ in range(3)]:
            old = val[ix]
            val[ix] = old + eps
            lp = S.loss_and_grad(params, X, f, ptr, col, layers)[0]
            val[ix] = old - eps
            lm = S.loss_and_grad(params, X, f, ptr, col, layers)[0]
            val[ix] = old
            assert g[name][ix] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-10), (name, ix)
    # within delta it is the squared error
    small = S.huber_loss(y + 0.01)
    assert small(y)[0] == pytest.approx(1e-4, rel=1e-9)


def test_gradient_error_bound_covers_the_bf16_rounding():
    """The first-order BF16 bound (gamma_k times the absolute-value pass) covers the
    deviation of the reference rounded at the kernels' BF16 points from the exact
    one, per block in the Frobenius norm, with and without the projection, and the
    loss bound covers the loss's deviation.  (A worst-case first-order bound is
    loose where a gradient sum cancels: on these random targets it reaches the
    size of the gradient; on solver states the GPU test measures 0.1-65 % of it.)"""
    k = S.bf16_rounding_points(3)
    assert k == 4 + 5 * 3 + 1
    assert S.BF16_U == 2.0 ** -8
    for layers, proj in ((2, False), (3, False), (3, True)):
        params, X, t, ptr, col, L = small_case(width=64, layers=layers)
        pw = None
        if proj:
            pw = np.linspace(1.0, 2.0, X.shape[0])
            pw /= pw.sum()
        _, g, _ = S.loss_and_grad(params, X, t, ptr, col, L, proj_w=pw)
        _, gb, _ = S.loss_and_grad(params, X, t, ptr, col, L, bf16=True, proj_w=pw)
        bound, lb = S.gradient_error_bound(params, X, t, ptr, col, L, proj_w=pw)
        assert set(bound) == set(g)
        ratios = []
        for key in g:
            if proj and key == "b_out":
                continue
            err, bnd = np.linalg.norm(gb[key] - g[key]), np.linalg.norm(bound[key])
            assert err <= bnd, (layers, proj, key)
            ratios.append(err / bnd)
        assert max(ratios) > 1e-3          # the deviation is of the order the bound describes
        lz, _, _ = S.loss_and_grad(params, X, t, ptr, col, L, proj_w=pw)
        lbf, _, _ = S.loss_and_grad(params, X, t, ptr, col, L, bf16=True, proj_w=pw)
        assert abs(lbf - lz) <= lb
