"""Pins of the FP64 oracle against closed forms, invariants and textbook special cases.

The paper prints no solution values, so every check here comes from the
mathematics of the method: element matrices of simple shapes, consistency of
linear elements, conservation of energy, reductions to 1-D schemes, known
analytic solutions of conduction and of the one-phase Stefan problem.
"""
import math

import numpy as np
import pytest
from scipy import optimize, special

from castgen import configs, meshes, rng

ALLOY = configs.ALLOY
K_AL, RHO_AL, C_AL = ALLOY[0], ALLOY[1], ALLOY[2]
ALPHA = K_AL / (RHO_AL * C_AL)


def no_latent(mat):
    return (mat[0], mat[1], mat[2], 0.0, 0.0, 0.0)


# ------------------------------------------------------------------ P-1, P-2
def test_p1_unit_right_tet(orc):
    Ke, V = orc.tet_ke([0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1], 2.0)
    expect = (2.0 / 6.0) * np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]])
    assert V == pytest.approx(1.0 / 6.0, rel=1e-15)
    assert np.max(np.abs(Ke - expect)) < 1e-15


def test_p1_kuhn_tet_is_path_laplacian(orc):
    h, k = 0.25, 3.0
    x = h * np.array([0, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 1], float)
    Ke, V = orc.tet_ke(x, k)
    lap = np.array([[1, -1, 0, 0], [-1, 2, -1, 0], [0, -1, 2, -1], [0, 0, -1, 1]], float)
    assert np.max(np.abs(Ke - k * h / 6.0 * lap)) < 1e-15
    assert V == pytest.approx(h ** 3 / 6.0, rel=1e-14)


def test_p1_cube_hex(orc):
    h, k, rho = 0.5, 2.0, 3.0
    x = h * meshes.HEX_CORNERS.astype(float)
    Ke, V = orc.hex_ke(x, k)
    for a in range(8):
        for b in range(8):
            nd = int(np.sum(meshes.HEX_CORNERS[a] != meshes.HEX_CORNERS[b]))
            expect = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}[nd] * k * h
            assert abs(Ke[a, b] - expect) < 1e-14, (a, b)
    assert V == pytest.approx(h ** 3, rel=1e-14)
    m = orc.elem_mass(8, x, rho)
    assert np.max(np.abs(m - rho * h ** 3 / 8)) < 1e-15


def test_p1_tet_lumping(orc):
    x = np.array([0, 0, 0, 2, 0, 0, 0, 3, 0, 0, 0, 4], float)
    m = orc.elem_mass(4, x, 5.0)
    assert np.allclose(m, 5.0 * (2 * 3 * 4 / 6.0) / 4.0, rtol=1e-15)


@pytest.mark.parametrize("kind", ["tet", "hex"])
def test_p2_element_invariants(orc, kind):
    """Rows sum to zero, K is symmetric and positive semi-definite, for jittered elements."""
    if kind == "tet":
        p = configs.tet_casting(n=6, region="cube", cube=(0.3, 0.7), permute=False)
        cells = p["conn"][:600]
        ke = lambda x: orc.tet_ke(x, 1.7)[0]
    else:
        p = configs.hex_cube(n=4)
        jit = rng.uniform(5, 0, p["xyz"].size, -0.15, 0.15).reshape(-1, 3) * (0.1 / 4)
        p["xyz"] = p["xyz"] + jit
        cells = p["conn"]
        ke = lambda x: orc.hex_ke(x, 1.7)[0]
    for c in cells:
        K = ke(p["xyz"][c])
        scale = np.max(np.abs(K))
        assert np.max(np.abs(K.sum(axis=1))) <= 1e-14 * scale
        assert np.max(np.abs(K - K.T)) <= 1e-15 * scale
        assert np.min(np.linalg.eigvalsh(0.5 * (K + K.T))) >= -1e-13 * scale


def test_inverted_element_rejected(orc):
    with pytest.raises(ValueError):
        orc.tet_ke([0, 0, 0, 0, 1, 0, 1, 0, 0, 0, 0, 1], 1.0)


# ------------------------------------------------------------------ P-3, P-7
def test_p3_lumped_mass_totals(orc):
    p = configs.tet_casting(n=8, region="cube", cube=(0.25, 0.75), permute=True)
    m = orc.lumped_mass(p)
    nm = orc.node_material(p)
    # the jitter keeps the outer boundary planar, so the domain volume is exact
    # (the jittered cast/mould surface moves volume between the two materials)
    rho = p["materials"][:, 1]
    assert np.sum(m / rho[nm]) == pytest.approx(0.1 ** 3, rel=1e-12)
    assert np.all(m > 0) and np.all(nm >= 0)
    # unjittered: casting cubes 2..5 of 8 make a 0.05 m cube
    q = configs.tet_casting(n=8, region="cube", cube=(0.25, 0.75), jitter=0.0, permute=True)
    mq, nq = orc.lumped_mass(q), orc.node_material(q)
    assert np.sum(mq[nq == 0]) == pytest.approx(rho[0] * 0.05 ** 3, rel=1e-12)
    assert np.sum(mq[nq == 1]) == pytest.approx(rho[1] * (0.1 ** 3 - 0.05 ** 3), rel=1e-12)


def test_p7_kuhn_interior_rows_are_7_point(orc):
    n, L = 4, 0.1
    h = L / n
    p = configs.tet_casting(n=n, region="none", jitter=0.0, permute=False, alloy=ALLOY)
    i, j, k = meshes.grid_ids(n)
    m = orc.lumped_mass(p)
    centre = 2 + 5 * (2 + 5 * 2)
    e = np.zeros(p["xyz"].shape[0])
    e[centre] = 1.0
    col = -orc.residual(p, e)               # column of the assembled K (K is symmetric)
    d = np.stack([i - 2, j - 2, k - 2], axis=1)
    dist = np.sum(np.abs(d), axis=1)
    kh = K_AL * h
    assert col[centre] == pytest.approx(6 * kh, rel=1e-13)
    axis = (dist == 1)
    assert np.allclose(col[axis], -kh, rtol=1e-13)
    assert np.max(np.abs(col[(dist > 1)])) < 1e-13 * kh
    assert m[centre] == pytest.approx(RHO_AL * h ** 3, rel=1e-13)


def test_p7_hex_interior_rows_are_27_point(orc):
    n, L = 4, 0.1
    h = L / n
    p = configs.hex_cube(n=n, noise_amp=0.0, dirichlet_x0=None)
    m1 = n + 1
    ids = np.arange(m1 ** 3)
    d = np.stack([ids % m1 - 2, (ids // m1) % m1 - 2, ids // (m1 * m1) - 2], axis=1)
    centre = 2 + m1 * (2 + m1 * 2)
    e = np.zeros(ids.size)
    e[centre] = 1.0
    col = -orc.residual(p, e)
    kh = K_AL * h
    cheb = np.max(np.abs(d), axis=1)
    nnz = np.sum(d != 0, axis=1)
    expect = np.where(cheb > 1, 0.0,
                      np.select([nnz == 0, nnz == 1, nnz == 2, nnz == 3],
                                [8 * kh / 3, 0.0, -kh / 6, -kh / 12]))
    assert np.max(np.abs(col - expect)) < 1e-12 * kh


# ------------------------------------------------------------------ P-4
@pytest.mark.parametrize("kind", ["tet", "hex"])
def test_p4_linear_patch(orc, kind):
    """A linear field with its boundary values held stays exact, also inside the mushy range."""
    if kind == "tet":
        p = configs.tet_casting(n=6, region="none", permute=True)
    else:
        p = configs.hex_cube(n=5, noise_amp=0.0, dirichlet_x0=None)
        i, j, k = meshes.grid_ids(5)
        inner = (i > 0) & (i < 5) & (j > 0) & (j < 5) & (k > 0) & (k < 5)
        jit = rng.uniform(9, 0, p["xyz"].size, -0.2, 0.2).reshape(-1, 3) * (0.1 / 5)
        p["xyz"] = p["xyz"] + np.where(inner[:, None], jit, 0.0)
    x = p["xyz"]
    lo, hi = x.min(axis=0), x.max(axis=0)
    bnd = np.nonzero(np.any((np.abs(x - lo) < 1e-12) | (np.abs(x - hi) < 1e-12), axis=1))[0]
    field = 630.0 + 150.0 * x[:, 0] - 80.0 * x[:, 1] + 40.0 * x[:, 2]   # 610..650 C: mushy
    p["dirichlet_nodes"] = bnd.astype(np.int32)
    p["dirichlet_T"] = field[bnd]
    p["T0"] = field.copy()
    dt = 0.9 * orc.stable_dt(p)
    H, T, fs = orc.run(p, dt, 1000)
    assert np.max(np.abs(T - field)) <= 1e-10
    assert np.all((fs > 0) & (fs < 1))


# ------------------------------------------------------------------ P-5, P-11(i)
def test_p5_energy_conserved_with_interface_and_phase_change(orc):
    p = configs.tet_casting(n=10, region="cube", permute=True)
    dt = 0.9 * orc.stable_dt(p)
    H, T, fs, D = orc.run(p, dt, 2000, diag=True)
    assert np.max(D[:, orc.D_RESID]) <= 1e-12
    assert np.all(D[:, orc.D_Q] == 0.0)
    # the casting lost heat to the mould and part of it is mushy or solid
    assert D[-1, orc.D_LATENT] < D[0, orc.D_LATENT]
    assert D[-1, orc.D_NONFINITE] == 0


def test_p11_zero_contact_decouples_sides(orc):
    p = configs.tet_casting(n=8, region="cube", permute=False, h_interface=0.0)
    m = orc.lumped_mass(p)
    cast = orc.node_material(p) == 0
    dt = 0.9 * orc.stable_dt(p)
    H0 = orc.initial_H(p)
    H, T, fs = orc.run(p, dt, 500)
    for side in (cast, ~cast):
        e0, e1 = np.sum(m[side] * H0[side]), np.sum(m[side] * H[side])
        assert abs(e1 - e0) <= 1e-12 * abs(e0)
    # nothing crossed: every mould node is still at its initial 25 C
    assert np.max(np.abs(T[~cast] - 25.0)) < 1e-9


def test_p5_energy_identity_with_dirichlet_reaction(orc):
    p = configs.config1()
    H, T, fs, D = orc.run(p, 0.284765625, 200, diag=True)
    assert np.max(D[:, orc.D_RESID]) <= 1e-12
    assert D[-1, orc.D_QCUM] < 0          # heat leaves through the chilled face


# ------------------------------------------------------------------ P-6
def ftcs_1d(T0, TD, n, h, dt, steps, mat):
    """Independent 1-D explicit enthalpy scheme on n+1 nodes, node 0 held at TD, far end insulated."""
    k, rho, c, Ts, Tl, L = mat

    def H_of(T):
        g = np.clip((T - Ts) / (Tl - Ts), 0.0, 1.0)
        return c * T + L * g

    def T_of(H):
        Hs, Hl = c * Ts, c * Tl + L
        return np.where(H <= Hs, H / c, np.where(H >= Hl, (H - L) / c,
                                                 Ts + (H - Hs) * (Tl - Ts) / (c * (Tl - Ts) + L)))

    T = np.full(n + 1, float(T0))
    T[0] = TD
    H = H_of(T)
    a = dt * k / (rho * h * h)
    for _ in range(steps):
        T = T_of(H)
        dH = np.zeros_like(H)
        dH[1:-1] = a * (T[:-2] - 2 * T[1:-1] + T[2:])
        dH[-1] = 2 * a * (T[-2] - T[-1])
        H = H + dH
    return T_of(H)


def test_p6_config1_without_noise_is_1d_ftcs(orc):
    p = configs.config1(noise_amp=0.0)
    H, T, fs = orc.run(p, 0.284765625, 200)
    ref = ftcs_1d(700.0, 25.0, 16, 0.1 / 16, 0.284765625, 200, ALLOY)
    i = np.arange(17 ** 3) % 17
    assert np.max(np.abs(T - ref[i])) <= 1e-10
    assert np.min(fs) < 1.0 and np.max(fs) > 0.0      # the front is inside the cube


# ------------------------------------------------------------------ P-8 and the dt bound
def test_p8_checkerboard_is_top_eigenvector(orc):
    n, L = 16, 0.1
    h = L / n
    p = configs.hex_cube(n=n, noise_amp=0.0, dirichlet_x0=None, material=no_latent(ALLOY))
    i = np.arange((n + 1) ** 3) % (n + 1)
    v = np.where(i % 2 == 0, 1.0, -1.0)
    m = orc.lumped_mass(p)
    lam = -orc.residual(p, v) / (m * C_AL) / v
    assert np.allclose(lam, 4 * ALPHA / h ** 2, rtol=1e-12)
    assert 4 * ALPHA / h ** 2 == pytest.approx(6.320988, rel=1e-6)
    # Gershgorin is 4/3 above the exact value for Q1 hexes
    assert orc.stable_dt(p) == pytest.approx(0.75 * h * h / (2 * ALPHA), rel=1e-12)


@pytest.mark.parametrize("factor,grows", [(1.05, True), (0.9, False)])
def test_p8_stability_threshold(orc, factor, grows):
    n, L = 8, 0.1
    h = L / n
    p = configs.hex_cube(n=n, noise_amp=0.0, dirichlet_x0=None, material=no_latent(ALLOY))
    i = np.arange((n + 1) ** 3) % (n + 1)
    p["T0"] = 400.0 + 10.0 * np.where(i % 2 == 0, 1.0, -1.0)
    dt = factor * h * h / (2 * ALPHA)
    H, T, fs = orc.run(p, dt, 200)
    amp = np.max(np.abs(T - 400.0))
    assert (amp > 10.0) == grows


def test_gershgorin_bound_brute_force(orc):
    """The bound equals 2 / max_i sum_j |A_ij| / (m_i c_i) of the densely assembled operator
    (conduction + Robin + interface), built column by column from residuals."""
    p = configs.tet_casting(n=4, region="cube", cube=(0.3, 0.7), permute=True)
    quads = np.array([[0, 1, 2]], np.int32)
    # one convective triangle on the outer boundary: a face of some tet on the x = 0 plane
    x = p["xyz"]
    on = np.nonzero(np.abs(x[:, 0]) < 1e-15)[0]
    for t in p["conn"]:
        f = [a for a in t if a in set(on)]
        if len(f) == 3:
            quads = np.array([f], np.int32)
            break
    p["flux_faces"], p["flux_q"] = quads, np.array([100.0])
    p["flux_h"], p["flux_Tinf"] = np.array([800.0]), np.array([25.0])
    N = x.shape[0]
    r0 = orc.residual(p, np.zeros(N))
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = -(orc.residual(p, e) - r0)
    m = orc.lumped_mass(p)
    c = p["materials"][orc.node_material(p), 2]
    lam = np.max(np.sum(np.abs(A), axis=1) / (m * c))
    assert orc.stable_dt(p) == pytest.approx(2.0 / lam, rel=1e-12)


def test_gershgorin_interior_rows_of_regular_kuhn_grid(orc):
    """Interior rows of the unjittered Kuhn grid give 12 alpha / h^2 (6kh + 6 kh over rho h^3 c)."""
    n = 4
    h = 0.1 / n
    p = configs.tet_casting(n=n, region="none", jitter=0.0, permute=False)
    centre = 2 + 5 * (2 + 5 * 2)
    e = np.zeros(p["xyz"].shape[0])
    e[centre] = 1.0
    col = orc.residual(p, e)
    m = orc.lumped_mass(p)
    assert np.sum(np.abs(col)) / (m[centre] * C_AL) == pytest.approx(12 * ALPHA / h ** 2, rel=1e-12)
    assert orc.stable_dt(p) <= h * h / (6 * ALPHA)


# ------------------------------------------------------------------ P-9
def erf_error(orc, nx, t_end=40.0):
    lx = 0.4
    h = lx / nx
    p = configs.hex_bar(nx=nx, ny=1, nz=1, lx=lx, ly=h, lz=h, material=no_latent(ALLOY))
    steps = int(math.ceil(t_end / (0.45 * h * h / ALPHA)))
    dt = t_end / steps
    H, T, fs = orc.run(p, dt, steps)
    x = p["xyz"][:, 0]
    exact = 25.0 + 675.0 * special.erf(x / (2 * math.sqrt(ALPHA * t_end)))
    return np.max(np.abs(T - exact))


def test_p9_erf_solution_converges_second_order(orc):
    e1, e2, e3 = erf_error(orc, 64), erf_error(orc, 128), erf_error(orc, 256)
    assert e3 < 0.1
    assert 3.2 < e1 / e2 < 5.0 and 3.2 < e2 / e3 < 5.0


# ------------------------------------------------------------------ P-10
def neumann_lambda(St):
    return optimize.brentq(lambda l: l * math.exp(l * l) * math.erf(l) - St / math.sqrt(math.pi), 1e-6, 5.0)


def front_and_profile(orc, nx, times):
    lx = 0.1
    h = lx / nx
    mat = (K_AL, RHO_AL, C_AL, 660.0, 660.0, 3.9e5)
    p = configs.hex_bar(nx=nx, ny=1, nz=1, lx=lx, ly=h, lz=h, T_init=660.0, material=mat)
    dt = 0.45 * h * h / ALPHA
    x = p["xyz"][:, 0]
    w = np.where((x == 0) | (x == lx), h / 2, h) / 4.0     # 4 nodes per x-plane
    out = []
    # liquid at the melting point: H = c T_m + L (T = T_m is ambiguous on the plateau)
    H = orc.initial_H(p)
    H[x > 0] = C_AL * 660.0 + 3.9e5
    t = 0.0
    for tt in times:
        steps = int(round((tt - t) / dt))
        H, T, fs = orc.run(p, dt, steps, H=H)
        t += steps * dt
        out.append((t, np.sum(w * fs), x, T, fs))
    return out


def test_p10_neumann_front(orc):
    St = C_AL * (660.0 - 25.0) / 3.9e5
    lam = neumann_lambda(St)
    assert lam == pytest.approx(0.717068, abs=2e-6)
    errs = {}
    for nx in (16, 32):
        worst = 0.0
        for t, s, x, T, fs in front_and_profile(orc, nx, [20.0, 40.0, 60.0, 75.0]):
            exact = 2 * lam * math.sqrt(ALPHA * t)
            worst = max(worst, abs(s - exact) / exact)
            behind = (fs == 1.0) & (x < 0.8 * s)
            prof = 25.0 + 635.0 * special.erf(x[behind] / (2 * math.sqrt(ALPHA * t))) / math.erf(lam)
            assert np.max(np.abs(T[behind] - prof)) < 6.0
        errs[nx] = worst
    assert errs[16] <= 0.02
    assert errs[32] < errs[16]


# ------------------------------------------------------------------ P-11
def lumped_two_body(orc, h_if, n=8):
    big_k = 1.0e4
    mat = (big_k, RHO_AL, C_AL, 0.0, 0.0, 0.0)
    p = configs.tet_casting(n=n, region="cube", cube=(0.3, 0.7), jitter=0.0, permute=False,
                            alloy=mat, mold=mat, T_pour=700.0, T_mold=25.0, h_interface=h_if)
    return p


def test_p11_lumped_contact_limit(orc):
    """Bi << 1: mean temperatures relax as exp(-h A (1/C_c + 1/C_m) t)."""
    h_if = 200.0
    p = lumped_two_body(orc, h_if)
    side = 4 / 8 * 0.1
    A = 6 * side ** 2
    Vc = side ** 3
    Cc = RHO_AL * C_AL * Vc
    Cm = RHO_AL * C_AL * (0.1 ** 3 - Vc)
    m = orc.lumped_mass(p)
    cast = orc.node_material(p) == 0
    dt = 0.9 * orc.stable_dt(p)
    steps = 400
    H, T, fs = orc.run(p, dt, steps)
    Tc = np.sum(m[cast] * T[cast]) / np.sum(m[cast])
    Tm = np.sum(m[~cast] * T[~cast]) / np.sum(m[~cast])
    expect = 675.0 * math.exp(-h_if * A * (1 / Cc + 1 / Cm) * steps * dt)
    Bi = h_if * side / 1.0e4
    assert abs((Tc - Tm) - expect) <= 5 * Bi * 675.0


def test_p11_large_contact_approaches_conforming(orc):
    """Same material on both sides: as h_i grows the split mesh tends to the conforming one."""
    mat = no_latent(ALLOY)
    n = 6
    common = dict(n=n, cube=(0.3, 0.7), jitter=0.2, jitter_seed=4, permute=False,
                  alloy=mat, mold=mat, T_pour=700.0, T_mold=25.0)
    conf = configs.tet_casting(region="none", **common)
    Ng = (n + 1) ** 3
    cube = np.repeat(meshes.cube_region_cells(n, 0.3, 0.7), 6)
    conn_g = meshes.kuhn_conn(n)
    tc = np.zeros(Ng, bool)
    tm = np.zeros(Ng, bool)
    tc[conn_g[cube].ravel()] = True
    tm[conn_g[~cube].ravel()] = True
    inner = tc & ~tm                                  # casting nodes off the interface
    conf["T0"] = np.where(inner, 700.0, 25.0)
    errs = []
    # beyond h_i ~ 1e4 the face-average coupling levels off near 0.1 K: an infinite
    # h_i forces each node to its sister face's mean, not to its own copy
    for h_if in (5e2, 1.5e3, 5e3):
        split = configs.tet_casting(region="cube", h_interface=h_if, **common)
        T0 = np.full(split["xyz"].shape[0], 25.0)
        T0[:Ng][inner] = 700.0                        # grid ids keep their numbering
        split["T0"] = T0
        dt = 0.9 * min(orc.stable_dt(split), orc.stable_dt(conf))
        steps = int(30.0 / dt)
        _, Ts, _ = orc.run(split, dt, steps)
        _, Tc, _ = orc.run(conf, dt, steps)
        errs.append(np.max(np.abs(Ts[:Ng] - Tc)))
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 0.01 * errs[0]


# ------------------------------------------------------------------ P-12, P-13
def test_p12_renumbering_invariance(orc):
    a = configs.tet_casting(n=8, region="cube", permute=False)
    b = configs.tet_casting(n=8, region="cube", permute=True)
    N = a["xyz"].shape[0]
    node_perm = rng.permutation(3, 0, N)
    dt = 0.9 * orc.stable_dt(a)
    assert orc.stable_dt(b) == pytest.approx(orc.stable_dt(a), rel=1e-12)
    _, Ta, fa = orc.run(a, dt, 300)
    _, Tb, fb = orc.run(b, dt, 300)
    assert np.max(np.abs(Tb[node_perm] - Ta)) <= 1e-12 * 700
    assert np.max(np.abs(fb[node_perm] - fa)) <= 1e-10


@pytest.mark.parametrize("n_parts", [1, 3, 8])
def test_p13_partitioned_equals_monolithic(orc, n_parts):
    p = configs.tet_casting(n=8, region="cube", permute=True)
    dt = 0.9 * orc.stable_dt(p)
    part = (np.arange(p["conn"].shape[0]) * 7919) % n_parts
    H1 = orc.run_partitioned(p, part, n_parts, dt, 100)
    H0, _, _ = orc.run(p, dt, 100)
    assert np.max(np.abs(H1 - H0)) <= 1e-12 * np.max(np.abs(H0))


# ------------------------------------------------------------------ P-14
@pytest.mark.parametrize("mat", [ALLOY, (150.0, 2700.0, 900.0, 660.0, 660.0, 3.9e5), configs.SAND])
def test_p14_enthalpy_relation(orc, mat):
    c, Ts, Tl, L = mat[2], mat[3], mat[4], mat[5]
    Hs, Hl = c * Ts, c * Tl + L
    H = np.concatenate([np.linspace(0, 2e6, 4001), [Hs, Hl, np.nextafter(Hs, 0), np.nextafter(Hl, 3e6)]])
    T = orc.T_of_H(mat, H)
    fs = orc.fs_of_H(mat, H)
    assert np.all((fs >= 0) & (fs <= 1))
    order = np.argsort(H)
    assert np.all(np.diff(T[order]) >= 0)
    assert np.all(np.diff(fs[order]) <= 0)
    if L > 0 and Tl > Ts:
        back = orc.H_of_T(mat, T)
        assert np.max(np.abs(back - H) / np.maximum(np.abs(H), 1.0)) <= 4 * np.finfo(float).eps
    if L > 0:
        assert orc.T_of_H(mat, [Hs])[0] == pytest.approx(Ts, abs=1e-12)
        assert orc.T_of_H(mat, [Hl])[0] == pytest.approx(Tl, abs=1e-12)
        assert orc.fs_of_H(mat, [Hs])[0] == 1.0 and orc.fs_of_H(mat, [Hl])[0] == 0.0
        # config-1 constants
        if Tl > Ts:
            assert orc.H_of_T(mat, [700.0])[0] == pytest.approx(1.02e6, rel=1e-15)
            assert Hs == 5.4e5 and Hl == 9.84e5
    else:
        assert np.all(fs == 1.0)


# ------------------------------------------------------------------ Robin / flux boundaries
def test_p15_robin_lumped_cooling(orc):
    """High conductivity cube cooled through one face: T relaxes as exp(-h A t / (rho c V))."""
    big_k = 5.0e4
    mat = (big_k, RHO_AL, C_AL, 0.0, 0.0, 0.0)
    h = 500.0
    p = configs.hex_cube(n=6, noise_amp=0.0, dirichlet_x0=None, robin_x0=(h, 25.0), material=mat,
                         T_pour=700.0)
    dt = 0.9 * orc.stable_dt(p)
    steps = 300
    H, T, fs, D = orc.run(p, dt, steps, diag=True)
    tau = RHO_AL * C_AL * 0.1 ** 3 / (h * 0.1 ** 2)
    expect = 25.0 + 675.0 * math.exp(-steps * dt / tau)
    m = orc.lumped_mass(p)
    Tbar = np.sum(m * T) / np.sum(m)
    Bi = h * 0.1 / big_k
    # explicit Euler on the lumped ODE plus O(Bi) spatial non-uniformity
    assert abs(Tbar - expect) <= 675.0 * (Bi + steps * (dt / tau) ** 2)
    assert np.max(D[:, orc.D_RESID]) < 1e-12


def test_p16_constant_flux_energy(orc):
    """With h = 0 the energy rises by -q A dt per step exactly (q is positive outward)."""
    p = configs.hex_cube(n=4, noise_amp=0.0, dirichlet_x0=None, robin_x0=(0.0, 25.0),
                         material=no_latent(ALLOY))
    p["flux_q"] = np.full(p["flux_q"].size, -2.0e4)     # 20 kW/m^2 into the cube
    dt = 0.5
    H, T, fs, D = orc.run(p, dt, 20, diag=True)
    A = 0.1 * 0.1
    dE = D[1:, orc.D_E] - D[:-1, orc.D_E]
    assert np.allclose(dE, 2.0e4 * A * dt, rtol=1e-10)
    assert np.allclose(D[:, orc.D_Q], 2.0e4 * A, rtol=1e-12)


# ------------------------------------------------------------------ diagnostics
def test_diagnostics_of_the_state(orc):
    """The latent heat still to release, the T range and the liquid count of the
    diagnostics against the returned state (numpy) and the closed form of the
    start: the cube is liquid but for its chilled face, which starts solid and
    whose nodes carry the half-cell layer of lumped mass (A h / 2), so
    rho L (V - A h / 2) of latent heat is left."""
    p = configs.config1()
    dt = 0.9 * orc.stable_dt(p)
    H, T, fs, D = orc.run(p, dt, 300, diag=True)
    m = orc.lumped_mass(p)
    L = ALLOY[5]
    h = 0.1 / 16
    assert D[0, orc.D_LATENT] == pytest.approx(RHO_AL * L * (0.1 ** 3 - 0.1 ** 2 * h / 2), rel=1e-12)
    assert D[0, orc.D_NLIQ] == p["xyz"].shape[0] - p["dirichlet_nodes"].size   # the chilled face starts solid
    assert D[-1, orc.D_LATENT] == pytest.approx(float(np.sum(m * L * (1.0 - fs))), rel=1e-12)
    assert D[-1, orc.D_TMIN] == T.min() and D[-1, orc.D_TMAX] == T.max()
    assert D[-1, orc.D_NLIQ] == np.count_nonzero(fs < 1.0)
    assert 0 < D[-1, orc.D_NLIQ] < D[0, orc.D_NLIQ]


def test_latent_heat_left_follows_the_neumann_front(orc):
    """Isothermal solidification of a bar from a chilled end: the latent heat still
    to release is rho L A (l - X(t)) with the Neumann front X = 2 lambda sqrt(alpha t)."""
    St = C_AL * (660.0 - 25.0) / 3.9e5
    lam = neumann_lambda(St)
    nx, lx = 32, 0.1
    h = lx / nx
    mat = (K_AL, RHO_AL, C_AL, 660.0, 660.0, 3.9e5)
    p = configs.hex_bar(nx=nx, ny=1, nz=1, lx=lx, ly=h, lz=h, T_init=660.0, material=mat)
    dt = 0.45 * h * h / ALPHA
    x = p["xyz"][:, 0]
    H = orc.initial_H(p)
    H[x > 0] = C_AL * 660.0 + 3.9e5
    steps = int(round(75.0 / dt))
    _, _, _, D = orc.run(p, dt, steps, H=H, diag=True)
    for n in (steps // 2, steps):
        t = n * dt
        front = 2 * lam * math.sqrt(ALPHA * t)
        exact = RHO_AL * 3.9e5 * h * h * (lx - front)
        assert abs(D[n, orc.D_LATENT] - exact) <= 0.02 * RHO_AL * 3.9e5 * h * h * front
