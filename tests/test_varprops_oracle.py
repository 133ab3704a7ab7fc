"""Pins of the oracle's temperature- and time-dependent properties: conductivity
k(T) per element (Sec. 2 after Eq. 1), interface coefficients that vary with
temperature and time (Eq. 8 and the remark that follows it), and a fixed
temperature that varies in time, uniformly (a shift) or node by node (Eq. 3 with
f(x, t), each fixed node with its own table against time).

Checked against: the constant-property run, an independent 1-D explicit scheme
with element-mean conductivity and a moving wall temperature (the noise-free hex
cube reduces to it), energy conservation where the couplings stay symmetric,
the energy identity with the prescribed change of fixed nodes counted as
inflow, and the lumped two-body recurrence with a time-varying contact.  The
per-node form: a constant schedule is the plain fixed temperature (bit for
bit), one schedule for every node is the shift, a bar whose two ends follow
their own histories is an independent two-wall 1-D scheme, and a linearly
rising wall on a semi-infinite solid converges at second order to the closed
form 4 beta t i^2erfc(x / 2 sqrt(alpha t)).
"""
import numpy as np
import pytest

from castgen import configs

ALLOY = configs.ALLOY
K_AL, RHO_AL, C_AL = ALLOY[0], ALLOY[1], ALLOY[2]
K_TAB = [(550.0, 180.0), (620.0, 150.0), (700.0, 95.0)]
SHIFT = [(0.0, 0.0), (15.0, 250.0), (40.0, 120.0)]


def test_table_values(orc):
    pts = [(0.0, 1.0), (10.0, 3.0), (20.0, -1.0)]
    for x, y in [(-5.0, 1.0), (0.0, 1.0), (5.0, 2.0), (10.0, 3.0), (15.0, 1.0), (20.0, -1.0), (99.0, -1.0)]:
        assert orc.table_value(pts, x) == pytest.approx(y, abs=1e-15)


def test_absent_tables_reproduce_the_constant_run(orc):
    p = configs.config2(n=8)
    v = orc.VarProps(2)
    dt = 0.9 * orc.stable_dt(p)
    assert orc.stable_dt_var(p, v) == orc.stable_dt(p)
    _, T, _ = orc.run(p, dt, 200)
    _, Tv, _ = orc.run_var(p, v, dt, 200)
    assert np.max(np.abs(Tv - T)) <= 1e-12


def _ftcs_1d_var(T0, TD, n, h, dt, steps, mat, k_of, shift_of):
    """1-D explicit enthalpy scheme on n+1 nodes with k((T_i + T_i+1)/2) per element,
    node 0 held at TD + shift(t), far end insulated (written independently)."""
    k0, rho, c, Ts, Tl, L = mat

    def H_of(T):
        return c * T + L * np.clip((T - Ts) / (Tl - Ts), 0.0, 1.0)

    def T_of(H):
        Hs, Hl = c * Ts, c * Tl + L
        return np.where(H <= Hs, H / c, np.where(H >= Hl, (H - L) / c,
                                                 Ts + (H - Hs) * (Tl - Ts) / (c * (Tl - Ts) + L)))

    T = np.full(n + 1, float(T0))
    T[0] = TD + shift_of(0.0)
    H = H_of(T)
    for s in range(steps):
        T = T_of(H)
        ke = np.array([k_of(0.5 * (T[i] + T[i + 1])) for i in range(n)])
        flux = ke * (T[1:] - T[:-1]) / h          # into node i from node i+1
        dH = np.zeros_like(H)
        dH[1:-1] = dt * (flux[1:] - flux[:-1]) / (rho * h)
        dH[-1] = -2.0 * dt * flux[-1] / (rho * h)
        H = H + dH
        H[0] = H_of(np.array([TD + shift_of((s + 1) * dt)]))[0]
    return T_of(H)


def test_hex_cube_with_k_of_T_and_a_moving_wall_is_the_1d_scheme(orc):
    p = configs.config1(noise_amp=0.0)
    v = orc.VarProps(1, k_of_T=[K_TAB], dir_of_t=SHIFT)
    dt = 0.9 * orc.stable_dt_var(p, v)
    H, T, fs = orc.run_var(p, v, dt, 200)
    ref = _ftcs_1d_var(700.0, 25.0, 16, 0.1 / 16, dt, 200, ALLOY,
                       lambda x: np.interp(x, [a for a, b in K_TAB], [b for a, b in K_TAB]),
                       lambda t: np.interp(t, [a for a, b in SHIFT], [b for a, b in SHIFT]))
    i = np.arange(17 ** 3) % 17
    assert np.max(np.abs(T - ref[i])) <= 1e-10
    assert np.min(fs) < 1.0 and np.max(fs) > 0.0
    assert 25.0 <= T.min() and T.max() <= 700.0 + 1e-9


def test_energy_identity_with_a_moving_wall(orc):
    p = configs.hex_bar(nx=16, ny=2, nz=2, lx=0.1, ly=0.0125, lz=0.0125)
    v = orc.VarProps(1, k_of_T=[K_TAB], dir_of_t=SHIFT)
    dt = 0.9 * orc.stable_dt_var(p, v)
    _, T, _, D = orc.run_var(p, v, dt, 600, diag=True)
    assert D[-1, orc.D_RESID] <= 1e-12
    assert abs(D[-1, orc.D_QCUM]) > 0


def test_symmetric_variable_contact_conserves_energy(orc):
    """Matched pairs with h(T) at the pair mean and h(t): every coupling is symmetric."""
    p = configs.tet_casting(n=8)
    v = orc.VarProps(2, k_of_T=[K_TAB, [(0.0, 0.4), (700.0, 1.2)]], h_of_T=[(100.0, 3.0), (650.0, 0.5)],
                     h_of_t=[(0.0, 1.0), (2.0, 0.2)])
    dt = 0.9 * orc.stable_dt_var(p, v)
    _, T, _, D = orc.run_var(p, v, dt, 400, diag=True)
    assert D[-1, orc.D_RESID] <= 1e-12
    _, T0, _ = orc.run(p, dt, 400)
    assert np.max(np.abs(T - T0)) > 1.0          # the properties do act


def test_lumped_two_body_with_a_time_varying_contact(orc):
    big_k, h_if = 1.0e4, 200.0
    mat = (big_k, RHO_AL, C_AL, 0.0, 0.0, 0.0)
    p = configs.tet_casting(n=8, region="cube", cube=(0.3, 0.7), jitter=0.0, permute=False,
                            alloy=mat, mold=mat, T_pour=700.0, T_mold=25.0, h_interface=h_if)
    ht = [(0.0, 1.0), (3.0, 0.25), (6.0, 2.0)]
    v = orc.VarProps(2, h_of_t=ht)
    side = 4 / 8 * 0.1
    A = 6 * side ** 2
    Cc = RHO_AL * C_AL * side ** 3
    Cm = RHO_AL * C_AL * (0.1 ** 3 - side ** 3)
    m = orc.lumped_mass(p)
    cast = orc.node_material(p) == 0
    dt = 0.9 * orc.stable_dt_var(p, v)
    steps = 400
    _, T, _ = orc.run_var(p, v, dt, steps)
    Tc = np.sum(m[cast] * T[cast]) / np.sum(m[cast])
    Tm = np.sum(m[~cast] * T[~cast]) / np.sum(m[~cast])
    phi = np.interp(np.arange(steps) * dt, [a for a, b in ht], [b for a, b in ht])
    expect = 675.0 * np.prod(1.0 - dt * h_if * A * (1 / Cc + 1 / Cm) * phi)
    Bi = h_if * 2.0 * side / big_k
    assert abs((Tc - Tm) - expect) <= 5 * Bi * 675.0


def test_stability_bound_takes_the_largest_properties(orc):
    p = configs.tet_casting(n=6)
    v = orc.VarProps(2, k_of_T=[K_TAB, None], h_of_T=[(0.0, 1.5), (500.0, 0.5)], h_of_t=[(0.0, 2.0), (1.0, 1.0)])
    q = dict(p)
    q["materials"] = np.array(p["materials"], dtype=float)
    q["materials"][0, 0] = 180.0
    q["if_h"] = np.asarray(p["if_h"]) * 3.0
    assert orc.stable_dt_var(p, v) == pytest.approx(orc.stable_dt(q), rel=1e-14)


def test_malformed_tables_are_refused(orc):
    p = configs.tet_casting(n=4)
    with pytest.raises(ValueError):
        orc.stable_dt_var(p, orc.VarProps(2, h_of_t=[(1.0, 1.0), (0.5, 2.0)]))


# ---------------------------------------------------------------- f(x, t) per node
def _faces(p, lx):
    x = p["xyz"][:, 0]
    return np.nonzero(x == 0.0)[0], np.nonzero(np.isclose(x, lx))[0]


def _with_walls(p, left, right):
    q = dict(p)
    q["dirichlet_nodes"] = np.concatenate([left, right]).astype(np.int32)
    q["dirichlet_T"] = np.zeros(left.size + right.size)
    return q


def test_a_constant_schedule_is_the_fixed_temperature(orc):
    p = configs.config1(noise_amp=2.0)
    nd = p["dirichlet_nodes"].size
    dt = 0.9 * orc.stable_dt(p)
    _, T, _ = orc.run_var(p, orc.VarProps(1), dt, 150)
    _, Ts, _ = orc.run_var(p, orc.VarProps(1, dir_sched=[[(0.0, 25.0)]] * nd), dt, 150)
    assert np.array_equal(T, Ts)


def test_one_schedule_for_every_node_is_the_shift(orc):
    p = configs.config1(noise_amp=2.0)
    nd = p["dirichlet_nodes"].size
    dt = 0.9 * orc.stable_dt(p)
    _, T, _ = orc.run_var(p, orc.VarProps(1, dir_of_t=SHIFT), dt, 300)
    sched = [(t, 25.0 + s) for t, s in SHIFT]
    _, Ts, _ = orc.run_var(p, orc.VarProps(1, dir_sched=[sched] * nd), dt, 300)
    assert np.max(np.abs(T - Ts)) <= 1e-10
    # both together: the schedule takes the place of T_D and the shift still adds
    _, Tb, _ = orc.run_var(p, orc.VarProps(1, dir_of_t=SHIFT, dir_sched=[[(0.0, 25.0)]] * nd), dt, 300)
    assert np.max(np.abs(T - Tb)) <= 1e-10


def _ftcs_1d_two_walls(T0, n, h, dt, steps, mat, left_of, right_of):
    """1-D explicit scheme on n+1 nodes, constant k, both ends prescribed (written
    independently of the oracle)."""
    k, rho, c, Ts, Tl, L = mat

    def H_of(T):
        return c * T + L * np.clip((T - Ts) / (Tl - Ts), 0.0, 1.0)

    def T_of(H):
        Hs, Hl = c * Ts, c * Tl + L
        return np.where(H <= Hs, H / c, np.where(H >= Hl, (H - L) / c,
                                                 Ts + (H - Hs) * (Tl - Ts) / (c * (Tl - Ts) + L)))

    T = np.full(n + 1, float(T0))
    T[0], T[-1] = left_of(0.0), right_of(0.0)
    H = H_of(T)
    for s in range(steps):
        T = T_of(H)
        flux = k * (T[1:] - T[:-1]) / h
        H[1:-1] = H[1:-1] + dt * (flux[1:] - flux[:-1]) / (rho * h)
        t = (s + 1) * dt
        H[0], H[-1] = H_of(np.array([left_of(t), right_of(t)]))
    return T_of(H)


def test_two_walls_with_their_own_schedules_is_the_1d_scheme(orc):
    """Each end of a bar follows its own piecewise-linear history (a ramp with a
    hold on one, an oscillation on the other): the nodes of the two faces read
    different tables at the same time."""
    lx, nx = 0.1, 16
    h = lx / nx
    p = configs.hex_bar(nx=nx, ny=1, nz=1, lx=lx, ly=h, lz=h, T_init=700.0)
    left, right = _faces(p, lx)
    q = _with_walls(p, left, right)
    L_s = [(0.0, 700.0), (8.0, 400.0), (20.0, 400.0), (30.0, 200.0)]
    R_s = [(0.0, 700.0), (5.0, 650.0), (10.0, 720.0), (15.0, 600.0), (25.0, 690.0)]
    v = orc.VarProps(1, dir_sched=[L_s] * left.size + [R_s] * right.size)
    dt = 0.9 * orc.stable_dt_var(q, v)
    steps = int(32.0 / dt)
    _, T, fs = orc.run_var(q, v, dt, steps)
    interp = lambda pts: (lambda t: np.interp(t, [a for a, b in pts], [b for a, b in pts]))
    ref = _ftcs_1d_two_walls(700.0, nx, h, dt, steps, ALLOY, interp(L_s), interp(R_s))
    i = np.rint(p["xyz"][:, 0] / h).astype(int)
    assert np.max(np.abs(T - ref[i])) <= 1e-9
    assert T[left].max() == pytest.approx(200.0, abs=1e-9) and T[right].max() == pytest.approx(690.0, abs=1e-9)
    assert np.min(fs) < 1.0 and np.max(fs) > 0.0        # the walls drive the bar through the mushy range


def _ramp_error(orc, nx, beta=5.0, t_end=40.0):
    lx = 0.4
    h = lx / nx
    k, rho, c = K_AL, RHO_AL, C_AL
    alpha = k / (rho * c)
    p = configs.hex_bar(nx=nx, ny=1, nz=1, lx=lx, ly=h, lz=h, T_init=25.0, material=(k, rho, c, 0.0, 0.0, 0.0))
    nd = p["dirichlet_nodes"].size
    v = orc.VarProps(1, dir_sched=[[(0.0, 25.0), (t_end, 25.0 + beta * t_end)]] * nd)
    steps = int(np.ceil(t_end / (0.45 * h * h / alpha)))
    _, T, _ = orc.run_var(p, v, t_end / steps, steps)
    from scipy import special
    z = p["xyz"][:, 0] / (2.0 * np.sqrt(alpha * t_end))
    i2 = (1.0 + 2.0 * z * z) * special.erfc(z) - 2.0 / np.sqrt(np.pi) * z * np.exp(-z * z)   # 4 i^2erfc(z)
    return np.max(np.abs(T - (25.0 + beta * t_end * i2)))


def test_linearly_rising_wall_is_the_closed_form(orc):
    """Semi-infinite solid whose surface temperature rises as T0 + beta t:
    T - T0 = 4 beta t i^2erfc(x / (2 sqrt(alpha t))) (the repeated integral of the
    complementary error function), approached at second order in h."""
    e1, e2, e3 = _ramp_error(orc, 64), _ramp_error(orc, 128), _ramp_error(orc, 256)
    assert e3 < 0.05          # of a 200 K rise
    assert 3.2 < e1 / e2 < 5.0 and 3.2 < e2 / e3 < 5.0


def test_energy_identity_with_a_schedule_that_varies_over_the_face(orc):
    p = configs.config1(noise_amp=2.0)
    d = p["dirichlet_nodes"]
    y = p["xyz"][d, 1] / 0.1
    dt = 0.9 * orc.stable_dt_var(p, orc.VarProps(1, k_of_T=[K_TAB]))
    sched = [[(0.0, 25.0 + 30.0 * yy), (150 * dt, 500.0 - 100.0 * yy), (600 * dt, 60.0)] for yy in y]
    v = orc.VarProps(1, k_of_T=[K_TAB], dir_sched=sched)
    assert orc.stable_dt_var(p, v) == pytest.approx(dt / 0.9, rel=1e-15)
    H, T, _, D = orc.run_var(p, v, dt, 400, diag=True)
    assert D[-1, orc.D_RESID] <= 1e-12
    t = 400 * dt
    assert np.max(np.abs(T[d] - np.array([np.interp(t, [a for a, b in s], [b for a, b in s]) for s in sched]))) <= 1e-9
    # the face is not uniform: the field is not that of the one-schedule run
    _, T1, _ = orc.run_var(p, orc.VarProps(1, k_of_T=[K_TAB], dir_sched=[sched[0]] * d.size), dt, 400)
    assert np.max(np.abs(T - T1)) > 1.0


def test_malformed_schedules_are_refused(orc):
    p = configs.config1()
    nd = p["dirichlet_nodes"].size
    with pytest.raises(ValueError):
        orc.stable_dt_var(p, orc.VarProps(1, dir_sched=[[(1.0, 25.0), (0.5, 30.0)]] * nd))
