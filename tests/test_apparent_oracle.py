"""Pins of the oracle's apparent-heat-capacity mode (Eq. 6 with Lemmon's element
value of dH/dT, Eq. 7, lumped and re-assembled every step, then Eq. 14).

Checked against what the mathematics fixes: the slope of the enthalpy relation
on elements inside one segment, gradients recovered by solving the element's
edge equations instead of shape-function sums, node relabelling, exact
agreement with the enthalpy form wherever the enthalpy relation is linear, and
Neumann's solidification front for a narrow freezing range.
"""
import math

import numpy as np
import pytest
from scipy import optimize

from castgen import configs, rng

ALLOY = configs.ALLOY
K_AL, RHO_AL, C_AL, TS, TL, L_AL = ALLOY
MUSHY = C_AL + L_AL / (TL - TS)


def _tet(seed):
    """A seeded, positively oriented tetrahedron of millimetre size."""
    x = rng.uniform(seed, 21, 12, -1e-3, 1e-3).reshape(4, 3)
    if np.dot(x[1] - x[0], np.cross(x[2] - x[0], x[3] - x[0])) < 0:
        x[[1, 2]] = x[[2, 1]]
    return x


def _H(T, mat=ALLOY):
    c, Ts, Tl, L = mat[2], mat[3], mat[4], mat[5]
    g = np.clip((np.asarray(T, float) - Ts) / (Tl - Ts), 0.0, 1.0) if L > 0 else 0.0
    return c * np.asarray(T, float) + L * g


@pytest.mark.parametrize("lo,hi,slope", [(300.0, 590.0, C_AL), (670.0, 900.0, C_AL), (605.0, 655.0, MUSHY)])
def test_lemmon_inside_one_segment_is_the_slope(orc, lo, hi, slope):
    for seed in range(10):
        x = _tet(seed)
        T = rng.uniform(seed, 22, 4, lo, hi)
        assert orc.lemmon_capacity(x, ALLOY, T, _H(T)) == pytest.approx(slope, rel=1e-11)


def test_lemmon_matches_gradients_solved_from_edges(orc):
    """grad v is the solution of (x_j - x_0) . g = v_j - v_0, j = 1..3."""
    for seed in range(40):
        x = _tet(seed)
        T = rng.uniform(seed, 23, 4, 560.0, 700.0)     # straddles both kinks
        H = _H(T)
        A = x[1:] - x[0]
        gT = np.linalg.solve(A, T[1:] - T[0])
        gH = np.linalg.solve(A, H[1:] - H[0])
        want = np.linalg.norm(gH) / np.linalg.norm(gT)
        assert orc.lemmon_capacity(x, ALLOY, T, H) == pytest.approx(want, rel=1e-9)


def test_lemmon_is_invariant_under_node_relabelling(orc):
    even = [(0, 1, 2, 3), (1, 2, 0, 3), (2, 0, 1, 3), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]
    for seed in range(10):
        x = _tet(seed)
        T = rng.uniform(seed, 24, 4, 580.0, 680.0)
        H = _H(T)
        ref = orc.lemmon_capacity(x, ALLOY, T, H)
        for p in even:
            p = list(p)
            assert orc.lemmon_capacity(x[p], ALLOY, T[p], H[p]) == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("T,want", [(630.0, MUSHY), (500.0, C_AL), (TS, C_AL), (TL, C_AL), (700.0, C_AL)])
def test_lemmon_uniform_element_takes_the_slope_at_its_temperature(orc, T, want):
    x = _tet(3)
    Te = np.full(4, T)
    assert orc.lemmon_capacity(x, ALLOY, Te, _H(Te)) == want


def test_isothermal_latent_material_and_hexahedra_rejected(orc):
    pure = (K_AL, RHO_AL, C_AL, 660.0, 660.0, L_AL)
    with pytest.raises(ValueError):
        orc.lemmon_capacity(_tet(0), pure, np.full(4, 650.0), np.full(4, 650.0 * C_AL))
    p = configs.tet_bar(nx=4, material=pure)
    with pytest.raises(ValueError):
        orc.run_apparent(p, 1e-3, 1)
    with pytest.raises(ValueError):
        orc.run_apparent(configs.hex_cube(n=3), 1e-3, 1)


def test_lumped_capacity_is_slope_times_mass_on_one_segment(orc):
    """All nodes inside one segment of their material: C_i = slope_i * m_i."""
    p = configs.tet_casting(n=6, T_pour=630.0, T_mold=25.0)
    H = orc.initial_H(p)
    Cn = orc.apparent_capacity(p, H)
    m = orc.lumped_mass(p)
    nm = orc.node_material(p)
    slope = np.where(nm == 0, MUSHY, configs.SAND[2])
    np.testing.assert_allclose(Cn, slope * m, rtol=1e-12)


def _equal_runs(orc, p, steps, tol):
    dt = 0.9 * orc.stable_dt(p)
    _, T, _, D = orc.run(p, dt, steps, diag=True)
    _, Ta, _, Da = orc.run_apparent(p, dt, steps, diag=True)
    assert np.max(np.abs(Ta - T)) <= tol
    assert Da[-1, orc.D_RESID] < 1e-12
    return T


def test_apparent_equals_enthalpy_without_latent_heat(orc):
    a = (K_AL, RHO_AL, C_AL, 0.0, 0.0, 0.0)
    p = configs.tet_casting(n=6, alloy=a)
    T = _equal_runs(orc, p, 60, 1e-9)
    assert np.ptp(T) > 100.0     # the field did change


def test_apparent_equals_enthalpy_where_the_relation_stays_linear(orc):
    """A freezing range wider than every temperature reached: each cast node
    stays in the mushy segment, where dH/dT is one constant."""
    wide = (K_AL, RHO_AL, C_AL, -1000.0, 5000.0, L_AL)
    p = configs.tet_casting(n=6, alloy=wide)
    _equal_runs(orc, p, 60, 1e-9)


def test_apparent_differs_from_enthalpy_across_the_kinks(orc):
    """With the real freezing range the two forms part, and the apparent form no
    longer conserves energy exactly (the missed-latent-heat effect)."""
    p = configs.tet_casting(n=6)
    dt = 0.9 * orc.stable_dt(p)
    _, T, _, D = orc.run(p, dt, 200, diag=True)
    _, Ta, _, Da = orc.run_apparent(p, dt, 200, diag=True)
    assert np.max(np.abs(Ta - T)) > 1e-3
    assert D[-1, orc.D_RESID] < 1e-12 < Da[-1, orc.D_RESID] < 0.05


def neumann_lambda(St):
    return optimize.brentq(lambda l: l * math.exp(l * l) * math.erf(l) - St / math.sqrt(math.pi), 1e-6, 5.0)


def _front_error(orc, nx, half):
    """Largest relative error of the solid-front position against Neumann's
    solution (melting point 660 C) at 20, 40, 60 and 75 s, for a freezing range
    660 +- half on a bar of Kuhn tetrahedra."""
    lx = 0.1
    h = lx / nx
    mat = (K_AL, RHO_AL, C_AL, 660.0 - half, 660.0 + half, L_AL)
    p = configs.tet_bar(nx=nx, lx=lx, T_init=660.0 + half, material=mat)
    x = p["xyz"][:, 0]
    w = np.where((x == 0) | (x == lx), h / 2, h) / 4.0
    alpha = K_AL / (RHO_AL * C_AL)
    lam = neumann_lambda(C_AL * (660.0 - 25.0) / L_AL)
    dt = 0.9 * orc.stable_dt(p)
    H = orc.initial_H(p)
    t, worst = 0.0, 0.0
    for tt in (20.0, 40.0, 60.0, 75.0):
        steps = int(round((tt - t) / dt))
        H, T, fs = orc.run_apparent(p, dt, steps, H=H)
        t += steps * dt
        exact = 2 * lam * math.sqrt(alpha * t)
        worst = max(worst, abs(np.sum(w * fs) - exact) / exact)
    return worst


def test_apparent_neumann_front(orc):
    e16, e32 = _front_error(orc, 16, 10.0), _front_error(orc, 32, 10.0)
    assert e16 < 0.03 and e32 < e16
