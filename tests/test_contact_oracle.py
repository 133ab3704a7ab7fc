"""Pins of the oracle's contact faces on non-matching cast/mould meshes (Eq. 8 with
the sister element found once at the start, end of Sec. 3).

Checked against: an independent numpy brute-force sister search, the matched
interface pairs (a matched mesh's contact faces must reproduce them), and the
lumped two-body relaxation of two highly conducting blocks joined through a
non-matching interface, whose closed form needs each face to use its own area.
"""
import math

import numpy as np
import pytest

from castgen import configs

ALLOY = configs.ALLOY
K_AL, RHO_AL, C_AL = ALLOY[0], ALLOY[1], ALLOY[2]


def _numpy_sisters(p):
    """Closest centroid of the other side, first index on ties (numpy argmin)."""
    x = np.asarray(p["xyz"], float)
    f = np.asarray(p["contact_faces"])
    side = np.asarray(p["contact_side"])
    c = ((x[f[:, 0]] + x[f[:, 1]]) + x[f[:, 2]]) / 3.0
    out = np.empty(f.shape[0], np.int64)
    for i in range(f.shape[0]):
        d = c[i] - c
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        d2[side == side[i]] = np.inf
        out[i] = int(np.argmin(d2))
    return out


@pytest.mark.parametrize("kw", [dict(), dict(n_cast=8, n_mold=4, cube=(0.25, 0.75), jitter=0.0, permute=False),
                                dict(n_cast=10, n_mold=8, jitter=0.2, jitter_seed=5, perm_seed=6)])
def test_sisters_match_a_numpy_brute_force(orc, kw):
    p = configs.tet_casting_nonmatching(**kw)
    s = orc.contact_sisters(p)
    ref = _numpy_sisters(p)
    assert np.array_equal(s, ref)
    side = np.asarray(p["contact_side"])
    assert np.all(side[s] != side)


def _matched_as_contact(p):
    """The matched interface pairs of a tet_casting mesh written as contact faces."""
    q = dict(p)
    n = p["if_a"].shape[0]
    q["contact_faces"] = np.concatenate([p["if_a"], p["if_b"]]).astype(np.int32)
    q["contact_side"] = np.concatenate([np.zeros(n, np.int32), np.ones(n, np.int32)])
    q["contact_h"] = np.concatenate([p["if_h"], p["if_h"]])
    q["if_a"] = np.zeros((0, 3), np.int32)
    q["if_b"] = np.zeros((0, 3), np.int32)
    q["if_h"] = np.zeros(0)
    return q


def test_matched_mesh_contact_equals_the_interface_pairs(orc):
    p = configs.tet_casting(n=8)
    q = _matched_as_contact(p)
    n = p["if_a"].shape[0]
    s = orc.contact_sisters(q)
    assert np.array_equal(s, np.concatenate([np.arange(n, 2 * n), np.arange(n)]))
    dt = 0.9 * orc.stable_dt(p)
    assert orc.stable_dt(q) == pytest.approx(orc.stable_dt(p), rel=1e-12)
    _, T, _, D = orc.run(p, dt, 200, diag=True)
    _, Tq, _, Dq = orc.run(q, dt, 200, diag=True)
    assert np.max(np.abs(Tq - T)) <= 1e-9
    assert Dq[-1, orc.D_RESID] <= 1e-12


def test_nonmatching_lumped_two_body_relaxation(orc):
    """Bi << 1 on both sides: the mean temperatures relax as the explicit two-body
    recurrence with each side exchanging h A (T_other - T_self), A the cube's area."""
    big_k, h_if = 1.0e4, 200.0
    mat = (big_k, RHO_AL, C_AL, 0.0, 0.0, 0.0)
    p = configs.tet_casting_nonmatching(n_cast=9, n_mold=6, cube=(1 / 3, 2 / 3), jitter=0.0, permute=False,
                                        alloy=mat, mold=mat, h_interface=h_if)
    side = 0.1 / 3
    A = 6 * side ** 2
    Cc = RHO_AL * C_AL * side ** 3
    Cm = RHO_AL * C_AL * (0.1 ** 3 - side ** 3)
    m = orc.lumped_mass(p)
    cast = orc.node_material(p) == 0
    dt = 0.9 * orc.stable_dt(p)
    steps = 400
    _, T, _, D = orc.run(p, dt, steps, diag=True)
    Tc = np.sum(m[cast] * T[cast]) / np.sum(m[cast])
    Tm = np.sum(m[~cast] * T[~cast]) / np.sum(m[~cast])
    expect = 675.0 * (1.0 - dt * h_if * A * (1 / Cc + 1 / Cm)) ** steps
    Bi = h_if * side / big_k
    assert abs((Tc - Tm) - expect) <= 5 * Bi * 675.0
    # near-uniform sides exchange almost symmetrically: little energy is created
    assert D[-1, orc.D_RESID] < 1e-3


def test_nonmatching_contact_does_not_conserve_energy_exactly(orc):
    p = configs.tet_casting_nonmatching()
    dt = 0.9 * orc.stable_dt(p)
    _, T, _, D = orc.run(p, dt, 300, diag=True)
    assert 1e-8 < D[-1, orc.D_RESID] < 1e-2
    assert np.all(np.isfinite(T))


def test_contact_stability_bound_by_brute_force(orc):
    """Gershgorin rows of the assembled operator including the contact links."""
    p = configs.tet_casting_nonmatching(n_cast=4, n_mold=4, cube=(0.25, 0.75), jitter=0.1, permute=False)
    N = p["xyz"].shape[0]
    K = np.zeros((N, N))
    for e in range(p["conn"].shape[0]):
        c = p["conn"][e]
        Ke, _ = orc.tet_ke(p["xyz"][c], p["materials"][p["elem_mat"][e]][0])
        K[np.ix_(c, c)] += Ke
    s = orc.contact_sisters(p)
    x = p["xyz"]
    for f, face in enumerate(p["contact_faces"]):
        a = 0.5 * np.linalg.norm(np.cross(x[face[1]] - x[face[0]], x[face[2]] - x[face[0]]))
        w = p["contact_h"][f] * a / 3.0
        for i in face:
            K[i, i] += w
            for j in p["contact_faces"][s[f]]:
                K[i, j] -= w / 3.0
    m = orc.lumped_mass(p)
    c = p["materials"][orc.node_material(p)][:, 2]
    lam = np.max(np.sum(np.abs(K), axis=1) / (m * c))
    assert orc.stable_dt(p) == pytest.approx(2.0 / lam, rel=1e-12)
    # and the residual is -K T with these contact rows
    T = np.linspace(20.0, 700.0, N)
    np.testing.assert_allclose(orc.residual(p, T), -K @ T, rtol=0, atol=1e-9 * np.max(np.abs(K @ T)))
