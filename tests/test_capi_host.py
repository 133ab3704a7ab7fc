"""CPU-only checks of the C interface: exported symbols, argument and call-order
errors, and the host preprocessing (lumping, stability bound, orderings,
blocks, colours) that runs before any device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from castgen import configs
from paper_1005_3158_amd import castfem as cf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "castfem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 20
    out = subprocess.check_output(["nm", "-D", "--defined-only", cf.LIB_PATH]).decode()
    exported = set(re.findall(r"\bT (fem_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert sorted(cf.EXPORTS) == names
    lib = cf.lib()
    for n in names:
        assert getattr(lib, n) is not None


def test_library_carries_gfx950_code_only():
    blob = open(cf.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob
    assert b"amdgcn-amd-amdhsa--gfx906" not in blob


def test_errors_and_call_order():
    with pytest.raises(cf.FemError) as e:
        cf.fem_create(cf.make_options(precision=7))
    assert e.value.code == -1
    ctx = cf.fem_create(None)
    with pytest.raises(cf.FemError) as e:
        cf.fem_finalize(ctx)
    assert e.value.code == -3
    with pytest.raises(cf.FemError) as e:
        cf.fem_step(ctx, 0.1, 1)
    assert e.value.code == -3
    assert "not bound" in cf.fem_last_error()
    p = configs.config2(n=4)
    # node in two materials: glue a casting tet onto a mould node
    bad = dict(p)
    conn = p["conn"].copy()
    cast = np.nonzero(p["elem_mat"] == 0)[0][0]
    mould_node = p["conn"][np.nonzero(p["elem_mat"] == 1)[0][0], 0]
    conn[cast, 0] = mould_node
    bad["conn"] = conn
    ctx2 = cf.fem_create(None)
    with pytest.raises(cf.FemError) as e:
        cf.setup_problem(ctx2, bad)
    assert e.value.code == -2
    # inverted element
    inv = dict(p)
    conn = p["conn"].copy()
    conn[0, [1, 2]] = conn[0, [2, 1]]
    inv["conn"] = conn
    ctx3 = cf.fem_create(None)
    with pytest.raises(cf.FemError) as e:
        cf.setup_problem(ctx3, inv)
    assert e.value.code == -2 and "inverted" in cf.fem_last_error()
    # out-of-range node
    oor = dict(p)
    conn = p["conn"].copy()
    conn[3, 2] = p["xyz"].shape[0]
    oor["conn"] = conn
    ctx4 = cf.fem_create(None)
    with pytest.raises(cf.FemError) as e:
        cf.setup_problem(ctx4, oor)
    assert e.value.code == -2
    # a failed finalize leaves the context usable
    cf.setup_problem(ctx4, p)
    for c in (ctx, ctx2, ctx3, ctx4):
        cf.fem_destroy(c)


def test_dt_bound_matches_oracle(orc):
    for p in (configs.config1(), configs.config2(n=10), configs.config4_trajectory(5001, n=6)):
        ctx = cf.fem_create(cf.make_options(scatter=cf.FEM_SCATTER_GLOBAL_ATOMIC))
        rep = cf.setup_problem(ctx, p)
        assert rep["dt_bound"] == pytest.approx(orc.stable_dt(p), rel=1e-12)
        cf.fem_destroy(ctx)


@pytest.mark.parametrize("ordering", [cf.FEM_ORDER_NONE, cf.FEM_ORDER_RCM, cf.FEM_ORDER_MORTON, cf.FEM_ORDER_HILBERT])
def test_orderings_are_permutations_and_shrink_bandwidth(ordering):
    p = configs.config2(n=16)
    ctx = cf.fem_create(cf.make_options(ordering=ordering, scatter=cf.FEM_SCATTER_GLOBAL_ATOMIC))
    rep = cf.setup_problem(ctx, p)
    perm = cf.fem_get_node_perm(ctx, p["xyz"].shape[0])
    assert np.array_equal(np.sort(perm), np.arange(perm.size))
    if ordering == cf.FEM_ORDER_NONE:
        assert np.array_equal(perm, np.arange(perm.size))
        assert rep["bandwidth_after"] == rep["bandwidth_before"]
    elif ordering == cf.FEM_ORDER_RCM:
        # the random input numbering has bandwidth ~N; RCM brings it near a grid plane
        assert rep["bandwidth_after"] < 0.1 * rep["bandwidth_before"]
    else:
        assert rep["bandwidth_after"] < rep["bandwidth_before"]
    cf.fem_destroy(ctx)


def test_blocks_and_colours_report():
    p = configs.config2(n=16)
    ctx = cf.fem_create(cf.make_options(scatter=cf.FEM_SCATTER_LDS_BLOCKED, lds_bytes=cf.lds_for_nodes(700), block_elems=4000))
    rep = cf.setup_problem(ctx, p)
    assert rep["max_local_nodes"] <= 700
    assert rep["n_blocks"] >= p["conn"].shape[0] // 4000
    assert 0 < rep["n_shared"] < p["xyz"].shape[0]
    assert rep["n_partials"] >= rep["n_shared"]    # interface nodes may sit in one block
    cf.fem_destroy(ctx)
    ctx = cf.fem_create(cf.make_options(scatter=cf.FEM_SCATTER_COLORED))
    rep = cf.setup_problem(ctx, p)
    assert 24 <= rep["n_colors"] <= 64      # 24 Kuhn tets share an interior node
    cf.fem_destroy(ctx)


def test_buffer_query_shapes():
    p = configs.config1()
    ctx = cf.fem_create(cf.make_options(precision=cf.FEM_PREC_FP64, scatter=cf.FEM_SCATTER_GLOBAL_ATOMIC))
    cf.setup_problem(ctx, p)
    bufs = {n: (b, a) for n, b, a in cf.fem_query_buffers(ctx)}
    N, E = p["xyz"].shape[0], p["conn"].shape[0]
    assert bufs["node_x"][0] >= 32 * N and bufs["T"][0] >= 16 * N and bufs["conn"][0] >= 32 * E
    assert all(a == 256 for b, a in bufs.values())
    with pytest.raises(cf.FemError) as e:
        cf.fem_bind_buffers(ctx, [0] * 3)
    assert e.value.code == -1
    cf.fem_destroy(ctx)


def test_apparent_mode_options_and_buffers():
    """The apparent-capacity mode: unknown model ids, hexahedra, other scatters and
    isothermal latent materials are refused; a tet problem gets the extra
    capacitance partials and material table."""
    with pytest.raises(cf.FemError) as e:
        cf.fem_create(cf.make_options(latent_model=5))
    assert e.value.code == -1
    app = cf.FEM_LATENT_APPARENT
    for prob, opts in ((configs.config1(), {}),
                       (configs.config2(n=6), dict(scatter=cf.FEM_SCATTER_COLORED)),
                       (configs.config2(n=6), dict(scatter=cf.FEM_SCATTER_GLOBAL_ATOMIC)),
                       (configs.tet_bar(nx=4, material=(150.0, 2700.0, 900.0, 660.0, 660.0, 3.9e5)), {})):
        ctx = cf.fem_create(cf.make_options(latent_model=app, **opts))
        with pytest.raises(cf.FemError) as e:
            cf.setup_problem(ctx, prob)
        assert e.value.code == -7
        cf.fem_destroy(ctx)
    p = configs.config2(n=6)
    sizes = {}
    for model in (cf.FEM_LATENT_ENTHALPY, app):
        ctx = cf.fem_create(cf.make_options(latent_model=model, lds_bytes=cf.lds_for_nodes(200, apparent=True)))
        rep = cf.setup_problem(ctx, p)
        sizes[model] = ({n: b for n, b, a in cf.fem_query_buffers(ctx)}, rep)
        cf.fem_destroy(ctx)
    bufs, rep = sizes[app]
    assert bufs["cap_partials"] >= 4 * rep["n_partials"] > 0
    assert bufs["app_mats"] > 0
    assert sizes[cf.FEM_LATENT_ENTHALPY][0]["cap_partials"] == 0


@pytest.mark.parametrize("kw", [dict(), dict(n_cast=8, n_mold=4, cube=(0.25, 0.75), jitter=0.0, permute=False),
                                dict(n_cast=10, n_mold=8, jitter=0.2, jitter_seed=5, perm_seed=6),
                                dict(n_cast=24, n_mold=12, jitter=0.1)])
def test_grid_sister_search_equals_the_oracle_brute_force(orc, kw):
    """The library's grid search and the oracle's all-pairs search pick the same
    sister for every contact face, ties included (structured faces are
    equidistant from several faces of the other side)."""
    p = configs.tet_casting_nonmatching(**kw)
    ctx = cf.fem_create(cf.make_options(scatter=cf.FEM_SCATTER_GLOBAL_ATOMIC))
    rep = cf.setup_problem(ctx, p)
    s = cf.fem_get_sisters(ctx, p["contact_faces"].shape[0])
    cf.fem_destroy(ctx)
    assert np.array_equal(s, orc.contact_sisters(p))
    assert rep["dt_bound"] == pytest.approx(orc.stable_dt(p), rel=1e-12)


def test_matched_faces_given_as_contact_find_their_partners():
    p = configs.tet_casting(n=10)
    n = p["if_a"].shape[0]
    ctx = cf.fem_create(cf.make_options(scatter=cf.FEM_SCATTER_GLOBAL_ATOMIC))
    cf.fem_upload_mesh(ctx, 4, p["xyz"], p["conn"], p["elem_mat"])
    cf.fem_set_materials(ctx, p["materials"])
    cf.fem_set_contact(ctx, np.concatenate([p["if_a"], p["if_b"]]), np.repeat([0, 1], n), np.full(2 * n, 1000.0))
    cf.fem_set_initial_T(ctx, p["T0"])
    cf.fem_finalize(ctx)
    s = cf.fem_get_sisters(ctx, 2 * n)
    cf.fem_destroy(ctx)
    assert np.array_equal(s, np.concatenate([np.arange(n, 2 * n), np.arange(n)]))
    with pytest.raises(cf.FemError) as e:
        ctx = cf.fem_create(None)
        cf.fem_upload_mesh(ctx, 4, p["xyz"], p["conn"], p["elem_mat"])
        cf.fem_set_materials(ctx, p["materials"])
        cf.fem_set_contact(ctx, p["if_a"], np.zeros(n, np.int32), np.full(n, 1000.0))   # one side only
        cf.fem_set_initial_T(ctx, p["T0"])
        cf.fem_finalize(ctx)
    assert e.value.code == -2
    cf.fem_destroy(ctx)


def test_variable_properties_bound_and_refusals(orc):
    """Host side of temperature- and time-dependent properties: the stability bound
    at the largest properties equals the oracle's; unsupported combinations and
    malformed tables are refused."""
    vp = dict(k_of_T=[[(550.0, 180.0), (700.0, 95.0)], None], h_of_T=[(100.0, 3.0), (650.0, 0.5)],
              h_of_t=[(0.0, 1.0), (1.0, 2.0)], dir_of_t=[(0.0, 0.0), (5.0, 30.0)])
    p = dict(configs.config2(n=8), varprops=vp)
    ctx = cf.fem_create(cf.make_options())
    rep = cf.setup_problem(ctx, p)
    cf.fem_destroy(ctx)
    assert rep["dt_bound"] == pytest.approx(orc.stable_dt_var(p, orc.VarProps(2, **vp)), rel=1e-12)
    for opts in (dict(scatter=cf.FEM_SCATTER_COLORED), dict(latent_model=cf.FEM_LATENT_APPARENT)):
        ctx = cf.fem_create(cf.make_options(**opts))
        with pytest.raises(cf.FemError) as e:
            cf.setup_problem(ctx, p)
        assert e.value.code == -7
        cf.fem_destroy(ctx)
    # a batch takes them too: every scenario's bound at its own largest properties
    b = configs.batch(n_scen=2, elems_range=(800, 1600))
    b["varprops"] = dict(h_of_t=[(0.0, 1.0), (1.0, 2.5)])
    ctx = cf.fem_create(cf.make_options())
    cf.setup_problem(ctx, b)
    bounds = cf.fem_stable_dt_scenarios(ctx, 2)
    cf.fem_destroy(ctx)
    for s, sp in enumerate(b["meta"]["scenarios"]):
        q = {k: v for k, v in b.items() if k != "varprops"}
        q["if_h"] = np.asarray(b["if_h"]) * 2.5
        ctx = cf.fem_create(cf.make_options())
        cf.setup_problem(ctx, q)
        assert bounds[s] == pytest.approx(cf.fem_stable_dt_scenarios(ctx, 2)[s], rel=1e-14)
        cf.fem_destroy(ctx)
    for bad in (dict(h_of_t=[(1.0, 1.0), (0.5, 2.0)]), dict(k_of_T=[[(0.0, -1.0)], None]),
                dict(h_of_T=[(0.0, float("nan"))])):
        ctx = cf.fem_create(cf.make_options())
        with pytest.raises(cf.FemError) as e:
            cf.setup_problem(ctx, dict(configs.config2(n=4), varprops=bad))
        assert e.value.code == -1
        cf.fem_destroy(ctx)


def test_dirichlet_schedule_checks_and_layout():
    """Host side of the node-by-node prescribed temperature: call order, malformed
    schedules, a schedule that no longer matches the fixed set, the colored scatter
    refused; a valid one makes the context one with variable properties (its
    buffers appear) and sets the fixed nodes' starting values to f(x, 0)."""
    p = configs.config1()
    nd = p["dirichlet_nodes"].size
    good = (np.array([0.0, 1.0, 3.0]), np.tile([40.0, 80.0, 20.0], (nd, 1)))
    ctx = cf.fem_create(cf.make_options())
    cf.fem_upload_mesh(ctx, p["elem_type"], p["xyz"], p["conn"], p["elem_mat"])
    cf.fem_set_materials(ctx, p["materials"])
    with pytest.raises(cf.FemError) as e:          # no fixed nodes yet
        cf.fem_set_dirichlet_schedule(ctx, *good)
    assert e.value.code == -3
    cf.fem_set_dirichlet(ctx, p["dirichlet_nodes"], p["dirichlet_T"])
    for times, values in ((np.array([0.0, 0.0]), np.zeros((nd, 2))), (np.arange(9.0), np.zeros((nd, 9))),
                          (np.array([0.0, 1.0]), np.full((nd, 2), np.nan))):
        with pytest.raises(cf.FemError) as e:
            cf.fem_set_dirichlet_schedule(ctx, times, values)
        assert e.value.code == -1
    cf.fem_set_dirichlet_schedule(ctx, *good)
    cf.fem_set_dirichlet(ctx, p["dirichlet_nodes"][:-1], p["dirichlet_T"][:-1])   # the set changed
    cf.fem_set_initial_T(ctx, p["T0"])
    with pytest.raises(cf.FemError) as e:
        cf.fem_finalize(ctx)
    assert e.value.code == -1
    cf.fem_destroy(ctx)
    q = dict(p, dirichlet_schedule=good)
    ctx = cf.fem_create(cf.make_options(scatter=cf.FEM_SCATTER_COLORED))
    with pytest.raises(cf.FemError) as e:
        cf.setup_problem(ctx, q)
    assert e.value.code == -7
    cf.fem_destroy(ctx)
    ctx = cf.fem_create(cf.make_options(lds_bytes=cf.lds_for_nodes(512)))
    cf.setup_problem(ctx, q)
    names = {n: b for n, b, _ in cf.fem_query_buffers(ctx)}
    cf.fem_destroy(ctx)
    assert names["dirichlet_schedule"] >= nd * 3 * 8
    assert names["var_tables_f64"] > 0
