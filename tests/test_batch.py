"""Batches of casting scenarios in one mesh: per-scenario stability bounds, time
steps and energy balances, compared with the oracle run on every scenario alone."""
import numpy as np
import pytest

from castgen import configs
from paper_1005_3158_amd import castfem as cf


def scenario_problem(sp, permute=True):
    """The scenario `sp` of configs.batch on its own (same seeds, same numbering)."""
    mold = (sp["k_mold"],) + configs.SAND[1:]
    return configs.tet_casting(n=sp["n"], region="cube", jitter_seed=sp["seed"], perm_seed=sp["seed"],
                               T_pour=sp["T_pour"], h_interface=sp["h_interface"], alloy=configs.ALLOY,
                               mold=mold, permute=permute)


@pytest.fixture(scope="module")
def small_batch():
    return configs.batch(n_scen=6, n_range=(5, 9))


def test_batch_bounds_match_each_scenario_alone(small_batch, orc):
    b = small_batch
    ctx = cf.fem_create(cf.make_options())
    cf.setup_problem(ctx, b)
    bounds = cf.fem_stable_dt_scenarios(ctx, 6)
    for s, sp in enumerate(b["meta"]["scenarios"]):
        assert bounds[s] == pytest.approx(orc.stable_dt(scenario_problem(sp)), rel=1e-12)
    assert cf.fem_stable_dt(ctx) == pytest.approx(bounds.min(), rel=1e-15)
    rep = cf.fem_get_report(ctx)
    assert rep["n_blocks"] >= 6
    cf.fem_destroy(ctx)


def test_interface_across_scenarios_is_rejected(small_batch):
    b = dict(small_batch)
    sc = b["meta"]["scenarios"]
    fb = b["if_b"].copy()
    fb[0] = fb[-1]                       # pair a face of scenario 0 with one of scenario 5
    b["if_b"] = fb
    ctx = cf.fem_create(cf.make_options())
    with pytest.raises(cf.FemError) as e:
        cf.setup_problem(ctx, b)
    assert e.value.code == -2 and "scenario" in cf.fem_last_error()
    cf.fem_destroy(ctx)
    assert sc[0]["node1"] <= sc[5]["node0"]


def test_scenario_table_errors():
    ctx = cf.fem_create(None)
    with pytest.raises(cf.FemError) as e:
        cf.fem_set_scenarios(ctx, [0, 1])
    assert e.value.code == -3                 # materials not set yet
    cf.fem_set_materials(ctx, np.array([configs.ALLOY, configs.SAND, configs.SAND]))
    with pytest.raises(cf.FemError):
        cf.fem_set_scenarios(ctx, np.array([0, 2, 2], np.int32))   # scenario 1 owns nothing
    cf.fem_destroy(ctx)


@pytest.mark.gpu
@pytest.mark.parametrize("scatter", ["lds", "atomic"])
def test_batch_matches_scenarios_run_alone(small_batch, orc, scatter):
    b = small_batch
    sc = b["meta"]["scenarios"]
    opts = dict(precision=cf.FEM_PREC_FP32_KAHAN, lds_bytes=cf.lds_for_nodes(300),
                scatter=cf.FEM_SCATTER_LDS_BLOCKED if scatter == "lds" else cf.FEM_SCATTER_GLOBAL_ATOMIC)
    s = cf.Solver(b, **opts)
    dt = 0.9 * s.stable_dt_scenarios()
    steps = 500
    s.step_batch(dt, steps)
    T, fs = s.T(), s.fs()
    reps = s.energy_scenarios()
    tot = s.energy()
    s.close()
    for k, sp in enumerate(sc):
        p = scenario_problem(sp)
        H_ref, T_ref, fs_ref = orc.run(p, dt[k], steps)
        Tk = T[sp["node0"]:sp["node1"]]
        err = float(np.max(np.abs(Tk - T_ref)))
        print("scenario %d (n=%d, dt=%.3e): max|dT| = %.3e K, residual %.2e" % (k, sp["n"], dt[k], err, reps[k]["residual"]))
        assert err <= 1e-3
        assert float(np.max(np.abs(fs[sp["node0"]:sp["node1"]] - fs_ref))) <= 1e-4
        assert reps[k]["residual"] <= 1e-5
        assert reps[k]["time"] == pytest.approx(dt[k] * steps, rel=1e-12)
    assert tot["E"] == pytest.approx(sum(r["E"] for r in reps), rel=1e-14)


K_CAST = [(550.0, 180.0), (620.0, 150.0), (700.0, 95.0)]
H_T = [(100.0, 3.0), (650.0, 0.5)]


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_with_variable_properties_matches_scenarios_run_alone(small_batch, orc, precision):
    """Temperature- and time-dependent properties in a batch: every scenario keeps
    its own device clock (its own dt), so h(t) of the contact is read at a
    different time in each; each scenario against the oracle's variable-property
    run of it alone."""
    b = dict(small_batch)
    sc = b["meta"]["scenarios"]
    nm = len(b["materials"])
    # the scenarios' steps are 0.07-0.32 s: 400 steps end between 30 and 130 s, and the
    # time factor changes throughout
    h_t = [(0.0, 1.0), (20.0, 0.2), (60.0, 2.5), (110.0, 0.6)]
    b["varprops"] = dict(k_of_T=[K_CAST if m % 2 == 0 else None for m in range(nm)], h_of_T=H_T, h_of_t=h_t)
    fp64 = precision == "fp64"
    prec = cf.FEM_PREC_FP64 if fp64 else cf.FEM_PREC_FP32_KAHAN
    s = cf.Solver(b, precision=prec, lds_bytes=cf.lds_for_nodes(300, prec))
    dt = 0.9 * s.stable_dt_scenarios()
    steps = 400
    s.step_batch(dt, steps)
    T = s.T()
    reps = s.energy_scenarios()
    s.close()
    assert np.ptp(dt) > 0.2 * dt.min()            # the clocks do differ
    for k, sp in enumerate(sc):
        p = scenario_problem(sp)
        assert b["materials"][2 * k][0] == p["materials"][0][0]
        vp = orc.VarProps(2, k_of_T=[K_CAST, None], h_of_T=H_T, h_of_t=h_t)
        assert orc.stable_dt_var(p, vp) == pytest.approx(dt[k] / 0.9, rel=1e-12)
        _, T_ref, _ = orc.run_var(p, vp, dt[k], steps)
        Tk = T[sp["node0"]:sp["node1"]]
        band = (T_ref >= configs.ALLOY[3] - 5.0) & (T_ref <= configs.ALLOY[4] + 5.0)
        err = np.abs(Tk - T_ref)
        off = float(err[~band].max()) if np.any(~band) else 0.0
        on = float(err[band].max()) if np.any(band) else 0.0
        print("scenario %d (n=%d, dt=%.3e, t_end=%.2f s): max|dT| off-front %.3e K, band %.3e K; residual %.2e"
              % (k, sp["n"], dt[k], dt[k] * steps, off, on, reps[k]["residual"]), flush=True)
        if fp64:
            assert max(off, on) <= 1e-8
            assert reps[k]["residual"] <= 1e-11
        else:
            assert off <= 1e-3 and on <= 0.05
        assert reps[k]["time"] == pytest.approx(dt[k] * steps, rel=1e-12)
