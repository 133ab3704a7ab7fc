"""The benchmark workload at full size, in the launch configuration the benchmark
times: 128^3 jittered Kuhn tets (12,582,912 tets, 2,181,347 nodes), alloy cube in
sand with h_i = 1000, FP32 state with compensated enthalpy, LDS-blocked scatter,
Hilbert ordering, the block shape autotuned as in the benchmark (the apparent,
variable-property and contact legs at 512-node blocks, as their benchmark legs),
steps in captured graphs.

- Three steps against the FP64 oracle at every node (the oracle takes ~5 s per step), also in
  the apparent-capacity form and with temperature- and time-dependent properties; the
  non-matching contact workload (16.3M tets) with all of its sisters and two steps.
- 400 steps against properties that hold at any size: the energy balance
  (FP64 E - E0 - Q_cum), finite values, and bitwise reproducibility of the
  fixed-point scatter (two runs give the same state).  The discrete maximum
  principle does not hold on jittered tets (the oracle's own 24^3 run undershoots
  the mould's 25 C by 4.6 K), so T bounds are not a property here.
"""
import numpy as np
import pytest

from castgen import configs

pytestmark = pytest.mark.gpu

BLOCK_NODES = 512   # the apparent, variable-property and contact legs


@pytest.fixture(scope="module")
def config2():
    return configs.config2()


def _solver(prob):
    from paper_1005_3158_amd import castfem as cf
    return cf.Solver(prob, precision=cf.FEM_PREC_FP32_KAHAN, scatter=cf.FEM_SCATTER_LDS_BLOCKED,
                     ordering=cf.FEM_ORDER_HILBERT)


def test_three_full_size_steps_match_the_oracle(config2, orc):
    dt = 0.9 * orc.stable_dt(config2)
    s = _solver(config2)
    try:
        assert s.report["n_elems"] == 12582912 and s.report["n_nodes"] == 2181347
        print("config 2: %d blocks, shared fraction %.3f" % (s.report["n_blocks"], s.report["shared_fraction"]),
              flush=True)
        s.step(dt, 3)
        T, fs = s.T(), s.fs()
    finally:
        s.close()
    _, T_ref, fs_ref = orc.run(config2, dt, 3)
    err = np.abs(T - T_ref)
    print("max|T - oracle| %.3e K, rms %.3e K; max|fs - oracle| %.3e" %
          (err.max(), np.sqrt(np.mean(err ** 2)), np.abs(fs - fs_ref).max()), flush=True)
    assert err.max() <= 1e-3
    assert np.abs(fs - fs_ref).max() <= 1e-4


def test_three_full_size_apparent_steps_match_the_oracle(config2, orc):
    """The apparent-heat-capacity form in the benchmark's launch shape (512-node
    blocks at its 32 B of LDS per node) against the oracle's apparent form."""
    from paper_1005_3158_amd import castfem as cf
    dt = 0.9 * orc.stable_dt(config2)
    s = cf.Solver(config2, precision=cf.FEM_PREC_FP32_KAHAN, latent_model=cf.FEM_LATENT_APPARENT,
                  lds_bytes=cf.lds_for_nodes(BLOCK_NODES, apparent=True))
    try:
        s.step(dt, 3)
        T, fs = s.T(), s.fs()
    finally:
        s.close()
    _, T_ref, fs_ref = orc.run_apparent(config2, dt, 3)
    err = np.abs(T - T_ref)
    print("apparent: max|T - oracle| %.3e K, rms %.3e K; max|fs - oracle| %.3e" %
          (err.max(), np.sqrt(np.mean(err ** 2)), np.abs(fs - fs_ref).max()), flush=True)
    assert err.max() <= 1e-3
    assert np.abs(fs - fs_ref).max() <= 1e-4


def test_three_full_size_steps_with_variable_properties_match_the_oracle(config2, orc):
    """k(T) of both materials, interface factors h(T) and h(t), in the benchmark's
    launch shape (512-node blocks), against the oracle's variable-property run."""
    from paper_1005_3158_amd import castfem as cf
    vp = dict(k_of_T=[[(550.0, 180.0), (620.0, 150.0), (700.0, 95.0)], [(0.0, 0.4), (700.0, 1.2)]],
              h_of_T=[(100.0, 3.0), (650.0, 0.5)], h_of_t=[(0.0, 1.0), (0.5, 0.3), (1.5, 1.5)])
    p = dict(config2, varprops=vp)
    props = orc.VarProps(2, **vp)
    dt = 0.9 * orc.stable_dt_var(p, props)
    s = cf.Solver(p, precision=cf.FEM_PREC_FP32_KAHAN, lds_bytes=cf.lds_for_nodes(BLOCK_NODES))
    try:
        s.step(dt, 3)
        T = s.T()
    finally:
        s.close()
    _, T_ref, _ = orc.run_var(p, props, dt, 3)
    err = np.abs(T - T_ref)
    print("variable properties: max|T - oracle| %.3e K" % err.max(), flush=True)
    assert err.max() <= 1e-3


def test_full_size_nonmatching_contact(orc):
    """The contact workload of the benchmark (16.3M tets, 159,744 contact faces): every
    sister equal to the oracle's all-pairs search, and two steps against the oracle."""
    from paper_1005_3158_amd import castfem as cf
    p = configs.tet_casting_nonmatching(n_cast=96, n_mold=128, jitter=0.15)
    nf = p["contact_faces"].shape[0]
    s = cf.Solver(p, precision=cf.FEM_PREC_FP32_KAHAN, lds_bytes=cf.lds_for_nodes(BLOCK_NODES))
    try:
        dt = 0.9 * s.stable_dt()
        sis = cf.fem_get_sisters(s.ctx, nf)
        s.step(dt, 2)
        T = s.T()
    finally:
        s.close()
    P = orc.Problem(p)
    assert np.array_equal(sis, P.sisters)
    _, T_ref, _ = orc.run(P, dt, 2)
    err = np.abs(T - T_ref)
    print("non-matching contact, %d faces: max|T - oracle| %.3e K" % (nf, err.max()), flush=True)
    assert err.max() <= 1e-3


def test_four_hundred_full_size_steps_keep_energy_and_are_reproducible(config2, orc):
    dt = 0.9 * orc.stable_dt(config2)
    H = []
    for run in range(2):
        s = _solver(config2)
        try:
            s.step(dt, 400)
            e = s.energy()
            H.append(s.H())
            print("run %d after 400 steps: energy residual %.2e, T in [%.3f, %.3f] K, %d liquid nodes" %
                  (run, e["residual"], e["T_min"], e["T_max"], e["n_liquid"]), flush=True)
            assert e["nonfinite"] == 0 and np.all(np.isfinite(H[-1]))
            assert e["residual"] <= 1e-9
        finally:
            s.close()
    assert np.array_equal(H[0], H[1])


def test_full_size_batch_matches_sampled_scenarios_run_alone(orc):
    """The 256-scenario batch (about 5.5e7 tets, 1.06e7 nodes) as the benchmark runs it
    (autotuned block size, per-scenario dt): the smallest, the median and the largest
    scenario against the oracle run on that scenario alone, at every node, and every
    scenario's FP64 energy balance."""
    from paper_1005_3158_amd import castfem as cf
    b = configs.batch()
    sc = b["meta"]["scenarios"]
    s = cf.Solver(b, precision=cf.FEM_PREC_FP32_KAHAN, scatter=cf.FEM_SCATTER_LDS_BLOCKED)
    try:
        print("config 3: %d tets, %d nodes, %d blocks of <= %d nodes" % (s.n_elems, s.n_nodes, s.report["n_blocks"],
                                                                        s.report["max_local_nodes"]), flush=True)
        dt = 0.9 * s.stable_dt_scenarios()
        steps = 20
        s.step_batch(dt, steps)
        T, fs = s.T(), s.fs()
        reps = s.energy_scenarios()
    finally:
        s.close()
    assert max(r["residual"] for r in reps) <= 1e-9
    assert all(r["nonfinite"] == 0 for r in reps)
    sizes = np.array([sp["elem1"] - sp["elem0"] for sp in sc])
    order = np.argsort(sizes)
    for k in (order[0], order[len(order) // 2], order[-1]):
        sp = sc[k]
        mold = (sp["k_mold"],) + configs.SAND[1:]
        p = configs.tet_casting(n=sp["n"], region="cube", jitter_seed=sp["seed"], perm_seed=sp["seed"],
                                T_pour=sp["T_pour"], h_interface=sp["h_interface"], alloy=configs.ALLOY, mold=mold)
        _, T_ref, fs_ref = orc.run(p, dt[k], steps)
        err = float(np.max(np.abs(T[sp["node0"]:sp["node1"]] - T_ref)))
        print("scenario %d (%d tets, dt %.3e s): max|T - oracle| %.3e K" % (k, sizes[k], dt[k], err), flush=True)
        assert err <= 1e-3
        assert float(np.max(np.abs(fs[sp["node0"]:sp["node1"]] - fs_ref))) <= 1e-4
