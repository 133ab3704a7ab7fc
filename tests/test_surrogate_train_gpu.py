"""Training of the surrogate on trajectories of the GPU solver (a reduced set of
config-4 chill trajectories), what it gains over the linear extrapolation it
corrects, and the accelerated run judged by the plain one.

The held-out truth comes from the FP64 oracle."""
import numpy as np
import pytest

from castgen import configs

pytestmark = pytest.mark.gpu

TRAIN_SEEDS = list(range(5000, 5016))
HELD_OUT = 5500
MAX_SNAP = 160


def _cf():
    from paper_1005_3158_amd import castfem as cf
    return cf


def _fixed_layout(cf):
    """FP32 blocked step with a pinned block size: solvers compared bit for bit must
    share one partition (the autotuner times its candidates and may pick another)."""
    return dict(precision=cf.FEM_PREC_FP32_KAHAN, lds_bytes=cf.lds_for_nodes(256))


def generate(solver, dt, max_snap):
    """States H^{16k}, H^{16k+1}, H^{16k+2} of every scenario until all are solid (or max_snap)."""
    import torch
    N = solver.n_nodes
    S = torch.empty((max_snap + 1, 3, N), dtype=torch.float32, device=solver.device)
    k = 0
    while k < max_snap:
        for j in range(3):
            solver.snapshot_H(S[k, j])
            solver.step_batch(dt, 1 if j < 2 else 14)
        k += 1
        if all(r["n_liquid"] == 0 for r in solver.energy_scenarios()):
            break
    solver.snapshot_H(S[k, 0])
    return S, k


@pytest.fixture(scope="module")
def trained():
    cf = _cf()
    b = configs.chill_batch(TRAIN_SEEDS)
    solver = cf.Solver(b, precision=cf.FEM_PREC_FP32_KAHAN)
    dt = 0.9 * solver.stable_dt_scenarios()
    S, n = generate(solver, dt, MAX_SNAP)
    sur = cf.Surrogate(solver, layers=3, max_samples=1, train=True, seed=11)
    losses = sur.train(S[0, 0], S[0, 1], S[0, 2], S[1, 0], 3 * solver.n_nodes, n, batch=1, epochs=30,
                       lr=2e-3, lr_final=2e-5, seed=3)
    params = sur.params()
    sur.close()
    solver.close()
    print("samples %d, loss per epoch %s" % (n, np.array2string(losses, precision=3)))
    return dict(params=params, losses=losses, n=n)


def test_training_reduces_the_loss(trained):
    L = trained["losses"]
    assert np.all(np.isfinite(L)) and trained["n"] >= 100
    assert L[-1] < 0.2 * L[0]


def test_trained_network_beats_linear_extrapolation_on_held_out_data(trained, orc):
    import torch
    cf = _cf()
    p = configs.config4_trajectory(HELD_OUT)
    dt = 0.9 * orc.stable_dt(p)
    starts = [64, 480, 960, 1440]
    H, at = {0: orc.initial_H(p)}, 0
    for n0 in starts:
        for n in (n0, n0 + 1, n0 + 2, n0 + 16):
            H[n], _, _ = orc.run(p, dt, n - at, H=H[at])
            at = n
    s = cf.Solver(p, **_fixed_layout(cf))
    s.step(dt, 0)
    sur = cf.Surrogate(s, layers=3, max_samples=len(starts))
    perm = s.node_perm()
    N = s.n_nodes

    def dev(states):
        a = np.empty((len(states), N), np.float32)
        for q, h in enumerate(states):
            a[q, perm] = h
        return torch.from_numpy(a).to(s.device)

    H0 = dev([H[n] for n in starts])
    H1 = dev([H[n + 1] for n in starts])
    H2 = dev([H[n + 2] for n in starts])
    out = torch.empty(len(starts) * N, dtype=torch.float64, device=s.device)
    errs = {}
    for name, params in (("extrapolation", np.zeros_like(trained["params"])), ("trained", trained["params"])):
        sur.set_params(params)
        sur.predict(H0, H1, H2, out, stride=N, slots=len(starts))
        got = out.cpu().numpy().reshape(len(starts), N)[:, perm]
        e = []
        for q, n0 in enumerate(starts):
            T_pred, _ = orc.state_T(p, got[q])
            T_true, _ = orc.state_T(p, H[n0 + 16])
            e.append(float(np.max(np.abs(T_pred - T_true))))
        errs[name] = np.array(e)
        print("%-13s max |T - T_plain| after one jump: %s K" % (name, np.array2string(errs[name], precision=4)))
    sur.close()
    s.close()
    assert np.mean(errs["trained"]) < 0.5 * np.mean(errs["extrapolation"])


def test_accelerated_run_against_the_plain_run(trained, orc):
    cf = _cf()
    p = configs.config4_trajectory(HELD_OUT)
    dt = 0.9 * orc.stable_dt(p)
    plain = cf.Solver(p, **_fixed_layout(cf))
    rp = plain.advance(dt, 200000, None, until_solid=True)
    acc = cf.Solver(p, **_fixed_layout(cf))
    sur = cf.Surrogate(acc, layers=3)
    sur.set_params(trained["params"])
    ra = acc.advance(dt, 200000, sur, until_solid=True)
    ref = cf.Solver(p, **_fixed_layout(cf))
    ref.step(dt, ra["steps"])
    err = float(np.max(np.abs(acc.T() - ref.T())))
    print("plain: %d steps %.3f s; surrogate: %d steps (%d computed, %d/%d jumps kept) %.3f s; "
          "max |T_sur - T_plain| = %.3f K; energy residual %.2e"
          % (rp["steps"], rp["wall_seconds"], ra["steps"], ra["plain_steps"], ra["jumps_accepted"],
             ra["jumps_accepted"] + ra["jumps_rejected"], ra["wall_seconds"], err, acc.energy()["residual"]))
    assert rp["solid"] == 1 and ra["solid"] == 1
    assert ra["jumps_accepted"] > 0 and ra["plain_steps"] < rp["steps"]
    assert abs(ra["steps"] - rp["steps"]) <= 16 * 8
    assert err <= 2.0
    sur.close()
    for s in (plain, acc, ref):
        s.close()
