"""Write the full-size reference samples of tests/golden/ from the FP64 oracle.

Calls only castgen (inputs) and oracle/ (the CPU reference, its multi-threaded
run, which is bitwise the serial one).  Run from the repository root:

    python tests/golden/make_full_size_golden.py config2   # ~40 min on 8 cores
    python tests/golden/make_full_size_golden.py config5   # ~40 min on 8 cores

config2: the 128^3 cast/mould mesh (12,582,912 tets) over its 2000 steps at
    dt = 0.9 x the oracle's stability bound.  Snapshots at steps 1000 and 2000
    hold every node whose oracle temperature lies in the liquidus-front band
    [T_sol - 5, T_liq + 5] and a seeded sample of all nodes.
config5: the 256^3 mesh with eight casting boxes (100,663,296 tets) over its
    first 100 steps.  The snapshot holds a seeded sample of the nodes the
    100 steps moved by more than 1e-3 K and a seeded sample of all nodes.
Each file also stores the step size, the oracle's energy diagnostics at the
snapshot steps and a digest of the inputs, so a change of the generator shows.
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from castgen import configs  # noqa: E402
from oracle import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
BAND = (configs.ALLOY[3] - 5.0, configs.ALLOY[4] + 5.0)


def input_digest(p):
    h = hashlib.sha256()
    for k in ("xyz", "conn", "elem_mat", "T0", "if_a", "if_b", "if_h", "materials"):
        h.update(np.ascontiguousarray(p[k]).tobytes())
    return h.hexdigest()[:32]


def snapshot(out, tag, step, H, P, diag, T0, sample, active_sample=None):
    T, fs = oracle.state_T(P, H)
    idx = [sample]
    if active_sample is not None:
        idx.append(active_sample(T))
    band = np.nonzero((T >= BAND[0]) & (T <= BAND[1]))[0]
    idx.append(band)
    idx = np.unique(np.concatenate(idx)).astype(np.int64)
    out[tag + "_step"] = np.int64(step)
    out[tag + "_idx"] = idx
    out[tag + "_T"] = T[idx]
    out[tag + "_fs"] = fs[idx]
    out[tag + "_band"] = band.astype(np.int64)
    out[tag + "_E"] = np.float64(diag[-1, oracle.D_E])
    out[tag + "_T_range"] = np.array([T.min(), T.max()])
    print("%s: step %d, %d band nodes, %d stored nodes, T in [%.4f, %.4f]"
          % (tag, step, band.size, idx.size, T.min(), T.max()), flush=True)


def run_config2():
    p = configs.config2()
    P = oracle.Problem(p)
    dt = 0.9 * oracle.stable_dt(P)
    N = p["xyz"].shape[0]
    sample = np.sort(np.random.default_rng(20).choice(N, 20000, replace=False))
    out = {"dt": np.float64(dt), "digest": np.array(input_digest(p)), "threads": np.int64(oracle.omp_threads())}
    H = oracle.initial_H(P)
    done, Qcum = 0, 0.0
    t0 = time.time()
    for stop in (250, 500, 750, 1000, 1250, 1500, 1750, 2000):
        H, _, _, D = oracle.run_omp(P, dt, stop - done, H=H, diag=True)
        Qcum += D[-1, oracle.D_QCUM]
        done = stop
        print("step %d (%.0f s)" % (done, time.time() - t0), flush=True)
        if stop in (1000, 2000):
            snapshot(out, "s%d" % stop, stop, H, P, D, p["T0"], sample)
            out["s%d_Qcum" % stop] = np.float64(Qcum)
    np.savez_compressed(os.path.join(HERE, "config2_front.npz"), **out)


def run_config5():
    p = configs.config5()
    P = oracle.Problem(p)
    t0 = time.time()
    dt = 0.9 * oracle.stable_dt(P)
    print("stability bound %.6e s (%.0f s)" % (dt / 0.9, time.time() - t0), flush=True)
    N = p["xyz"].shape[0]
    sample = np.sort(np.random.default_rng(50).choice(N, 20000, replace=False))
    T0 = oracle.state_T(P, oracle.initial_H(P))[0]

    def active(T):
        moved = np.nonzero(np.abs(T - T0) > 1e-3)[0]
        print("nodes moved by more than 1e-3 K: %d" % moved.size, flush=True)
        return np.sort(np.random.default_rng(51).choice(moved, min(40000, moved.size), replace=False))

    out = {"dt": np.float64(dt), "digest": np.array(input_digest(p)), "threads": np.int64(oracle.omp_threads())}
    H, _, _, D = oracle.run_omp(P, dt, 100, diag=True)
    print("100 steps (%.0f s)" % (time.time() - t0), flush=True)
    snapshot(out, "s100", 100, H, P, D, T0, sample, active)
    out["s100_Qcum"] = np.float64(D[-1, oracle.D_QCUM])
    np.savez_compressed(os.path.join(HERE, "config5_spot.npz"), **out)


if __name__ == "__main__":
    {"config2": run_config2, "config5": run_config5}[sys.argv[1]]()
