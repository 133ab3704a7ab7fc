"""ctypes front end of the FP64 CPU oracle (castfem_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark are the only callers.  The product path
never imports this module.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "castfem_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ORC_NDIAG = 9
D_E, D_LATENT, D_Q, D_QCUM, D_TMIN, D_TMAX, D_NLIQ, D_NONFINITE, D_RESID = range(9)


SRC_OMP = os.path.join(HERE, "castfem_oracle_omp.c")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(force=False):
    """Compile the oracle with gcc (plain -O2, no fast-math), and the same source
    once more with its multi-threaded run (bitwise the serial run)."""
    for src, lib_, extra in ((SRC, LIB, []), (SRC_OMP, LIB_OMP, ["-fopenmp"])):
        deps = (SRC, src, os.path.join(HERE, "castfem_oracle.h"))
        if force or not os.path.exists(lib_) or os.path.getmtime(lib_) < max(os.path.getmtime(d) for d in deps):
            tmp = lib_ + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared"] + extra + ["-o", tmp, src, "-lm"])
            os.replace(tmp, lib_)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB)
        d = C.c_double
        _lib.orc_H_of_T.restype = d
        _lib.orc_T_of_H.restype = d
        _lib.orc_fs_of_H.restype = d
        for f in (_lib.orc_H_of_T, _lib.orc_T_of_H, _lib.orc_fs_of_H):
            f.argtypes = [C.c_void_p, d]
    return _lib


class _Problem(C.Structure):
    _fields_ = [
        ("elem_type", C.c_int32), ("n_nodes", C.c_int64), ("xyz", C.c_void_p),
        ("n_elems", C.c_int64), ("conn", C.c_void_p), ("elem_mat", C.c_void_p),
        ("n_mat", C.c_int32), ("materials", C.c_void_p),
        ("n_dir", C.c_int64), ("dir_nodes", C.c_void_p), ("dir_T", C.c_void_p),
        ("n_flux", C.c_int64), ("flux_npf", C.c_int32), ("flux_faces", C.c_void_p),
        ("flux_q", C.c_void_p), ("flux_h", C.c_void_p), ("flux_Tinf", C.c_void_p),
        ("n_if", C.c_int64), ("if_a", C.c_void_p), ("if_b", C.c_void_p), ("if_h", C.c_void_p),
        ("n_contact", C.c_int64), ("contact_faces", C.c_void_p), ("contact_side", C.c_void_p),
        ("contact_h", C.c_void_p), ("contact_sister", C.c_void_p),
    ]


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a.size else None


class Problem:
    """Holds contiguous copies of a problem dict and the C struct pointing at them.
    Contact faces (non-matching meshes) get their sisters by the oracle's brute-force
    search when the problem is built."""

    def __init__(self, prob):
        f8 = lambda k: np.ascontiguousarray(prob[k], dtype=np.float64)
        i4 = lambda k: np.ascontiguousarray(prob[k], dtype=np.int32)
        self.keep = dict(
            xyz=f8("xyz"), conn=i4("conn"), elem_mat=i4("elem_mat"), materials=f8("materials"),
            dir_nodes=i4("dirichlet_nodes"), dir_T=f8("dirichlet_T"),
            flux_faces=i4("flux_faces"), flux_q=f8("flux_q"), flux_h=f8("flux_h"),
            flux_Tinf=f8("flux_Tinf"), if_a=i4("if_a"), if_b=i4("if_b"), if_h=f8("if_h"))
        k = self.keep
        self.T0 = np.ascontiguousarray(prob["T0"], dtype=np.float64)
        self.n_nodes = k["xyz"].shape[0]
        ff = k["flux_faces"]
        self.s = _Problem(
            int(prob["elem_type"]), self.n_nodes, _ptr(k["xyz"]),
            k["conn"].shape[0], _ptr(k["conn"]), _ptr(k["elem_mat"]),
            k["materials"].shape[0], _ptr(k["materials"]),
            k["dir_nodes"].size, _ptr(k["dir_nodes"]), _ptr(k["dir_T"]),
            ff.shape[0] if ff.size else 0, ff.shape[1] if ff.ndim == 2 else 3, _ptr(ff),
            _ptr(k["flux_q"]), _ptr(k["flux_h"]), _ptr(k["flux_Tinf"]),
            k["if_a"].shape[0] if k["if_a"].size else 0, _ptr(k["if_a"]), _ptr(k["if_b"]),
            _ptr(k["if_h"]), 0, None, None, None, None)
        cf = prob.get("contact_faces")
        if cf is not None and np.size(cf):
            k["contact_faces"] = np.ascontiguousarray(cf, dtype=np.int32).reshape(-1, 3)
            k["contact_side"] = np.ascontiguousarray(prob["contact_side"], dtype=np.int32)
            k["contact_h"] = np.ascontiguousarray(prob["contact_h"], dtype=np.float64)
            n = k["contact_faces"].shape[0]
            self.s.n_contact = n
            self.s.contact_faces = _ptr(k["contact_faces"])
            self.s.contact_side = _ptr(k["contact_side"])
            self.s.contact_h = _ptr(k["contact_h"])
            k["contact_sister"] = np.zeros(n, np.int32)
            _check(lib().orc_contact_sisters(C.byref(self.s), _ptr(k["contact_sister"])), "contact_sisters")
            self.s.contact_sister = _ptr(k["contact_sister"])
        self.sisters = k.get("contact_sister")

    @property
    def ref(self):
        return C.byref(self.s)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))


def _as_problem(p):
    return p if isinstance(p, Problem) else Problem(p)


def tet_ke(x, k):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(12)
    Ke = np.zeros(16)
    V = C.c_double()
    _check(lib().orc_tet_ke(_ptr(x), C.c_double(k), _ptr(Ke), C.byref(V)), "tet_ke")
    return Ke.reshape(4, 4), V.value


def hex_ke(x, k):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(24)
    Ke = np.zeros(64)
    V = C.c_double()
    _check(lib().orc_hex_ke(_ptr(x), C.c_double(k), _ptr(Ke), C.byref(V)), "hex_ke")
    return Ke.reshape(8, 8), V.value


def elem_mass(elem_type, x, rho):
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    m = np.zeros(elem_type)
    _check(lib().orc_elem_mass(C.c_int32(elem_type), _ptr(x), C.c_double(rho), _ptr(m)), "elem_mass")
    return m


def _mat(mat):
    a = np.ascontiguousarray(mat, dtype=np.float64).reshape(6)
    return a, _ptr(a)


def H_of_T(mat, T):
    a, p = _mat(mat)
    return np.array([lib().orc_H_of_T(p, float(t)) for t in np.ravel(T)])


def T_of_H(mat, H):
    a, p = _mat(mat)
    return np.array([lib().orc_T_of_H(p, float(h)) for h in np.ravel(H)])


def fs_of_H(mat, H):
    a, p = _mat(mat)
    return np.array([lib().orc_fs_of_H(p, float(h)) for h in np.ravel(H)])


def lumped_mass(prob):
    P = _as_problem(prob)
    m = np.zeros(P.n_nodes)
    _check(lib().orc_lumped_mass(P.ref, _ptr(m)), "lumped_mass")
    return m


def node_material(prob):
    P = _as_problem(prob)
    nm = np.zeros(P.n_nodes, np.int32)
    _check(lib().orc_node_material(P.ref, _ptr(nm)), "node_material")
    return nm


def residual(prob, T):
    P = _as_problem(prob)
    T = np.ascontiguousarray(T, dtype=np.float64)
    r = np.zeros(P.n_nodes)
    _check(lib().orc_residual(P.ref, _ptr(T), _ptr(r)), "residual")
    return r


def stable_dt(prob):
    P = _as_problem(prob)
    dt = C.c_double()
    _check(lib().orc_stable_dt(P.ref, C.byref(dt)), "stable_dt")
    return dt.value


def initial_H(prob, T0=None):
    P = _as_problem(prob)
    if T0 is None:
        T0 = P.T0
    T0 = np.ascontiguousarray(T0, dtype=np.float64)
    H = np.zeros(P.n_nodes)
    _check(lib().orc_initial_H(P.ref, _ptr(T0), _ptr(H)), "initial_H")
    return H


def state_T(prob, H):
    P = _as_problem(prob)
    H = np.ascontiguousarray(H, dtype=np.float64)
    T = np.zeros(P.n_nodes)
    fs = np.zeros(P.n_nodes)
    _check(lib().orc_state_T(P.ref, _ptr(H), _ptr(T), _ptr(fs)), "state_T")
    return T, fs


def run(prob, dt, n_steps, H=None, diag=False):
    """n explicit steps from H (default: the initial state of prob).  Returns (H, T, fs[, diag])."""
    P = _as_problem(prob)
    H = initial_H(P) if H is None else np.array(H, dtype=np.float64)
    D = np.zeros((n_steps + 1, ORC_NDIAG)) if diag else None
    _check(lib().orc_run(P.ref, C.c_double(dt), C.c_int64(n_steps), _ptr(H),
                         _ptr(D) if diag else None), "run")
    T, fs = state_T(P, H)
    return (H, T, fs, D) if diag else (H, T, fs)


_lib_omp = None


def _omp():
    global _lib_omp
    if _lib_omp is None:
        build()
        _lib_omp = C.CDLL(LIB_OMP)
        _lib_omp.orc_omp_threads.restype = C.c_int32
    return _lib_omp


def omp_threads():
    """Threads the multi-threaded run uses by default (OpenMP's own count)."""
    return int(_omp().orc_omp_threads())


def run_omp(prob, dt, n_steps, H=None, diag=False, threads=0):
    """run() over all host cores (threads = 0: OpenMP's default), bitwise equal to run():
    the same element routines, each node's element sum in the serial order."""
    P = _as_problem(prob)
    H = initial_H(P) if H is None else np.array(H, dtype=np.float64)
    D = np.zeros((n_steps + 1, ORC_NDIAG)) if diag else None
    _check(_omp().orc_run_omp(P.ref, C.c_double(dt), C.c_int64(n_steps), _ptr(H),
                              _ptr(D) if diag else None, C.c_int32(threads)), "run_omp")
    T, fs = state_T(P, H)
    return (H, T, fs, D) if diag else (H, T, fs)


def run_partitioned(prob, elem_part, n_parts, dt, n_steps, H=None):
    P = _as_problem(prob)
    H = initial_H(P) if H is None else np.array(H, dtype=np.float64)
    ep = np.ascontiguousarray(elem_part, dtype=np.int32)
    _check(lib().orc_run_partitioned(P.ref, C.c_int32(n_parts), _ptr(ep), C.c_double(dt),
                                     C.c_int64(n_steps), _ptr(H)), "run_partitioned")
    return H


def lemmon_capacity(x, mat, T, H):
    """Lemmon's dH/dT of one linear tetrahedron (Eq. 7) from nodal T and H."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(12)
    a, pm = _mat(mat)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(4)
    H = np.ascontiguousarray(H, dtype=np.float64).reshape(4)
    c = C.c_double()
    _check(lib().orc_lemmon_capacity(_ptr(x), pm, _ptr(T), _ptr(H), C.byref(c)), "lemmon_capacity")
    return c.value


def apparent_capacity(prob, H):
    """Row-sum lumped apparent capacitance C_i (J/K) of the state H (tetrahedra)."""
    P = _as_problem(prob)
    H = np.ascontiguousarray(H, dtype=np.float64)
    Cn = np.zeros(P.n_nodes)
    _check(lib().orc_apparent_capacity(P.ref, _ptr(H), _ptr(Cn)), "apparent_capacity")
    return Cn


def run_apparent(prob, dt, n_steps, H=None, diag=False):
    """n explicit steps of the apparent-heat-capacity mode (Eq. 6-7, Eq. 14) from H
    (default: the initial state).  Returns (H, T, fs[, diag]) as run()."""
    P = _as_problem(prob)
    H = initial_H(P) if H is None else np.array(H, dtype=np.float64)
    D = np.zeros((n_steps + 1, ORC_NDIAG)) if diag else None
    _check(lib().orc_run_apparent(P.ref, C.c_double(dt), C.c_int64(n_steps), _ptr(H),
                                  _ptr(D) if diag else None), "run_apparent")
    T, fs = state_T(P, H)
    return (H, T, fs, D) if diag else (H, T, fs)


def contact_sisters(prob):
    """Sister face of every contact face (brute-force closest centroid, other side)."""
    return _as_problem(prob).sisters


def contact_sisters_of(prob, faces):
    """Sisters of the listed contact faces only, by the same brute-force search
    (for meshes whose all-pairs search would take long).  prob: a problem dict."""
    x = np.ascontiguousarray(prob["xyz"], dtype=np.float64)
    cf = np.ascontiguousarray(prob["contact_faces"], dtype=np.int32).reshape(-1, 3)
    side = np.ascontiguousarray(prob["contact_side"], dtype=np.int32)
    s = _Problem()
    s.elem_type, s.n_nodes, s.xyz = 4, x.shape[0], _ptr(x)
    s.n_contact, s.contact_faces, s.contact_side = cf.shape[0], _ptr(cf), _ptr(side)
    f = np.ascontiguousarray(faces, dtype=np.int64)
    out = np.zeros(f.size, np.int32)
    _check(lib().orc_contact_sisters_of(C.byref(s), C.c_int64(f.size), _ptr(f), _ptr(out)), "contact_sisters_of")
    return out


# ------------------------------------------- temperature- and time-dependent properties
ORC_TABLE = 17


class _VarProps(C.Structure):
    _fields_ = [("k_of_T", C.c_void_p), ("h_of_T", C.c_void_p), ("h_of_t", C.c_void_p), ("dir_of_t", C.c_void_p),
                ("dir_sched", C.c_void_p)]


def table(points):
    """[(x, y), ...] (at most 8, increasing x) -> the oracle's 17-double table; None -> n = 0."""
    t = np.zeros(ORC_TABLE)
    if points is not None and len(points):
        pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
        t[0] = pts.shape[0]
        t[1:1 + pts.shape[0]] = pts[:, 0]
        t[9:9 + pts.shape[0]] = pts[:, 1]
    return t


class VarProps:
    """k_of_T: per material a point list or None; h_of_T, h_of_t, dir_of_t: point lists or None;
    dir_sched: per fixed node (in the order of dirichlet_nodes) a point list (t, T) or None."""

    def __init__(self, n_mat, k_of_T=None, h_of_T=None, h_of_t=None, dir_of_t=None, dir_sched=None):
        self.k = np.concatenate([table(k_of_T[q] if k_of_T else None) for q in range(n_mat)])
        self.hT, self.ht, self.dt = table(h_of_T), table(h_of_t), table(dir_of_t)
        self.sched = None if dir_sched is None else np.concatenate([table(s) for s in dir_sched] or [np.zeros(0)])
        self.s = _VarProps(_ptr(self.k), _ptr(self.hT), _ptr(self.ht), _ptr(self.dt),
                           _ptr(self.sched) if self.sched is not None and self.sched.size else None)

    @property
    def ref(self):
        return C.byref(self.s)


def table_value(points, x):
    lib().orc_table.restype = C.c_double
    t = table(points)
    return lib().orc_table(_ptr(t), C.c_double(x))


def residual_var(prob, props, T, t):
    P = _as_problem(prob)
    T = np.ascontiguousarray(T, dtype=np.float64)
    r = np.zeros(P.n_nodes)
    _check(lib().orc_residual_var(P.ref, props.ref, _ptr(T), C.c_double(t), _ptr(r)), "residual_var")
    return r


def stable_dt_var(prob, props):
    P = _as_problem(prob)
    dt = C.c_double()
    _check(lib().orc_stable_dt_var(P.ref, props.ref, C.byref(dt)), "stable_dt_var")
    return dt.value


def initial_H_var(prob, props, t0=0.0):
    """Initial enthalpy with every fixed node at f(t0) + shift(t0) (f: its schedule, else T_D)."""
    P = _as_problem(prob)
    H = initial_H(P)
    if P.keep["dir_nodes"].size and (props.dt[0] > 0 or props.sched is not None):
        lib().orc_table.restype = C.c_double
        shift = lib().orc_table(_ptr(props.dt), C.c_double(t0)) if props.dt[0] > 0 else 0.0
        nm = node_material(P)
        mats = P.keep["materials"]
        for d, (i, TD) in enumerate(zip(P.keep["dir_nodes"], P.keep["dir_T"])):
            if props.sched is not None:
                TD = lib().orc_table(_ptr(props.sched[ORC_TABLE * d:ORC_TABLE * (d + 1)]), C.c_double(t0))
            H[i] = H_of_T(mats[nm[i]], TD + shift)[0]
    return H


def run_var(prob, props, dt, n_steps, H=None, t0=0.0, diag=False):
    """n explicit steps with temperature- and time-dependent properties from time t0.
    Returns (H, T, fs[, diag]) as run()."""
    P = _as_problem(prob)
    H = initial_H_var(P, props, t0) if H is None else np.array(H, dtype=np.float64)
    D = np.zeros((n_steps + 1, ORC_NDIAG)) if diag else None
    _check(lib().orc_run_var(P.ref, props.ref, C.c_double(t0), C.c_double(dt), C.c_int64(n_steps), _ptr(H),
                             _ptr(D) if diag else None), "run_var")
    T, fs = state_T(P, H)
    return (H, T, fs, D) if diag else (H, T, fs)
