"""ctypes binding of libcastfem.so: the C functions under their own names, plus
`Solver`, which owns the device buffers through torch.

Every step of the casting path runs in the HIP library; this module only
marshals arguments.  If the library is missing the import fails loudly.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcastfem.so")

FEM_OK = 0
ERRORS = {-1: "FEM_E_INVALID_ARG", -2: "FEM_E_MESH", -3: "FEM_E_STATE", -4: "FEM_E_UNSTABLE",
          -5: "FEM_E_NONFINITE", -6: "FEM_E_HIP", -7: "FEM_E_UNSUPPORTED"}
FEM_TET4, FEM_HEX8 = 4, 8
FEM_PREC_FP64, FEM_PREC_FP32_KAHAN = 0, 1
FEM_ORDER_NONE, FEM_ORDER_RCM, FEM_ORDER_MORTON, FEM_ORDER_HILBERT = 0, 1, 2, 3
FEM_SCATTER_GLOBAL_ATOMIC, FEM_SCATTER_LDS_BLOCKED, FEM_SCATTER_COLORED = 0, 1, 2
FEM_LATENT_ENTHALPY, FEM_LATENT_APPARENT = 0, 1
# LDS bytes per block-local node of the blocked element kernel, by precision
LDS_PER_NODE = {FEM_PREC_FP64: 48, FEM_PREC_FP32_KAHAN: 28}


LDS_PER_NODE_APPARENT = {FEM_PREC_FP64: 52, FEM_PREC_FP32_KAHAN: 32}


def lds_for_nodes(nodes, precision=FEM_PREC_FP32_KAHAN, apparent=False):
    """lds_bytes option that caps an LDS block at `nodes` local nodes (apparent:
    for the apparent-heat-capacity form, whose kernels hold more per node)."""
    return (LDS_PER_NODE_APPARENT if apparent else LDS_PER_NODE)[precision] * int(nodes)

EXPORTS = [
    "fem_create", "fem_destroy", "fem_last_error", "fem_set_stream", "fem_upload_mesh", "fem_set_materials",
    "fem_set_dirichlet", "fem_set_flux_faces", "fem_set_interface", "fem_set_initial_T", "fem_finalize",
    "fem_query_buffers", "fem_bind_buffers", "fem_get_report", "fem_stable_dt", "fem_step", "fem_step_no_alloc", "fem_read_T",
    "fem_read_fs", "fem_read_H", "fem_energy", "fem_read_state", "fem_write_state", "fem_get_node_perm",
    "fem_time_kernels", "fem_copy_kernel", "fem_copy_kernel_nt", "fem_set_scenarios", "fem_stable_dt_scenarios", "fem_step_batch",
    "fem_energy_scenarios", "fem_sur_create", "fem_sur_destroy", "fem_sur_query_buffers", "fem_sur_bind_buffers",
    "fem_sur_n_params", "fem_sur_get_params", "fem_sur_set_params", "fem_sur_features", "fem_sur_loss_grad",
    "fem_sur_train", "fem_sur_predict", "fem_snapshot_H", "fem_advance", "fem_sur_generate", "fem_sur_save",
    "fem_sur_load", "fem_set_contact", "fem_get_sisters", "fem_set_variable_properties",
    "fem_set_dirichlet_schedule",
]


class FemError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__("%s failed: %s (%s)" % (fn, msg, ERRORS.get(code, code)))
        self.code = code


class fem_table(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad", C.c_int32), ("x", C.c_double * 8), ("y", C.c_double * 8)]


def make_table(points):
    """[(x, y), ...] with increasing x (at most 8) -> fem_table; None -> n = 0."""
    t = fem_table()
    if points is not None:
        for j, (x, y) in enumerate(points):
            t.x[j], t.y[j] = x, y
        t.n = len(points)
    return t


class fem_options(C.Structure):
    _fields_ = [("device", C.c_int32), ("precision", C.c_int32), ("ordering", C.c_int32),
                ("scatter", C.c_int32), ("block_elems", C.c_int32), ("allow_unstable", C.c_int32),
                ("lds_bytes", C.c_int32), ("threads", C.c_int32), ("latent_model", C.c_int32),
                ("reserved", C.c_int32 * 7)]


class fem_material(C.Structure):
    _fields_ = [("k", C.c_double), ("rho", C.c_double), ("c", C.c_double), ("T_sol", C.c_double),
                ("T_liq", C.c_double), ("L", C.c_double)]


class fem_prep_report(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("n_blocks", C.c_int64),
                ("n_shared", C.c_int64), ("n_partials", C.c_int64), ("max_local_nodes", C.c_int64),
                ("n_colors", C.c_int64), ("bandwidth_before", C.c_int64), ("bandwidth_after", C.c_int64),
                ("block_elems", C.c_int64), ("shared_fraction", C.c_double), ("dt_bound", C.c_double),
                ("setup_seconds", C.c_double), ("contact_search_seconds", C.c_double), ("n_contact", C.c_int64),
                ("block_threads", C.c_int64), ("reserved", C.c_int64 * 1)]


class fem_buffer_desc(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("bytes", C.c_int64), ("alignment", C.c_int64)]


class fem_energy_report(C.Structure):
    _fields_ = [("E", C.c_double), ("E0", C.c_double), ("latent", C.c_double), ("Q_cum", C.c_double),
                ("residual", C.c_double), ("T_min", C.c_double), ("T_max", C.c_double),
                ("n_liquid", C.c_int64), ("nonfinite", C.c_int64), ("steps", C.c_int64), ("time", C.c_double)]


class fem_kernel_times(C.Structure):
    _fields_ = [("ms_element", C.c_double), ("ms_combine", C.c_double), ("launches_element", C.c_int64),
                ("launches_combine", C.c_int64), ("bytes_element", C.c_double), ("bytes_combine", C.c_double)]


class fem_sur_options(C.Structure):
    _fields_ = [("width", C.c_int32), ("layers", C.c_int32), ("horizon", C.c_int32), ("max_samples", C.c_int32),
                ("train", C.c_int32), ("loss", C.c_int32), ("extrapolation", C.c_int32), ("no_projection", C.c_int32),
                ("reserved", C.c_int32 * 4),
                ("seed", C.c_uint64)]


class fem_advance_report(C.Structure):
    _fields_ = [("steps", C.c_int64), ("plain_steps", C.c_int64), ("jumps_accepted", C.c_int64),
                ("jumps_rejected", C.c_int64), ("solid", C.c_int32), ("pad", C.c_int32),
                ("wall_seconds", C.c_double), ("max_residual", C.c_double), ("rejected_fs", C.c_int64),
                ("rejected_energy", C.c_int64), ("rejected_verify", C.c_int64), ("reserved", C.c_int64 * 1)]


def _as_dict(s):
    return {k: (list(getattr(s, k)) if k == "reserved" else getattr(s, k)) for k, _ in s._fields_ if k != "reserved"}


_lib = None


def lib():
    """Load libcastfem.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        # torch first: the process then holds torch's HIP runtime, which the
        # library resolves to as well (loading the library first would bring in
        # a second runtime, and torch's GPU calls then find no device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcastfem.so is not built: run __graft_entry__.build() "
                              "(or python paper_1005_3158_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        L.fem_last_error.restype = C.c_char_p
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "fem_create": [vp, vp], "fem_destroy": [vp], "fem_set_stream": [vp, vp],
            "fem_upload_mesh": [vp, i32, i64, vp, i64, vp, vp], "fem_set_materials": [vp, i32, vp],
            "fem_set_dirichlet": [vp, i64, vp, vp], "fem_set_flux_faces": [vp, i64, i32, vp, vp, vp, vp],
            "fem_set_interface": [vp, i64, vp, vp, vp], "fem_set_initial_T": [vp, vp],
            "fem_finalize": [vp, vp], "fem_query_buffers": [vp, vp, vp], "fem_bind_buffers": [vp, vp, i32],
            "fem_get_report": [vp, vp], "fem_stable_dt": [vp, vp], "fem_step": [vp, dp, i64],
            "fem_step_no_alloc": [vp, dp, i64],
            "fem_read_T": [vp, vp], "fem_read_fs": [vp, vp], "fem_read_H": [vp, vp], "fem_energy": [vp, vp],
            "fem_read_state": [vp, vp, vp], "fem_write_state": [vp, vp, i64], "fem_get_node_perm": [vp, vp],
            "fem_time_kernels": [vp, dp, i64, vp], "fem_copy_kernel": [vp, vp, vp, i64, i32, vp],
            "fem_copy_kernel_nt": [vp, vp, vp, i64, i32, vp],
            "fem_set_scenarios": [vp, i32, vp], "fem_stable_dt_scenarios": [vp, vp],
            "fem_step_batch": [vp, vp, i64], "fem_energy_scenarios": [vp, vp],
            "fem_sur_create": [vp, vp, vp], "fem_sur_destroy": [vp], "fem_sur_query_buffers": [vp, vp, vp],
            "fem_sur_bind_buffers": [vp, vp, i32], "fem_sur_n_params": [vp, vp],
            "fem_sur_get_params": [vp, vp, i64], "fem_sur_set_params": [vp, vp, i64],
            "fem_sur_features": [vp, vp, vp, vp, i64, i64, vp],
            "fem_sur_loss_grad": [vp, vp, vp, vp, vp, i64, i64, vp, vp],
            "fem_sur_train": [vp, vp, vp, vp, vp, i64, i64, i32, i32, C.c_float, C.c_float, C.c_uint64, vp],
            "fem_sur_predict": [vp, vp, vp, vp, i64, i64, vp], "fem_snapshot_H": [vp, vp],
            "fem_advance": [vp, vp, vp, i64, i32, dp, dp, dp, vp], "fem_sur_generate": [vp, vp, i64, i32, vp],
            "fem_sur_save": [vp, C.c_char_p], "fem_sur_load": [vp, C.c_char_p],
            "fem_set_contact": [vp, i64, vp, vp, vp], "fem_get_sisters": [vp, vp],
            "fem_set_variable_properties": [vp, i32, vp, vp, vp, vp],
            "fem_set_dirichlet_schedule": [vp, i32, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        _lib = L
    return _lib


def _call(name, *args):
    rc = getattr(lib(), name)(*args)
    if rc != FEM_OK:
        raise FemError(rc, name, lib().fem_last_error().decode())
    return rc


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


# ------------------------------------------------------------ same-name wrappers
def fem_create(opt=None):
    ctx = C.c_void_p()
    _call("fem_create", C.byref(ctx), C.byref(opt) if opt is not None else None)
    return ctx


def fem_destroy(ctx):
    _call("fem_destroy", ctx)


def fem_last_error():
    return lib().fem_last_error().decode()


def fem_set_stream(ctx, stream_ptr):
    _call("fem_set_stream", ctx, C.c_void_p(stream_ptr))


def fem_upload_mesh(ctx, elem_type, xyz, conn, elem_mat):
    xyz = np.ascontiguousarray(xyz, np.float64)
    conn = np.ascontiguousarray(conn, np.int32)
    em = np.ascontiguousarray(elem_mat, np.int32)
    _call("fem_upload_mesh", ctx, int(elem_type), xyz.shape[0], _p(xyz), conn.shape[0], _p(conn), _p(em))


def fem_set_materials(ctx, materials):
    m = np.ascontiguousarray(materials, np.float64).reshape(-1, 6)
    arr = (fem_material * m.shape[0])(*[fem_material(*row) for row in m])
    _call("fem_set_materials", ctx, m.shape[0], arr)


def fem_set_dirichlet(ctx, nodes, values):
    n = np.ascontiguousarray(nodes, np.int32)
    v = np.ascontiguousarray(values, np.float64)
    _call("fem_set_dirichlet", ctx, n.size, _p(n), _p(v))


def fem_set_flux_faces(ctx, faces, q, h, T_inf):
    f = np.ascontiguousarray(faces, np.int32)
    npf = f.shape[1] if f.ndim == 2 and f.size else 3
    nf = f.shape[0] if f.size else 0
    _call("fem_set_flux_faces", ctx, nf, npf, _p(f), _p(np.ascontiguousarray(q, np.float64)),
          _p(np.ascontiguousarray(h, np.float64)), _p(np.ascontiguousarray(T_inf, np.float64)))


def fem_set_interface(ctx, face_a, face_b, h):
    a = np.ascontiguousarray(face_a, np.int32)
    b = np.ascontiguousarray(face_b, np.int32)
    hh = np.ascontiguousarray(h, np.float64)
    _call("fem_set_interface", ctx, hh.size, _p(a), _p(b), _p(hh))


def fem_set_contact(ctx, faces, side, h):
    f = np.ascontiguousarray(faces, np.int32).reshape(-1, 3)
    sd = np.ascontiguousarray(side, np.int32)
    hh = np.ascontiguousarray(h, np.float64)
    _call("fem_set_contact", ctx, hh.size, _p(f), _p(sd), _p(hh))


def fem_set_variable_properties(ctx, n_mat, k_of_T=None, h_of_T=None, h_of_t=None, dir_of_t=None):
    """k_of_T: per material a point list or None; the others: point lists or None."""
    ks = (fem_table * n_mat)(*[make_table(k_of_T[q] if k_of_T else None) for q in range(n_mat)])
    tabs = [make_table(t) for t in (h_of_T, h_of_t, dir_of_t)]
    _call("fem_set_variable_properties", ctx, int(n_mat), C.cast(ks, C.c_void_p),
          *[C.cast(C.byref(t), C.c_void_p) for t in tabs])


def fem_set_dirichlet_schedule(ctx, times, values):
    """times: n common times; values: (fixed nodes x n) temperatures, in the order of fem_set_dirichlet."""
    t = np.ascontiguousarray(times, dtype=np.float64)
    v = np.ascontiguousarray(values, dtype=np.float64)
    _call("fem_set_dirichlet_schedule", ctx, int(t.size), _p(t), _p(v))


def fem_get_sisters(ctx, n):
    out = np.empty(n, np.int32)
    _call("fem_get_sisters", ctx, _p(out))
    return out


def fem_set_initial_T(ctx, T0):
    t = np.ascontiguousarray(T0, np.float64)
    _call("fem_set_initial_T", ctx, _p(t))


def fem_set_scenarios(ctx, material_scenario):
    ms = np.ascontiguousarray(material_scenario, np.int32)
    _call("fem_set_scenarios", ctx, int(ms.max()) + 1, _p(ms))


def fem_stable_dt_scenarios(ctx, n_scen):
    out = np.empty(n_scen, np.float64)
    _call("fem_stable_dt_scenarios", ctx, _p(out))
    return out


def fem_step_batch(ctx, dt_per_scenario, n_steps):
    dt = np.ascontiguousarray(dt_per_scenario, np.float64)
    _call("fem_step_batch", ctx, _p(dt), int(n_steps))


def fem_energy_scenarios(ctx, n_scen):
    arr = (fem_energy_report * n_scen)()
    _call("fem_energy_scenarios", ctx, arr)
    return [_as_dict(r) for r in arr]


def fem_finalize(ctx):
    rep = fem_prep_report()
    _call("fem_finalize", ctx, C.byref(rep))
    return _as_dict(rep)


def fem_get_report(ctx):
    rep = fem_prep_report()
    _call("fem_get_report", ctx, C.byref(rep))
    return _as_dict(rep)


def fem_query_buffers(ctx):
    n = C.c_int32(0)
    _call("fem_query_buffers", ctx, None, C.byref(n))
    arr = (fem_buffer_desc * n.value)()
    _call("fem_query_buffers", ctx, arr, C.byref(n))
    return [(d.name.decode(), d.bytes, d.alignment) for d in arr]


def fem_bind_buffers(ctx, ptrs):
    arr = (C.c_void_p * len(ptrs))(*[C.c_void_p(p) if p else None for p in ptrs])
    _call("fem_bind_buffers", ctx, arr, len(ptrs))


def fem_stable_dt(ctx):
    dt = C.c_double()
    _call("fem_stable_dt", ctx, C.byref(dt))
    return dt.value


def fem_step(ctx, dt, n_steps):
    _call("fem_step", ctx, float(dt), int(n_steps))


def fem_step_no_alloc(ctx, dt, n_steps):
    _call("fem_step_no_alloc", ctx, float(dt), int(n_steps))


def _read(name, ctx, n):
    out = np.empty(n, np.float64)
    _call(name, ctx, _p(out))
    return out


def fem_read_T(ctx, n):
    return _read("fem_read_T", ctx, n)


def fem_read_fs(ctx, n):
    return _read("fem_read_fs", ctx, n)


def fem_read_H(ctx, n):
    return _read("fem_read_H", ctx, n)


def fem_energy(ctx):
    rep = fem_energy_report()
    _call("fem_energy", ctx, C.byref(rep))
    return _as_dict(rep)


def fem_read_state(ctx):
    nb = C.c_int64(0)
    _call("fem_read_state", ctx, None, C.byref(nb))
    buf = np.empty(nb.value, np.uint8)
    _call("fem_read_state", ctx, _p(buf), C.byref(nb))
    return buf


def fem_write_state(ctx, buf):
    b = np.ascontiguousarray(buf, np.uint8)
    _call("fem_write_state", ctx, _p(b), b.size)


def fem_get_node_perm(ctx, n):
    out = np.empty(n, np.int32)
    _call("fem_get_node_perm", ctx, _p(out))
    return out


def fem_time_kernels(ctx, dt, n_steps):
    t = fem_kernel_times()
    _call("fem_time_kernels", ctx, float(dt), int(n_steps), C.byref(t))
    return _as_dict(t)


def fem_copy_kernel(ctx, dst_ptr, src_ptr, nbytes, repeats):
    ms = C.c_double()
    _call("fem_copy_kernel", ctx, C.c_void_p(dst_ptr), C.c_void_p(src_ptr), int(nbytes), int(repeats), C.byref(ms))
    return ms.value


def fem_copy_kernel_nt(ctx, dst_ptr, src_ptr, nbytes, repeats):
    ms = C.c_double()
    _call("fem_copy_kernel_nt", ctx, C.c_void_p(dst_ptr), C.c_void_p(src_ptr), int(nbytes), int(repeats),
          C.byref(ms))
    return ms.value


# ------------------------------------------------------------ surrogate
FEM_SUR_LOSS_H, FEM_SUR_LOSS_T, FEM_SUR_LOSS_HUBER = 0, 1, 2
FEM_SUR_EXTRAP_LINEAR, FEM_SUR_EXTRAP_QUADRATIC = 0, 1


def fem_sur_create(ctx, width=64, layers=3, horizon=16, max_samples=1, train=False, seed=0, loss=FEM_SUR_LOSS_H,
                   extrapolation=FEM_SUR_EXTRAP_LINEAR, projection=True):
    o = fem_sur_options()
    o.width, o.layers, o.horizon, o.max_samples, o.train, o.seed = width, layers, horizon, max_samples, int(train), seed
    o.loss, o.extrapolation, o.no_projection = loss, extrapolation, int(not projection)
    s = C.c_void_p()
    _call("fem_sur_create", C.byref(s), ctx, C.byref(o))
    return s


def fem_sur_destroy(s):
    _call("fem_sur_destroy", s)


def fem_sur_query_buffers(s):
    n = C.c_int32(0)
    _call("fem_sur_query_buffers", s, None, C.byref(n))
    arr = (fem_buffer_desc * n.value)()
    _call("fem_sur_query_buffers", s, arr, C.byref(n))
    return [(d.name.decode(), d.bytes, d.alignment) for d in arr]


def fem_sur_bind_buffers(s, ptrs):
    arr = (C.c_void_p * len(ptrs))(*[C.c_void_p(p) if p else None for p in ptrs])
    _call("fem_sur_bind_buffers", s, arr, len(ptrs))


def fem_sur_n_params(s):
    n = C.c_int64()
    _call("fem_sur_n_params", s, C.byref(n))
    return n.value


def fem_sur_get_params(s):
    out = np.empty(fem_sur_n_params(s), np.float32)
    _call("fem_sur_get_params", s, _p(out), out.size)
    return out


def fem_sur_save(s, path):
    _call("fem_sur_save", s, os.fsencode(path))


def fem_sur_load(s, path):
    _call("fem_sur_load", s, os.fsencode(path))


def fem_sur_set_params(s, params):
    p = np.ascontiguousarray(params, np.float32)
    _call("fem_sur_set_params", s, _p(p), p.size)


N_FEAT = 12


def fem_sur_features(s, H0_ptr, H1_ptr, H2_ptr, stride, slots, n_nodes):
    out = np.empty((slots * n_nodes, N_FEAT), np.float32)
    _call("fem_sur_features", s, C.c_void_p(H0_ptr), C.c_void_p(H1_ptr), C.c_void_p(H2_ptr), int(stride), int(slots),
          _p(out))
    return out


def fem_sur_loss_grad(s, H0_ptr, H1_ptr, H2_ptr, Ht_ptr, stride, slots):
    g = np.empty(fem_sur_n_params(s), np.float32)
    loss = C.c_double()
    _call("fem_sur_loss_grad", s, C.c_void_p(H0_ptr), C.c_void_p(H1_ptr), C.c_void_p(H2_ptr), C.c_void_p(Ht_ptr),
          int(stride), int(slots), C.byref(loss), _p(g))
    return loss.value, g


def fem_sur_train(s, H0_ptr, H1_ptr, H2_ptr, Ht_ptr, stride, n_samples, batch, epochs, lr, lr_final, seed):
    losses = np.zeros(max(int(epochs), 1), np.float64)
    _call("fem_sur_train", s, C.c_void_p(H0_ptr), C.c_void_p(H1_ptr), C.c_void_p(H2_ptr), C.c_void_p(Ht_ptr),
          int(stride), int(n_samples), int(batch), int(epochs), float(lr), float(lr_final), int(seed), _p(losses))
    return losses[:int(epochs)]


def fem_sur_predict(s, H0_ptr, H1_ptr, H2_ptr, stride, slots, out_ptr):
    _call("fem_sur_predict", s, C.c_void_p(H0_ptr), C.c_void_p(H1_ptr), C.c_void_p(H2_ptr), int(stride), int(slots),
          C.c_void_p(out_ptr))


def fem_sur_generate(s, dt_per_scenario, n_chunks, jump_every, S_ptr):
    dt = np.ascontiguousarray(np.atleast_1d(dt_per_scenario), np.float64)
    _call("fem_sur_generate", s, _p(dt), int(n_chunks), int(jump_every), C.c_void_p(S_ptr))


def fem_snapshot_H(ctx, out_ptr):
    _call("fem_snapshot_H", ctx, C.c_void_p(out_ptr))


def fem_advance(ctx, sur, dt_per_scenario, max_steps, until_solid=True, energy_tol=1e-4, fs_tol=1e-6, verify_tol=3.0):
    dt = np.ascontiguousarray(np.atleast_1d(dt_per_scenario), np.float64)
    rep = fem_advance_report()
    _call("fem_advance", ctx, sur, _p(dt), int(max_steps), int(bool(until_solid)), float(energy_tol),
          float(fs_tol), float(verify_tol), C.byref(rep))
    return _as_dict(rep)


# ------------------------------------------------------------ convenience
def make_options(precision=FEM_PREC_FP32_KAHAN, ordering=FEM_ORDER_HILBERT, scatter=FEM_SCATTER_LDS_BLOCKED,
                 block_elems=0, device=0, allow_unstable=False, lds_bytes=0, threads=0,
                 latent_model=FEM_LATENT_ENTHALPY):
    o = fem_options()
    o.device, o.precision, o.ordering, o.scatter = device, precision, ordering, scatter
    o.block_elems, o.allow_unstable, o.lds_bytes, o.threads = block_elems, int(allow_unstable), lds_bytes, threads
    o.latent_model = latent_model
    return o


def setup_problem(ctx, prob):
    """Upload a problem dict (castgen layout) and finalize; returns the prep report."""
    fem_upload_mesh(ctx, prob["elem_type"], prob["xyz"], prob["conn"], prob["elem_mat"])
    fem_set_materials(ctx, prob["materials"])
    if np.size(prob.get("dirichlet_nodes", [])):
        fem_set_dirichlet(ctx, prob["dirichlet_nodes"], prob["dirichlet_T"])
    if np.size(prob.get("flux_faces", [])):
        fem_set_flux_faces(ctx, prob["flux_faces"], prob["flux_q"], prob["flux_h"], prob["flux_Tinf"])
    if np.size(prob.get("if_h", [])):
        fem_set_interface(ctx, prob["if_a"], prob["if_b"], prob["if_h"])
    if np.size(prob.get("contact_h", [])):
        fem_set_contact(ctx, prob["contact_faces"], prob["contact_side"], prob["contact_h"])
    if prob.get("varprops"):
        fem_set_variable_properties(ctx, len(prob["materials"]), **prob["varprops"])
    if prob.get("dirichlet_schedule") is not None:
        fem_set_dirichlet_schedule(ctx, *prob["dirichlet_schedule"])
    fem_set_initial_T(ctx, prob["T0"])
    if "mat_scenario" in prob:
        fem_set_scenarios(ctx, prob["mat_scenario"])
    return fem_finalize(ctx)


def _allocate(torch, device, descs):
    """torch-owned device buffers for a list of (name, bytes, alignment); returns (tensors, aligned pointers)."""
    bufs, ptrs = [], []
    for name, nbytes, align in descs:
        if nbytes:
            t = torch.empty(nbytes + align, dtype=torch.uint8, device=device)
            p = t.data_ptr()
            bufs.append(t)
            ptrs.append(p + (-p) % align)
        else:
            ptrs.append(0)
    return bufs, ptrs


class Solver:
    """One casting problem on one GPU: torch allocates the device buffers and
    the stream, the library borrows them."""

    def __init__(self, prob, device=0, stream=None, **opts):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("castfem.Solver needs a ROCm GPU")
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.n_nodes = prob["xyz"].shape[0]
        self.n_elems = prob["conn"].shape[0]
        self.n_scen = int(np.max(prob["mat_scenario"])) + 1 if "mat_scenario" in prob else 1
        self.ctx = fem_create(make_options(device=device, **opts))
        self.report = setup_problem(self.ctx, prob)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        fem_set_stream(self.ctx, self.stream.cuda_stream)
        self.buffers, ptrs = _allocate(torch, self.device, fem_query_buffers(self.ctx))
        fem_bind_buffers(self.ctx, ptrs)
        self.report = fem_get_report(self.ctx)

    def stable_dt(self):
        return fem_stable_dt(self.ctx)

    def step(self, dt, n):
        fem_step(self.ctx, dt, n)

    def T(self):
        return fem_read_T(self.ctx, self.n_nodes)

    def fs(self):
        return fem_read_fs(self.ctx, self.n_nodes)

    def H(self):
        return fem_read_H(self.ctx, self.n_nodes)

    def energy(self):
        return fem_energy(self.ctx)

    def stable_dt_scenarios(self):
        return fem_stable_dt_scenarios(self.ctx, self.n_scen)

    def step_batch(self, dt_per_scenario, n):
        fem_step_batch(self.ctx, dt_per_scenario, n)

    def energy_scenarios(self):
        return fem_energy_scenarios(self.ctx, self.n_scen)

    def node_perm(self):
        return fem_get_node_perm(self.ctx, self.n_nodes)

    def snapshot_H(self, out):
        """Current enthalpy (device numbering) into the float32 CUDA tensor `out` (n_nodes)."""
        assert out.dtype == self.torch.float32 and out.is_cuda and out.numel() >= self.n_nodes
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        fem_snapshot_H(self.ctx, out.data_ptr())
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def advance(self, dt_per_scenario, max_steps, surrogate=None, until_solid=True, energy_tol=1e-4, fs_tol=1e-6,
                verify_tol=3.0):
        return fem_advance(self.ctx, surrogate.sur if surrogate is not None else None, dt_per_scenario, max_steps,
                           until_solid, energy_tol, fs_tol, verify_tol)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.ctx is not None:
            self.synchronize()
            fem_destroy(self.ctx)
            self.ctx = None
            self.buffers = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """The learned surrogate of a Solver; torch allocates its device buffers."""

    def __init__(self, solver, layers=3, horizon=16, max_samples=1, train=False, seed=0, loss=FEM_SUR_LOSS_H,
                 extrapolation=FEM_SUR_EXTRAP_LINEAR, projection=True):
        self.solver = solver
        self.torch = solver.torch
        self.n_nodes = solver.n_nodes
        self.sur = fem_sur_create(solver.ctx, 64, layers, horizon, max_samples, train, seed, loss, extrapolation,
                                  projection)
        self.buffers, ptrs = _allocate(self.torch, solver.device, fem_sur_query_buffers(self.sur))
        fem_sur_bind_buffers(self.sur, ptrs)

    def _sync_in(self):
        self.solver.stream.wait_stream(self.torch.cuda.current_stream(self.solver.device))

    def params(self):
        return fem_sur_get_params(self.sur)

    def set_params(self, p):
        fem_sur_set_params(self.sur, p)

    def save(self, path):
        fem_sur_save(self.sur, path)

    def load(self, path):
        fem_sur_load(self.sur, path)

    def _states(self, tensors, stride, slots):
        """Device pointers of float32 CUDA tensors (or views), each checked to reach `slots`
        states `stride` floats apart within its storage."""
        need = (slots - 1) * stride + self.n_nodes
        for t in tensors:
            assert t.dtype == self.torch.float32 and t.is_cuda and t.is_contiguous()
            st = t.untyped_storage()
            avail = (st.data_ptr() + st.nbytes() - t.data_ptr()) // 4
            if avail < need:
                raise ValueError("state tensor too small for %d states of stride %d" % (slots, stride))
        return [t.data_ptr() for t in tensors]

    def features(self, H0, H1, H2, stride=None, slots=1):
        stride = self.n_nodes if stride is None else stride
        ptrs = self._states((H0, H1, H2), stride, slots)
        self._sync_in()
        return fem_sur_features(self.sur, *ptrs, stride, slots, self.n_nodes)

    def loss_grad(self, H0, H1, H2, Ht, stride=None, slots=1):
        stride = self.n_nodes if stride is None else stride
        ptrs = self._states((H0, H1, H2, Ht), stride, slots)
        self._sync_in()
        return fem_sur_loss_grad(self.sur, *ptrs, stride, slots)

    def train(self, H0, H1, H2, Ht, stride, n_samples, batch=1, epochs=1, lr=1e-3, lr_final=1e-5, seed=0):
        """Tensors may be views into one buffer (e.g. states [k][0..2] with Ht = the next [k][0])."""
        ptrs = self._states((H0, H1, H2, Ht), stride, n_samples)
        self._sync_in()
        return fem_sur_train(self.sur, *ptrs, stride, n_samples, batch, epochs, lr, lr_final, seed)

    def generate(self, dt_per_scenario, n_chunks, jump_every, S):
        """Chunks of explicit states (H^n, H^n+1, H^n+2, H^n+horizon) into S, a float32 CUDA
        tensor of shape (>= n_chunks, 4, n_nodes); see fem_sur_generate."""
        assert S.dtype == self.torch.float32 and S.is_cuda and S.is_contiguous()
        assert S.dim() == 3 and S.shape[0] >= n_chunks and S.shape[1] == 4 and S.shape[2] == self.n_nodes
        self._sync_in()
        fem_sur_generate(self.sur, dt_per_scenario, n_chunks, jump_every, S.data_ptr())
        self.torch.cuda.current_stream(self.solver.device).wait_stream(self.solver.stream)

    def predict(self, H0, H1, H2, out, stride=None, slots=1):
        stride = self.n_nodes if stride is None else stride
        ptrs = self._states((H0, H1, H2), stride, slots)
        assert out.dtype == self.torch.float64 and out.is_cuda and out.numel() >= slots * self.n_nodes
        self._sync_in()
        fem_sur_predict(self.sur, *ptrs, stride, slots, out.data_ptr())

    def close(self):
        if self.sur is not None:
            self.solver.synchronize()
            fem_sur_destroy(self.sur)
            self.sur = None
            self.buffers = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
