"""Seeded problem builders for the casting workloads.

A problem is a dict of host arrays in the layout the C interface takes:

  elem_type      4 (tet4) or 8 (hex8)
  xyz            (N, 3) float64, metres
  conn           (E, nen) int32, 0-based node ids
  elem_mat       (E,) int32 material index
  materials      (M, 6) float64 rows [k, rho, c, T_sol, T_liq, L] (SI, deg C)
  dirichlet_nodes, dirichlet_T        fixed-temperature nodes
  flux_faces (nf, npf) int32, flux_q, flux_h, flux_Tinf     Robin faces
  if_a, if_b (np, 3) int32, if_h       matched cast/mold interface triangles
  T0             (N,) float64 initial temperature
  meta           dict describing the recipe (sizes, seeds)

The workloads follow the casting setting of the paper (aluminium-like alloy
poured into a sand mould, heat crossing the cast/mould contact through an
interface heat-transfer coefficient) on synthetic meshes, since the paper's
meshes are not published.  No finite-element arithmetic lives here.
"""
import numpy as np

from . import meshes, rng

# [k, rho, c, T_sol, T_liq, L]
ALLOY = (150.0, 2700.0, 900.0, 600.0, 660.0, 3.9e5)
SAND = (0.6, 1500.0, 1000.0, 0.0, 0.0, 0.0)


def box_hex_grid(nx, ny, nz, lx, ly, lz):
    """Hex8 grid of nx*ny*nz boxes on [0,lx]x[0,ly]x[0,lz]; node (i,j,k) id = i + (nx+1)(j + (ny+1)k)."""
    mx, my, mz = nx + 1, ny + 1, nz + 1
    ids = np.arange(mx * my * mz, dtype=np.int64)
    i, j, k = ids % mx, (ids // mx) % my, ids // (mx * my)
    xyz = np.stack([i * (lx / nx), j * (ly / ny), k * (lz / nz)], axis=1)
    c = np.arange(nx * ny * nz, dtype=np.int64)
    ci, cj, ck = c % nx, (c // nx) % ny, c // (nx * ny)
    base = ci + mx * (cj + my * ck)
    offs = np.array([a + mx * (b + my * cc) for (a, b, cc) in meshes.HEX_CORNERS], dtype=np.int64)
    conn = base[:, None] + offs[None, :]
    return xyz, conn, (i, j, k)


def x0_quads(nx, ny, nz):
    """Quad faces of a box hex grid on the plane x = 0, nodes ordered around the face."""
    mx, my = nx + 1, ny + 1
    q = []
    for k in range(nz):
        for j in range(ny):
            a = 0 + mx * (j + my * k)
            b = 0 + mx * (j + 1 + my * k)
            c = 0 + mx * (j + 1 + my * (k + 1))
            d = 0 + mx * (j + my * (k + 1))
            q.append((a, b, c, d))
    return np.array(q, dtype=np.int64)


def smooth_noise(xyz, length, seed, modes=8):
    """sum_m a_m sin(2 pi k_m.x / length + phi_m), k_m in {0..3}^3 without 0, scaled to max |.| = 1."""
    ks = []
    off = 0
    while len(ks) < modes:
        v = (rng.u64(seed, 7, 3, off) % np.uint64(4)).astype(np.int64)
        off += 3
        if np.any(v):
            ks.append(v)
    a = rng.uniform(seed, 8, modes, 0.5, 1.0)
    phi = rng.uniform(seed, 9, modes, 0.0, 2.0 * np.pi)
    s = np.zeros(xyz.shape[0])
    for m in range(modes):
        s += a[m] * np.sin(2.0 * np.pi * (xyz @ ks[m].astype(np.float64)) / length + phi[m])
    return s / np.max(np.abs(s))


def _empty_faces(problem):
    problem.setdefault("dirichlet_nodes", np.zeros(0, np.int32))
    problem.setdefault("dirichlet_T", np.zeros(0))
    problem.setdefault("flux_faces", np.zeros((0, 3), np.int32))
    problem.setdefault("flux_q", np.zeros(0))
    problem.setdefault("flux_h", np.zeros(0))
    problem.setdefault("flux_Tinf", np.zeros(0))
    problem.setdefault("if_a", np.zeros((0, 3), np.int32))
    problem.setdefault("if_b", np.zeros((0, 3), np.int32))
    problem.setdefault("if_h", np.zeros(0))
    return problem


def hex_cube(n=16, length=0.1, T_pour=700.0, noise_amp=2.0, noise_seed=1,
             dirichlet_x0=25.0, robin_x0=None, material=ALLOY):
    """The 0.1 m alloy cube as n^3 hex8 elements.

    dirichlet_x0: temperature held on the x = 0 face (None for none).
    robin_x0: (h, T_inf) of a convective chill on the x = 0 face, or None.
    The initial field is T_pour plus seeded smooth noise of amplitude noise_amp.
    """
    xyz, conn, (i, j, k) = box_hex_grid(n, n, n, length, length, length)
    N = xyz.shape[0]
    T0 = np.full(N, float(T_pour))
    if noise_amp:
        T0 = T0 + noise_amp * smooth_noise(xyz, length, noise_seed)
    prob = dict(elem_type=8, xyz=xyz, conn=conn.astype(np.int32),
                elem_mat=np.zeros(conn.shape[0], np.int32),
                materials=np.array([material], dtype=np.float64), T0=T0,
                meta=dict(kind="hex_cube", n=n, length=length, T_pour=T_pour,
                          noise_amp=noise_amp, noise_seed=noise_seed))
    if dirichlet_x0 is not None:
        d = np.nonzero(i == 0)[0]
        prob["dirichlet_nodes"] = d.astype(np.int32)
        prob["dirichlet_T"] = np.full(d.size, float(dirichlet_x0))
    if robin_x0 is not None:
        q = x0_quads(n, n, n)
        prob["flux_faces"] = q.astype(np.int32)
        prob["flux_q"] = np.zeros(q.shape[0])
        prob["flux_h"] = np.full(q.shape[0], float(robin_x0[0]))
        prob["flux_Tinf"] = np.full(q.shape[0], float(robin_x0[1]))
    return _empty_faces(prob)


def hex_bar(nx=64, ny=4, nz=4, lx=0.4, ly=0.025, lz=0.025, T_init=700.0, T_wall=25.0, material=ALLOY):
    """A bar of hexes along x with a fixed temperature on x = 0 (semi-infinite conduction setting)."""
    xyz, conn, (i, j, k) = box_hex_grid(nx, ny, nz, lx, ly, lz)
    d = np.nonzero(i == 0)[0]
    prob = dict(elem_type=8, xyz=xyz, conn=conn.astype(np.int32),
                elem_mat=np.zeros(conn.shape[0], np.int32),
                materials=np.array([material], dtype=np.float64),
                T0=np.full(xyz.shape[0], float(T_init)),
                dirichlet_nodes=d.astype(np.int32), dirichlet_T=np.full(d.size, float(T_wall)),
                meta=dict(kind="hex_bar", nx=nx, ny=ny, nz=nz, lx=lx))
    return _empty_faces(prob)


def box_kuhn_conn(nx, ny, nz):
    """Kuhn split of the boxes of box_hex_grid(nx, ny, nz, ...): six positively
    oriented tetrahedra per box, ids as in box_hex_grid."""
    mx, my = nx + 1, ny + 1
    c = np.arange(nx * ny * nz, dtype=np.int64)
    base = c % nx + mx * ((c // nx) % ny + my * (c // (nx * ny)))
    tets = []
    for order, odd in meshes._AXIS_ORDERS:
        v = [0, 0, 0]
        path = [tuple(v)]
        for ax in order:
            v = list(v)
            v[ax] = 1
            path.append(tuple(v))
        if odd:
            path[1], path[2] = path[2], path[1]
        tets.append([a + mx * (b + my * cc) for (a, b, cc) in path])
    return (base[:, None, None] + np.array(tets, dtype=np.int64)[None]).reshape(-1, 4)


def tet_bar(nx=64, ny=1, nz=1, lx=0.1, ly=None, lz=None, T_init=700.0, T_wall=25.0, material=ALLOY):
    """hex_bar split into Kuhn tetrahedra (fixed temperature on x = 0)."""
    h = lx / nx
    ly = h * ny if ly is None else ly
    lz = h * nz if lz is None else lz
    xyz, _, (i, j, k) = box_hex_grid(nx, ny, nz, lx, ly, lz)
    conn = box_kuhn_conn(nx, ny, nz)
    d = np.nonzero(i == 0)[0]
    prob = dict(elem_type=4, xyz=xyz, conn=conn.astype(np.int32),
                elem_mat=np.zeros(conn.shape[0], np.int32),
                materials=np.array([material], dtype=np.float64),
                T0=np.full(xyz.shape[0], float(T_init)),
                dirichlet_nodes=d.astype(np.int32), dirichlet_T=np.full(d.size, float(T_wall)),
                meta=dict(kind="tet_bar", nx=nx, ny=ny, nz=nz, lx=lx))
    return _empty_faces(prob)


def tet_casting(n=128, length=0.1, region="cube", cube=(0.2, 0.8), boxes_seed=6, n_boxes=8,
                jitter=0.2, jitter_seed=2, perm_seed=3, T_pour=700.0, T_mold=25.0,
                h_interface=1000.0, alloy=ALLOY, mold=SAND, permute=True):
    """Jittered Kuhn-tet cast+mold mesh of the cube [0, length]^3 with an adiabatic outer boundary.

    region: "cube" (cubes whose centre lies in [cube[0], cube[1]]^3 are casting),
            "boxes" (union of `n_boxes` seeded boxes), or "none" (all casting).
    Nodes on the cast/mold interface are duplicated; each interface triangle is
    listed once as a (casting copy, mold copy) pair with coefficient h_interface.
    With permute, node ids and element order are seeded random permutations.
    """
    conn_grid = meshes.kuhn_conn(n)
    if jitter:
        xyz01, redrawn = meshes.jitter_grid(n, conn_grid, jitter, jitter_seed)
    else:
        xyz01, redrawn = meshes.grid_xyz(n, 1.0), 0
    ncell = n ** 3
    if region == "cube":
        cell_cast = meshes.cube_region_cells(n, cube[0], cube[1])
        boxes = None
    elif region == "boxes":
        boxes = meshes.random_boxes(boxes_seed, n_boxes)
        cell_cast = meshes.boxes_region_cells(n, boxes)
    elif region == "none":
        cell_cast = np.ones(ncell, dtype=bool)
        boxes = None
    else:
        raise ValueError(region)
    elem_is_cast = np.repeat(cell_cast, 6)
    Ng = (n + 1) ** 3
    if np.all(elem_is_cast):
        conn, dup, copy_id = conn_grid, np.zeros(0, np.int64), np.full(Ng, -1, np.int64)
        fa, fb = np.zeros((0, 3), np.int64), np.zeros((0, 3), np.int64)
    else:
        conn, dup, copy_id = meshes.split_materials(conn_grid, elem_is_cast, Ng)
        fa, fb = meshes.interface_faces(conn_grid, elem_is_cast, dup, copy_id)
    xyz = np.concatenate([xyz01, xyz01[dup]], axis=0) * length
    N = xyz.shape[0]
    node_is_cast = np.zeros(N, dtype=bool)
    node_is_cast[conn[elem_is_cast].ravel()] = True
    T0 = np.where(node_is_cast, float(T_pour), float(T_mold))
    materials = np.array([alloy, mold], dtype=np.float64)
    prob = dict(elem_type=4, xyz=xyz, conn=conn.astype(np.int32),
                elem_mat=np.where(elem_is_cast, 0, 1).astype(np.int32),
                materials=materials, T0=T0,
                if_a=fa.astype(np.int32), if_b=fb.astype(np.int32),
                if_h=np.full(fa.shape[0], float(h_interface)),
                meta=dict(kind="tet_casting", n=n, length=length, region=region, cube=cube,
                          boxes=boxes, jitter=jitter, jitter_seed=jitter_seed, perm_seed=perm_seed,
                          redrawn_nodes=int(redrawn), n_dup=int(dup.size)))
    prob = _empty_faces(prob)
    if permute:
        node_perm = rng.permutation(perm_seed, 0, N)
        elem_perm = rng.permutation(perm_seed, 1, conn.shape[0])
        prob = meshes.apply_permutations(prob, node_perm, elem_perm)
    return prob


def plane_triangles(conn, on_plane):
    """Faces of a tet mesh whose three nodes lie on one of the given planes
    (on_plane: list of per-node boolean masks) and that belong to one
    tetrahedron only, (n, 3) node ids."""
    f = np.concatenate([conn[:, [1, 2, 3]], conn[:, [0, 2, 3]], conn[:, [0, 1, 3]], conn[:, [0, 1, 2]]])
    ok = np.zeros(f.shape[0], dtype=bool)
    for m in on_plane:
        ok |= np.all(m[f], axis=1)
    f = f[ok]
    s = np.sort(f, axis=1)
    _, inv, cnt = np.unique(s, axis=0, return_inverse=True, return_counts=True)
    return f[cnt[inv.ravel()] == 1]


def _jitter_interior(xyz, conn, interior, h, amp, seed, stream):
    """U(+-amp h) per coordinate on the interior nodes; the nodes of any tet left with
    6V < 0.1 h^3 go back to their grid position until none is left."""
    off = rng.uniform(seed, stream, xyz.size, -amp * h, amp * h).reshape(xyz.shape)
    off[~interior] = 0.0
    while True:
        x = xyz + off
        bad = meshes._six_volume(x, conn) < 0.1 * h ** 3
        if not np.any(bad):
            return x
        off[conn[bad].ravel()] = 0.0


def tet_casting_nonmatching(n_cast=12, n_mold=8, length=0.1, cube=(0.25, 0.75), T_pour=700.0, T_mold=25.0,
                            h_interface=1000.0, alloy=ALLOY, mold=SAND, jitter=0.15, jitter_seed=2, perm_seed=3,
                            permute=True):
    """A casting cube and its sand mould meshed separately (the paper's cast and mould
    grids with no coincident interface nodes).

    Mould: Kuhn tets of an n_mold^3 grid of [0, length]^3 without the cells of the cube
    [cube[0], cube[1]]^3 (whose faces must lie on grid planes).  Casting: Kuhn tets of an
    n_cast^3 grid of the cube itself.  The two meshes share no nodes; every boundary
    triangle on the cube's surface is a contact face, side 0 for the mould and side 1 for
    the casting, with coefficient h_interface; the sister pairing is left to the solver.
    Nodes off every boundary plane are jittered by U(+-jitter h).
    """
    lo, hi = cube
    if abs(lo * n_mold - round(lo * n_mold)) > 1e-9 or abs(hi * n_mold - round(hi * n_mold)) > 1e-9:
        raise ValueError("the cube must lie on mould grid planes")
    # mould part
    cm = meshes.kuhn_conn(n_mold)
    keep = ~np.repeat(meshes.cube_region_cells(n_mold, lo, hi), 6)
    cm = cm[keep]
    used = np.unique(cm)
    ids = np.full((n_mold + 1) ** 3, -1, np.int64)
    ids[used] = np.arange(used.size)
    cm = ids[cm]
    g = np.stack(meshes.grid_ids(n_mold), axis=1)[used]
    xm = meshes.grid_xyz(n_mold, 1.0)[used] * length
    planes_m = {0, int(round(lo * n_mold)), int(round(hi * n_mold)), n_mold}
    inner_m = np.ones(used.size, dtype=bool)
    for ax in range(3):
        inner_m &= ~np.isin(g[:, ax], list(planes_m))
    xm = _jitter_interior(xm, cm, inner_m, length / n_mold, jitter, jitter_seed, 30)
    # casting part
    cc = meshes.kuhn_conn(n_cast)
    gc = np.stack(meshes.grid_ids(n_cast), axis=1)
    xc = (lo + (hi - lo) * meshes.grid_xyz(n_cast, 1.0)) * length
    inner_c = np.all((gc > 0) & (gc < n_cast), axis=1)
    xc = _jitter_interior(xc, cc, inner_c, (hi - lo) * length / n_cast, jitter, jitter_seed, 31)
    nm = xm.shape[0]
    xyz = np.concatenate([xm, xc], axis=0)
    conn = np.concatenate([cm, cc + nm], axis=0)
    elem_mat = np.concatenate([np.ones(cm.shape[0], np.int32), np.zeros(cc.shape[0], np.int32)])
    # contact faces: mould triangles on the cube's six faces, then the casting's boundary triangles
    a, b = int(round(lo * n_mold)), int(round(hi * n_mold))
    in_sq = [np.all((np.delete(g, ax, axis=1) >= a) & (np.delete(g, ax, axis=1) <= b), axis=1) for ax in range(3)]
    bm = plane_triangles(cm, [(g[:, ax] == v) & in_sq[ax] for ax in range(3) for v in (a, b)])
    bc = plane_triangles(cc, [gc[:, ax] == v for ax in range(3) for v in (0, n_cast)]) + nm
    faces = np.concatenate([bm, bc], axis=0)
    side = np.concatenate([np.zeros(bm.shape[0], np.int32), np.ones(bc.shape[0], np.int32)])
    N = xyz.shape[0]
    T0 = np.concatenate([np.full(nm, float(T_mold)), np.full(xc.shape[0], float(T_pour))])
    prob = dict(elem_type=4, xyz=xyz, conn=conn.astype(np.int32), elem_mat=elem_mat,
                materials=np.array([alloy, mold], dtype=np.float64), T0=T0,
                contact_faces=faces.astype(np.int32), contact_side=side,
                contact_h=np.full(faces.shape[0], float(h_interface)),
                meta=dict(kind="tet_casting_nonmatching", n_cast=n_cast, n_mold=n_mold, length=length, cube=cube,
                          jitter=jitter, jitter_seed=jitter_seed, perm_seed=perm_seed))
    prob = _empty_faces(prob)
    if permute:
        node_perm = rng.permutation(perm_seed, 0, N)
        elem_perm = rng.permutation(perm_seed, 1, conn.shape[0])
        prob = meshes.apply_permutations(prob, node_perm, elem_perm)
    return prob


def config1(**kw):
    """16^3 hex8 alloy cube, noise seed 1, 25 C on x = 0, adiabatic elsewhere."""
    return hex_cube(**kw)


def config2(n=128, **kw):
    """128^3 jittered Kuhn tets, inner casting cube [0.2, 0.8]^3 in sand, h_i = 1000, jitter 2, perm 3."""
    kw.setdefault("jitter_seed", 2)
    kw.setdefault("perm_seed", 3)
    return tet_casting(n=n, region="cube", **kw)


def config5(n=256, **kw):
    """256^3 jittered Kuhn tets, casting = union of 8 seeded boxes (seed 6), jitter 7, perm 8."""
    kw.setdefault("boxes_seed", 6)
    kw.setdefault("jitter_seed", 7)
    kw.setdefault("perm_seed", 8)
    return tet_casting(n=n, region="boxes", **kw)


def chill_params(seed):
    """Pour temperature U(680, 760) C and chill coefficient log-uniform on [300, 3000] W/m^2K."""
    u = rng.uniform(seed, 11, 2)
    T_pour = 680.0 + 80.0 * u[0]
    h = float(np.exp(np.log(300.0) + (np.log(3000.0) - np.log(300.0)) * u[1]))
    return T_pour, h


def config4_trajectory(seed, n=16):
    """Alloy cube with a convective chill (h, 25 C) on x = 0 and a uniform pour temperature."""
    T_pour, h = chill_params(seed)
    return hex_cube(n=n, T_pour=T_pour, noise_amp=0.0, dirichlet_x0=None, robin_x0=(h, 25.0))


def chill_batch(seeds, n=16):
    """config4_trajectory of every seed as one disjoint problem (scenario s = seeds[s],
    material s); meta['scenarios'] lists node0/node1, T_pour and h of each."""
    parts, sc = [], []
    n0 = 0
    for s, seed in enumerate(seeds):
        p = config4_trajectory(seed, n)
        T_pour, h = chill_params(seed)
        N = p["xyz"].shape[0]
        sc.append(dict(seed=int(seed), T_pour=T_pour, h=h, node0=n0, node1=n0 + N))
        parts.append((p, n0))
        n0 += N
    cat = lambda key: np.concatenate([q[key] for q, _ in parts], axis=0)
    prob = dict(
        elem_type=8,
        xyz=cat("xyz"),
        conn=np.concatenate([q["conn"] + off for q, off in parts], axis=0).astype(np.int32),
        elem_mat=np.concatenate([q["elem_mat"] + s for s, (q, _) in enumerate(parts)]).astype(np.int32),
        materials=np.array([ALLOY] * len(parts), dtype=np.float64),
        T0=cat("T0"),
        flux_faces=np.concatenate([q["flux_faces"] + off for q, off in parts], axis=0).astype(np.int32),
        flux_q=cat("flux_q"), flux_h=cat("flux_h"), flux_Tinf=cat("flux_Tinf"),
        mat_scenario=np.arange(len(parts), dtype=np.int32),
        meta=dict(kind="chill_batch", n=n, scenarios=sc))
    return _empty_faces(prob)


def batch_scenarios(n_scen=256, seed=4, elems_range=(20000, 400000), n_range=None):
    """Parameters of a batch of casting scenarios (one dict per scenario).

    Scenario s uses seed 4000 + s for its jitter and numbering; its size is drawn as
    E_s ~ U(elems_range) and n_s = round((E_s / 6)^(1/3)) cubes per axis (or n_s
    ~ U{n_range} when given); pour temperature U(680, 760) C, contact coefficient
    log-uniform on [300, 3000] W/m^2K, mould conductivity U(0.4, 1.5) W/mK.
    """
    u = rng.uniform(seed, 21, 4 * n_scen).reshape(n_scen, 4)
    out = []
    for s in range(n_scen):
        if n_range is None:
            E_s = elems_range[0] + (elems_range[1] - elems_range[0]) * u[s, 0]
            n_s = int(round((E_s / 6.0) ** (1.0 / 3.0)))
        else:
            n_s = int(n_range[0] + min(int(u[s, 0] * (n_range[1] - n_range[0] + 1)), n_range[1] - n_range[0]))
        out.append(dict(
            n=n_s, seed=4000 + s,
            T_pour=680.0 + 80.0 * u[s, 1],
            h_interface=float(np.exp(np.log(300.0) + (np.log(3000.0) - np.log(300.0)) * u[s, 2])),
            k_mold=0.4 + 1.1 * u[s, 3]))
    return out


def batch(n_scen=256, seed=4, elems_range=(20000, 400000), n_range=None, permute=True):
    """A batch of cast+mould scenarios as one disjoint problem.

    Scenario s owns materials 2s (alloy) and 2s+1 (its sand mould); node and
    element ranges of every scenario are listed in meta['scenarios'] (input
    numbering: nodes [node0, node1), elements [elem0, elem1)).
    """
    params = batch_scenarios(n_scen, seed, elems_range, n_range)
    parts = []
    mats = []
    n0 = e0 = 0
    for s, sp in enumerate(params):
        mold = (sp["k_mold"], SAND[1], SAND[2], SAND[3], SAND[4], SAND[5])
        p = tet_casting(n=sp["n"], region="cube", jitter_seed=sp["seed"], perm_seed=sp["seed"],
                        T_pour=sp["T_pour"], h_interface=sp["h_interface"], alloy=ALLOY, mold=mold,
                        permute=permute)
        N, E = p["xyz"].shape[0], p["conn"].shape[0]
        sp.update(node0=n0, node1=n0 + N, elem0=e0, elem1=e0 + E, mat_cast=2 * s, mat_mold=2 * s + 1)
        parts.append((p, n0))
        mats += [ALLOY, mold]
        n0 += N
        e0 += E
    cat = lambda key, shift: np.concatenate([q[key] + (off if shift else 0) for q, off in parts], axis=0)
    prob = dict(
        elem_type=4,
        xyz=np.concatenate([q["xyz"] for q, _ in parts], axis=0),
        conn=np.concatenate([q["conn"] + off for q, off in parts], axis=0).astype(np.int32),
        elem_mat=np.concatenate([q["elem_mat"] + 2 * s for s, (q, _) in enumerate(parts)]).astype(np.int32),
        materials=np.array(mats, dtype=np.float64),
        T0=np.concatenate([q["T0"] for q, _ in parts]),
        if_a=np.concatenate([q["if_a"] + off for q, off in parts], axis=0).astype(np.int32),
        if_b=np.concatenate([q["if_b"] + off for q, off in parts], axis=0).astype(np.int32),
        if_h=np.concatenate([q["if_h"] for q, _ in parts]),
        mat_scenario=np.repeat(np.arange(n_scen, dtype=np.int32), 2),
        meta=dict(kind="batch", n_scen=n_scen, seed=seed, scenarios=params))
    return _empty_faces(prob)
