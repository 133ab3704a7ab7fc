"""Seeded synthetic cast+mold meshes (the paper's own meshes are not available).

Everything here builds input arrays only: node coordinates, element
connectivity, element materials, boundary sets and the matched interface face
pairs.  None of the finite-element arithmetic (element matrices, lumping,
fluxes, the enthalpy relation) lives in this package.

Grid conventions
* A structured n^3 grid of cubes on [0, 1]^3 (scaled by `length`), grid node
  (i, j, k) has id i + (n+1)*(j + (n+1)*k).
* Hex8 nodes follow the usual trilinear ordering: bottom face counter-clockwise
  (0,0,0) (1,0,0) (1,1,0) (0,1,0), then the top face in the same order.
* Tet4 meshes split each cube into the 6 Kuhn (Freudenthal) tetrahedra that
  share the (0,0,0)-(1,1,1) diagonal, one per ordering of the three axes.  The
  split is conforming.  Odd orderings swap their two middle vertices so that
  every tetrahedron is positively oriented on the unjittered grid.
"""
import numpy as np

from . import rng

HEX_CORNERS = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                        (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], dtype=np.int64)

# axis orderings and whether they are odd permutations
_AXIS_ORDERS = [((0, 1, 2), False), ((0, 2, 1), True), ((1, 0, 2), True),
                ((1, 2, 0), False), ((2, 0, 1), False), ((2, 1, 0), True)]


def grid_ids(n):
    """(i, j, k) index arrays of all (n+1)^3 grid nodes in id order."""
    m = n + 1
    ids = np.arange(m ** 3, dtype=np.int64)
    return ids % m, (ids // m) % m, ids // (m * m)


def grid_xyz(n, length=1.0):
    i, j, k = grid_ids(n)
    h = 1.0 / n
    return np.stack([i * h, j * h, k * h], axis=1) * length


def cell_base_ids(n):
    """Grid id of the (0,0,0) corner of every cube, cube id order c = i + n*(j + n*k)."""
    c = np.arange(n ** 3, dtype=np.int64)
    i, j, k = c % n, (c // n) % n, c // (n * n)
    m = n + 1
    return i + m * (j + m * k)


def _corner_offset(n, a, b, c):
    m = n + 1
    return a + m * (b + m * c)


def hex_conn(n):
    base = cell_base_ids(n)
    offs = np.array([_corner_offset(n, *cn) for cn in HEX_CORNERS], dtype=np.int64)
    return base[:, None] + offs[None, :]


def kuhn_conn(n):
    """(6 n^3, 4) grid-node connectivity; tet t belongs to cube t // 6."""
    base = cell_base_ids(n)
    tets = []
    for order, odd in _AXIS_ORDERS:
        p = np.zeros(3, dtype=np.int64)
        path = [tuple(p)]
        for ax in order:
            p = p.copy()
            p[ax] = 1
            path.append(tuple(p))
        if odd:
            path[1], path[2] = path[2], path[1]
        tets.append([_corner_offset(n, *v) for v in path])
    offs = np.array(tets, dtype=np.int64)            # (6, 4)
    conn = base[:, None, None] + offs[None, :, :]    # (ncell, 6, 4)
    return conn.reshape(-1, 4)


def _six_volume(xyz, conn):
    """Signed 6*volume of tetrahedra; used only to reject badly jittered input meshes."""
    x0 = xyz[conn[:, 0]]
    d1 = xyz[conn[:, 1]] - x0
    d2 = xyz[conn[:, 2]] - x0
    d3 = xyz[conn[:, 3]] - x0
    return np.einsum("ij,ij->i", d1, np.cross(d2, d3))


def jitter_grid(n, conn, amp, seed, min_six_vol=0.1, max_rounds=32):
    """Grid coordinates on [0,1]^3 moved by U(-amp*h, amp*h) per coordinate.

    A coordinate on a boundary plane of the unit cube is not moved, so boundary
    nodes slide within their face and the domain volume is exact.  Any node of
    a tetrahedron whose 6*volume drops below `min_six_vol`*h^3 is re-drawn from
    the next sub-stream, up to `max_rounds` times.  Returns (xyz, n_redrawn).
    """
    h = 1.0 / n
    i, j, k = grid_ids(n)
    idx = np.stack([i, j, k], axis=1)
    N = idx.shape[0]
    free = (idx > 0) & (idx < n)                      # movable coordinates
    base = idx * h

    def draw(stream, nodes):
        d = np.empty((nodes.size, 3))
        for a in range(3):
            d[:, a] = rng.uniform(seed, stream * 4 + a, N, -amp * h, amp * h)[nodes]
        return d

    all_nodes = np.arange(N)
    xyz = base + np.where(free, draw(0, all_nodes), 0.0)
    redrawn = 0
    for rnd in range(1, max_rounds + 1):
        v6 = _six_volume(xyz, conn)
        bad = np.nonzero(v6 < min_six_vol * h ** 3)[0]
        if bad.size == 0:
            break
        nodes = np.unique(conn[bad].ravel())
        redrawn += nodes.size
        xyz[nodes] = base[nodes] + np.where(free[nodes], draw(rnd, nodes), 0.0)
    else:
        raise RuntimeError("jitter re-draw did not converge")
    return xyz, redrawn


def cube_region_cells(n, lo, hi):
    """Boolean per cube: unjittered centre inside [lo, hi]^3."""
    c = np.arange(n ** 3, dtype=np.int64)
    ijk = np.stack([c % n, (c // n) % n, c // (n * n)], axis=1)
    centre = (ijk + 0.5) / n
    return np.all((centre >= lo) & (centre <= hi), axis=1)


def boxes_region_cells(n, boxes):
    """Boolean per cube: unjittered centre inside the union of axis-aligned boxes (lo3, hi3)."""
    c = np.arange(n ** 3, dtype=np.int64)
    ijk = np.stack([c % n, (c // n) % n, c // (n * n)], axis=1)
    centre = (ijk + 0.5) / n
    inside = np.zeros(n ** 3, dtype=bool)
    for lo, hi in boxes:
        inside |= np.all((centre >= np.asarray(lo)) & (centre <= np.asarray(hi)), axis=1)
    return inside


def random_boxes(seed, count=8):
    """`count` boxes: centres U(0.25,0.75)^3, half-widths U(0.05,0.15) per axis, clipped to [0.1,0.9]."""
    c = rng.uniform(seed, 100, 3 * count, 0.25, 0.75).reshape(count, 3)
    w = rng.uniform(seed, 101, 3 * count, 0.05, 0.15).reshape(count, 3)
    return [(np.clip(c[b] - w[b], 0.1, 0.9), np.clip(c[b] + w[b], 0.1, 0.9)) for b in range(count)]


def split_materials(conn, elem_is_cast, n_grid_nodes):
    """Duplicate every grid node touched by both casting and mold elements.

    The mold keeps the grid id; the casting copy of duplicated node g gets id
    n_grid_nodes + rank of g among the duplicated nodes.  Returns the new
    connectivity, the duplicated grid ids (sorted) and the casting-copy ids.
    """
    touched_cast = np.zeros(n_grid_nodes, dtype=bool)
    touched_mold = np.zeros(n_grid_nodes, dtype=bool)
    touched_cast[conn[elem_is_cast].ravel()] = True
    touched_mold[conn[~elem_is_cast].ravel()] = True
    dup = np.nonzero(touched_cast & touched_mold)[0]
    copy_id = np.full(n_grid_nodes, -1, dtype=np.int64)
    copy_id[dup] = n_grid_nodes + np.arange(dup.size)
    new_conn = conn.copy()
    cc = new_conn[elem_is_cast]
    cid = copy_id[cc]
    cc = np.where(cid >= 0, cid, cc)
    new_conn[elem_is_cast] = cc
    return new_conn, dup, copy_id


def interface_faces(conn_grid, elem_is_cast, dup, copy_id):
    """Matched interface triangles between casting and mold tetrahedra.

    A triangle is on the interface when it is a face of a casting tet and of a
    mold tet (compared through grid ids).  Returns (face_cast, face_mold), each
    (n_pairs, 3): the casting copies and the mold ids of the same grid nodes in
    the same order.
    """
    if dup.size == 0:
        return np.zeros((0, 3), np.int64), np.zeros((0, 3), np.int64)
    compact = np.full(copy_id.shape[0], -1, dtype=np.int64)
    compact[dup] = np.arange(dup.size)
    nd = np.int64(dup.size)

    def faces_of(mask):
        t = conn_grid[mask]
        out = []
        for omit in range(4):
            keep = [a for a in range(4) if a != omit]
            f = t[:, keep]
            ok = np.all(compact[f] >= 0, axis=1)
            out.append(f[ok])
        f = np.concatenate(out, axis=0)
        s = np.sort(compact[f], axis=1)
        key = (s[:, 0] * nd + s[:, 1]) * nd + s[:, 2]
        return f, key

    fc, kc = faces_of(elem_is_cast)
    fm, km = faces_of(~elem_is_cast)
    common, ic, im = np.intersect1d(kc, km, assume_unique=False, return_indices=True)
    face_grid = fc[ic]
    order = np.argsort(common)
    face_grid = face_grid[order]
    return copy_id[face_grid], face_grid


def apply_permutations(prob, node_perm, elem_perm):
    """Renumber nodes (new id = node_perm[old]) and reorder elements (new row r = old row elem_perm[r])."""
    inv = np.empty_like(node_perm)
    inv[node_perm] = np.arange(node_perm.size)
    out = dict(prob)
    out["xyz"] = prob["xyz"][inv]
    out["T0"] = prob["T0"][inv]
    out["conn"] = node_perm[prob["conn"][elem_perm]].astype(np.int32)
    out["elem_mat"] = prob["elem_mat"][elem_perm]
    for key in ("dirichlet_nodes", "flux_faces", "if_a", "if_b", "contact_faces"):
        if key in prob and prob[key] is not None and np.size(prob[key]):
            out[key] = node_perm[prob[key]].astype(np.int32)
    return out
