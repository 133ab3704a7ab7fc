// Host preprocessing of the casting step (see prep.hpp).
#include "prep.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "elem.hpp"

namespace castfem {

namespace {

[[noreturn]] void fail(int code, const std::string &msg) { throw PrepError{code, msg}; }

// phase timing on stderr when CASTFEM_PREP_TIMING is set
struct PhaseTimer {
    bool on = std::getenv("CASTFEM_PREP_TIMING") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char *what) {
        if (!on) return;
        auto n = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[castfem prep] %-28s %8.3f s\n", what, std::chrono::duration<double>(n - t).count());
        t = n;
    }
};

V3<double> node_x(const std::vector<double> &xyz, int64_t i) {
    return {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
}

// indices 0..n-1 stably sorted by 64-bit key (LSD radix sort over 11-bit
// digits; digits above the largest key and digits equal for every key are skipped)
template <class I>
std::vector<I> sort_by_key(const std::vector<uint64_t> &key) {
    const size_t n = key.size();
    std::vector<I> idx(n), tmp(n);
    for (size_t i = 0; i < n; ++i) idx[i] = (I)i;
    uint64_t kmax = 0;
    for (size_t i = 0; i < n; ++i) kmax = std::max(kmax, key[i]);
    std::vector<uint64_t> k(key), ktmp(n);
    constexpr int DIG = 11, RAD = 1 << DIG;
    std::vector<size_t> cnt(RAD + 1);
    for (int shift = 0; shift < 64 && (kmax >> shift) != 0; shift += DIG) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t i = 0; i < n; ++i) cnt[((k[i] >> shift) & (RAD - 1)) + 1]++;
        bool trivial = false;
        for (int d = 1; d <= RAD; ++d)
            if (cnt[d] == n) trivial = true;
        if (trivial) continue;
        for (int d = 0; d < RAD; ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < n; ++i) {
            size_t pos = cnt[(k[i] >> shift) & (RAD - 1)]++;
            tmp[pos] = idx[i];
            ktmp[pos] = k[i];
        }
        idx.swap(tmp);
        k.swap(ktmp);
    }
    return idx;
}

// area of a triangle, or of a quad as half the norm of the cross product of its diagonals
double face_area(const std::vector<double> &xyz, const int32_t *f, int npf) {
    V3<double> u, v;
    if (npf == 3) {
        u = sub3(node_x(xyz, f[1]), node_x(xyz, f[0]));
        v = sub3(node_x(xyz, f[2]), node_x(xyz, f[0]));
    } else {
        u = sub3(node_x(xyz, f[2]), node_x(xyz, f[0]));
        v = sub3(node_x(xyz, f[3]), node_x(xyz, f[1]));
    }
    V3<double> w = cross3(u, v);
    return 0.5 * std::sqrt(dot3(w, w));
}

// node -> incident element slots (e * nen + a), CSR
void node_elem_csr(const Problem &p, std::vector<int64_t> &ptr, std::vector<int64_t> &inc) {
    ptr.assign(p.N + 1, 0);
    const int64_t tot = p.E * p.nen;
    for (int64_t s = 0; s < tot; ++s) ptr[p.conn[s] + 1]++;
    for (int64_t i = 0; i < p.N; ++i) ptr[i + 1] += ptr[i];
    inc.resize(tot);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t s = 0; s < tot; ++s) inc[fill[p.conn[s]]++] = s;
}

void elem_ke(const Problem &p, int64_t e, double Ke[8][8]) {
    const int32_t *c = &p.conn[e * p.nen];
    double k = p.mats[p.emat[e]].k;
    if (p.nen == 4) {
        double K4[4][4];
        tet_ke<double>(node_x(p.xyz, c[0]), node_x(p.xyz, c[1]), node_x(p.xyz, c[2]), node_x(p.xyz, c[3]), k, K4);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) Ke[a][b] = K4[a][b];
    } else {
        V3<double> x[8];
        for (int a = 0; a < 8; ++a) x[a] = node_x(p.xyz, c[a]);
        double m[8];
        hex_ke_mass<double>(x, k, 1.0, Ke, m);
    }
}

}  // namespace

// ---------------------------------------------------------------- base data
void prep_base(const Problem &p, Base &b) {
    if (p.nen != 4 && p.nen != 8) fail(FEM_E_STATE, "no mesh uploaded");
    if (p.mats.empty()) fail(FEM_E_STATE, "no materials set");
    if ((int64_t)p.T0.size() != p.N) fail(FEM_E_STATE, "no initial temperature set");
    for (size_t q = 0; q < p.mats.size(); ++q) {
        const fem_material &m = p.mats[q];
        if (!(m.k > 0) || !(m.rho > 0) || !(m.c > 0) || !(m.L >= 0) || !(m.T_liq >= m.T_sol))
            fail(FEM_E_INVALID_ARG, "material " + std::to_string(q) + " has invalid properties");
    }
    const int nen = p.nen;
    const int64_t N = p.N, E = p.E;
    PhaseTimer tm;
    b.elem_abs_max = 0.0;
    // node materials
    b.nmat.assign(N, -1);
    for (int64_t e = 0; e < E; ++e) {
        int32_t mt = p.emat[e];
        if (mt < 0 || mt >= (int32_t)p.mats.size()) fail(FEM_E_MESH, "element " + std::to_string(e) + " has no valid material");
        for (int a = 0; a < nen; ++a) {
            int32_t n = p.conn[e * nen + a];
            if (n < 0 || n >= N) fail(FEM_E_MESH, "element " + std::to_string(e) + " refers to node out of range");
            if (b.nmat[n] >= 0 && b.nmat[n] != mt)
                fail(FEM_E_MESH, "node " + std::to_string(n) + " belongs to two materials (duplicate interface nodes)");
            b.nmat[n] = mt;
        }
    }
    for (int64_t i = 0; i < N; ++i)
        if (b.nmat[i] < 0) fail(FEM_E_MESH, "node " + std::to_string(i) + " is in no element");
    if (!p.mat_scen.empty()) {
        if ((int64_t)p.mat_scen.size() != (int64_t)p.mats.size()) fail(FEM_E_STATE, "scenario table does not match the materials");
        for (int32_t sc : p.mat_scen)
            if (sc < 0 || sc >= p.n_scen) fail(FEM_E_INVALID_ARG, "scenario id out of range");
    }
    tm.mark("node materials");
    // lumped capacitance, element orientation
    b.m.assign(N, 0.0);
    for (int64_t e = 0; e < E; ++e) {
        const int32_t *c = &p.conn[e * nen];
        double rho = p.mats[p.emat[e]].rho;
        if (nen == 4) {
            double D = tet_six_vol<double>(node_x(p.xyz, c[0]), node_x(p.xyz, c[1]), node_x(p.xyz, c[2]), node_x(p.xyz, c[3]));
            if (!(D > 0)) fail(FEM_E_MESH, "tetrahedron " + std::to_string(e) + " is inverted or degenerate");
            double w = rho * D / 24.0;  // rho V / 4
            for (int a = 0; a < 4; ++a) b.m[c[a]] += w;
        } else {
            V3<double> x[8];
            for (int a = 0; a < 8; ++a) x[a] = node_x(p.xyz, c[a]);
            double Ke[8][8], me[8];
            double mindet = hex_ke_mass<double>(x, 1.0, rho, Ke, me);
            if (!(mindet > 0)) fail(FEM_E_MESH, "hexahedron " + std::to_string(e) + " is inverted or degenerate");
            for (int a = 0; a < 8; ++a) b.m[c[a]] += me[a];
        }
    }
    tm.mark("lumping");
    // fixed temperatures and the initial field
    b.fixed.assign(N, 0);
    b.T_init = p.T0;
    for (size_t d = 0; d < p.dir_nodes.size(); ++d) {
        int32_t n = p.dir_nodes[d];
        if (n < 0 || n >= N) fail(FEM_E_MESH, "fixed-temperature node out of range");
        b.fixed[n] = 1;
        b.T_init[n] = p.dir_T[d];
    }
    for (int64_t i = 0; i < N; ++i)
        if (!std::isfinite(b.T_init[i])) fail(FEM_E_INVALID_ARG, "initial temperature not finite");
    // convective / flux faces: r_i += a_i - b_i T_i
    b.robin_a.assign(N, 0.0);
    b.robin_b.assign(N, 0.0);
    const int64_t nf = p.npf ? (int64_t)p.flux_faces.size() / p.npf : 0;
    b.any_robin = nf > 0;
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t *fn = &p.flux_faces[f * p.npf];
        for (int a = 0; a < p.npf; ++a)
            if (fn[a] < 0 || fn[a] >= N) fail(FEM_E_MESH, "flux face node out of range");
        double A = face_area(p.xyz, fn, p.npf) / p.npf;
        for (int a = 0; a < p.npf; ++a) {
            b.robin_a[fn[a]] += A * (-p.flux_q[f] + p.flux_h[f] * p.flux_Tinf[f]);
            b.robin_b[fn[a]] += A * p.flux_h[f];
        }
    }
    // interface pairs as symmetric node links: node i of one face and node j of
    // its sister face share w = h A / 9, so r_i += sum_j w_ij (T_j - T_i)
    struct Trip {
        int32_t i, j;
        double w;
    };
    std::vector<Trip> t;
    const int64_t npair = (int64_t)p.if_h.size();
    t.reserve(npair * 18);
    b.pair_w.assign(npair, 0.0);
    for (int64_t f = 0; f < npair; ++f) {
        const int32_t *fa = &p.if_a[3 * f], *fb = &p.if_b[3 * f];
        for (int a = 0; a < 3; ++a)
            if (fa[a] < 0 || fa[a] >= N || fb[a] < 0 || fb[a] >= N) fail(FEM_E_MESH, "interface face node out of range");
        if (p.scen_of_mat(b.nmat[fa[0]]) != p.scen_of_mat(b.nmat[fb[0]]))
            fail(FEM_E_MESH, "interface pair " + std::to_string(f) + " joins two scenarios");
        double A = face_area(p.xyz, fa, 3);
        double w = p.if_h[f] * A / 9.0;
        b.pair_w[f] = w;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                t.push_back({fa[a], fb[c], w});
                t.push_back({fb[c], fa[a], w});
            }
    }
    // contact faces of non-matching meshes: node i of face f takes w = h A_f / 9
    // towards each node of f's sister (one direction only: the sister's own
    // links go to its own sister, so the exchange is not symmetric)
    const int64_t ncf = (int64_t)p.contact_h.size();
    if (ncf > 0) {
        for (int64_t f = 0; f < 3 * ncf; ++f)
            if (p.contact_faces[f] < 0 || p.contact_faces[f] >= N) fail(FEM_E_MESH, "contact face node out of range");
        const auto ts0 = std::chrono::steady_clock::now();
        contact_sisters(p, b.nmat, b.sisters);
        b.sister_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts0).count();
        tm.mark("sister search");
        t.reserve(t.size() + ncf * 9);
        for (int64_t f = 0; f < ncf; ++f) {
            const int32_t *fa = &p.contact_faces[3 * f], *fs = &p.contact_faces[3 * b.sisters[f]];
            const double w = p.contact_h[f] * face_area(p.xyz, fa, 3) / 9.0;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) t.push_back({fa[a], fs[c], w});
        }
    } else {
        b.sisters.clear();
    }
    // CSR by node of trips [t0, t1) of t, equal (i, j) merged
    auto to_csr = [&](size_t t0, size_t t1, std::vector<int32_t> &ptr, std::vector<int32_t> &node,
                      std::vector<double> &wt) {
        std::sort(t.begin() + t0, t.begin() + t1,
                  [](const Trip &x, const Trip &y) { return x.i != y.i ? x.i < y.i : x.j < y.j; });
        ptr.assign(N + 1, 0);
        node.clear();
        wt.clear();
        for (size_t s = t0; s < t1;) {
            size_t u = s;
            double w = 0;
            while (u < t1 && t[u].i == t[s].i && t[u].j == t[s].j) w += t[u++].w;
            node.push_back(t[s].j);
            wt.push_back(w);
            ptr[t[s].i + 1]++;
            s = u;
        }
        for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
    };
    // the contact links alone (before the trips are sorted together)
    to_csr((size_t)npair * 18, t.size(), b.clptr, b.clnode, b.clw);
    to_csr(0, t.size(), b.lptr, b.lnode, b.lw);
    tm.mark("boundary terms");
    // stability bound: Gershgorin rows of the assembled operator over m_i c_i
    std::vector<int64_t> ptr, inc;
    node_elem_csr(p, ptr, inc);
    tm.mark("node-element lists");
    double lam = 0.0;
    std::vector<double> lam_s(p.n_scen, 0.0);
    b.kabs.assign(N, 0.0);
#pragma omp parallel
    {
        std::vector<int32_t> cols;
        std::vector<double> vals;
        std::vector<double> lam_st(p.n_scen, 0.0);
        double lam_t = 0.0, eabs_t = 0.0;
#pragma omp for schedule(dynamic, 4096)
        for (int64_t i = 0; i < N; ++i) {
            cols.clear();
            vals.clear();
            double Ke[8][8];
            double eabs = 0.0;  // sum over elements of sum_j |K^e_ij|
            for (int64_t s = ptr[i]; s < ptr[i + 1]; ++s) {
                int64_t e = inc[s] / nen;
                int a = (int)(inc[s] % nen);
                elem_ke(p, e, Ke);
                for (int c = 0; c < nen; ++c) {
                    int32_t j = p.conn[e * nen + c];
                    size_t q = 0;
                    while (q < cols.size() && cols[q] != j) ++q;
                    if (q == cols.size()) {
                        cols.push_back(j);
                        vals.push_back(0.0);
                    }
                    vals[q] += Ke[a][c];
                    eabs += std::fabs(Ke[a][c]);
                }
            }
            // interface couplings may be summed in the element blocks too
            for (int32_t s = b.lptr[i]; s < b.lptr[i + 1]; ++s) eabs += 2.0 * b.lw[s];
            if (eabs > eabs_t) eabs_t = eabs;
            double kabs = 0.0;
            for (double v : vals) kabs += std::fabs(v);
            b.kabs[i] = kabs;
            double row = b.robin_b[i] + kabs;
            for (int32_t s = b.lptr[i]; s < b.lptr[i + 1]; ++s) row += 2.0 * b.lw[s];
            double li = row / (b.m[i] * p.mats[b.nmat[i]].c);
            if (li > lam_t) lam_t = li;
            const int32_t sc = p.scen_of_mat(b.nmat[i]);
            if (li > lam_st[sc]) lam_st[sc] = li;
        }
#pragma omp critical
        {
            if (lam_t > lam) lam = lam_t;
            if (eabs_t > b.elem_abs_max) b.elem_abs_max = eabs_t;
            for (int32_t sc = 0; sc < p.n_scen; ++sc) lam_s[sc] = std::max(lam_s[sc], lam_st[sc]);
        }
    }
    b.dt_bound = lam > 0 ? 2.0 / lam : INFINITY;
    b.dt_scen.resize(p.n_scen);
    for (int32_t sc = 0; sc < p.n_scen; ++sc) b.dt_scen[sc] = lam_s[sc] > 0 ? 2.0 / lam_s[sc] : INFINITY;
    // temperature span of the data: initial field, fixed values, ambient temperatures
    double tlo = INFINITY, thi = -INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        tlo = std::min(tlo, b.T_init[i]);
        thi = std::max(thi, b.T_init[i]);
    }
    for (double t : p.flux_Tinf) {
        tlo = std::min(tlo, t);
        thi = std::max(thi, t);
    }
    b.T_span = std::max(thi - tlo, 1.0);
    tm.mark("stability bound");
}

// Uniform grid over the face centroids (cell size = the mean longest edge, so a
// cell holds a few centroids of a surface mesh); cells are found by binary
// search in the centroids sorted by cell key.  A query visits the rings of cells
// around its own (Chebyshev distance r = 0, 1, ...) and stops once no unvisited
// cell can hold a centroid closer than the best so far: every centroid in a cell
// at ring distance r + 1 or more lies at least r times the cell size away.
void contact_sisters(const Problem &p, const std::vector<int32_t> &nmat, std::vector<int32_t> &sister) {
    const int64_t nf = (int64_t)p.contact_h.size();
    if ((int64_t)p.contact_side.size() != nf || (int64_t)p.contact_faces.size() != 3 * nf)
        fail(FEM_E_INVALID_ARG, "contact arrays of different lengths");
    std::vector<double> c(3 * nf);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, edge = 0.0;
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t *fn = &p.contact_faces[3 * f];
        for (int j = 0; j < 3; ++j) {
            c[3 * f + j] = ((p.xyz[3 * fn[0] + j] + p.xyz[3 * fn[1] + j]) + p.xyz[3 * fn[2] + j]) / 3.0;
            lo[j] = std::min(lo[j], c[3 * f + j]);
            hi[j] = std::max(hi[j], c[3 * f + j]);
        }
        double e = 0.0;
        for (int a = 0; a < 3; ++a) {
            const V3<double> d = sub3(node_x(p.xyz, fn[(a + 1) % 3]), node_x(p.xyz, fn[a]));
            e = std::max(e, std::sqrt(dot3(d, d)));
        }
        edge += e;
        if (p.contact_side[f] != 0 && p.contact_side[f] != 1) fail(FEM_E_INVALID_ARG, "contact side must be 0 or 1");
    }
    double cell = nf ? edge / (double)nf : 1.0;
    int64_t dim[3];
    for (;;) {
        if (!(cell > 0) || !std::isfinite(cell)) cell = 1.0;
        double cells = 1.0;
        for (int j = 0; j < 3; ++j) {
            dim[j] = (int64_t)std::floor((hi[j] - lo[j]) / cell) + 1;
            cells *= (double)dim[j];
        }
        if (cells < 1e15) break;
        cell *= 2.0;
    }
    auto cell_of = [&](const double *x, int j) {
        return std::min<int64_t>(dim[j] - 1, std::max<int64_t>(0, (int64_t)std::floor((x[j] - lo[j]) / cell)));
    };
    auto key_of = [&](int64_t ix, int64_t iy, int64_t iz) { return (uint64_t)((ix * dim[1] + iy) * dim[2] + iz); };
    // per side: faces sorted by cell key
    std::vector<std::pair<uint64_t, int32_t>> grid[2];
    for (int64_t f = 0; f < nf; ++f) {
        const double *x = &c[3 * f];
        grid[p.contact_side[f]].push_back({key_of(cell_of(x, 0), cell_of(x, 1), cell_of(x, 2)), (int32_t)f});
    }
    for (auto &g : grid) std::sort(g.begin(), g.end());
    auto scen = [&](int64_t f) { return p.scen_of_mat(nmat[p.contact_faces[3 * f]]); };
    sister.assign(nf, -1);
    const int64_t rmax = std::max(dim[0], std::max(dim[1], dim[2]));
    bool missing = false;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t f = 0; f < nf; ++f) {
        const auto &g = grid[1 - p.contact_side[f]];
        const double *a = &c[3 * f];
        const int64_t q[3] = {cell_of(a, 0), cell_of(a, 1), cell_of(a, 2)};
        const int32_t sf = scen(f);
        double best = INFINITY;
        int64_t arg = -1;
        for (int64_t r = 0; r <= rmax; ++r) {
            for (int64_t ix = q[0] - r; ix <= q[0] + r; ++ix) {
                if (ix < 0 || ix >= dim[0]) continue;
                for (int64_t iy = q[1] - r; iy <= q[1] + r; ++iy) {
                    if (iy < 0 || iy >= dim[1]) continue;
                    const bool face_xy = ix == q[0] - r || ix == q[0] + r || iy == q[1] - r || iy == q[1] + r;
                    for (int64_t iz = q[2] - r; iz <= q[2] + r; iz += (face_xy ? 1 : 2 * r > 0 ? 2 * r : 1)) {
                        if (iz < 0 || iz >= dim[2]) continue;
                        const uint64_t k = key_of(ix, iy, iz);
                        auto it = std::lower_bound(g.begin(), g.end(), std::make_pair(k, (int32_t)INT32_MIN));
                        for (; it != g.end() && it->first == k; ++it) {
                            const int64_t h = it->second;
                            if (scen(h) != sf) continue;
                            const double *b = &c[3 * h];
                            const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
                            const double d2 = (dx * dx + dy * dy) + dz * dz;
                            if (d2 < best || (d2 == best && h < arg)) {
                                best = d2;
                                arg = h;
                            }
                        }
                    }
                }
            }
            const double reach = (double)r * cell;
            if (arg >= 0 && best < reach * reach * (1.0 - 1e-9)) break;
        }
        if (arg < 0) {
#pragma omp atomic write
            missing = true;
        } else {
            sister[f] = (int32_t)arg;
        }
    }
    if (missing) fail(FEM_E_MESH, "a contact face has no face on the other side in its scenario");
}

int64_t bandwidth(const Problem &p, const Base &b, const std::vector<int32_t> *perm) {
    auto id = [&](int32_t n) -> int64_t { return perm ? (*perm)[n] : n; };
    int64_t bw = 0;
    for (int64_t e = 0; e < p.E; ++e) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int a = 0; a < p.nen; ++a) {
            int64_t v = id(p.conn[e * p.nen + a]);
            lo = std::min(lo, v);
            hi = std::max(hi, v);
        }
        bw = std::max(bw, hi - lo);
    }
    for (int64_t i = 0; i < p.N; ++i)
        for (int32_t s = b.lptr[i]; s < b.lptr[i + 1]; ++s) bw = std::max(bw, std::abs(id((int32_t)i) - id(b.lnode[s])));
    return bw;
}

// ---------------------------------------------------------------- orderings
namespace {

// Node graph (element edges and interface links), CSR with sorted unique neighbours.
void node_graph(const Problem &p, const Base &b, std::vector<int64_t> &gptr, std::vector<int32_t> &adj) {
    std::vector<int64_t> ptr, inc;
    node_elem_csr(p, ptr, inc);
    const int64_t N = p.N;
    std::vector<int32_t> deg(N);
#pragma omp parallel
    {
        std::vector<int32_t> nb;
#pragma omp for schedule(dynamic, 4096)
        for (int64_t i = 0; i < N; ++i) {
            nb.clear();
            for (int64_t s = ptr[i]; s < ptr[i + 1]; ++s) {
                int64_t e = inc[s] / p.nen;
                for (int c = 0; c < p.nen; ++c) {
                    int32_t j = p.conn[e * p.nen + c];
                    if (j != i) nb.push_back(j);
                }
            }
            for (int32_t s = b.lptr[i]; s < b.lptr[i + 1]; ++s) nb.push_back(b.lnode[s]);
            std::sort(nb.begin(), nb.end());
            deg[i] = (int32_t)(std::unique(nb.begin(), nb.end()) - nb.begin());
        }
    }
    gptr.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) gptr[i + 1] = gptr[i] + deg[i];
    adj.resize(gptr[N]);
#pragma omp parallel
    {
        std::vector<int32_t> nb;
#pragma omp for schedule(dynamic, 4096)
        for (int64_t i = 0; i < N; ++i) {
            nb.clear();
            for (int64_t s = ptr[i]; s < ptr[i + 1]; ++s) {
                int64_t e = inc[s] / p.nen;
                for (int c = 0; c < p.nen; ++c) {
                    int32_t j = p.conn[e * p.nen + c];
                    if (j != i) nb.push_back(j);
                }
            }
            for (int32_t s = b.lptr[i]; s < b.lptr[i + 1]; ++s) nb.push_back(b.lnode[s]);
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
            std::copy(nb.begin(), nb.end(), adj.begin() + gptr[i]);
        }
    }
}

// breadth-first level structure from `root` over unvisited-in-component nodes;
// returns the last level and the depth
int bfs_levels(const std::vector<int64_t> &gptr, const std::vector<int32_t> &adj, int32_t root,
               std::vector<int32_t> &mark, int32_t stamp, std::vector<int32_t> &last) {
    std::vector<int32_t> cur{root}, nxt;
    mark[root] = stamp;
    int depth = 0;
    for (;;) {
        nxt.clear();
        for (int32_t u : cur)
            for (int64_t s = gptr[u]; s < gptr[u + 1]; ++s) {
                int32_t v = adj[s];
                if (mark[v] != stamp) {
                    mark[v] = stamp;
                    nxt.push_back(v);
                }
            }
        if (nxt.empty()) break;
        cur.swap(nxt);
        ++depth;
    }
    last = cur;
    return depth;
}

}  // namespace

// Reverse Cuthill-McKee: per connected component, a pseudo-peripheral start
// node (repeated breadth-first searches from a minimum-degree node of the last
// level while the depth grows), then a breadth-first numbering that visits
// neighbours in increasing degree, reversed at the end.
std::vector<int32_t> order_rcm(const Problem &p, const Base &b) {
    std::vector<int64_t> gptr;
    std::vector<int32_t> adj;
    node_graph(p, b, gptr, adj);
    const int64_t N = p.N;
    auto deg = [&](int32_t u) { return gptr[u + 1] - gptr[u]; };
    std::vector<int32_t> order;
    order.reserve(N);
    std::vector<uint8_t> done(N, 0);
    std::vector<int32_t> mark(N, -1);
    int32_t stamp = 0;
    // nodes by degree, to seed each component at a low-degree node
    std::vector<uint64_t> dkey(N);
    for (int64_t i = 0; i < N; ++i) dkey[i] = (uint64_t)deg((int32_t)i);
    std::vector<int32_t> bydeg = sort_by_key<int32_t>(dkey);
    std::vector<int32_t> last, nb;
    for (int32_t seed : bydeg) {
        if (done[seed]) continue;
        int32_t root = seed;
        int depth = bfs_levels(gptr, adj, root, mark, stamp++, last);
        for (int it = 0; it < 16; ++it) {
            int32_t best = last[0];
            for (int32_t v : last)
                if (deg(v) < deg(best)) best = v;
            int d2 = bfs_levels(gptr, adj, best, mark, stamp++, last);
            if (d2 <= depth) break;
            depth = d2;
            root = best;
        }
        size_t head = order.size();
        order.push_back(root);
        done[root] = 1;
        while (head < order.size()) {
            int32_t u = order[head++];
            nb.clear();
            for (int64_t s = gptr[u]; s < gptr[u + 1]; ++s)
                if (!done[adj[s]]) {
                    nb.push_back(adj[s]);
                    done[adj[s]] = 1;
                }
            std::stable_sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) { return deg(x) < deg(y); });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::vector<int32_t> perm(N);
    for (int64_t r = 0; r < N; ++r) perm[order[N - 1 - r]] = (int32_t)r;
    return perm;
}

namespace {

// Hilbert index of a point with `bits`-bit coordinates: the axes are turned
// into the transposed Hilbert form by Skilling's inverse-undo and Gray-code
// passes ("Programming the Hilbert curve", AIP Conf. Proc. 707, 2004), then
// the bits are interleaved, most significant level first.
uint64_t hilbert3(uint32_t X[3], int bits) {
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int bit = bits - 1; bit >= 0; --bit)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> bit) & 1u);
    return h;
}

uint64_t morton3(const uint32_t X[3], int bits) {
    uint64_t h = 0;
    for (int bit = bits - 1; bit >= 0; --bit)
        for (int i = 2; i >= 0; --i) h = (h << 1) | ((X[i] >> bit) & 1u);
    return h;
}

struct Quant {
    double lo[3], scale[3];
    int bits = 21;
    // `count` points will be keyed: about 2^4 cells per point and axis resolve them
    Quant(const std::vector<double> &xyz, int64_t N, int64_t count) {
        bits = 4;
        while (bits < 21 && ((int64_t)1 << (3 * (bits - 4))) < count) ++bits;
        double hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = INFINITY;
            hi[d] = -INFINITY;
        }
        for (int64_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], xyz[3 * i + d]);
                hi[d] = std::max(hi[d], xyz[3 * i + d]);
            }
        double ext = 0;
        for (int d = 0; d < 3; ++d) ext = std::max(ext, hi[d] - lo[d]);
        for (int d = 0; d < 3; ++d) scale[d] = ext > 0 ? ((1u << bits) - 1) / ext : 0.0;
    }
    uint64_t key(double x, double y, double z, bool hilbert) const {
        double v[3] = {x, y, z};
        uint32_t X[3];
        for (int d = 0; d < 3; ++d) {
            double q = (v[d] - lo[d]) * scale[d];
            X[d] = (uint32_t)std::min(std::max(q, 0.0), (double)((1u << bits) - 1));
        }
        return hilbert ? hilbert3(X, bits) : morton3(X, bits);
    }
};

}  // namespace

std::vector<int32_t> order_sfc(const Problem &p, bool hilbert) {
    const int64_t N = p.N;
    Quant qz(p.xyz, N, N);
    std::vector<uint64_t> key(N);
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) key[i] = qz.key(p.xyz[3 * i], p.xyz[3 * i + 1], p.xyz[3 * i + 2], hilbert);
    std::vector<int32_t> idx = sort_by_key<int32_t>(key);
    std::vector<int32_t> perm(N);
    for (int64_t r = 0; r < N; ++r) perm[idx[r]] = (int32_t)r;
    return perm;
}

// ---------------------------------------------------------------- layout
namespace {

// element order for a node ordering: SFC key of the centroid for curve
// orderings, the smallest and largest renumbered node otherwise; the keys of
// the ordered elements in `keys`
std::vector<int64_t> element_order(const Problem &p, const std::vector<int32_t> &perm, int ordering,
                                   std::vector<uint64_t> &keys) {
    const int64_t E = p.E;
    const int nen = p.nen;
    std::vector<uint64_t> key(E);
    if (ordering == FEM_ORDER_NONE) {
        for (int64_t e = 0; e < E; ++e) key[e] = (uint64_t)e;
    } else if (ordering == FEM_ORDER_MORTON || ordering == FEM_ORDER_HILBERT) {
        Quant qz(p.xyz, p.N, E);
#pragma omp parallel for
        for (int64_t e = 0; e < E; ++e) {
            double c[3] = {0, 0, 0};
            for (int a = 0; a < nen; ++a)
                for (int d = 0; d < 3; ++d) c[d] += p.xyz[3 * (int64_t)p.conn[e * nen + a] + d];
            key[e] = qz.key(c[0] / nen, c[1] / nen, c[2] / nen, ordering == FEM_ORDER_HILBERT);
        }
    } else {
#pragma omp parallel for
        for (int64_t e = 0; e < E; ++e) {
            uint64_t lo = UINT64_MAX, hi = 0;
            for (int a = 0; a < nen; ++a) {
                uint64_t v = (uint64_t)perm[p.conn[e * nen + a]];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            key[e] = (lo << 32) | hi;
        }
    }
    std::vector<int64_t> order = ordering == FEM_ORDER_NONE ? std::vector<int64_t>() : sort_by_key<int64_t>(key);
    if (ordering == FEM_ORDER_NONE) {
        order.resize(E);
        std::iota(order.begin(), order.end(), 0);
    }
    keys.resize(E);
    for (int64_t r = 0; r < E; ++r) keys[r] = key[order[r]];
    return order;
}

// matched interface pairs in the same kind of order: the centroid of face a (which
// face b shares) for curve orderings, the smallest and largest renumbered node of
// the six otherwise, after every element without an ordering
std::vector<int64_t> pair_order(const Problem &p, const std::vector<int32_t> &perm, int ordering,
                                std::vector<uint64_t> &keys) {
    const int64_t P = (int64_t)p.if_h.size();
    std::vector<uint64_t> key(P);
    if (ordering == FEM_ORDER_NONE) {
        for (int64_t f = 0; f < P; ++f) key[f] = (uint64_t)(p.E + f);
    } else if (ordering == FEM_ORDER_MORTON || ordering == FEM_ORDER_HILBERT) {
        Quant qz(p.xyz, p.N, p.E);
        for (int64_t f = 0; f < P; ++f) {
            double c[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d) c[d] += p.xyz[3 * (int64_t)p.if_a[3 * f + a] + d];
            key[f] = qz.key(c[0] / 3, c[1] / 3, c[2] / 3, ordering == FEM_ORDER_HILBERT);
        }
    } else {
        for (int64_t f = 0; f < P; ++f) {
            uint64_t lo = UINT64_MAX, hi = 0;
            for (int a = 0; a < 6; ++a) {
                const uint64_t v = (uint64_t)perm[a < 3 ? p.if_a[3 * f + a] : p.if_b[3 * f + a - 3]];
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
            key[f] = (lo << 32) | hi;
        }
    }
    std::vector<int64_t> order = sort_by_key<int64_t>(key);
    keys.resize(P);
    for (int64_t r = 0; r < P; ++r) keys[r] = key[order[r]];
    return order;
}

}  // namespace

void prep_order(const Problem &p, const Base &b, int ordering, Ordering &ord) {
    PhaseTimer tm;
    if (ordering == FEM_ORDER_RCM) ord.perm = order_rcm(p, b);
    else if (ordering == FEM_ORDER_MORTON) ord.perm = order_sfc(p, false);
    else if (ordering == FEM_ORDER_HILBERT) ord.perm = order_sfc(p, true);
    else if (ordering == FEM_ORDER_NONE) {
        ord.perm.resize(p.N);
        std::iota(ord.perm.begin(), ord.perm.end(), 0);
    } else fail(FEM_E_INVALID_ARG, "unknown ordering");
    tm.mark("node ordering");
    ord.eorder = element_order(p, ord.perm, ordering, ord.ekey);
    ord.porder = pair_order(p, ord.perm, ordering, ord.pkey);
    ord.escen.assign(p.E, 0);
    ord.pscen.assign(ord.porder.size(), 0);
    tm.mark("element ordering");
    if (p.n_scen > 1) {
        // a batch is numbered scenario by scenario (the ordering applies
        // inside each scenario), so no block ever spans two scenarios
        std::vector<int32_t> nm(p.N, 0);
        for (int64_t e = 0; e < p.E; ++e)
            for (int a = 0; a < p.nen; ++a) nm[p.conn[e * p.nen + a]] = p.emat[e];
        std::vector<uint64_t> key(p.N);
        for (int64_t i = 0; i < p.N; ++i) key[i] = ((uint64_t)p.scen_of_mat(nm[i]) << 32) | (uint32_t)ord.perm[i];
        std::vector<int32_t> idx = sort_by_key<int32_t>(key);
        for (int64_t r = 0; r < p.N; ++r) ord.perm[idx[r]] = (int32_t)r;
        std::vector<uint64_t> ekey(p.E);
        for (int64_t r = 0; r < p.E; ++r) ekey[r] = ((uint64_t)p.scen_of_mat(p.emat[ord.eorder[r]]) << 40) | (uint64_t)r;
        std::vector<int64_t> eidx = sort_by_key<int64_t>(ekey);
        std::vector<int64_t> e2(p.E);
        std::vector<uint64_t> k2(p.E);
        for (int64_t r = 0; r < p.E; ++r) {
            e2[r] = ord.eorder[eidx[r]];
            k2[r] = ord.ekey[eidx[r]];
            ord.escen[r] = (uint64_t)p.scen_of_mat(p.emat[e2[r]]);
        }
        ord.eorder.swap(e2);
        ord.ekey.swap(k2);
        // interface pairs likewise (a pair never joins two scenarios)
        const int64_t P = (int64_t)ord.porder.size();
        std::vector<uint64_t> pk(P);
        for (int64_t r = 0; r < P; ++r) pk[r] = ((uint64_t)p.scen_of_mat(nm[p.if_a[3 * ord.porder[r]]]) << 40) | (uint64_t)r;
        std::vector<int64_t> pidx = sort_by_key<int64_t>(pk);
        std::vector<int64_t> p2(P);
        std::vector<uint64_t> q2(P);
        for (int64_t r = 0; r < P; ++r) {
            p2[r] = ord.porder[pidx[r]];
            q2[r] = ord.pkey[pidx[r]];
            ord.pscen[r] = (uint64_t)p.scen_of_mat(nm[p.if_a[3 * p2[r]]]);
        }
        ord.porder.swap(p2);
        ord.pkey.swap(q2);
        tm.mark("scenario-major order");
    }
}

void prep_layout(const Problem &p, const Base &b, const PrepOptions &o, const Ordering &ord, Layout &L) {
    const int64_t N = p.N, E = p.E;
    const int nen = p.nen;
    L.nen = nen;
    L.N = N;
    L.E = E;
    L.dt_bound = b.dt_bound;
    L.xtra.clear();
    L.n_partial_slots = 0;
    // 1. locality ordering of nodes and elements
    std::vector<int32_t> perm = ord.perm;
    std::vector<int64_t> eorder = ord.eorder;

    // matched interface pairs as block elements (blocked enthalpy step): their
    // couplings leave the node links, which keep the contact faces alone
    const bool pairs_in_blocks = o.interface_in_blocks && o.scatter == FEM_SCATTER_LDS_BLOCKED && !ord.porder.empty();
    const std::vector<int32_t> &lptr = pairs_in_blocks ? b.clptr : b.lptr;
    const std::vector<int32_t> &lnode = pairs_in_blocks ? b.clnode : b.lnode;
    const std::vector<double> &lw = pairs_in_blocks ? b.clw : b.lw;
    auto has_bc = [&](int64_t i) {
        return b.robin_b[i] != 0.0 || b.robin_a[i] != 0.0 || lptr[i + 1] > lptr[i];
    };
    L.vconn.clear();
    L.vw.clear();

    // 2. element blocks (LDS-blocked scatter) and the final node numbering
    if (o.scatter == FEM_SCATTER_LDS_BLOCKED) {
        if (o.max_local_nodes > 65535) fail(FEM_E_INVALID_ARG, "block node cap above 65535");
        std::vector<int64_t> stamp(N, -1);
        // the elements (in eorder) and the interface pairs (in ord.porder) of
        // every block: both streams are sorted by (scenario, key), and a block
        // takes the next item of their merge until a cap or a scenario change
        struct Blk {
            int64_t e0, ne, v0, nv;
        };
        std::vector<Blk> blk;
        const int64_t P = pairs_in_blocks ? (int64_t)ord.porder.size() : 0;
        auto item_nodes = [&](bool pair, int64_t k, int32_t *nd) {
            if (!pair) {
                for (int a = 0; a < nen; ++a) nd[a] = p.conn[eorder[k] * nen + a];
                return nen;
            }
            const int64_t f = ord.porder[k];
            for (int a = 0; a < 3; ++a) {
                nd[a] = p.if_a[3 * f + a];
                nd[3 + a] = p.if_b[3 * f + a];
            }
            return 6;
        };
        int64_t cur = 0, nloc = 0, e0 = 0, v0 = 0, ie = 0, iv = 0;
        int32_t cur_scen = -1;
        while (ie < E || iv < P) {
            const bool pair = iv < P && (ie >= E || ord.pscen[iv] < ord.escen[ie] ||
                                         (ord.pscen[iv] == ord.escen[ie] && ord.pkey[iv] < ord.ekey[ie]));
            int32_t nd[8];
            const int k = item_nodes(pair, pair ? iv : ie, nd);
            int nnew = 0;
            for (int a = 0; a < k; ++a) nnew += stamp[nd[a]] != cur;
            const int64_t cnt = (ie - e0) + (iv - v0);
            const int32_t sc = pair ? (int32_t)ord.pscen[iv] : p.scen_of_mat(p.emat[eorder[ie]]);
            if (cur_scen < 0) cur_scen = sc;
            if (cnt > 0 && (cnt + 1 > o.block_elems || nloc + nnew > o.max_local_nodes || sc != cur_scen)) {
                cur_scen = sc;
                blk.push_back({e0, ie - e0, v0, iv - v0});
                ++cur;
                e0 = ie;
                v0 = iv;
                nloc = 0;
                nnew = k;
                for (int a = 0; a < k; ++a)
                    for (int q = 0; q < a; ++q)
                        if (nd[q] == nd[a]) --nnew;
            }
            for (int a = 0; a < k; ++a) stamp[nd[a]] = cur;
            nloc += nnew;
            if (pair) ++iv;
            else ++ie;
        }
        if ((ie - e0) + (iv - v0) > 0) blk.push_back({e0, ie - e0, v0, iv - v0});
        const int64_t nb = (int64_t)blk.size();
        // blocks touching each node; owner block of private nodes
        std::vector<int32_t> nblk(N, 0), owner(N, -1);
        std::fill(stamp.begin(), stamp.end(), -1);
        auto block_nodes = [&](int64_t q, auto &&visit) {
            int32_t nd[8];
            for (int64_t s = blk[q].e0; s < blk[q].e0 + blk[q].ne; ++s)
                for (int a = 0, k = item_nodes(false, s, nd); a < k; ++a) visit(nd[a]);
            for (int64_t v = blk[q].v0; v < blk[q].v0 + blk[q].nv; ++v)
                for (int a = 0, k = item_nodes(true, v, nd); a < k; ++a) visit(nd[a]);
        };
        for (int64_t q = 0; q < nb; ++q)
            block_nodes(q, [&](int32_t n) {
                if (stamp[n] != q) {
                    stamp[n] = q;
                    nblk[n]++;
                    if (owner[n] < 0) owner[n] = (int32_t)q;
                }
            });
        // private nodes grouped by owner block, in ordering rank within a block;
        // shared nodes after them ordered by first block then rank
        std::vector<int32_t> priv, shar;
        // nodes with boundary terms or a fixed temperature are always shared,
        // so all boundary inflow is computed by the node kernel
        auto special = [&](int64_t i) { return has_bc(i) || b.fixed[i]; };
        for (int64_t i = 0; i < N; ++i) (nblk[i] == 1 && !special(i) ? priv : shar).push_back((int32_t)i);
        auto by_owner_rank = [&](std::vector<int32_t> &v) {
            std::vector<uint64_t> key(v.size());
            for (size_t r = 0; r < v.size(); ++r) key[r] = ((uint64_t)owner[v[r]] << 32) | (uint32_t)perm[v[r]];
            std::vector<int64_t> o2 = sort_by_key<int64_t>(key);
            std::vector<int32_t> out(v.size());
            for (size_t r = 0; r < v.size(); ++r) out[r] = v[o2[r]];
            v.swap(out);
        };
        by_owner_rank(priv);
        by_owner_rank(shar);
        // shared nodes carrying boundary inflow (Robin faces, fixed temperature)
        // come first: only the node-kernel workgroups covering them reduce it
        auto inflow = [&](int32_t i) { return b.fixed[i] || b.robin_b[i] != 0.0 || b.robin_a[i] != 0.0; };
        const auto inflow_end = std::stable_partition(shar.begin(), shar.end(), inflow);
        // then the other nodes with boundary terms (interface links), so that the
        // node-kernel workgroups that follow have none; then the nodes in at most
        // PARTIAL_SLOTS blocks, then the few in more: only the workgroups covering
        // those read extra partials
        const auto bc_end = std::stable_partition(inflow_end, shar.end(), [&](int32_t i) { return has_bc(i); });
        std::stable_partition(bc_end, shar.end(), [&](int32_t i) { return nblk[i] <= PARTIAL_SLOTS; });
        L.n_inflow = (int64_t)(inflow_end - shar.begin());
        L.n_private = (int64_t)priv.size();
        std::vector<int32_t> fin(N);
        for (size_t r = 0; r < priv.size(); ++r) fin[priv[r]] = (int32_t)r;
        for (size_t r = 0; r < shar.size(); ++r) fin[shar[r]] = (int32_t)(priv.size() + r);
        perm.swap(fin);
        // per block: private range, shared list, local connectivity
        std::vector<int64_t> priv_begin(nb + 1, 0);
        for (int32_t n : priv) priv_begin[owner[n] + 1]++;
        for (int64_t q = 0; q < nb; ++q) priv_begin[q + 1] += priv_begin[q];
        L.blocks.resize(nb);
        L.sh_list.clear();
        L.lconn.resize(E * nen);
        L.vconn.assign(6 * P, 0);
        L.vw.assign(P, 0.0);
        L.max_local = 0;
        std::vector<int32_t> local(N, -1);
        std::vector<int32_t> shl;
        std::vector<uint64_t> cmask;
        std::vector<int32_t> bcol;
        std::vector<int64_t> bord;
        for (int64_t q = 0; q < nb; ++q) {
            BlockInfo &bi = L.blocks[q];
            bi.e_begin = (int32_t)blk[q].e0;
            bi.n_e = (int32_t)blk[q].ne;
            bi.v_begin = (int32_t)blk[q].v0;
            bi.n_v = (int32_t)blk[q].nv;
            bi.int_base = (int32_t)priv_begin[q];
            bi.n_int = (int32_t)(priv_begin[q + 1] - priv_begin[q]);
            shl.clear();
            block_nodes(q, [&](int32_t n) {
                if (perm[n] >= L.n_private) shl.push_back(perm[n]);
            });
            std::sort(shl.begin(), shl.end());
            shl.erase(std::unique(shl.begin(), shl.end()), shl.end());
            bi.sh_begin = (int32_t)L.sh_list.size();
            bi.n_sh = (int32_t)shl.size();
            bi.pad0 = bi.pad1 = 0;
            L.sh_list.insert(L.sh_list.end(), shl.begin(), shl.end());
            for (size_t r = 0; r < shl.size(); ++r) local[shl[r]] = bi.n_int + (int32_t)r;
            const int64_t nl = bi.n_int + bi.n_sh;
            L.max_local = std::max<int64_t>(L.max_local, nl);
            const int64_t b0 = blk[q].e0, b1 = blk[q].e0 + blk[q].ne;
            auto local_id = [&](int64_t s, int a) {
                int32_t g = perm[p.conn[eorder[s] * nen + a]];
                int32_t l = g < L.n_private ? g - bi.int_base : local[g];
                if (l < 0 || l >= nl) fail(FEM_E_MESH, "internal: block numbering");
                return l;
            };
            if (o.color_in_block) {
                // greedy colouring inside the block, then elements ordered by
                // colour: the elements of one wavefront then touch distinct
                // nodes and their LDS additions do not collide on one address
                cmask.assign(2 * nl, 0);
                bcol.resize(b1 - b0);
                int ncol = 0;
                for (int64_t s = b0; s < b1; ++s) {
                    uint64_t f0 = 0, f1 = 0;
                    for (int a = 0; a < nen; ++a) {
                        int32_t l = local_id(s, a);
                        f0 |= cmask[2 * l];
                        f1 |= cmask[2 * l + 1];
                    }
                    int k;
                    if (~f0) k = __builtin_ctzll(~f0);
                    else if (~f1) k = 64 + __builtin_ctzll(~f1);
                    else fail(FEM_E_UNSUPPORTED, "block colouring needs more than 128 colours");
                    bcol[s - b0] = k;
                    ncol = std::max(ncol, k + 1);
                    for (int a = 0; a < nen; ++a) cmask[2 * local_id(s, a) + (k >> 6)] |= 1ull << (k & 63);
                }
                std::vector<int64_t> cstart(ncol + 1, 0);
                for (int64_t s = b0; s < b1; ++s) cstart[bcol[s - b0] + 1]++;
                for (int c = 0; c < ncol; ++c) cstart[c + 1] += cstart[c];
                bord.resize(b1 - b0);
                for (int64_t s = b0; s < b1; ++s) bord[cstart[bcol[s - b0]]++] = eorder[s];
                std::copy(bord.begin(), bord.end(), eorder.begin() + b0);
            }
            for (int64_t s = b0; s < b1; ++s)
                for (int a = 0; a < nen; ++a) L.lconn[s * nen + a] = (uint16_t)local_id(s, a);
            // interface pairs: face a then face b, in local ids, with their coupling
            for (int64_t v = blk[q].v0; v < blk[q].v0 + blk[q].nv; ++v) {
                int32_t nd[8];
                item_nodes(true, v, nd);
                for (int a = 0; a < 6; ++a) {
                    const int32_t g = perm[nd[a]];
                    const int32_t l = g < L.n_private ? g - bi.int_base : local[g];
                    if (l < 0 || l >= nl) fail(FEM_E_MESH, "internal: block numbering of an interface pair");
                    L.vconn[v * 6 + a] = (uint16_t)l;
                }
                L.vw[v] = b.pair_w[ord.porder[v]];
            }
        }
        if (L.max_local > o.max_local_nodes) fail(FEM_E_INVALID_ARG, "internal: block above node cap");
        // tets with 12-bit local ids: 6 bytes of connectivity per element instead of 8
        L.lconn12.clear();
        if (nen == 4 && L.max_local <= 4096) {
            L.lconn12.assign(3 * ((E + 1) / 2), 0u);
            for (int64_t e = 0; e < E; e += 2) {
                uint64_t v[2] = {0, 0};
                for (int h = 0; h < 2 && e + h < E; ++h)
                    for (int a = 0; a < 4; ++a) v[h] |= (uint64_t)L.lconn[(e + h) * 4 + a] << (12 * a);
                const uint64_t lo = v[0] | (v[1] << 48);
                uint32_t *w = &L.lconn12[3 * (e / 2)];
                w[0] = (uint32_t)lo;
                w[1] = (uint32_t)(lo >> 32);
                w[2] = (uint32_t)(v[1] >> 16);
            }
        }
        // partial slots: the j-th block (in block order) of shared node s writes
        // slot j < PARTIAL_SLOTS at j * nsh + s (slot-major, so the combine's
        // loads are coalesced and need no index; unused slots stay zero), and
        // the rest at PARTIAL_SLOTS * nsh + comb_ptr[s] + j - PARTIAL_SLOTS
        const int64_t nsh = N - L.n_private;
        L.comb_ptr.assign(nsh + 1, 0);
        for (int64_t s = 0; s < nsh; ++s)
            L.comb_ptr[s + 1] = std::max<int32_t>(nblk[shar[s]] - PARTIAL_SLOTS, 0);
        for (int64_t s = 0; s < nsh; ++s) L.comb_ptr[s + 1] += L.comb_ptr[s];
        L.sh_pos.resize(L.sh_list.size());
        std::vector<int32_t> rank(nsh, 0);
        for (size_t slot = 0; slot < L.sh_list.size(); ++slot) {
            const int64_t s = L.sh_list[slot] - L.n_private;
            const int32_t j = rank[s]++;
            L.sh_pos[slot] = j < PARTIAL_SLOTS ? (int32_t)(j * nsh + s)
                                               : (int32_t)(PARTIAL_SLOTS * nsh + L.comb_ptr[s] + j - PARTIAL_SLOTS);
        }
        for (int64_t s = 0; s < nsh; ++s)
            if (rank[s] != nblk[shar[s]]) fail(FEM_E_MESH, "internal: partial slots");
        L.n_partial_slots = PARTIAL_SLOTS * nsh + L.comb_ptr[nsh];
        L.xtra.assign(N, 0);
        for (int64_t s = 0; s < nsh; ++s) L.xtra[L.n_private + s] = nblk[shar[s]] > PARTIAL_SLOTS;
        L.bc_first = L.n_private;
        L.n_bc_slots = nsh;
        L.block_elems = o.block_elems;
    } else {
        L.bc_first = 0;
        L.n_bc_slots = N;
        L.n_private = 0;
        L.n_inflow = N;
    }

    // 3. colouring (colour by colour scatter): greedy first-fit in element order
    if (o.scatter == FEM_SCATTER_COLORED) {
        std::vector<uint64_t> used(2 * N, 0);
        std::vector<int32_t> col(E);
        int ncol = 0;
        for (int64_t s = 0; s < E; ++s) {
            const int32_t *c = &p.conn[eorder[s] * nen];
            uint64_t f0 = 0, f1 = 0;
            for (int a = 0; a < nen; ++a) {
                f0 |= used[2 * c[a]];
                f1 |= used[2 * c[a] + 1];
            }
            int k;
            if (~f0) k = __builtin_ctzll(~f0);
            else if (~f1) k = 64 + __builtin_ctzll(~f1);
            else fail(FEM_E_UNSUPPORTED, "element colouring needs more than 128 colours");
            col[s] = k;
            ncol = std::max(ncol, k + 1);
            for (int a = 0; a < nen; ++a) used[2 * c[a] + (k >> 6)] |= 1ull << (k & 63);
        }
        std::vector<uint64_t> ckey(col.begin(), col.end());
        std::vector<int64_t> idx = sort_by_key<int64_t>(ckey);
        std::vector<int64_t> e2(E);
        for (int64_t s = 0; s < E; ++s) e2[s] = eorder[idx[s]];
        eorder.swap(e2);
        L.color_ptr.assign(ncol + 1, 0);
        for (int64_t s = 0; s < E; ++s) L.color_ptr[col[s] + 1]++;
        for (int c = 0; c < ncol; ++c) L.color_ptr[c + 1] += L.color_ptr[c];
    }

    // 4. arrays in the final numbering
    L.perm = perm;
    L.iperm.assign(N, 0);
    for (int64_t i = 0; i < N; ++i) L.iperm[perm[i]] = (int32_t)i;
    L.xyz.resize(3 * N);
    L.nflag.resize(N);
    L.m.resize(N);
    L.T_init.resize(N);
    for (int64_t n = 0; n < N; ++n) {
        int64_t i = L.iperm[n];
        for (int d = 0; d < 3; ++d) L.xyz[3 * n + d] = p.xyz[3 * i + d];
        L.nflag[n] = (uint32_t)b.nmat[i] | (b.fixed[i] ? NODE_FIXED : 0u) | (has_bc(i) ? NODE_BC : 0u) |
                     (!L.xtra.empty() && L.xtra[n] ? NODE_XTRA : 0u);
        L.m[n] = b.m[i];
        L.T_init[n] = b.T_init[i];
    }
    L.conn.resize(E * nen);
    for (int64_t s = 0; s < E; ++s)
        for (int a = 0; a < nen; ++a) L.conn[s * nen + a] = perm[p.conn[eorder[s] * nen + a]];
    // boundary slots
    L.robin_a.clear();
    L.robin_b.clear();
    if (b.any_robin) {
        L.robin_a.resize(L.n_bc_slots);
        L.robin_b.resize(L.n_bc_slots);
    }
    L.link_ptr.assign(L.n_bc_slots + 1, 0);
    L.link_node.clear();
    L.link_w.clear();
    for (int64_t s = 0; s < L.n_bc_slots; ++s) {
        int64_t i = L.iperm[L.bc_first + s];
        if (b.any_robin) {
            L.robin_a[s] = b.robin_a[i];
            L.robin_b[s] = b.robin_b[i];
        }
        for (int32_t q = lptr[i]; q < lptr[i + 1]; ++q) {
            L.link_node.push_back(perm[lnode[q]]);
            L.link_w.push_back(lw[q]);
        }
        L.link_ptr[s + 1] = (int32_t)L.link_node.size();
    }
    // a private node never carries boundary terms
    for (int64_t n = 0; n < L.n_private; ++n)
        if (has_bc(L.iperm[n]) || b.fixed[L.iperm[n]]) fail(FEM_E_MESH, "internal: boundary node classed private");
    // scenario segments of the final numbering
    L.seg_begin.clear();
    L.seg_scen.clear();
    for (int64_t n = 0; n < N; ++n) {
        const int32_t sc = p.scen_of_mat(b.nmat[L.iperm[n]]);
        if (L.seg_scen.empty() || sc != L.seg_scen.back() || n - L.seg_begin.back() >= SEG_NODES) {
            L.seg_begin.push_back((int32_t)n);
            L.seg_scen.push_back(sc);
        }
    }
    L.seg_begin.push_back((int32_t)N);
    L.bw_before = bandwidth(p, b, nullptr);
    L.bw_after = bandwidth(p, b, &L.perm);
}

}  // namespace castfem
