/*
 * Plain FP64 CPU oracle of the explicit finite-element casting step.
 * TEST INFRASTRUCTURE ONLY: see castfem_oracle.h for what may use it.
 *
 * Build: gcc -O2 -fPIC -shared -std=c99 castfem_oracle.c -lm (no fast-math,
 * so every expression rounds as written).
 */
#include "castfem_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ERR_ARG  (-1)
#define ORC_ERR_MESH (-2)

/* ---------------------------------------------------------------- helpers */

static double det3(const double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* inverse by the adjugate; returns the determinant */
static double inv3(const double J[3][3], double Ji[3][3])
{
    double d = det3(J);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / d;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / d;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / d;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / d;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / d;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / d;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / d;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / d;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / d;
    return d;
}

/* reference-cube sign of hex node a along each axis: (0,0,0) (1,0,0) (1,1,0) (0,1,0) then top */
static const double HEX_SGN[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

/* shape functions and reference derivatives of the trilinear hexahedron */
static void hex_shape(const double xi[3], double N[8], double dN[8][3])
{
    for (int a = 0; a < 8; ++a) {
        double f0 = 1.0 + xi[0] * HEX_SGN[a][0];
        double f1 = 1.0 + xi[1] * HEX_SGN[a][1];
        double f2 = 1.0 + xi[2] * HEX_SGN[a][2];
        N[a] = 0.125 * f0 * f1 * f2;
        dN[a][0] = 0.125 * HEX_SGN[a][0] * f1 * f2;
        dN[a][1] = 0.125 * HEX_SGN[a][1] * f0 * f2;
        dN[a][2] = 0.125 * HEX_SGN[a][2] * f0 * f1;
    }
}

/* J[i][j] = d x_j / d xi_i for shape-function reference derivatives dN (nen x 3) */
static void jacobian(int nen, const double *x, const double (*dN)[3], double J[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int a = 0; a < nen; ++a) s += dN[a][i] * x[3 * a + j];
            J[i][j] = s;
        }
}

/* grad_x N_a = J^{-1} grad_xi N_a */
static void phys_grad(int nen, const double Ji[3][3], const double (*dN)[3], double (*g)[3])
{
    for (int a = 0; a < nen; ++a)
        for (int i = 0; i < 3; ++i)
            g[a][i] = Ji[i][0] * dN[a][0] + Ji[i][1] * dN[a][1] + Ji[i][2] * dN[a][2];
}

/* ------------------------------------------------------ element matrices */

/* Linear tetrahedron: N0 = 1 - xi - eta - zeta, N1 = xi, N2 = eta, N3 = zeta.
 * K^e_ab = k V grad N_a . grad N_b (the Galerkin conduction matrix of Sec. 3). */
int orc_tet_ke(const double x[12], double k, double Ke[16], double *vol)
{
    static const double dN[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double J[3][3], Ji[3][3], g[4][3];
    jacobian(4, x, dN, J);
    double d = det3(J);
    if (!(d > 0.0)) return ORC_ERR_MESH;
    inv3(J, Ji);
    phys_grad(4, Ji, dN, g);
    double V = d / 6.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            Ke[4 * a + b] = k * V * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
    if (vol) *vol = V;
    return 0;
}

/* Trilinear hexahedron, 2x2x2 Gauss-Legendre (points +-1/sqrt(3), weights 1). */
int orc_hex_ke(const double x[24], double k, double Ke[64], double *vol)
{
    const double gp = 1.0 / sqrt(3.0);
    double V = 0.0;
    memset(Ke, 0, 64 * sizeof(double));
    for (int q = 0; q < 8; ++q) {
        double xi[3] = {HEX_SGN[q][0] * gp, HEX_SGN[q][1] * gp, HEX_SGN[q][2] * gp};
        double N[8], dN[8][3], J[3][3], Ji[3][3], g[8][3];
        hex_shape(xi, N, dN);
        jacobian(8, x, (const double (*)[3])dN, J);
        double d = det3(J);
        if (!(d > 0.0)) return ORC_ERR_MESH;
        inv3(J, Ji);
        phys_grad(8, Ji, (const double (*)[3])dN, g);
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
                Ke[8 * a + b] += k * d * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
        V += d;
    }
    if (vol) *vol = V;
    return 0;
}

/* Row-sum lumping: the a-th row of the consistent capacitance rho int N_a N_b dV
 * summed over b is rho int N_a dV because the shape functions sum to one. */
int orc_elem_mass(int32_t elem_type, const double *x, double rho, double *m)
{
    if (elem_type == 4) {
        double Ke[16], V;
        int rc = orc_tet_ke(x, 1.0, Ke, &V);
        if (rc) return rc;
        for (int a = 0; a < 4; ++a) m[a] = rho * V / 4.0;
        return 0;
    }
    if (elem_type == 8) {
        const double gp = 1.0 / sqrt(3.0);
        for (int a = 0; a < 8; ++a) m[a] = 0.0;
        for (int q = 0; q < 8; ++q) {
            double xi[3] = {HEX_SGN[q][0] * gp, HEX_SGN[q][1] * gp, HEX_SGN[q][2] * gp};
            double N[8], dN[8][3], J[3][3];
            hex_shape(xi, N, dN);
            jacobian(8, x, (const double (*)[3])dN, J);
            double d = det3(J);
            if (!(d > 0.0)) return ORC_ERR_MESH;
            for (int a = 0; a < 8; ++a) m[a] += rho * N[a] * d;
        }
        return 0;
    }
    return ORC_ERR_ARG;
}

/* ------------------------------------------------- enthalpy relation */

/* H(T) = c T + L g(T), g the liquid fraction rising linearly from 0 at T_sol to 1 at T_liq. */
double orc_H_of_T(const double mat[6], double T)
{
    double c = mat[2], Ts = mat[3], Tl = mat[4], L = mat[5];
    double g;
    if (L == 0.0) g = 0.0;
    else if (T <= Ts) g = 0.0;
    else if (T >= Tl) g = 1.0;
    else g = (T - Ts) / (Tl - Ts);
    return c * T + L * g;
}

/* Inverse of orc_H_of_T; an isothermal change (T_sol == T_liq) holds T = T_sol on the plateau. */
double orc_T_of_H(const double mat[6], double H)
{
    double c = mat[2], Ts = mat[3], Tl = mat[4], L = mat[5];
    if (L == 0.0) return H / c;
    double Hs = c * Ts, Hl = c * Tl + L;
    if (H <= Hs) return H / c;
    if (H >= Hl) return (H - L) / c;
    if (Tl == Ts) return Ts;
    return Ts + (H - Hs) * (Tl - Ts) / (c * (Tl - Ts) + L);
}

/* fraction solid 1 - g; materials without latent heat count as solid */
double orc_fs_of_H(const double mat[6], double H)
{
    double c = mat[2], Ts = mat[3], Tl = mat[4], L = mat[5];
    if (L == 0.0) return 1.0;
    double Hs = c * Ts, Hl = c * Tl + L;
    if (H <= Hs) return 1.0;
    if (H >= Hl) return 0.0;
    return 1.0 - (H - Hs) / (Hl - Hs);
}

/* --------------------------------------------------------- mesh checks */

static int gather_x(const orc_problem *p, int64_t e, double *x)
{
    int nen = p->elem_type;
    for (int a = 0; a < nen; ++a) {
        int64_t n = p->conn[e * nen + a];
        if (n < 0 || n >= p->n_nodes) return ORC_ERR_MESH;
        x[3 * a + 0] = p->xyz[3 * n + 0];
        x[3 * a + 1] = p->xyz[3 * n + 1];
        x[3 * a + 2] = p->xyz[3 * n + 2];
    }
    return 0;
}

static int elem_ke(const orc_problem *p, int64_t e, double *Ke)
{
    double x[24];
    int rc = gather_x(p, e, x);
    if (rc) return rc;
    int32_t mt = p->elem_mat[e];
    if (mt < 0 || mt >= p->n_mat) return ORC_ERR_MESH;
    double k = p->materials[6 * mt + 0];
    return p->elem_type == 4 ? orc_tet_ke(x, k, Ke, NULL) : orc_hex_ke(x, k, Ke, NULL);
}

int orc_node_material(const orc_problem *p, int32_t *node_mat)
{
    if (p->elem_type != 4 && p->elem_type != 8) return ORC_ERR_ARG;
    for (int64_t i = 0; i < p->n_nodes; ++i) node_mat[i] = -1;
    int nen = p->elem_type;
    for (int64_t e = 0; e < p->n_elems; ++e) {
        int32_t mt = p->elem_mat[e];
        if (mt < 0 || mt >= p->n_mat) return ORC_ERR_MESH;
        for (int a = 0; a < nen; ++a) {
            int64_t n = p->conn[e * nen + a];
            if (n < 0 || n >= p->n_nodes) return ORC_ERR_MESH;
            if (node_mat[n] >= 0 && node_mat[n] != mt) return ORC_ERR_MESH;
            node_mat[n] = mt;
        }
    }
    return 0;
}

int orc_lumped_mass(const orc_problem *p, double *m)
{
    int nen = p->elem_type;
    if (nen != 4 && nen != 8) return ORC_ERR_ARG;
    for (int64_t i = 0; i < p->n_nodes; ++i) m[i] = 0.0;
    for (int64_t e = 0; e < p->n_elems; ++e) {
        double x[24], me[8];
        int rc = gather_x(p, e, x);
        if (rc) return rc;
        int32_t mt = p->elem_mat[e];
        if (mt < 0 || mt >= p->n_mat) return ORC_ERR_MESH;
        rc = orc_elem_mass(nen, x, p->materials[6 * mt + 1], me);
        if (rc) return rc;
        for (int a = 0; a < nen; ++a) m[p->conn[e * nen + a]] += me[a];
    }
    return 0;
}

/* ------------------------------------------------------- face geometry */

/* area of a triangle, or of a quad as half the cross product of its diagonals */
static double face_area(const double *xyz, const int32_t *f, int npf)
{
    double u[3], v[3], w[3];
    if (npf == 3) {
        for (int j = 0; j < 3; ++j) {
            u[j] = xyz[3 * f[1] + j] - xyz[3 * f[0] + j];
            v[j] = xyz[3 * f[2] + j] - xyz[3 * f[0] + j];
        }
    } else {
        for (int j = 0; j < 3; ++j) {
            u[j] = xyz[3 * f[2] + j] - xyz[3 * f[0] + j];
            v[j] = xyz[3 * f[3] + j] - xyz[3 * f[1] + j];
        }
    }
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
    return 0.5 * sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
}

static int check_faces(const orc_problem *p)
{
    if (p->n_flux > 0 && p->flux_npf != 3 && p->flux_npf != 4) return ORC_ERR_ARG;
    for (int64_t f = 0; f < p->n_flux * p->flux_npf; ++f)
        if (p->flux_faces[f] < 0 || p->flux_faces[f] >= p->n_nodes) return ORC_ERR_MESH;
    for (int64_t f = 0; f < 3 * p->n_if; ++f)
        if (p->if_a[f] < 0 || p->if_a[f] >= p->n_nodes || p->if_b[f] < 0 || p->if_b[f] >= p->n_nodes)
            return ORC_ERR_MESH;
    for (int64_t d = 0; d < p->n_dir; ++d)
        if (p->dir_nodes[d] < 0 || p->dir_nodes[d] >= p->n_nodes) return ORC_ERR_MESH;
    for (int64_t f = 0; f < p->n_contact; ++f) {
        for (int a = 0; a < 3; ++a)
            if (p->contact_faces[3 * f + a] < 0 || p->contact_faces[3 * f + a] >= p->n_nodes) return ORC_ERR_MESH;
        if (p->contact_side[f] != 0 && p->contact_side[f] != 1) return ORC_ERR_ARG;
    }
    return 0;
}

static void face_centroid(const orc_problem *p, int64_t f, double c[3])
{
    const int32_t *fn = p->contact_faces + 3 * f;
    for (int j = 0; j < 3; ++j)
        c[j] = ((p->xyz[3 * fn[0] + j] + p->xyz[3 * fn[1] + j]) + p->xyz[3 * fn[2] + j]) / 3.0;
}

/* the sister of face f by a scan over every face of the other side (centroids c) */
static int64_t sister_of(const orc_problem *p, int64_t f, const double *c)
{
    double best = INFINITY;
    int64_t arg = -1;
    const double *a = c + 3 * f;
    for (int64_t g = 0; g < p->n_contact; ++g) {
        if (p->contact_side[g] == p->contact_side[f]) continue;
        const double *b = c + 3 * g;
        double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 < best) {
            best = d2;
            arg = g;
        }
    }
    return arg;
}

int orc_contact_sisters_of(const orc_problem *p, int64_t n, const int64_t *faces, int32_t *sister)
{
    int rc = check_faces(p);
    if (rc) return rc;
    double *c = malloc((size_t)(3 * p->n_contact + 1) * sizeof(double));
    if (!c) return ORC_ERR_ARG;
    for (int64_t f = 0; f < p->n_contact; ++f) face_centroid(p, f, c + 3 * f);
    for (int64_t k = 0; k < n && rc == 0; ++k) {
        if (faces[k] < 0 || faces[k] >= p->n_contact) { rc = ORC_ERR_ARG; break; }
        int64_t s = sister_of(p, faces[k], c);
        if (s < 0) rc = ORC_ERR_MESH;   /* no face on the other side */
        else sister[k] = (int32_t)s;
    }
    free(c);
    return rc;
}

int orc_contact_sisters(const orc_problem *p, int32_t *sister)
{
    int64_t *all = malloc((size_t)(p->n_contact + 1) * sizeof(int64_t));
    if (!all) return ORC_ERR_ARG;
    for (int64_t f = 0; f < p->n_contact; ++f) all[f] = f;
    int rc = orc_contact_sisters_of(p, p->n_contact, all, sister);
    free(all);
    return rc;
}

/* flux face f: r_i += (A/n)(-q - h (T_i - Tinf)) at each of its n nodes (nodal quadrature) */
static void add_flux_face(const orc_problem *p, int64_t f, const double *T, double *r)
{
    int npf = p->flux_npf;
    const int32_t *fn = p->flux_faces + f * npf;
    double A = face_area(p->xyz, fn, npf);
    for (int a = 0; a < npf; ++a) {
        int32_t i = fn[a];
        r[i] += (A / npf) * (-p->flux_q[f] - p->flux_h[f] * (T[i] - p->flux_Tinf[f]));
    }
}

/* interface pair f: each node of one side sees the mean temperature of the other
 * side's face as ambient, r_i += h (A/3)(Tbar_other - T_i); A from side a */
static void add_interface_pair(const orc_problem *p, int64_t f, const double *T, double *r)
{
    const int32_t *fa = p->if_a + 3 * f, *fb = p->if_b + 3 * f;
    double A = face_area(p->xyz, fa, 3);
    double ta = (T[fa[0]] + T[fa[1]] + T[fa[2]]) / 3.0;
    double tb = (T[fb[0]] + T[fb[1]] + T[fb[2]]) / 3.0;
    for (int a = 0; a < 3; ++a) {
        r[fa[a]] += p->if_h[f] * (A / 3.0) * (tb - T[fa[a]]);
        r[fb[a]] += p->if_h[f] * (A / 3.0) * (ta - T[fb[a]]);
    }
}

/* contact face f: each of its nodes sees the mean temperature of the sister
 * face as ambient, r_i += h (A_f / 3)(Tbar_sister - T_i), A_f the face's own area */
static void add_contact_face(const orc_problem *p, int64_t f, const double *T, double *r)
{
    const int32_t *fa = p->contact_faces + 3 * f, *fs = p->contact_faces + 3 * p->contact_sister[f];
    double A = face_area(p->xyz, fa, 3);
    double ts = (T[fs[0]] + T[fs[1]] + T[fs[2]]) / 3.0;
    for (int a = 0; a < 3; ++a) r[fa[a]] += p->contact_h[f] * (A / 3.0) * (ts - T[fa[a]]);
}

static int check_sisters(const orc_problem *p)
{
    if (p->n_contact > 0 && !p->contact_sister) return ORC_ERR_ARG;
    for (int64_t f = 0; f < p->n_contact; ++f) {
        int32_t s = p->contact_sister[f];
        if (s < 0 || s >= p->n_contact || p->contact_side[s] == p->contact_side[f]) return ORC_ERR_ARG;
    }
    return 0;
}

/* ------------------------------------------------------------ residual */

int orc_residual(const orc_problem *p, const double *T, double *r)
{
    int nen = p->elem_type;
    if (nen != 4 && nen != 8) return ORC_ERR_ARG;
    int rc = check_faces(p);
    if (rc == 0) rc = check_sisters(p);
    if (rc) return rc;
    for (int64_t i = 0; i < p->n_nodes; ++i) r[i] = 0.0;
    double Ke[64];
    for (int64_t e = 0; e < p->n_elems; ++e) {
        rc = elem_ke(p, e, Ke);
        if (rc) return rc;
        const int32_t *cn = p->conn + e * nen;
        for (int a = 0; a < nen; ++a) {
            double s = 0.0;
            for (int b = 0; b < nen; ++b) s += Ke[nen * a + b] * T[cn[b]];
            r[cn[a]] -= s;
        }
    }
    for (int64_t f = 0; f < p->n_flux; ++f) add_flux_face(p, f, T, r);
    for (int64_t f = 0; f < p->n_if; ++f) add_interface_pair(p, f, T, r);
    for (int64_t f = 0; f < p->n_contact; ++f) add_contact_face(p, f, T, r);
    return 0;
}

/* ------------------------------------------------------ stability bound */

/* lambda_hat = max_i [sum_j |K_ij| + sum_{flux faces at i} (A/n) h
 *                     + sum_{interface pairs at i} 2 h A / 3] / (m_i c_i),
 * the Gershgorin bound of M^-1 (K + boundary terms) with the sensible heat c
 * (the smallest dH/dT of the enthalpy relation); dt_bound = 2 / lambda_hat. */
int orc_stable_dt(const orc_problem *p, double *dt_bound)
{
    int nen = p->elem_type;
    int64_t N = p->n_nodes, E = p->n_elems;
    int rc = check_faces(p);
    if (rc) return rc;
    double *m = malloc(N * sizeof(double));
    double *extra = calloc(N, sizeof(double));
    int32_t *nmat = malloc(N * sizeof(int32_t));
    int64_t *ptr = calloc(N + 1, sizeof(int64_t));
    int64_t *inc = malloc(E * nen * sizeof(int64_t));
    if (!m || !extra || !nmat || !ptr || !inc) { rc = ORC_ERR_ARG; goto done; }
    if ((rc = orc_lumped_mass(p, m))) goto done;
    if ((rc = orc_node_material(p, nmat))) goto done;
    /* node -> incident (element, local index) list */
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nen; ++a) ptr[p->conn[e * nen + a] + 1]++;
    for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
    {
        int64_t *fill = malloc(N * sizeof(int64_t));
        if (!fill) { rc = ORC_ERR_ARG; goto done; }
        memcpy(fill, ptr, N * sizeof(int64_t));
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nen; ++a) inc[fill[p->conn[e * nen + a]]++] = e * nen + a;
        free(fill);
    }
    for (int64_t f = 0; f < p->n_flux; ++f) {
        const int32_t *fn = p->flux_faces + f * p->flux_npf;
        double A = face_area(p->xyz, fn, p->flux_npf);
        for (int a = 0; a < p->flux_npf; ++a) extra[fn[a]] += (A / p->flux_npf) * p->flux_h[f];
    }
    for (int64_t f = 0; f < p->n_if; ++f) {
        double A = face_area(p->xyz, p->if_a + 3 * f, 3);
        for (int a = 0; a < 3; ++a) {
            extra[p->if_a[3 * f + a]] += 2.0 * p->if_h[f] * A / 3.0;
            extra[p->if_b[3 * f + a]] += 2.0 * p->if_h[f] * A / 3.0;
        }
    }
    /* a contact face adds h A / 3 to the diagonal of each of its nodes and the
     * same in total to the off-diagonals (its sister's three nodes) */
    for (int64_t f = 0; f < p->n_contact; ++f) {
        double A = face_area(p->xyz, p->contact_faces + 3 * f, 3);
        for (int a = 0; a < 3; ++a) extra[p->contact_faces[3 * f + a]] += 2.0 * p->contact_h[f] * A / 3.0;
    }
    {
        double lam = 0.0;
        int64_t cap = 64;
        int32_t *cols = malloc(cap * sizeof(int32_t));
        double *vals = malloc(cap * sizeof(double));
        double Ke[64];
        for (int64_t i = 0; i < N && rc == 0; ++i) {
            if (nmat[i] < 0) continue;
            int64_t nc = 0;
            for (int64_t t = ptr[i]; t < ptr[i + 1]; ++t) {
                int64_t e = inc[t] / nen;
                int a = (int)(inc[t] % nen);
                if ((rc = elem_ke(p, e, Ke))) break;
                for (int b = 0; b < nen; ++b) {
                    int32_t j = p->conn[e * nen + b];
                    int64_t s = 0;
                    while (s < nc && cols[s] != j) ++s;
                    if (s == nc) {
                        if (nc == cap) {
                            cap *= 2;
                            cols = realloc(cols, cap * sizeof(int32_t));
                            vals = realloc(vals, cap * sizeof(double));
                        }
                        cols[nc] = j;
                        vals[nc] = 0.0;
                        ++nc;
                    }
                    vals[s] += Ke[nen * a + b];
                }
            }
            double row = extra[i];
            for (int64_t s = 0; s < nc; ++s) row += fabs(vals[s]);
            double li = row / (m[i] * p->materials[6 * nmat[i] + 2]);
            if (li > lam) lam = li;
        }
        free(cols);
        free(vals);
        if (rc == 0) *dt_bound = lam > 0.0 ? 2.0 / lam : INFINITY;
    }
done:
    free(m); free(extra); free(nmat); free(ptr); free(inc);
    return rc;
}

/* --------------------------------------------------------------- state */

static unsigned char *dirichlet_mask(const orc_problem *p)
{
    unsigned char *mask = calloc(p->n_nodes, 1);
    if (!mask) return NULL;
    for (int64_t d = 0; d < p->n_dir; ++d) mask[p->dir_nodes[d]] = 1;
    return mask;
}

int orc_initial_H(const orc_problem *p, const double *T0, double *H)
{
    int32_t *nmat = malloc(p->n_nodes * sizeof(int32_t));
    if (!nmat) return ORC_ERR_ARG;
    int rc = orc_node_material(p, nmat);
    if (rc == 0) rc = check_faces(p);
    if (rc == 0) {
        for (int64_t i = 0; i < p->n_nodes; ++i)
            H[i] = nmat[i] >= 0 ? orc_H_of_T(p->materials + 6 * nmat[i], T0[i]) : 0.0;
        for (int64_t d = 0; d < p->n_dir; ++d) {
            int32_t i = p->dir_nodes[d];
            if (nmat[i] >= 0) H[i] = orc_H_of_T(p->materials + 6 * nmat[i], p->dir_T[d]);
        }
    }
    free(nmat);
    return rc;
}

static void state_T_nm(const orc_problem *p, const int32_t *nmat, const double *H, double *T, double *fs)
{
    for (int64_t i = 0; i < p->n_nodes; ++i) {
        const double *mt = nmat[i] >= 0 ? p->materials + 6 * nmat[i] : NULL;
        if (T) T[i] = mt ? orc_T_of_H(mt, H[i]) : 0.0;
        if (fs) fs[i] = mt ? orc_fs_of_H(mt, H[i]) : 1.0;
    }
}

int orc_state_T(const orc_problem *p, const double *H, double *T, double *fs)
{
    int32_t *nmat = malloc(p->n_nodes * sizeof(int32_t));
    if (!nmat) return ORC_ERR_ARG;
    int rc = orc_node_material(p, nmat);
    if (rc == 0) state_T_nm(p, nmat, H, T, fs);
    free(nmat);
    return rc;
}

/* boundary inflow of one residual evaluation: Robin/flux terms everywhere
 * plus the reaction -r_i at fixed-temperature nodes (interface terms cancel) */
static double boundary_inflow(const orc_problem *p, const double *T, const double *r)
{
    double Q = 0.0;
    for (int64_t f = 0; f < p->n_flux; ++f) {
        const int32_t *fn = p->flux_faces + f * p->flux_npf;
        double A = face_area(p->xyz, fn, p->flux_npf);
        for (int a = 0; a < p->flux_npf; ++a)
            Q += (A / p->flux_npf) * (-p->flux_q[f] - p->flux_h[f] * (T[fn[a]] - p->flux_Tinf[f]));
    }
    for (int64_t d = 0; d < p->n_dir; ++d) Q -= r[p->dir_nodes[d]];
    return Q;
}

static void fill_diag(const orc_problem *p, const int32_t *nmat, const double *m, const double *H,
                      const double *T, double Q, double Qcum, double E0, double Eref, double *dg)
{
    double E = 0.0, lat = 0.0, tmin = INFINITY, tmax = -INFINITY;
    int64_t nliq = 0, nonfinite = 0;
    for (int64_t i = 0; i < p->n_nodes; ++i) {
        if (nmat[i] < 0) continue;
        const double *mt = p->materials + 6 * nmat[i];
        double fs = orc_fs_of_H(mt, H[i]);
        E += m[i] * H[i];
        lat += m[i] * mt[5] * (1.0 - fs);
        if (T[i] < tmin) tmin = T[i];
        if (T[i] > tmax) tmax = T[i];
        if (mt[5] > 0.0 && fs < 1.0) ++nliq;
        if (!isfinite(H[i])) ++nonfinite;
    }
    dg[ORC_D_E] = E;
    dg[ORC_D_LATENT] = lat;
    dg[ORC_D_Q] = Q;
    dg[ORC_D_QCUM] = Qcum;
    dg[ORC_D_TMIN] = tmin;
    dg[ORC_D_TMAX] = tmax;
    dg[ORC_D_NLIQ] = (double)nliq;
    dg[ORC_D_NONFINITE] = (double)nonfinite;
    double E0v = isnan(E0) ? E : E0;
    dg[ORC_D_RESID] = fabs(E - E0v - Qcum) / fabs(E0v - Eref);
}

int orc_run(const orc_problem *p, double dt, int64_t n_steps, double *H, double *diag)
{
    int64_t N = p->n_nodes;
    double *m = malloc(N * sizeof(double));
    double *T = malloc(N * sizeof(double));
    double *r = malloc(N * sizeof(double));
    int32_t *nmat = malloc(N * sizeof(int32_t));
    unsigned char *fixed = dirichlet_mask(p);
    int rc = 0;
    if (!m || !T || !r || !nmat || !fixed) { rc = ORC_ERR_ARG; goto done; }
    if ((rc = orc_lumped_mass(p, m))) goto done;
    if ((rc = orc_node_material(p, nmat))) goto done;
    double Eref = 0.0, E0 = NAN, Qcum = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (nmat[i] >= 0) Eref += m[i] * orc_H_of_T(p->materials + 6 * nmat[i], 25.0);
    for (int64_t n = 0; n <= n_steps; ++n) {
        /* T^n = T(H^n) */
        state_T_nm(p, nmat, H, T, NULL);
        /* r^n = F^n - K T^n */
        if ((rc = orc_residual(p, T, r))) goto done;
        double Q = boundary_inflow(p, T, r);
        if (diag) {
            fill_diag(p, nmat, m, H, T, Q, Qcum, E0, Eref, diag + n * ORC_NDIAG);
            if (n == 0) E0 = diag[ORC_D_E];
        }
        if (n == n_steps) break;
        /* H^{n+1} = H^n + dt r^n / m at free nodes */
        for (int64_t i = 0; i < N; ++i)
            if (!fixed[i] && nmat[i] >= 0) H[i] = H[i] + dt * r[i] / m[i];
        Qcum += dt * Q;
    }
done:
    free(m); free(T); free(r); free(nmat); free(fixed);
    return rc;
}

/* ------------------------------------- apparent heat capacity (Eq. 6-7) */

/* gradients of the four shape functions of a linear tetrahedron; *vol = volume */
static int tet_grads(const double x[12], double g[4][3], double *vol)
{
    static const double dN[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double J[3][3], Ji[3][3];
    jacobian(4, x, dN, J);
    double d = det3(J);
    if (!(d > 0.0)) return ORC_ERR_MESH;
    inv3(J, Ji);
    phys_grad(4, Ji, dN, g);
    *vol = d / 6.0;
    return 0;
}

/* Lemmon's element value of dH/dT (Eq. 7): |grad H| / |grad T| with H and T
 * interpolated linearly from the nodal values, so both gradients are constant
 * on the element.  Where grad T vanishes the ratio is undefined and the slope of
 * the enthalpy relation at the mean nodal temperature is taken: c + L/(T_liq -
 * T_sol) strictly inside the mushy interval, c elsewhere. */
int orc_lemmon_capacity(const double x[12], const double mat[6], const double T[4], const double H[4],
                        double *c_app)
{
    double g[4][3], V;
    double c = mat[2], Ts = mat[3], Tl = mat[4], L = mat[5];
    if (L > 0.0 && !(Tl > Ts)) return ORC_ERR_ARG;
    int rc = tet_grads(x, g, &V);
    if (rc) return rc;
    /* the shape functions sum to one, so the gradients are sums over the
     * differences to node 0; a uniform field then has exactly zero gradient */
    double gT[3] = {0, 0, 0}, gH[3] = {0, 0, 0};
    for (int a = 1; a < 4; ++a)
        for (int i = 0; i < 3; ++i) {
            gT[i] += (T[a] - T[0]) * g[a][i];
            gH[i] += (H[a] - H[0]) * g[a][i];
        }
    double nT = gT[0] * gT[0] + gT[1] * gT[1] + gT[2] * gT[2];
    double nH = gH[0] * gH[0] + gH[1] * gH[1] + gH[2] * gH[2];
    if (nT > 0.0) {
        *c_app = sqrt(nH / nT);
    } else {
        double Tm = (T[0] + T[1] + T[2] + T[3]) / 4.0;
        *c_app = (L > 0.0 && Tm > Ts && Tm < Tl) ? c + L / (Tl - Ts) : c;
    }
    return 0;
}

/* lumped capacitance C_i = sum over elements at i of rho C_app V / 4 (row-sum
 * lumping of the element capacitance rho C_app int N_a N_b dV) */
static int apparent_lumped(const orc_problem *p, const double *T, const double *H, double *C)
{
    for (int64_t i = 0; i < p->n_nodes; ++i) C[i] = 0.0;
    for (int64_t e = 0; e < p->n_elems; ++e) {
        double x[12], Te[4], He[4], g[4][3], V, capp;
        int rc = gather_x(p, e, x);
        if (rc) return rc;
        int32_t mt = p->elem_mat[e];
        if (mt < 0 || mt >= p->n_mat) return ORC_ERR_MESH;
        const int32_t *cn = p->conn + 4 * e;
        for (int a = 0; a < 4; ++a) {
            Te[a] = T[cn[a]];
            He[a] = H[cn[a]];
        }
        if ((rc = orc_lemmon_capacity(x, p->materials + 6 * mt, Te, He, &capp))) return rc;
        if ((rc = tet_grads(x, g, &V))) return rc;
        for (int a = 0; a < 4; ++a) C[cn[a]] += p->materials[6 * mt + 1] * capp * V / 4.0;
    }
    return 0;
}

int orc_apparent_capacity(const orc_problem *p, const double *H, double *C)
{
    if (p->elem_type != 4) return ORC_ERR_ARG;
    double *T = malloc(p->n_nodes * sizeof(double));
    if (!T) return ORC_ERR_ARG;
    int rc = orc_state_T(p, H, T, NULL);
    if (rc == 0) rc = apparent_lumped(p, T, H, C);
    free(T);
    return rc;
}

int orc_run_apparent(const orc_problem *p, double dt, int64_t n_steps, double *H, double *diag)
{
    if (p->elem_type != 4) return ORC_ERR_ARG;
    for (int32_t q = 0; q < p->n_mat; ++q)
        if (p->materials[6 * q + 5] > 0.0 && !(p->materials[6 * q + 4] > p->materials[6 * q + 3]))
            return ORC_ERR_ARG;
    int64_t N = p->n_nodes;
    double *m = malloc(N * sizeof(double));
    double *T = malloc(N * sizeof(double));
    double *r = malloc(N * sizeof(double));
    double *Cn = malloc(N * sizeof(double));
    int32_t *nmat = malloc(N * sizeof(int32_t));
    unsigned char *fixed = dirichlet_mask(p);
    int rc = 0;
    if (!m || !T || !r || !Cn || !nmat || !fixed) { rc = ORC_ERR_ARG; goto done; }
    if ((rc = orc_lumped_mass(p, m))) goto done;
    if ((rc = orc_node_material(p, nmat))) goto done;
    double Eref = 0.0, E0 = NAN, Qcum = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (nmat[i] >= 0) Eref += m[i] * orc_H_of_T(p->materials + 6 * nmat[i], 25.0);
    for (int64_t n = 0; n <= n_steps; ++n) {
        state_T_nm(p, nmat, H, T, NULL);
        /* r^n = F^n - K T^n, as in the enthalpy form */
        if ((rc = orc_residual(p, T, r))) goto done;
        double Q = boundary_inflow(p, T, r);
        if (diag) {
            fill_diag(p, nmat, m, H, T, Q, Qcum, E0, Eref, diag + n * ORC_NDIAG);
            if (n == 0) E0 = diag[ORC_D_E];
        }
        if (n == n_steps) break;
        /* C^n from the current field (Eq. 7, lumped), then Eq. 14:
         * T^{n+1} = T^n + dt (C^n)^-1 r^n, and the state keeps H(T^{n+1}) */
        if ((rc = apparent_lumped(p, T, H, Cn))) goto done;
        for (int64_t i = 0; i < N; ++i)
            if (!fixed[i] && nmat[i] >= 0) H[i] = orc_H_of_T(p->materials + 6 * nmat[i], T[i] + dt * r[i] / Cn[i]);
        Qcum += dt * Q;
    }
done:
    free(m); free(T); free(r); free(Cn); free(nmat); free(fixed);
    return rc;
}

/* ------------------------------- temperature- and time-dependent properties */

double orc_table(const double *tab, double x)
{
    int n = (int)tab[0];
    const double *xs = tab + 1, *ys = tab + 9;
    if (x <= xs[0]) return ys[0];
    if (x >= xs[n - 1]) return ys[n - 1];
    int j = 0;
    while (j + 2 < n && !(x < xs[j + 1])) ++j;   /* bounded: a NaN x ends in the last segment */
    return ys[j] + (ys[j + 1] - ys[j]) * (x - xs[j]) / (xs[j + 1] - xs[j]);
}

static int table_ok(const double *tab)
{
    if (!tab) return 1;
    int n = (int)tab[0];
    if (n < 0 || n > 8 || (double)n != tab[0]) return 0;
    for (int j = 0; j + 1 < n; ++j)
        if (!(tab[1 + j] < tab[2 + j])) return 0;
    return 1;
}

static int has(const double *tab) { return tab && tab[0] > 0; }

static int check_var(const orc_problem *p, const orc_varprops *v)
{
    if (!table_ok(v->h_of_T) || !table_ok(v->h_of_t) || !table_ok(v->dir_of_t)) return ORC_ERR_ARG;
    if (v->dir_sched)
        for (int64_t d = 0; d < p->n_dir; ++d)
            if (!table_ok(v->dir_sched + ORC_TABLE * d) || !has(v->dir_sched + ORC_TABLE * d)) return ORC_ERR_ARG;
    if (v->k_of_T)
        for (int32_t q = 0; q < p->n_mat; ++q)
            if (!table_ok(v->k_of_T + ORC_TABLE * q)) return ORC_ERR_ARG;
    return 0;
}

/* interface coefficient factor of the node pair (i, j) at time t */
static double h_factor(const orc_varprops *v, double Ti, double Tj, double t)
{
    double f = 1.0;
    if (has(v->h_of_T)) f *= orc_table(v->h_of_T, (Ti + Tj) / 2.0);
    if (has(v->h_of_t)) f *= orc_table(v->h_of_t, t);
    return f;
}

int orc_residual_var(const orc_problem *p, const orc_varprops *v, const double *T, double t, double *r)
{
    int nen = p->elem_type;
    if (nen != 4 && nen != 8) return ORC_ERR_ARG;
    int rc = check_faces(p);
    if (rc == 0) rc = check_sisters(p);
    if (rc == 0) rc = check_var(p, v);
    if (rc) return rc;
    for (int64_t i = 0; i < p->n_nodes; ++i) r[i] = 0.0;
    double Ke[64];
    for (int64_t e = 0; e < p->n_elems; ++e) {
        const int32_t *cn = p->conn + e * nen;
        int32_t mt = p->elem_mat[e];
        if (mt < 0 || mt >= p->n_mat) return ORC_ERR_MESH;
        /* K^e is linear in k: build it for k = 1 and scale by k(mean T^n of the element) */
        double x[24];
        if ((rc = gather_x(p, e, x))) return rc;
        rc = nen == 4 ? orc_tet_ke(x, 1.0, Ke, NULL) : orc_hex_ke(x, 1.0, Ke, NULL);
        if (rc) return rc;
        double k = p->materials[6 * mt + 0];
        if (v->k_of_T && has(v->k_of_T + ORC_TABLE * mt)) {
            double Tm = 0.0;
            for (int a = 0; a < nen; ++a) Tm += T[cn[a]];
            k = orc_table(v->k_of_T + ORC_TABLE * mt, Tm / nen);
        }
        for (int a = 0; a < nen; ++a) {
            double s = 0.0;
            for (int b = 0; b < nen; ++b) s += Ke[nen * a + b] * T[cn[b]];
            r[cn[a]] -= k * s;
        }
    }
    for (int64_t f = 0; f < p->n_flux; ++f) add_flux_face(p, f, T, r);
    /* interface pairs and contact faces, node pair by node pair: node i of a face
     * and node j of the face it sees exchange h f_ij (A/9)(T_j - T_i) */
    for (int64_t f = 0; f < p->n_if; ++f) {
        const int32_t *fa = p->if_a + 3 * f, *fb = p->if_b + 3 * f;
        double A = face_area(p->xyz, fa, 3);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                int32_t i = fa[a], j = fb[b];
                double w = p->if_h[f] * (A / 9.0) * h_factor(v, T[i], T[j], t);
                r[i] += w * (T[j] - T[i]);
                r[j] += w * (T[i] - T[j]);
            }
    }
    for (int64_t f = 0; f < p->n_contact; ++f) {
        const int32_t *fa = p->contact_faces + 3 * f, *fs = p->contact_faces + 3 * p->contact_sister[f];
        double A = face_area(p->xyz, fa, 3);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                int32_t i = fa[a], j = fs[b];
                r[i] += p->contact_h[f] * (A / 9.0) * h_factor(v, T[i], T[j], t) * (T[j] - T[i]);
            }
    }
    return 0;
}

/* the largest value a table (or its constant) takes */
static double table_max(const double *tab, double constant)
{
    if (!has(tab)) return constant;
    double m = tab[9];
    for (int j = 1; j < (int)tab[0]; ++j) m = fmax(m, tab[9 + j]);
    return m;
}

/* Gershgorin bound with every property at its largest value: the conduction part
 * of a material scaled by max k / k, the interface parts by the largest factors */
int orc_stable_dt_var(const orc_problem *p, const orc_varprops *v, double *dt_bound)
{
    int rc = check_var(p, v);
    if (rc) return rc;
    int32_t nm = p->n_mat;
    double *mats = malloc((size_t)(6 * nm + 1) * sizeof(double));
    double *ifh = malloc((size_t)(p->n_if + 1) * sizeof(double));
    double *ch = malloc((size_t)(p->n_contact + 1) * sizeof(double));
    if (!mats || !ifh || !ch) { free(mats); free(ifh); free(ch); return ORC_ERR_ARG; }
    for (int32_t q = 0; q < nm; ++q) {
        for (int j = 0; j < 6; ++j) mats[6 * q + j] = p->materials[6 * q + j];
        if (v->k_of_T) mats[6 * q] = table_max(v->k_of_T + ORC_TABLE * q, mats[6 * q]);
    }
    double hf = table_max(v->h_of_T, 1.0) * table_max(v->h_of_t, 1.0);
    for (int64_t f = 0; f < p->n_if; ++f) ifh[f] = p->if_h[f] * hf;
    for (int64_t f = 0; f < p->n_contact; ++f) ch[f] = p->contact_h[f] * hf;
    orc_problem q = *p;
    q.materials = mats;
    q.if_h = ifh;
    q.contact_h = ch;
    rc = orc_stable_dt(&q, dt_bound);
    free(mats); free(ifh); free(ch);
    return rc;
}

int orc_run_var(const orc_problem *p, const orc_varprops *v, double t0, double dt, int64_t n_steps, double *H,
                double *diag)
{
    int64_t N = p->n_nodes;
    double *m = malloc(N * sizeof(double));
    double *T = malloc(N * sizeof(double));
    double *r = malloc(N * sizeof(double));
    int32_t *nmat = malloc(N * sizeof(int32_t));
    int rc = check_var(p, v);
    if (!m || !T || !r || !nmat) rc = ORC_ERR_ARG;
    if (rc) goto done;
    if ((rc = orc_lumped_mass(p, m))) goto done;
    if ((rc = orc_node_material(p, nmat))) goto done;
    double Eref = 0.0, E0 = NAN, Qcum = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (nmat[i] >= 0) Eref += m[i] * orc_H_of_T(p->materials + 6 * nmat[i], 25.0);
    for (int64_t n = 0; n <= n_steps; ++n) {
        double t = t0 + (double)n * dt;
        state_T_nm(p, nmat, H, T, NULL);
        if ((rc = orc_residual_var(p, v, T, t, r))) goto done;
        double Q = boundary_inflow(p, T, r);
        if (diag) {
            fill_diag(p, nmat, m, H, T, Q, Qcum, E0, Eref, diag + n * ORC_NDIAG);
            if (n == 0) E0 = diag[ORC_D_E];
        }
        if (n == n_steps) break;
        /* free nodes: H += dt r / m; fixed nodes: H(f(t + dt) + shift(t + dt)) with
         * f the node's schedule or its constant T_D; the boundary supplies the change */
        unsigned char *fixed = dirichlet_mask(p);
        if (!fixed) { rc = ORC_ERR_ARG; goto done; }
        for (int64_t i = 0; i < N; ++i)
            if (!fixed[i] && nmat[i] >= 0) H[i] = H[i] + dt * r[i] / m[i];
        free(fixed);
        double shift = has(v->dir_of_t) ? orc_table(v->dir_of_t, t + dt) : 0.0;
        for (int64_t d = 0; d < p->n_dir; ++d) {
            int32_t i = p->dir_nodes[d];
            if (nmat[i] < 0) continue;
            double TD = v->dir_sched ? orc_table(v->dir_sched + ORC_TABLE * d, t + dt) : p->dir_T[d];
            double Hn = orc_H_of_T(p->materials + 6 * nmat[i], TD + shift);
            Qcum += m[i] * (Hn - H[i]);
            H[i] = Hn;
        }
        Qcum += dt * Q;
    }
done:
    free(m); free(T); free(r); free(nmat);
    return rc;
}

/* ----------------------------------------------- partitioned algorithm */

int orc_run_partitioned(const orc_problem *p, int32_t n_parts, const int32_t *elem_part,
                        double dt, int64_t n_steps, double *H)
{
    int64_t N = p->n_nodes, E = p->n_elems;
    int nen = p->elem_type;
    if (n_parts < 1 || (nen != 4 && nen != 8)) return ORC_ERR_ARG;
    for (int64_t e = 0; e < E; ++e)
        if (elem_part[e] < 0 || elem_part[e] >= n_parts) return ORC_ERR_ARG;
    int rc = check_faces(p);
    if (rc == 0) rc = check_sisters(p);
    if (rc) return rc;
    /* per partition: local capacitance C^l and local residual R^l over all nodes
     * (only the nodes of the partition are ever non-zero) */
    double *Cl = calloc((size_t)n_parts * N, sizeof(double));
    double *Rl = malloc((size_t)n_parts * N * sizeof(double));
    double *T = malloc(N * sizeof(double));
    int32_t *nmat = malloc(N * sizeof(int32_t));
    unsigned char *fixed = dirichlet_mask(p);
    if (!Cl || !Rl || !T || !nmat || !fixed) { rc = ORC_ERR_ARG; goto done; }
    if ((rc = orc_node_material(p, nmat))) goto done;
    for (int64_t e = 0; e < E; ++e) {
        double x[24], me[8];
        if ((rc = gather_x(p, e, x))) goto done;
        if ((rc = orc_elem_mass(nen, x, p->materials[6 * p->elem_mat[e] + 1], me))) goto done;
        double *C = Cl + (size_t)elem_part[e] * N;
        for (int a = 0; a < nen; ++a) C[p->conn[e * nen + a]] += me[a];
    }
    for (int64_t n = 0; n < n_steps; ++n) {
        state_T_nm(p, nmat, H, T, NULL);
        for (size_t s = 0; s < (size_t)n_parts * N; ++s) Rl[s] = 0.0;
        double Ke[64];
        for (int64_t e = 0; e < E; ++e) {
            if ((rc = elem_ke(p, e, Ke))) goto done;
            double *R = Rl + (size_t)elem_part[e] * N;
            const int32_t *cn = p->conn + e * nen;
            for (int a = 0; a < nen; ++a) {
                double s = 0.0;
                for (int b = 0; b < nen; ++b) s += Ke[nen * a + b] * T[cn[b]];
                R[cn[a]] -= s;
            }
        }
        for (int64_t f = 0; f < p->n_flux; ++f) add_flux_face(p, f, T, Rl + (size_t)(f % n_parts) * N);
        for (int64_t f = 0; f < p->n_if; ++f) add_interface_pair(p, f, T, Rl + (size_t)(f % n_parts) * N);
        for (int64_t f = 0; f < p->n_contact; ++f) add_contact_face(p, f, T, Rl + (size_t)(f % n_parts) * N);
        /* exchange: sum the partition-local values at every node, then update */
        for (int64_t i = 0; i < N; ++i) {
            if (fixed[i] || nmat[i] < 0) continue;
            double C = 0.0, R = 0.0;
            for (int32_t q = 0; q < n_parts; ++q) {
                C += Cl[(size_t)q * N + i];
                R += Rl[(size_t)q * N + i];
            }
            H[i] = H[i] + dt * R / C;
        }
    }
done:
    free(Cl); free(Rl); free(T); free(nmat); free(fixed);
    return rc;
}
