/*
 * Plain FP64 CPU oracle of the explicit finite-element casting step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  The product
 * path never calls it and shares no code, header or table with it.
 *
 * What it computes (R. Tavakoli, "Improvement cache efficiency of explicit
 * finite element procedure and its application to parallel casting
 * solidification simulation", 2006):
 *   - conduction with phase change in enthalpy form, dH/dt = div(k grad T)
 *     (Sec. 2, Eq. 1 and Eq. 5), with the enthalpy-temperature relation of
 *     Eq. 11 for a linear latent release between solidus and liquidus;
 *   - Galerkin linear tetrahedra (Sec. 3, Eq. 9) and trilinear hexahedra,
 *     with the row-sum lumped capacitance (Sec. 3);
 *   - convective/flux boundaries (Eq. 4) and the cast/mould contact
 *     conductance (Eq. 8) with the sister-face average as ambient
 *     temperature (end of Sec. 3);
 *   - the fully explicit update (Eq. 10 with theta = 0, i.e. Eq. 14),
 *     assembled element by element (Eq. 15-18), written here for the nodal
 *     enthalpy state: H_i += dt * r_i / m_i with r = F - K T;
 *   - the partition-local sums with shared-node exchange of Eq. 19-22;
 *   - the paper's own latent-heat treatment as a second mode: the apparent heat
 *     capacity form of Eq. 6 with Lemmon's element-wise dH/dT of Eq. 7, lumped
 *     and re-assembled every step, advancing T by Eq. 14.
 * Every routine is a direct loop over elements, faces or nodes in double
 * precision with no blocking, fusion or reordering.
 *
 * Conventions: SI units, temperatures in deg C, specific enthalpy in J/kg with
 * H = 0 at 0 C.  A material row is {k, rho, c, T_sol, T_liq, L}.  Indices are
 * 0-based.  Every function returns 0 on success and a negative value on bad
 * input (inverted element, index out of range, node shared by two materials).
 */
#ifndef CASTFEM_ORACLE_H
#define CASTFEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t elem_type;          /* 4 = linear tetrahedron, 8 = trilinear hexahedron */
    int64_t n_nodes;
    const double *xyz;          /* n_nodes x 3 */
    int64_t n_elems;
    const int32_t *conn;        /* n_elems x elem_type */
    const int32_t *elem_mat;    /* n_elems */
    int32_t n_mat;
    const double *materials;    /* n_mat x 6 */
    int64_t n_dir;
    const int32_t *dir_nodes;
    const double *dir_T;
    int64_t n_flux;
    int32_t flux_npf;           /* 3 or 4 nodes per flux face */
    const int32_t *flux_faces;  /* n_flux x flux_npf */
    const double *flux_q, *flux_h, *flux_Tinf;
    int64_t n_if;
    const int32_t *if_a, *if_b; /* n_if x 3 each: matched faces on the two sides */
    const double *if_h;
    /* contact faces of non-matching meshes: triangles on side 0 or 1 of a contact
     * surface; the sister of each face (orc_contact_sisters) must be given before
     * any residual is evaluated */
    int64_t n_contact;
    const int32_t *contact_faces;   /* n_contact x 3 */
    const int32_t *contact_side;    /* n_contact, 0 or 1 */
    const double *contact_h;        /* n_contact */
    const int32_t *contact_sister;  /* n_contact, or NULL when n_contact == 0 */
} orc_problem;

/* per-state diagnostics written by orc_run, ORC_NDIAG doubles per state */
enum {
    ORC_D_E = 0,        /* sum_i m_i H_i */
    ORC_D_LATENT = 1,   /* sum_i m_i L_i (1 - fs_i): latent heat still to release */
    ORC_D_Q = 2,        /* boundary heat inflow rate of the step leaving this state (W) */
    ORC_D_QCUM = 3,     /* sum over earlier steps of dt * Q */
    ORC_D_TMIN = 4,
    ORC_D_TMAX = 5,
    ORC_D_NLIQ = 6,     /* number of phase-change nodes with fs < 1 */
    ORC_D_NONFINITE = 7,
    ORC_D_RESID = 8,    /* |E - E0 - QCUM| / |E0 - E_ref|, E_ref = sum m_i H_i(25 C) */
    ORC_NDIAG = 9
};

/* Element conductance matrix of a linear tetrahedron, row-major 4x4; *vol = volume. */
int orc_tet_ke(const double x[12], double k, double Ke[16], double *vol);
/* Element conductance matrix of a trilinear hexahedron by 2x2x2 Gauss-Legendre. */
int orc_hex_ke(const double x[24], double k, double Ke[64], double *vol);
/* Row-sum lumped capacitance weights rho * int N_a dV of one element. */
int orc_elem_mass(int32_t elem_type, const double *x, double rho, double *m);

/* Enthalpy relation of one material (Eq. 11 with linear latent release). */
double orc_H_of_T(const double mat[6], double T);
double orc_T_of_H(const double mat[6], double H);
double orc_fs_of_H(const double mat[6], double H);

/* m_i for every node; also validates the mesh. */
int orc_lumped_mass(const orc_problem *p, double *m);
/* Material of every node (-1 for nodes in no element); error if a node has two. */
int orc_node_material(const orc_problem *p, int32_t *node_mat);
/* Sister of every contact face (end of Sec. 3: the closest element of the other
 * region, found once at the start): the face of the other side whose centroid
 * (x0 + x1 + x2) / 3 is nearest in squared Euclidean distance, ties to the lower
 * face index; by brute force over all pairs. */
int orc_contact_sisters(const orc_problem *p, int32_t *sister);
/* The same search for the n faces listed in `faces` only (sister[k] for faces[k]). */
int orc_contact_sisters_of(const orc_problem *p, int64_t n, const int64_t *faces, int32_t *sister);
/* r = F(T) - K T: element conduction, flux faces, interface pairs and contact
 * faces (node i of face f: h_f (A_f / 3) (mean T of the sister face - T_i)). */
int orc_residual(const orc_problem *p, const double *T, double *r);
/* Explicit stability bound 2 / lambda_hat with the Gershgorin estimate of M^-1 K. */
int orc_stable_dt(const orc_problem *p, double *dt_bound);
/* H_i = H(T0_i), Dirichlet temperatures overriding T0. */
int orc_initial_H(const orc_problem *p, const double *T0, double *H);
/* T and fs of every node from the enthalpy state. */
int orc_state_T(const orc_problem *p, const double *H, double *T, double *fs);
/* n explicit steps of the enthalpy update in place on H; diag (n_steps+1) x ORC_NDIAG or NULL. */
int orc_run(const orc_problem *p, double dt, int64_t n_steps, double *H, double *diag);
/* The same steps with the mesh split into n_parts element partitions (Eq. 19-22):
   local capacitances and residuals per partition, then a sum over partitions at
   shared nodes.  Face terms are given to partition (face index mod n_parts). */
int orc_run_partitioned(const orc_problem *p, int32_t n_parts, const int32_t *elem_part,
                        double dt, int64_t n_steps, double *H);

/* Apparent heat capacity (Eq. 6) with Lemmon's element value of dH/dT (Eq. 7),
 * linear tetrahedra only; materials with L > 0 need T_liq > T_sol.
 * orc_lemmon_capacity: C_app of one element from nodal T and H (x as for orc_tet_ke).
 * orc_apparent_capacity: row-sum lumped C_i = sum_e rho C_app V / 4 (J/K) of a state.
 * orc_run_apparent: n explicit steps T^{n+1} = T^n + dt r^n / C^n (Eq. 14 with C
 * re-assembled from the current field every step), the state kept as H = H(T);
 * diag as for orc_run. */
int orc_lemmon_capacity(const double x[12], const double mat[6], const double T[4], const double H[4],
                        double *c_app);
int orc_apparent_capacity(const orc_problem *p, const double *H, double *C);
int orc_run_apparent(const orc_problem *p, double dt, int64_t n_steps, double *H, double *diag);

/* Temperature- and time-dependent properties (Sec. 2 after Eq. 1, Eq. 3 with
 * f(x, t), Eq. 8 with h_i(t, T)).  A table is ORC_TABLE doubles {n, x_0..x_7,
 * y_0..y_7}: n points with increasing x, linear in between and constant beyond
 * the ends; n = 0 leaves the quantity constant.
 *   k_of_T:   n_mat tables, the conductivity of each material against T; an
 *             element takes k at the mean of its nodal T^n (K re-weighted per
 *             element per step);
 *   h_of_T:   factor on every interface coefficient (matched pairs and contact
 *             faces) against T: each node-to-node coupling i-j of a face uses the
 *             factor at (T_i + T_j) / 2;
 *   h_of_t:   factor on every interface coefficient against time;
 *   dir_of_t: shift added to every fixed temperature against time:
 *             T_i(t) = T_D,i + shift(t);
 *   dir_sched: the prescribed temperature f(x_i, t) of every fixed node as its
 *             own table against time (n_dir tables in the order of dir_nodes),
 *             taking the place of T_D,i: T_i(t) = f_i(t) + shift(t).
 * orc_residual_var: r = F - K T at time t with these properties.
 * orc_run_var: n explicit steps from time t0 (the state H must hold the fixed
 *   temperatures of t0); the prescribed change of a fixed node's enthalpy counts
 *   as boundary inflow in the diagnostics. */
enum { ORC_TABLE = 17 };
typedef struct {
    const double *k_of_T;     /* n_mat x ORC_TABLE, or NULL */
    const double *h_of_T;     /* ORC_TABLE, or NULL */
    const double *h_of_t;     /* ORC_TABLE, or NULL */
    const double *dir_of_t;   /* ORC_TABLE, or NULL */
    const double *dir_sched;  /* n_dir x ORC_TABLE, or NULL */
} orc_varprops;

double orc_table(const double *tab, double x);
int orc_residual_var(const orc_problem *p, const orc_varprops *v, const double *T, double t, double *r);
int orc_stable_dt_var(const orc_problem *p, const orc_varprops *v, double *dt_bound);
int orc_run_var(const orc_problem *p, const orc_varprops *v, double t0, double dt, int64_t n_steps, double *H,
                double *diag);

#ifdef __cplusplus
}
#endif
#endif
