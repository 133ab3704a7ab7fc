/*
 * The explicit run of castfem_oracle.c spread over the host's cores, with the
 * same result bit for bit.
 *
 * TEST INFRASTRUCTURE ONLY, like the serial oracle: the test-suite, the
 * scripts that write stored expected values, and the CPU-baseline leg of the
 * benchmark are its only users.
 *
 * It includes the serial oracle's source, so every element matrix, lumped
 * mass, flux term and enthalpy relation is the same function.  What differs is
 * only who does which additions:
 *   - the element contributions s_{e,a} = (K^e T^e)_a of every element are
 *     formed in parallel (each by the serial oracle's own loop) into a table;
 *   - every node then subtracts its own contributions in increasing element
 *     order, which is the order in which the serial element loop reaches it,
 *     starting from the same 0.0;
 *   - the flux, interface and contact loops, the boundary inflow and the
 *     diagnostics run serially, exactly as in orc_run;
 *   - the enthalpy update and T(H) are per node, hence order-free.
 * So the residual of every node, and with it the whole trajectory, is that of
 * orc_run (a CPU test holds the two equal bit for bit).
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -std=c99 castfem_oracle_omp.c -lm
 */
#include "castfem_oracle.c"

#include <omp.h>

int orc_run_omp(const orc_problem *p, double dt, int64_t n_steps, double *H, double *diag, int32_t n_threads)
{
    const int nen = p->elem_type;
    if (nen != 4 && nen != 8) return ORC_ERR_ARG;
    if (n_threads > 0) omp_set_num_threads(n_threads);
    const int64_t N = p->n_nodes, E = p->n_elems;
    double *m = malloc(N * sizeof(double));
    double *T = malloc(N * sizeof(double));
    double *r = malloc(N * sizeof(double));
    int32_t *nmat = malloc(N * sizeof(int32_t));
    int64_t *ptr = calloc(N + 1, sizeof(int64_t));
    int64_t *inc = malloc((size_t)(E * nen + 1) * sizeof(int64_t));
    double *contrib = malloc((size_t)(E * nen + 1) * sizeof(double));
    unsigned char *fixed = dirichlet_mask(p);
    int rc = 0;
    if (!m || !T || !r || !nmat || !ptr || !inc || !contrib || !fixed) { rc = ORC_ERR_ARG; goto done; }
    if ((rc = orc_lumped_mass(p, m))) goto done;
    if ((rc = orc_node_material(p, nmat))) goto done;
    if ((rc = check_faces(p))) goto done;
    if ((rc = check_sisters(p))) goto done;
    /* incidences of every node, (e, a) as e * nen + a, in increasing e
     * (orc_node_material has checked every index) */
    for (int64_t k = 0; k < E * nen; ++k) ptr[p->conn[k] + 1]++;
    for (int64_t i = 0; i < N; ++i) ptr[i + 1] += ptr[i];
    {
        int64_t *fill = malloc((N + 1) * sizeof(int64_t));
        if (!fill) { rc = ORC_ERR_ARG; goto done; }
        memcpy(fill, ptr, (N + 1) * sizeof(int64_t));
        for (int64_t k = 0; k < E * nen; ++k) inc[fill[p->conn[k]]++] = k;
        free(fill);
    }
    double Eref = 0.0, E0 = NAN, Qcum = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (nmat[i] >= 0) Eref += m[i] * orc_H_of_T(p->materials + 6 * nmat[i], 25.0);
    for (int64_t n = 0; n <= n_steps; ++n) {
        /* T^n = T(H^n) */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            T[i] = nmat[i] >= 0 ? orc_T_of_H(p->materials + 6 * nmat[i], H[i]) : 0.0;
        /* element contributions, then each node's sum in element order */
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t e = 0; e < E; ++e) {
            double Ke[64];
            if (elem_ke(p, e, Ke)) {
                bad = 1;
                continue;
            }
            const int32_t *cn = p->conn + e * nen;
            for (int a = 0; a < nen; ++a) {
                double s = 0.0;
                for (int b = 0; b < nen; ++b) s += Ke[nen * a + b] * T[cn[b]];
                contrib[e * nen + a] = s;
            }
        }
        if (bad) { rc = ORC_ERR_MESH; goto done; }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            double ri = 0.0;
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) ri -= contrib[inc[k]];
            r[i] = ri;
        }
        for (int64_t f = 0; f < p->n_flux; ++f) add_flux_face(p, f, T, r);
        for (int64_t f = 0; f < p->n_if; ++f) add_interface_pair(p, f, T, r);
        for (int64_t f = 0; f < p->n_contact; ++f) add_contact_face(p, f, T, r);
        double Q = boundary_inflow(p, T, r);
        if (diag) {
            fill_diag(p, nmat, m, H, T, Q, Qcum, E0, Eref, diag + n * ORC_NDIAG);
            if (n == 0) E0 = diag[ORC_D_E];
        }
        if (n == n_steps) break;
        /* H^{n+1} = H^n + dt r^n / m at free nodes */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            if (!fixed[i] && nmat[i] >= 0) H[i] = H[i] + dt * r[i] / m[i];
        Qcum += dt * Q;
    }
done:
    free(m); free(T); free(r); free(nmat); free(ptr); free(inc); free(contrib); free(fixed);
    return rc;
}

/* threads an OpenMP region of this library would use */
int32_t orc_omp_threads(void)
{
    return (int32_t)omp_get_max_threads();
}
