/*
 * castfem: explicit finite-element casting-solidification step on MI355X (gfx950).
 *
 * Method (R. Tavakoli, "Improvement cache efficiency of explicit finite element
 * procedure and its application to parallel casting solidification
 * simulation", 2006):
 *   - heat conduction with phase change, written for the nodal specific
 *     enthalpy H (Sec. 2, Eq. 1 and Eq. 5) with T = T(H) from the enthalpy
 *     relation of Eq. 11 (linear latent release between solidus and liquidus);
 *   - Galerkin linear tetrahedra (Sec. 3, Eq. 9) or trilinear hexahedra,
 *     row-sum lumped capacitance (Sec. 3);
 *   - fully explicit update (Eq. 10 with theta = 0, i.e. Eq. 14) assembled
 *     element by element (Eq. 15-18): H_i += dt * r_i / m_i, r = F - K T;
 *   - flux/convective boundaries (Eq. 4) and cast/mould contact conductance
 *     (Eq. 8) whose ambient temperature is the mean of the sister face on the
 *     other side (end of Sec. 3);
 *   - element blocks with private/shared nodes and a sum of partial residuals
 *     at shared nodes (Eq. 19-22, Sec. 4.1.2 and the cache blocking of
 *     Sec. 4.2), here held in LDS per workgroup.
 *
 * Conventions
 *   - SI units, temperatures in deg C, specific enthalpy J/kg with H = 0 at 0 C.
 *   - Indices are 0-based int32; counts are int64.
 *   - Every function returns FEM_OK (0) or a negative FEM_E_* code and, on
 *     error, sets a thread-local message read by fem_last_error().  No C++
 *     exception crosses this interface.  A setup call that fails leaves the
 *     context as it was.
 *   - Host arrays passed in are owned by the caller and copied during the call.
 *   - Device buffers are owned by the caller (allocated after
 *     fem_query_buffers) and borrowed by the context until fem_destroy.  The
 *     library allocates no device memory of its own.
 *   - Work is enqueued on the stream given to fem_set_stream.  Stepping is
 *     asynchronous; read-back calls synchronise that stream.  A failure of
 *     asynchronous work is reported by the next synchronising call.
 */
#ifndef CASTFEM_H
#define CASTFEM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
enum {
    FEM_OK = 0,
    FEM_E_INVALID_ARG = -1,   /* null pointer, bad size or enum value */
    FEM_E_MESH = -2,          /* inverted element, node in two materials, index out of range */
    FEM_E_STATE = -3,         /* call out of order (e.g. step before bind) */
    FEM_E_UNSTABLE = -4,      /* dt above the explicit stability bound */
    FEM_E_NONFINITE = -5,     /* the state holds NaN or Inf */
    FEM_E_HIP = -6,           /* a HIP runtime call failed */
    FEM_E_UNSUPPORTED = -7    /* option combination not built */
};

enum { FEM_TET4 = 4, FEM_HEX8 = 8 };
enum { FEM_PREC_FP64 = 0, FEM_PREC_FP32_KAHAN = 1 };
enum { FEM_ORDER_NONE = 0, FEM_ORDER_RCM = 1, FEM_ORDER_MORTON = 2, FEM_ORDER_HILBERT = 3 };
enum { FEM_SCATTER_GLOBAL_ATOMIC = 0, FEM_SCATTER_LDS_BLOCKED = 1, FEM_SCATTER_COLORED = 2 };
/* Latent-heat model.
 * ENTHALPY: the nodal enthalpy is advanced, H_i += dt r_i / m_i, T = T(H)
 *   (Eq. 5 and Eq. 11); conserves energy exactly.
 * APPARENT: the paper's apparent heat capacity (Eq. 6) with Lemmon's element
 *   value of dH/dT (Eq. 7): per element C_app = |grad H| / |grad T| from the
 *   linear interpolants of the nodal H(T_j) and T_j (where grad T = 0, the slope
 *   of H(T) at the element's mean temperature), lumped to
 *   C_i = sum_e rho C_app V / 4 and re-assembled every step; the update is
 *   T_i += dt r_i / C_i (Eq. 14) and the state keeps H_i = H(T_i), so energy is
 *   no longer conserved exactly where elements straddle the solidus or
 *   liquidus.  Linear tetrahedra and the LDS-blocked scatter only; a material
 *   with L > 0 needs T_liq > T_sol.  Not accepted by the surrogate. */
enum { FEM_LATENT_ENTHALPY = 0, FEM_LATENT_APPARENT = 1 };

typedef struct fem_ctx fem_ctx;

/* A piecewise-linear table: n points (at most 8) with increasing x, linear
 * between them and constant beyond the ends; n = 0 means "not given". */
typedef struct {
    int32_t n, pad;
    double x[8], y[8];
} fem_table;

typedef struct {
    int32_t device;          /* HIP device ordinal */
    int32_t precision;       /* FEM_PREC_* */
    int32_t ordering;        /* FEM_ORDER_*: node/element locality reordering */
    int32_t scatter;         /* FEM_SCATTER_* */
    int32_t block_elems;     /* LDS-blocked: elements per block; 0 = autotune */
    int32_t allow_unstable;  /* nonzero: fem_step accepts dt above the bound */
    int32_t lds_bytes;       /* LDS-blocked: LDS budget per workgroup; 0 = default */
    int32_t threads;         /* LDS-blocked: threads per workgroup; 0 = default (256) */
    int32_t latent_model;    /* FEM_LATENT_*; 0 = enthalpy */
    int32_t reserved[7];     /* must be zero */
} fem_options;

/* One material: conductivity k (W/mK), density rho (kg/m^3), specific heat c
 * (J/kgK), solidus and liquidus (C) and latent heat L (J/kg).  L = 0: no phase
 * change (fraction solid reported as 1).  T_sol == T_liq: isothermal change. */
typedef struct {
    double k, rho, c, T_sol, T_liq, L;
} fem_material;

typedef struct {
    int64_t n_nodes, n_elems;
    int64_t n_blocks;            /* LDS-blocked: element blocks */
    int64_t n_shared;            /* LDS-blocked: nodes touched by more than one block */
    int64_t n_partials;          /* LDS-blocked: (block, shared node) partial slots */
    int64_t max_local_nodes;     /* LDS-blocked: largest block node set */
    int64_t n_colors;            /* colored: element colours */
    int64_t bandwidth_before;    /* max |i - j| over coupled nodes, input numbering */
    int64_t bandwidth_after;     /* the same after reordering */
    int64_t block_elems;         /* elements per block in use */
    double shared_fraction;      /* n_shared / n_nodes */
    double dt_bound;             /* explicit stability bound (s) */
    double setup_seconds;        /* host time of fem_finalize */
    double contact_search_seconds;   /* host time of the sister search (fem_set_contact) */
    int64_t n_contact;           /* contact faces */
    int64_t block_threads;       /* LDS-blocked: threads per element block in use */
    int64_t reserved[1];
} fem_prep_report;

typedef struct {
    char name[32];
    int64_t bytes;               /* size the caller must allocate (may be 0) */
    int64_t alignment;           /* required alignment of the device pointer */
} fem_buffer_desc;

typedef struct {
    double E;                /* sum_i m_i H_i (J), FP64 */
    double E0;               /* E of the initial state */
    double latent;           /* sum_i m_i L_i (1 - fs_i): latent heat still to release */
    double Q_cum;            /* sum over steps of dt * boundary inflow (J) */
    double residual;         /* |E - E0 - Q_cum| / |E0 - E_ref|, E_ref = sum m_i H_i(25 C) */
    double T_min, T_max;
    int64_t n_liquid;        /* phase-change nodes with fraction solid < 1 */
    int64_t nonfinite;       /* nodes whose enthalpy is NaN or Inf */
    int64_t steps;           /* steps taken since the initial state */
    double time;             /* simulated time (s); the largest over scenarios for a batch */
} fem_energy_report;

typedef struct {
    double ms_element;       /* mean duration of one element (block) kernel launch */
    double ms_combine;       /* mean duration of one node update / shared combine launch */
    int64_t launches_element, launches_combine;
    double bytes_element;    /* algorithmic bytes per element-kernel launch */
    double bytes_combine;    /* algorithmic bytes per combine-kernel launch */
} fem_kernel_times;

/* ------------------------------------------------------------ lifecycle */
/* Create a context.  opt may be NULL for the defaults (device 0, FP32 with
 * Kahan-compensated enthalpy, Hilbert ordering, LDS-blocked scatter,
 * autotuned block size).  *out receives the handle. */
int fem_create(fem_ctx **out, const fem_options *opt);
/* Release host memory of the context.  Device buffers stay with the caller. */
int fem_destroy(fem_ctx *ctx);
/* Message of the last failing call on this thread ("" if none). */
const char *fem_last_error(void);
/* Stream (a hipStream_t) for all device work; NULL = the null stream, which
 * disables graph capture of fem_step. */
int fem_set_stream(fem_ctx *ctx, void *hip_stream);

/* ------------------------------------------------------------ problem */
/* Mesh (Sec. 3): xyz is n_nodes x 3 (m), conn is n_elems x elem_type node ids
 * with positive orientation (tet: (x1-x0).((x2-x0)x(x3-x0)) > 0; hex: the
 * usual bottom-then-top ordering), elem_mat the material of every element.
 * Nodes on a cast/mould interface must be duplicated, one copy per side, so
 * that every node belongs to one material (checked by fem_finalize). */
int fem_upload_mesh(fem_ctx *ctx, int32_t elem_type, int64_t n_nodes, const double *xyz,
                    int64_t n_elems, const int32_t *conn, const int32_t *elem_mat);
/* Material table (Eq. 1, Eq. 11); n_mat entries indexed by elem_mat. */
int fem_set_materials(fem_ctx *ctx, int32_t n_mat, const fem_material *m);
/* Fixed temperatures (Eq. 3, constant in time): n node ids and their values.
 * A fixed node keeps H(T_value) and its residual counts as boundary inflow. */
int fem_set_dirichlet(fem_ctx *ctx, int64_t n, const int32_t *node, const double *T_value);
/* Flux/convective faces (Eq. 4): -k dT/dn = q + h (T - T_inf).  face_nodes is
 * nf x nodes_per_face (3 or 4); each node of face f receives
 * (A_f / nodes_per_face) (-q_f - h_f (T_i - T_inf_f)).  A quad's area is half
 * the norm of the cross product of its diagonals.  Faces not listed are
 * adiabatic. */
int fem_set_flux_faces(fem_ctx *ctx, int64_t nf, int32_t nodes_per_face, const int32_t *face_nodes,
                       const double *q, const double *h, const double *T_inf);
/* Cast/mould contact (Eq. 8, sister faces at the end of Sec. 3): npairs
 * triangles face_a[3] / face_b[3] on the two sides of the interface with
 * coefficient h_i.  Node i of one side receives h_i (A/3) (mean T of the
 * other face - T_i), A the area of face_a. */
int fem_set_interface(fem_ctx *ctx, int64_t npairs, const int32_t *face_a, const int32_t *face_b,
                      const double *h_i);
/* Cast/mould contact on non-matching meshes (Eq. 8 with the sister element of
 * the end of Sec. 3): nf triangles face_nodes[3], each on side 0 or 1 of a
 * contact surface, with coefficient h.  fem_finalize gives every face a sister:
 * the face of the other side, in the same scenario, whose centroid
 * ((x_0 + x_1) + x_2) / 3 is nearest in squared Euclidean distance (FP64; ties
 * go to the lower face index), found by a uniform-grid search over the
 * centroids.  Node i of face f then receives h_f (A_f / 3) (mean T of the
 * sister's nodes - T_i), A_f the area of f itself.  The two sides of a
 * non-matching surface do not exchange equal and opposite heat, so energy is
 * not conserved exactly (fem_energy reports the drift).  May be combined with
 * fem_set_interface.  Errors: FEM_E_MESH if a face has no face of the other
 * side in its scenario. */
int fem_set_contact(fem_ctx *ctx, int64_t nf, const int32_t *face_nodes, const int32_t *side, const double *h);
/* After fem_finalize: the sister of every contact face (nf int32, caller-owned). */
int fem_get_sisters(const fem_ctx *ctx, int32_t *sister);
/* Temperature- and time-dependent properties (Sec. 2 after Eq. 1; Eq. 3 with
 * f(x, t); Eq. 8 and the remark after it), any of them NULL or n = 0 for none:
 *   k_of_T[n_mat]: conductivity of each material against T (W/mK); each element
 *     takes k at the mean of its nodal T^n, so K is re-weighted per element and
 *     step;
 *   h_of_T: factor on every interface coefficient (fem_set_interface and
 *     fem_set_contact) against temperature; the coupling of node i to node j of
 *     the face it sees uses the factor at (T_i + T_j) / 2;
 *   h_of_t: factor on every interface coefficient against time t (s);
 *   dir_of_t: shift added to every fixed temperature: T_i(t) = T_D,i + shift(t);
 *     the prescribed change of a fixed node's enthalpy counts as boundary inflow.
 * Time starts at 0 at fem_bind_buffers and advances on the device, in a batch
 * (fem_set_scenarios) per scenario by that scenario's dt.  The stability bound
 * takes every property at its largest value.  Supported with the enthalpy form
 * and the LDS-blocked scatter; the surrogate and fem_write_state refuse such a
 * context (FEM_E_UNSUPPORTED).
 * Call before fem_finalize. */
int fem_set_variable_properties(fem_ctx *ctx, int32_t n_mat, const fem_table *k_of_T, const fem_table *h_of_T,
                                const fem_table *h_of_t, const fem_table *dir_of_t);
/* Prescribed temperature as a function of place and time, T = f(x, t) on the
 * fixed-temperature boundary (Eq. 3), node by node: n_times common times
 * times[0] < ... < times[n_times - 1] (s, 1 <= n_times <= 8) and, for the k-th
 * node of fem_set_dirichlet (in its order), its temperatures at those times in
 * values[k * n_times .. k * n_times + n_times - 1] (C), linear in between and
 * constant beyond the ends.  The schedule takes the place of the constant
 * values of fem_set_dirichlet (a node starts at f(x, 0)); a dir_of_t shift of
 * fem_set_variable_properties still adds.  The prescribed change of a fixed
 * node's enthalpy counts as boundary inflow.  Both arrays are host memory,
 * copied.  Makes the context one with variable properties (the same limits:
 * enthalpy form, LDS-blocked scatter, no surrogate or state restore; in a
 * batch each fixed node follows its schedule on its scenario's clock).  Call after fem_set_dirichlet and before fem_finalize; errors:
 * FEM_E_STATE (no fixed nodes, or after fem_finalize), FEM_E_INVALID_ARG (count
 * out of range, times not increasing, a value not finite). */
int fem_set_dirichlet_schedule(fem_ctx *ctx, int32_t n_times, const double *times, const double *values);
/* Initial temperature of every node (Eq. 2); fixed nodes take their value. */
int fem_set_initial_T(fem_ctx *ctx, const double *T0);
/* Batch of independent casting scenarios in one mesh: material_scenario[m]
 * (one entry per material, set after fem_set_materials) names the scenario of
 * material m, 0 <= id < n_scen, every scenario owning at least one material.
 * Elements of different scenarios may not share nodes and no interface pair
 * may join two scenarios (checked by fem_finalize, FEM_E_MESH).  Each
 * scenario has its own time step (fem_step_batch), stability bound and energy
 * balance.  Without this call the whole problem is scenario 0. */
int fem_set_scenarios(fem_ctx *ctx, int32_t n_scen, const int32_t *material_scenario);

/* Validate, lump, reorder, block, colour and bound dt (host work only, no
 * device call).  rep may be NULL. */
int fem_finalize(fem_ctx *ctx, fem_prep_report *rep);
/* Device buffers the context needs.  Call with d == NULL to get the count in
 * *n; then with an array of *n descriptors. */
int fem_query_buffers(const fem_ctx *ctx, fem_buffer_desc *d, int32_t *n);
/* Hand over device pointers in the order of fem_query_buffers, upload the
 * static data and the initial state (and autotune the block size when
 * requested).  Synchronises the stream. */
int fem_bind_buffers(fem_ctx *ctx, void *const *dev_ptrs, int32_t n);
/* Report of the finalized layout (valid after fem_finalize; block fields are
 * final after fem_bind_buffers). */
int fem_get_report(const fem_ctx *ctx, fem_prep_report *rep);

/* ------------------------------------------------------------ stepping */
/* Explicit stability bound: 2 / max_i [sum_j |K_ij| + boundary terms] / (m_i c_i)
 * (Gershgorin on the lumped system with the sensible heat c; Eq. 13 states
 * only the scaling rho c l^2 / k). */
int fem_stable_dt(const fem_ctx *ctx, double *dt);
/* n_steps explicit steps of size dt (Eq. 14 in enthalpy form), enqueued on the
 * stream; repeated calls reuse a captured hipGraph. */
int fem_step(fem_ctx *ctx, double dt, int64_t n_steps);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): fem_step without any
 * allocation.  Every launch is enqueued eagerly (no graph is built), a new dt
 * is written into the device material table by a kernel, and the partial
 * residuals of the shared nodes live in the library's static device scratch
 * of 32 MiB (file-scope, one copy per GPU, kept until the process ends)
 * instead of the bound `partials` buffer; each call clears the part it uses
 * with a fill kernel.  Results are those of fem_step bit for bit.  All calls
 * on one GPU share that scratch: calls that overlap on one GPU (two streams,
 * two threads) race.  Enthalpy form, one scenario and the LDS-blocked scatter
 * only (else FEM_E_UNSUPPORTED); a mesh needing more than 32 MiB of partials
 * (about 4 * shared nodes * 4 bytes in FP32) is refused with FEM_E_UNSUPPORTED.
 * Other errors as fem_step. */
int fem_step_no_alloc(fem_ctx *ctx, double dt, int64_t n_steps);
/* Stability bound of every scenario (n_scen doubles). */
int fem_stable_dt_scenarios(const fem_ctx *ctx, double *dt_bounds);
/* n_steps steps of every scenario at once, scenario s with its own dt
 * (dt_per_scenario[n_scen]); each checked against that scenario's bound. */
int fem_step_batch(fem_ctx *ctx, const double *dt_per_scenario, int64_t n_steps);

/* ------------------------------------------------------------ read-back */
/* Temperature / fraction solid / enthalpy of every node in the caller's
 * numbering (n_nodes doubles).  Synchronous. */
int fem_read_T(fem_ctx *ctx, double *T_host);
int fem_read_fs(fem_ctx *ctx, double *fs_host);
int fem_read_H(fem_ctx *ctx, double *H_host);
/* FP64 energy balance of the current state (wavefront partials summed in a
 * fixed order), over all scenarios.  Synchronous; FEM_E_NONFINITE if any
 * enthalpy is NaN or Inf. */
int fem_energy(fem_ctx *ctx, fem_energy_report *rep);
/* The same per scenario: reps[n_scen]. */
int fem_energy_scenarios(fem_ctx *ctx, fem_energy_report *reps);
/* Checkpoint of the evolving state (enthalpy with its compensation, the
 * current temperatures, fraction solid, step count, time, energy budget), every
 * per-node array in input-node order, so that it restores into any layout of
 * the same problem (another ordering, block size or autotuner choice).  With
 * buf == NULL *bytes receives the size.  fem_write_state refuses a checkpoint
 * of another node count, precision or scenario count (FEM_E_INVALID_ARG). */
int fem_read_state(fem_ctx *ctx, void *buf, int64_t *bytes);
int fem_write_state(fem_ctx *ctx, const void *buf, int64_t bytes);
/* New (device) id of every input node (n_nodes int32). */
int fem_get_node_perm(const fem_ctx *ctx, int32_t *perm);

/* ------------------------------------------------------------ measurement */
/* Run n_steps without a graph, each step kernel timed by start and stop events
 * of its own launch on the context stream (the dispatch gap between launches
 * is not counted), and return the mean launch durations and the algorithmic
 * bytes per launch (16 B per element, 48 B per node split between kernels;
 * 44 B per node in the apparent-capacity form, which reads no 1/m_i). */
int fem_time_kernels(fem_ctx *ctx, double dt, int64_t n_steps, fem_kernel_times *out);
/* Device-to-device copy of `bytes` (multiple of 16) by a plain vector kernel on
 * the context stream; the reference for measured bandwidth and counters. */
int fem_copy_kernel(fem_ctx *ctx, void *dst, const void *src, int64_t bytes, int32_t repeats, double *ms_per_copy);
/* The same copy with non-temporal loads and stores over up to 32,768
 * workgroups: the streaming-bandwidth ceiling the element kernel is compared
 * with.  Same arguments and errors as fem_copy_kernel. */
int fem_copy_kernel_nt(fem_ctx *ctx, void *dst, const void *src, int64_t bytes, int32_t repeats, double *ms_per_copy);

/* ------------------------------------------------------------ surrogate */
/* A learned message-passing surrogate that jumps the enthalpy state `horizon`
 * explicit steps ahead (not part of the paper; the explicit step of Eq. 14 is
 * its fallback and the reference for its error).  From three consecutive
 * explicit states H0 = H^n, H1 = H^{n+1}, H2 = H^{n+2} it predicts, per node i,
 * with m = horizon - 2, q = m (m + 1) / 2, r = H2 - H1 and a = (H2 - H1) - (H1 - H0),
 *   H^{n+horizon}_i = base_i + mu_i s_i (y_i - ybar),
 * base = H2 + m r (linear extrapolation, the default) or
 * base = H2 + m r + q a (quadratic; fem_sur_options.extrapolation).
 * s_i = |m r_i| + |q a_i| + 0.01 K c_i is the node's activity over the window;
 * mu_i = 1 at a free phase-change node whose H2 lies within 2 (|m r_i| + |q a_i|)
 * of the solidus enthalpy c T_sol or the liquidus enthalpy c T_liq + L,
 * else 0: the network corrects the
 * extrapolation only where a kink of T(H) makes it fail.  ybar is the mean of
 * y weighted by m_i mu_i s_i over the node's scenario (m_i the lumped mass),
 * which makes the correction energy-neutral.
 * y = output of a network of `layers` residual message-passing layers of
 * width 64 over the mesh graph (nodes sharing an element, mean aggregation):
 *   h_0 = relu(x W_in + b_in);  h_l = h_{l-1} + relu([h_{l-1}, mean_nbr h_{l-1}] W_l + b_l);
 *   y = h_L . w_out + b_out.
 * Node features x (12): (T(H2) - 25)/700, fs(H2), latent-heat flag, Robin,
 * interface and conduction strengths b_i dt/(m_i c_i), 2 sum w_ij dt/(m_i c_i),
 * sum_j |K_ij| dt/(m_i c_i), m r / s, q a / s, 1, ln(s / (c 1 K)) / 8, and
 * clip((H2 - H_liq) / s, -4, 4) / 4, clip((H2 - H_sol) / s, -4, 4) / 4 (0 for
 * materials without latent heat).
 * Activations and weights are BF16 on the matrix cores with FP32
 * accumulation; parameters, gradients and Adam moments are FP32.
 * Parameters are one FP32 vector: W_in [12 x 64] row-major, b_in [64], then per
 * layer W_l [128 x 64] row-major and b_l [64], then w_out [64], b_out [1].
 * State arrays passed in are float32 device arrays in the context's device
 * numbering (fem_get_node_perm); state q of a call starts at q * stride.
 * Features use the context's current time step (per scenario), i.e. that of
 * its last fem_step, fem_step_batch or fem_advance call. */
typedef struct fem_sur fem_sur;

/* Training loss, a mean over all nodes of the states of a step, with y' = y - ybar:
 *   FEM_SUR_LOSS_H: mu (y' - t)^2 with t = (Ht - base) / s, the enthalpy error
 *   relative to the node's activity;
 *   FEM_SUR_LOSS_T: ((T(base + mu s y') - T(Ht)) / 10 K)^2, the temperature error
 *   (gradient through the branch of T(H) the prediction lies on);
 *   FEM_SUR_LOSS_HUBER: the enthalpy error e = y' - t with e^2 replaced by
 *   0.1 (2|e| - 0.1) beyond |e| = 0.1, at masked nodes. */
enum { FEM_SUR_LOSS_H = 0, FEM_SUR_LOSS_T = 1, FEM_SUR_LOSS_HUBER = 2 };
enum { FEM_SUR_EXTRAP_LINEAR = 0, FEM_SUR_EXTRAP_QUADRATIC = 1 };

typedef struct {
    int32_t width;         /* must be 64 */
    int32_t layers;        /* 1..4 */
    int32_t horizon;       /* explicit steps per chunk (two computed, the rest jumped), >= 3 */
    int32_t max_samples;   /* states per forward / backward pass (rows = max_samples * n_nodes < 2^31) */
    int32_t train;         /* nonzero: size the training buffers too */
    int32_t loss;          /* FEM_SUR_LOSS_*: what the training loss measures */
    int32_t extrapolation; /* FEM_SUR_EXTRAP_*: the base the network corrects */
    int32_t no_projection; /* nonzero: y is used as it is (ybar = 0), the correction is not energy-neutral
                              (for studying the projection and checking gradients without its cancellation) */
    int32_t reserved[4];   /* must be zero */
    uint64_t seed;         /* initial parameters (He-normal, counter-based generator) */
} fem_sur_options;

typedef struct {
    int64_t steps;         /* explicit steps the state advanced in the call */
    int64_t plain_steps;   /* of these, steps computed by the explicit kernels */
    int64_t jumps_accepted;
    int64_t jumps_rejected;
    int32_t solid;         /* 1: every phase-change node has fraction solid 1 */
    int32_t pad;
    double wall_seconds;   /* host wall-clock of the call */
    double max_residual;   /* largest energy residual of an accepted jump */
    int64_t rejected_fs;   /* jumps rejected by the fraction-solid (or NaN) check */
    int64_t rejected_energy; /* jumps rejected by the energy residual */
    int64_t rejected_verify; /* jumps rejected by the one-step verification */
    int64_t reserved[1];
} fem_advance_report;

/* Surrogate on a bound context (graph and node strengths from its layout). */
int fem_sur_create(fem_sur **out, fem_ctx *ctx, const fem_sur_options *opt);
int fem_sur_destroy(fem_sur *s);
/* Device buffers of the surrogate, as fem_query_buffers / fem_bind_buffers;
 * binding uploads the graph and sets the initial parameters.  Synchronous. */
int fem_sur_query_buffers(const fem_sur *s, fem_buffer_desc *d, int32_t *n);
int fem_sur_bind_buffers(fem_sur *s, void *const *dev_ptrs, int32_t n);
int fem_sur_n_params(const fem_sur *s, int64_t *n);
/* Copy the FP32 parameter vector out / in (host arrays of n floats); setting
 * resets the Adam moments.  Synchronous. */
int fem_sur_get_params(fem_sur *s, float *host, int64_t n);
int fem_sur_set_params(fem_sur *s, const float *host, int64_t n);
/* Write the parameters to a file (path: NUL-terminated; created or replaced):
 * the bytes "CASTSUR1", int32 width, layers, horizon, extrapolation, int64
 * n_params, then n_params FP32 values, all in host byte order.  Load reads
 * such a file into a surrogate of the same width, layers, horizon and
 * extrapolation (FEM_E_INVALID_ARG otherwise, or for a truncated or oversized
 * file, leaving the parameters unchanged) and clears the Adam moments, as
 * fem_sur_set_params does.  Synchronous. */
int fem_sur_save(fem_sur *s, const char *path);
int fem_sur_load(fem_sur *s, const char *path);
/* Features (as rounded to BF16) of `slots` states: X_host[slots * n_nodes * 12]. */
int fem_sur_features(fem_sur *s, const float *H0, const float *H1, const float *H2, int64_t stride, int64_t slots,
                     float *X_host);
/* Training loss (fem_sur_options.loss) over all nodes of `slots` states and its
 * gradient with respect to the parameters (grad_host: n_params floats). */
int fem_sur_loss_grad(fem_sur *s, const float *H0, const float *H1, const float *H2, const float *Ht, int64_t stride,
                      int64_t slots, double *loss, float *grad_host);
/* Adam training: `epochs` passes over n_samples (H0, H1, H2, Ht) states in a
 * seeded shuffled order, `batch` states per step, learning rate decaying from
 * lr to lr_final on a cosine.  loss_per_epoch (may be NULL): epochs doubles. */
int fem_sur_train(fem_sur *s, const float *H0, const float *H1, const float *H2, const float *Ht, int64_t stride,
                  int64_t n_samples, int32_t batch, int32_t epochs, float lr, float lr_final, uint64_t seed,
                  double *loss_per_epoch);
/* Predicted H^{n+horizon} of `slots` states into H_out (device, slots * n_nodes doubles). */
int fem_sur_predict(fem_sur *s, const float *H0, const float *H1, const float *H2, int64_t stride, int64_t slots,
                    double *H_out);
/* Training data from explicit trajectories that also pass through the
 * network's own jumps: n_chunks chunks of `horizon` explicit steps of every
 * scenario (dt_per_scenario[n_scen]); chunk k writes H^n, H^{n+1}, H^{n+2} and
 * H^{n+horizon} (float32, device numbering) to S_dev[(4k + j) * n_nodes ...].
 * With jump_every = J > 0, every J-th chunk is followed by returning to
 * H^{n+2} and jumping with the current network (as fem_advance would, without
 * the gates), so that the next chunks start from a jumped state.  Advances
 * the context's state and clock.  Synchronous. */
int fem_sur_generate(fem_sur *s, const double *dt_per_scenario, int64_t n_chunks, int32_t jump_every, float *S_dev);
/* Current enthalpy of every node (device numbering) into a float32 device array. */
int fem_snapshot_H(fem_ctx *ctx, float *H_dev);
/* Advance every scenario (dt_per_scenario[n_scen]) until max_steps or, with
 * until_solid, until every phase-change node has fraction solid 1 (checked
 * after every chunk).  s == NULL: plain explicit steps in chunks of 16.
 * Otherwise chunks of `horizon` steps: explicit steps to H^n, H^{n+1},
 * H^{n+2}, the surrogate's jump to H^{n+horizon}, and one explicit step from
 * the jump (which is also the next chunk's first step).  The jump is kept only
 * if, in every scenario:
 *   - no phase-change node's fraction solid fell by more than fs_tol below its
 *     value at H^{n+2}, and no enthalpy is NaN or Inf;
 *   - the explicit step from the jump agrees with the extrapolation: at every
 *     free node |dT/dH| |dH - dH_ext| <= verify_tol (K), dH_ext the increment
 *     the extrapolation implies for that step (a wrong jump relaxes fast in
 *     the first explicit step after it);
 *   - |dE - dQ| / |E_n - E_ref| <= energy_tol, with dE the FP64 energy change
 *     since the last check, dQ the exact boundary inflow of the explicit steps
 *     in between plus their mean rate over the jumped steps, E_n the energy at
 *     the last check and E_ref that of the scenario at 25 C.
 * A rejected jump returns the state to H^{n+2} and horizon - 2 explicit steps
 * follow.  The extrapolated inflow of kept jumps enters Q_cum of the energy
 * reports.  Synchronous. */
int fem_advance(fem_ctx *ctx, fem_sur *s, const double *dt_per_scenario, int64_t max_steps, int32_t until_solid,
                double energy_tol, double fs_tol, double verify_tol, fem_advance_report *rep);

#ifdef __cplusplus
}
#endif
#endif
