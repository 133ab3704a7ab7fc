// Internal state of a castfem context, shared by the C interface of the
// explicit step (capi.cpp) and of the learned surrogate (surrogate.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/castfem.h"
#include "apparent.hpp"
#include "kernels.hpp"
#include "varprops.hpp"
#include "prep.hpp"

namespace castfem {

// thread-local message of the last failing call; returns `code`
int set_err(int code, const std::string &msg);
const char *last_error();

#define HIPCHECK(x)                                                                                   \
    do {                                                                                              \
        hipError_t e_ = (x);                                                                          \
        if (e_ != hipSuccess) throw PrepError{FEM_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

enum Stage { ST_NEW = 0, ST_FINAL = 1, ST_BOUND = 2 };

enum Buf {
    B_NODE_X, B_T, B_H, B_INV_M, B_FS, B_MATS, B_CONN, B_R, B_LCONN, B_BLOCKS, B_SH_LIST, B_PARTIALS,
    B_COMB_PTR, B_SH_POS, B_ROBIN, B_LINK_PTR, B_LINK_NODE, B_LINK_W, B_DIAG, B_QNODE, B_FLAGS, B_SEG,
    B_CAP_PARTIALS, B_APP_MATS, B_VAR_TABS_F, B_VAR_TABS_D, B_T_FIXED, B_TIME, B_NODE_WIN, B_SCHED, B_VAR_SCEN, B_VCONN, B_VW, B_COUNT
};
inline const char *const BUF_NAMES[B_COUNT] = {"node_x", "T", "H", "inv_m", "fs", "mats", "conn", "r", "lconn", "blocks",
                                  "sh_list", "partials", "comb_ptr", "sh_pos", "robin", "link_ptr",
                                  "link_node", "link_w", "diag", "qnode", "flags", "segments",
                                  "cap_partials", "app_mats", "var_tables_f32", "var_tables_f64", "T_fixed",
                                  "time", "node_windows", "dirichlet_schedule", "var_scenarios", "pair_conn", "pair_w"};
constexpr int64_t ALIGN = 256;
constexpr int GRAPH_STEPS = 16;  // steps per captured graph (even: both parities)
constexpr size_t MAX_BLOCK_LDS = 160 * 1024 - 2048;  // gfx950 LDS per workgroup, less static use

struct Candidate {
    PrepOptions o;
    int threads = 256;
    Layout L;
    double ms = -1;
};

inline MatDev make_mat(const fem_material &m, double dt) {
    MatDev d{};
    d.c = m.c;
    d.inv_c = 1.0 / m.c;
    d.Ts = m.T_sol;
    d.Tl = m.T_liq;
    d.L = m.L;
    d.Hs = m.c * m.T_sol;
    d.Hl = m.c * m.T_liq + m.L;
    d.latent = m.L > 0 ? 1 : 0;
    d.slope = (m.L > 0 && m.T_liq > m.T_sol) ? (m.T_liq - m.T_sol) / (m.c * (m.T_liq - m.T_sol) + m.L) : 0.0;
    d.inv_dH = m.L > 0 ? 1.0 / (d.Hl - d.Hs) : 0.0;
    d.dt = dt;
    d.k = m.k;
    d.kf = (float)m.k;
    d.dtf = (float)dt;
    return d;
}

// enthalpy relation on the host (initial state and read-back of fraction solid)
inline double h_of_t(const fem_material &m, double T) {
    double g = 0.0;
    if (m.L > 0 && T > m.T_sol) g = T >= m.T_liq ? 1.0 : (T - m.T_sol) / (m.T_liq - m.T_sol);
    return m.c * T + m.L * g;
}

inline void t_of_h(const MatDev &M, double H, double &T, double &fs) {
    if (!M.latent || H <= M.Hs) {
        T = H * M.inv_c;
        fs = 1.0;
    } else if (H >= M.Hl) {
        T = (H - M.L) * M.inv_c;
        fs = 0.0;
    } else {
        T = M.Ts + (H - M.Hs) * M.slope;
        fs = 1.0 - (H - M.Hs) * M.inv_dH;
    }
}

// value of a table at x (n >= 1): linear between points, constant beyond the ends
inline double tab_eval_host(const Tab<double> &t, double x) {
    const int n = t.n;
    if (x <= t.x[0]) return t.y[0];
    if (x >= t.x[n - 1]) return t.y[n - 1];
    int j = 0;
    while (j + 2 < n && !(x < t.x[j + 1])) ++j;
    return t.y[j] + (t.y[j + 1] - t.y[j]) * (x - t.x[j]) / (t.x[j + 1] - t.x[j]);
}
// the largest value of a table, or `constant` if it is not given
inline double tab_max(const Tab<double> &t, double constant) {
    if (t.n == 0) return constant;
    double m = t.y[0];
    for (int j = 1; j < t.n; ++j) m = std::max(m, t.y[j]);
    return m;
}

}  // namespace castfem

using namespace castfem;

struct fem_ctx {
    fem_options opt{};
    Problem prob;
    bool have_mesh = false;
    Stage stage = ST_NEW;
    Base base;
    std::vector<Candidate> cands;
    int chosen = 0;
    hipStream_t stream = nullptr;
    int64_t sizes[B_COUNT] = {};
    void *ptr[B_COUNT] = {};
    Dev dev;
    AppDev app;                 // apparent-capacity mode: the step's view of the buffers
    double cap_bound = 0;       // apparent mode: bound on any node's lumped capacitance (J/K)
    // temperature- and time-dependent properties: n_mat conductivity tables, then
    // h(T), h(t) and the fixed-temperature shift (empty: constant properties)
    std::vector<Tab<double>> vtabs;
    // prescribed temperature node by node: common times and, per fixed node in
    // the order of fem_set_dirichlet, its values at them (empty: none)
    std::vector<double> sched_t, sched_T;
    VarDev vdev;
    std::vector<MatDev> mats_host;
    float x_scale = 1.0f;       // FP32 node coordinates: metres per fixed-point unit
    int parity = 0;
    int64_t steps = 0;
    double E0 = 0, Eref = 0, lat0 = 0, tmin0 = 0, tmax0 = 0;
    int64_t nliq0 = 0;
    // per scenario (a single problem is scenario 0)
    std::vector<double> E0_s, Eref_s, time_s, dt_s;
    std::vector<double> Qx_s;   // boundary inflow estimated over steps the surrogate jumped
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // the device state diagnostics (`diag`) belong to the current state: the
    // last state change was a graph of GRAPH_STEPS steps, whose last node
    // reduces them (every other state change clears this)
    bool diag_fresh = false;
    double setup_seconds = 0;

    Layout &L() { return cands[chosen].L; }
    const Layout &L() const { return cands[chosen].L; }
    size_t rsize() const { return opt.precision == FEM_PREC_FP64 ? 8 : 4; }
    bool apparent() const { return opt.latent_model == FEM_LATENT_APPARENT; }
    bool variable() const { return !vtabs.empty(); }
    // the fixed-temperature shift at time t (0 without variable properties)
    double dir_shift(double t) const;
    // node_x.w carries the material index instead of the conductivity
    bool mat_in_node_x() const { return apparent() || variable(); }
};


namespace castfem {

// helpers of capi.cpp used by the surrogate interface
void set_dt(fem_ctx *c, double dt);
void set_dt_scen(fem_ctx *c, const std::vector<double> &dt);
void eager_steps(fem_ctx *c, int64_t n);
// one step of the context's latent-heat model (see enqueue_step)
hipError_t enqueue_ctx_step(const fem_ctx *c, int parity, hipStream_t s, hipEvent_t *ev);
void run_steps(fem_ctx *c, int64_t n);
void check_bound(fem_ctx *c, int fn_stage);
void energy_scenarios(fem_ctx *ctx, fem_energy_report *reps);
// the parts of energy_scenarios: device-to-host copies of the state
// diagnostics and inflow (enqueued; valid after a stream sync), and the
// fixed-order host reduction into per-scenario reports
void energy_copies(fem_ctx *ctx, std::vector<double> &dg, std::vector<double> &qn);
void energy_reduce(const fem_ctx *ctx, const std::vector<double> &dg, const std::vector<double> &qn,
                   fem_energy_report *reps);

template <class F>
int guarded(F &&f) {
    try {
        f();
        set_err(FEM_OK, "");
        return FEM_OK;
    } catch (const PrepError &e) {
        return set_err(e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return set_err(FEM_E_INVALID_ARG, "host allocation failed");
    } catch (const std::exception &e) {
        return set_err(FEM_E_INVALID_ARG, e.what());
    } catch (...) {
        return set_err(FEM_E_INVALID_ARG, "unknown error");
    }
}

}  // namespace castfem
