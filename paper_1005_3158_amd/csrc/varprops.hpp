// Temperature- and time-dependent properties on the LDS-blocked enthalpy step:
// element conductivity k(T) at the element's mean temperature (Sec. 2 after
// Eq. 1: K re-weighted per element and step), interface coefficients scaled by
// factors of temperature and time (Eq. 8 and the remark after it), and fixed
// temperatures that vary in time, uniformly or node by node (Eq. 3 with f(x, t)).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace castfem {

constexpr int TAB_POINTS = 8;

// a piecewise-linear table: n points with increasing x, constant beyond the ends
template <class R>
struct Tab {
    int32_t n, pad;
    R x[TAB_POINTS], y[TAB_POINTS];
};

// index of the time and temperature tables after the n_mat conductivity tables
enum { TAB_H_OF_T = 0, TAB_H_OF_TIME = 1, TAB_DIR_OF_TIME = 2, TAB_GLOBAL = 3 };

struct VarDev {
    Dev d;                              // node_x.w holds the node's material index
    const Tab<float> *tabs_f = nullptr; // n_mat conductivity tables, then the TAB_GLOBAL tables
    const Tab<double> *tabs_d = nullptr;
    const double *T_fixed = nullptr;    // per node: the fixed temperature before its time shift
    // time of the state held in T buffer 0 and 1, per scenario: time[parity * n_scen + scenario]
    double *time = nullptr;
    const int32_t *mat_scen = nullptr;  // [n_mat]: scenario of each material
    const int32_t *scen_mat = nullptr;  // [n_scen]: a material of each scenario (its dt)
    int32_t n_scen = 1;
    // prescribed temperature f(x, t) node by node: n_sched common times and, per
    // shared slot s < n_inflow (every fixed node has one), its n_sched values
    // (rows of other slots unused); n_sched = 0: the constant T_fixed
    const double *sched = nullptr;
    int32_t n_sched = 0;
    double sched_t[TAB_POINTS] = {};
};

__host__ __device__ inline bool tab_given(int32_t n) { return n > 0; }

// One step reading T buffer `parity`; ev as for enqueue_step.
hipError_t enqueue_step_var(const VarDev &v, int parity, hipStream_t s, hipEvent_t *ev);
hipError_t set_var_lds_limit(int prec, int nen, size_t bytes);

}  // namespace castfem
