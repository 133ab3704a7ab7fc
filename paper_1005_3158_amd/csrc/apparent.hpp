// Apparent-heat-capacity step (Eq. 6 of the paper with Lemmon's element value
// of dH/dT, Eq. 7) on the LDS-blocked layout of the enthalpy step.
//
// Per element of a linear tetrahedron, with G = D grad T and G_f = D grad f
// (f the liquid fraction of Eq. 11, D = 6 V):
//   C_app = |c G + L G_f| / |G|  (= |grad H| / |grad T|),
//   or, where G = 0, the slope of H(T) at the element's mean temperature;
// the element adds rho C_app V / 4 to the lumped capacitance of each of its
// nodes (row-sum lumping, re-assembled every step), and the node update is the
// explicit step of Eq. 14 in temperature: T += dt r / C, with the state kept
// as H = H(T) so that the energy diagnostics of the enthalpy form apply.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace castfem {

// material constants of the apparent-capacity element kernel
struct AppMat {
    double k, rho, c, L, Ts, Tl, inv_dT;   // inv_dT = 1 / (T_liq - T_sol), 0 without latent heat
    float kf, rhof, cf, Lf, Tsf, Tlf, inv_dTf, pad;
};

struct AppDev {
    Dev d;                      // node_x.w holds the node's material index
    void *cap_partials = nullptr;   // R per (block, shared node): partial capacitance
    const AppMat *amats = nullptr;
    double cx_scale = 1.0, cx_inv = 1.0;   // FP32: fixed-point scale 2^S of capacitance sums and 2^-S
    float cx_limit = 0.0f;                 // largest element capacitance that fits (C * 2^S < 2^31)
};

// LDS bytes per local node: x, y, z, T; residual and capacitance accumulators (FP32:
// 64- and 32-bit fixed point); material
inline size_t lds_per_node_apparent(int prec) { return prec == FEM_PREC_FP64 ? 52 : 32; }

// One step reading T buffer `parity`; ev as for enqueue_step.
hipError_t enqueue_step_apparent(const AppDev &a, int parity, hipStream_t s, hipEvent_t *ev);
hipError_t set_apparent_lds_limit(int prec, size_t bytes);

}  // namespace castfem
