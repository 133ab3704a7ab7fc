// Device layout and launchers of the message-passing surrogate (gfx950).
//
// Network (width WIDTH, LAYERS message-passing layers), per node row r:
//   h_0 = relu(X W_in + b_in)                      X: 12 features padded to 16
//   h_l = h_{l-1} + relu([h_{l-1}, A h_{l-1}] W_l + b_l)     A: mean over mesh neighbours
//   y   = h_L . w_out + b_out
// Activations are BF16, products run on MFMA (v_mfma_f32_16x16x16_bf16) with
// FP32 accumulation; parameters, gradients and Adam moments are FP32.
//
// The jump H = base + mu s (y - ybar): base the time extrapolation over the
// window, s = |m r| + |q a| + c EPS_T the node's activity over it, mu = 1 at a
// free phase-change node whose H2 lies within REACH activities of a kink of
// T(H) (the only places the extrapolation fails), else 0, and ybar the
// m mu s weighted mean of y over the scenario (energy-neutral correction).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"

namespace castfem {
namespace sur {

constexpr int WIDTH = 64;
constexpr int NFEAT = 12;       // input features
constexpr int KIN = 16;         // features padded to the MFMA K step
constexpr int MAX_LAYERS = 4;
constexpr float T_REF = 25.0f, T_SCALE = 700.0f, DT_SCALE = 10.0f;
constexpr double EPS_T = 0.01;   // K: activity floor of the correction scale
constexpr double REACH = 2.0;    // a kink within REACH activities of H2 enables the correction
enum { LOSS_H = 0, LOSS_T = 1, LOSS_HUBER = 2 };
constexpr float HUBER_DELTA = 0.1f;   // Huber loss: quadratic within a tenth of the node's activity

typedef uint16_t bf16;

// parameter offsets in the FP32 parameter vector
struct ParamLayout {
    int layers = 3;
    int64_t w_in = 0, b_in = 0, w[MAX_LAYERS] = {}, b[MAX_LAYERS] = {}, w_out = 0, b_out = 0, total = 0;
    void build(int L) {
        layers = L;
        int64_t o = 0;
        w_in = o;  o += NFEAT * WIDTH;          // row-major [NFEAT x WIDTH]
        b_in = o;  o += WIDTH;
        for (int l = 0; l < L; ++l) {
            w[l] = o;  o += 2 * WIDTH * WIDTH;  // row-major [2 WIDTH x WIDTH]
            b[l] = o;  o += WIDTH;
        }
        w_out = o; o += WIDTH;
        b_out = o; o += 1;
        total = o;
    }
};

struct SurDev {
    int64_t N = 0;            // nodes of the mesh (device numbering of the context)
    int layers = 3;
    int horizon = 16;         // explicit steps per jump
    int loss_mode = LOSS_H;   // LOSS_H, LOSS_HUBER: target (Ht - base) / s; LOSS_T: target T(Ht)
    int project = 1;          // 0: the output is used as it is (no energy-neutral projection)
    int quadratic = 0;        // base: 0 linear through H1, H2; 1 quadratic through H0, H1, H2
    ParamLayout pl;
    // graph: mean over mesh neighbours
    const int32_t *nbr_ptr = nullptr, *nbr = nullptr;
    const float *inv_deg = nullptr;
    // per-node strengths per unit time (times dt: per step), N x 4:
    // b_i / (m_i c_i), 2 sum_j w_ij / (m_i c_i), sum_j |K_ij| / (m_i c_i),
    // and the lumped mass m_i / sum over the node's scenario (0 at fixed nodes)
    const float *coef = nullptr;
    // energy-neutral correction: per node its scenario; node segments of one
    // scenario each (the context's), and the segments of every scenario (CSR)
    const int32_t *scen = nullptr;
    const int32_t *seg_begin = nullptr;
    int64_t n_seg = 0, n_scen = 1;
    const int32_t *scen_seg_ptr = nullptr, *scen_seg = nullptr;
    double *seg_part = nullptr;           // slots x n_seg x 2
    double *scen_sum = nullptr;           // slots x n_scen x 2: the projected sum and sum m mu s
    const uint32_t *flags = nullptr;      // N: material | flags (shared with the context)
    const void *mats = nullptr;           // MatDev table of the context
    // parameters
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    bf16 *wt_in = nullptr;                // [WIDTH x KIN]   W_in transposed, zero-padded
    bf16 *wt[MAX_LAYERS] = {};            // [WIDTH x 2 WIDTH] W_l transposed
    bf16 *wr[MAX_LAYERS] = {};            // [2 WIDTH x WIDTH] W_l as is (for dU = dZ W_l^T)
    // activations for R rows
    int64_t rows = 0;                     // capacity in rows
    bf16 *X = nullptr;                    // R x KIN
    bf16 *Zin = nullptr;                  // R x WIDTH pre-activation of the encoder
    bf16 *U[MAX_LAYERS] = {};             // R x 2 WIDTH: [h_{l-1}, A h_{l-1}]
    bf16 *Z[MAX_LAYERS] = {};             // R x WIDTH pre-activations
    bf16 *HL = nullptr;                   // R x WIDTH last hidden state
    float *y = nullptr;                   // R outputs
    double *base = nullptr;               // R: extrapolated enthalpy
    float *scale = nullptr;               // R: mu_i s_i (0 where the extrapolation stands)
    float *target = nullptr;              // R: training target (see loss_mode)
    // backward
    float *dH = nullptr;                  // R x WIDTH
    bf16 *dZ = nullptr;                   // R x WIDTH
    float *dU = nullptr;                  // R x 2 WIDTH
    float *partials = nullptr;            // reduction partials
    float *partials2 = nullptr;           // second pass of the reduction of partials
    float *dy = nullptr;                  // R: dL/dy of the unprojected output
    int64_t n_partial_blocks = 0;
    double *loss_part = nullptr;          // per workgroup loss partials
    // jumps of the solver state
    double *H0 = nullptr, *H1 = nullptr, *H2 = nullptr;  // N: the three explicit states a jump starts from
    float2 *H2_pair = nullptr;            // N (FP32 state): the enthalpy pairs at H2, bit for bit (null in FP64)
    double *Hn = nullptr;                 // N: the predicted state (the next chunk's H0)
    double *rext = nullptr;               // N: increment the extrapolation expects one step past the horizon
    int32_t *check = nullptr;             // 2 x per workgroup: nodes whose f_s fell; nodes failing the verification
};

// rows handled by one workgroup of the weight-gradient product
constexpr int GRAD_ROWS = 512;
constexpr int PARTIAL_GROUP = 64;     // partials summed per group in the first reduction pass

// features, extrapolated base, scale and (Ht != null) targets of `slots`
// states: slot q is sample idx[q] (q if idx is null) at offset sample * stride
hipError_t features(const SurDev &s, const void *H0, const void *H1, const void *H2, int h_is_double,
                    const float *Ht, int64_t stride, const int32_t *idx, int64_t slots, hipStream_t st);
// store: keep what the backward pass needs (pre-activations, neighbour means);
// project: apply the energy-neutral projection to y (otherwise only the
// per-scenario sums are formed, for write_jump to subtract)
hipError_t forward(const SurDev &s, int64_t rows, int store, int project, hipStream_t st);
hipError_t loss_and_dy(const SurDev &s, int64_t rows, hipStream_t st);      // writes loss partials, dH of the output
hipError_t backward(const SurDev &s, int64_t rows, hipStream_t st);
hipError_t adam(const SurDev &s, float lr, float b1, float b2, float eps, int step, hipStream_t st);
hipError_t refresh_bf16(const SurDev &s, hipStream_t st);
hipError_t apply(const SurDev &s, int64_t rows, double *H_out, hipStream_t st);   // H = base + scale * y

// solver state <-> surrogate (d: the context's device layout, T buffer `parity`)
// (keep_qnode, if not null: also the per-node inflow sums, d.n_inflow doubles)
// FP64 copy of the enthalpy state into out (and of the inflow sums into
// keep_qnode, and of the raw FP32 pairs into pair_out, when not null)
hipError_t state_to_f64(const Dev &d, double *out, double *keep_qnode, hipStream_t st, float2 *pair_out = nullptr);
// features of one state whose H2 is the solver's current state (kept in s.H2, the
// FP32 pairs and keep_qnode as state_to_f64 keeps them), from FP64 copies H0, H1
hipError_t features_live(const SurDev &s, const Dev &d, const double *H0, const double *H1, double *keep_qnode,
                         hipStream_t st);
hipError_t state_to_f32(const Dev &d, float *out, hipStream_t st);
// write H = base + scale * (y - the scenario's weighted mean of y) (one state slot,
// unprojected y) into the solver state with its T and fraction solid; counts
// per workgroup the nodes whose fraction solid fell by more than fs_tol below
// that of s.H2
hipError_t write_jump(const SurDev &s, const Dev &d, int parity, float fs_tol, hipStream_t st);
// put the state back to s.H2
// (kept_qnode, if not null: also the per-node inflow sums saved with H2)
hipError_t restore_h2(const SurDev &s, const Dev &d, int parity, const double *kept_qnode, hipStream_t st);
// after one explicit step from the predicted state s.Hn: count per workgroup
// the free nodes whose increment departs from the extrapolated one, s.rext, by
// more than tol (in K: |dT/dH (s.Hn)| |(H - s.Hn) - s.rext| > tol)
hipError_t verify_jump(const SurDev &s, const Dev &d, float tol, hipStream_t st);
__host__ __device__ inline int64_t check_blocks(int64_t N) { return (N + 255) / 256; }

}  // namespace sur
}  // namespace castfem
