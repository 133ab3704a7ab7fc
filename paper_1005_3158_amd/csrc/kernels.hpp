// Device-side data layout of one context and the step launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "prep.hpp"

namespace castfem {

// material constants of the enthalpy relation, precomputed in FP64 on the host
struct MatDev {
    double c, inv_c, Ts, Tl, L, Hs, Hl, slope, inv_dH, dt;
    double k;
    float kf, dtf;
    int32_t latent, pad;
};

// number of FP64 values in one per-workgroup diagnostics record
constexpr int NDIAG = 6;
enum { DG_E = 0, DG_LAT = 1, DG_TMIN = 2, DG_TMAX = 3, DG_NLIQ = 4, DG_NONFIN = 5 };

struct Dev {
    int prec = FEM_PREC_FP32_KAHAN;
    int nen = 4;
    int scatter = FEM_SCATTER_LDS_BLOCKED;
    int64_t N = 0, E = 0;
    // nodes
    void *node_x = nullptr;   // R4 per node: x, y, z (FP32: fixed-point integer bits), and k or the material
    float x_scale = 1.0f;     // FP32: metres per coordinate unit (a power of two)
    void *T = nullptr;        // R[2N] ping-pong temperatures
    void *H = nullptr;        // float2 (hi, lo) or double per node
    void *inv_m = nullptr;    // R per node
    void *fs = nullptr;       // R per node
    const MatDev *mats = nullptr;
    // elements
    const int32_t *conn = nullptr;      // global-atomic / coloured
    void *r = nullptr;                  // R[N] residual (global-atomic / coloured)
    // LDS-blocked local connectivity: 16-bit ids, NEN per element; or, with
    // conn12 (tets in blocks of at most 4096 nodes), two tets per three words
    // with 12-bit ids (see step::conn_load)
    const uint16_t *lconn = nullptr;
    int32_t conn12 = 0;
    // matched interface pairs as block elements: six local ids per pair (face a,
    // face b; BlockInfo::v_begin / n_v) and the coupling w (R) of each
    const uint16_t *vconn = nullptr;
    const void *vw = nullptr;
    const BlockInfo *blocks = nullptr;
    const int32_t *sh_list = nullptr;
    void *partials = nullptr;           // R per partial slot (see Layout::comb_ptr)
    const int32_t *node_win = nullptr;  // per node-kernel workgroup: first row of its material window, or -1
    const int32_t *comb_ptr = nullptr, *sh_pos = nullptr;
    const uint32_t *flags = nullptr;    // material | flag bits per node
    // boundary slots
    const void *robin = nullptr;        // R2 (a, b) per slot or null
    const int32_t *link_ptr = nullptr, *link_node = nullptr;
    const void *link_w = nullptr;       // R per link
    // diagnostics
    double *diag = nullptr;             // state diagnostics: NDIAG per node segment
    double *qnode = nullptr;            // per inflow slot: sum over steps of dt * boundary inflow
    int64_t n_inflow = 0;               // node-kernel slots 0..n_inflow-1 may carry boundary inflow
    const int32_t *seg_begin = nullptr; // single-scenario node segments
    int64_t n_seg = 0;
    int32_t n_mat = 0;
    // sizes and launch shape
    int64_t n_private = 0, n_blocks = 0, n_bc_slots = 0, bc_first = 0;
    int threads = 256;
    size_t lds_bytes = 0;
    int n_colors = 0;
    const int32_t *color_ptr_host = nullptr;
    double fx_scale = 1.0, fx_inv = 1.0; // FP32 blocked path: fixed-point scale 2^S and 2^-S
    float fx_limit = 0.0f;              // largest element contribution that fits (|r| * 2^S < 2^50)
    int64_t node_blocks = 0;            // workgroups of the node kernel
};

constexpr int NODE_THREADS = 256;
// rows of a material-table window staged in LDS by the step kernels
constexpr int MAT_WINDOW = 8;

inline int64_t node_grid(int64_t n) { return (n + NODE_THREADS - 1) / NODE_THREADS; }

// LDS bytes per local node of the blocked kernel
inline size_t lds_per_node(int prec) { return prec == FEM_PREC_FP64 ? 48 : 28; }
// dynamic LDS of the blocked kernel for blocks of at most max_local nodes (one
// spare node slot that the gather's tail lanes write)
inline size_t block_lds_bytes(int prec, int64_t max_local) { return (size_t)(max_local + 1) * lds_per_node(prec); }

// Enqueue one explicit step reading T buffer `parity` and writing 1 - parity.
// If ev is not null, ev[0..1] bracket the element kernel(s) and ev[2..3] the
// node kernel.
hipError_t enqueue_step(const Dev &d, int parity, hipStream_t s, hipEvent_t *ev);
// Reduce the state diagnostics of T buffer `parity` into d.diag.
hipError_t enqueue_state_diag(const Dev &d, int parity, hipStream_t s);
// Allow the blocked element kernel `bytes` of dynamic LDS.
hipError_t set_block_lds_limit(int prec, int nen, size_t bytes);
// Plain vector copy of n16 16-byte words.
hipError_t enqueue_copy(void *dst, const void *src, int64_t n16, hipStream_t s);
// The same with non-temporal loads and stores and up to 32,768 workgroups.
hipError_t enqueue_copy_nt(void *dst, const void *src, int64_t n16, hipStream_t s);

// Allocation-free stepping: bytes of the library's static device scratch (the
// partial residuals of fem_step_no_alloc), its address on `device` (which must
// be current; resolved once per device), a zero fill and a dt update of the
// material table by kernels (no copy, no allocation).
constexpr int64_t SCRATCH_BYTES = 32ll << 20;
hipError_t scratch_address(int device, void **out);
hipError_t enqueue_zero(void *p, int64_t bytes, hipStream_t s);
hipError_t enqueue_set_dt(MatDev *mats, int n, double dt, hipStream_t s);
// Copy check counts, diagnostics and inflow sums into page-locked host memory the device can write.
hipError_t enqueue_stage(int32_t *dst_chk, const int32_t *chk, int64_t n_chk, double *dst_dg, const double *dg,
                         int64_t n_dg, double *dst_qn, const double *qn, int64_t n_qn, hipStream_t s);

}  // namespace castfem
