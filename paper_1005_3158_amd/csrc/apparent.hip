// gfx950 kernels of the apparent-heat-capacity step (Eq. 6-7 of the paper),
// on the LDS-blocked layout of the enthalpy step.
//
// One step is two launches, as in the enthalpy form:
//   element phase: a workgroup gathers its block's nodes (coordinates,
//     temperature, material) into LDS; each element adds its conduction
//     residual -K^e T^e and its lumped capacitance rho C_app V / 4 to LDS
//     accumulators (64-bit fixed point for FP32, so the sums are bitwise
//     reproducible); private nodes are updated in place and each shared node
//     gets one residual and one capacitance partial;
//   node phase: per shared node the sums of both partials, the flux and
//     interface terms, and the update.
// The update T += dt r / C (Eq. 14 with the re-assembled C of Eq. 6) runs in
// FP64 from T(H) of the stored state, and the state stores H(T_new).
//
#include "apparent.hpp"

#include <hip/hip_ext.h>

#include <cfloat>
#include <type_traits>

#include "elem.hpp"
#include "step_common.hpp"

namespace castfem {
namespace {

using step::boundary_terms;
using step::fx_from;
using step::fx_to;
using step::h_of_t;
using step::LDS_MATS;
using step::stage_table;
using step::t_of_h;
using step::VT;
using step::xcd_remap;

// the constants one element needs, in the working precision (held in registers)
template <class R>
struct MatR {
    R k, rho, c, L, Ts, Tl, inv_dT;
};
__device__ __forceinline__ MatR<float> mat_r(const AppMat &m, float) {
    return {m.kf, m.rhof, m.cf, m.Lf, m.Tsf, m.Tlf, m.inv_dTf};
}
__device__ __forceinline__ MatR<double> mat_r(const AppMat &m, double) {
    return {m.k, m.rho, m.c, m.L, m.Ts, m.Tl, m.inv_dT};
}

// clamp to [0, 1] (one v_med3 in FP32)
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }

// sqrt(hh / g2) for g2 > 0: FP32 with the hardware square root and reciprocal
// square root (about 1 ulp each; the FP32 path rounds its inputs far more),
// FP64 correctly rounded
__device__ __forceinline__ float lemmon_ratio(float hh, float g2) {
    return __builtin_amdgcn_sqrtf(hh) * __builtin_amdgcn_rsqf(g2);
}
__device__ __forceinline__ double lemmon_ratio(double hh, double g2) { return sqrt(hh / g2); }

// Residual r = -K^e T^e and lumped capacitance share rho C_app V / 4 of a
// linear tetrahedron.  With edges d_j = x_j - x_0, c_1 = d_2 x d_3 (cyclic),
// D = d_1 . c_1 = 6 V: G = sum_j (T_j - T_0) c_j = D grad T and, with the liquid
// fraction f, G_f = D grad f; grad H = (c G + L G_f) / D, so C_app = |c G + L G_f| / |G|.
template <class R>
__device__ __forceinline__ void tet_app(const typename VT<R>::V4 *p, const MatR<R> M, R re[4], R &cap) {
    const V3<R> x0 = {p[0].x, p[0].y, p[0].z};
    const V3<R> d1 = sub3(V3<R>{p[1].x, p[1].y, p[1].z}, x0);
    const V3<R> d2 = sub3(V3<R>{p[2].x, p[2].y, p[2].z}, x0);
    const V3<R> d3 = sub3(V3<R>{p[3].x, p[3].y, p[3].z}, x0);
    const V3<R> c1 = cross3(d2, d3), c2 = cross3(d3, d1), c3 = cross3(d1, d2);
    const R D = dot3(d1, c1);
    const R a1 = p[1].w - p[0].w, a2 = p[2].w - p[0].w, a3 = p[3].w - p[0].w;
    const V3<R> G = {a1 * c1.x + a2 * c2.x + a3 * c3.x, a1 * c1.y + a2 * c2.y + a3 * c3.y,
                     a1 * c1.z + a2 * c2.z + a3 * c3.z};
    const R s = -M.k * recip(R(6) * D);
    re[1] = s * dot3(c1, G);
    re[2] = s * dot3(c2, G);
    re[3] = s * dot3(c3, G);
    re[0] = -(re[1] + re[2] + re[3]);
    // liquid fraction; inv_dT = 0 (no latent heat) gives f = 0 everywhere
    const R ts = M.Ts, idt = M.inv_dT;
    auto frac = [&](R T) { return clamp01((T - ts) * idt); };
    const R f0 = frac(p[0].w);
    const R b1 = frac(p[1].w) - f0, b2 = frac(p[2].w) - f0, b3 = frac(p[3].w) - f0;
    const R c = M.c, L = M.L;
    const V3<R> GH = {c * G.x + L * (b1 * c1.x + b2 * c2.x + b3 * c3.x),
                      c * G.y + L * (b1 * c1.y + b2 * c2.y + b3 * c3.y),
                      c * G.z + L * (b1 * c1.z + b2 * c2.z + b3 * c3.z)};
    const R g2 = dot3(G, G);
    R capp;
    if (g2 > R(0)) {
        capp = lemmon_ratio(dot3(GH, GH), g2);
    } else {
        // uniform element: the slope of H(T) at its temperature
        const R tm = (((p[0].w + p[1].w) + p[2].w) + p[3].w) * R(0.25);
        capp = (idt > R(0) && tm > ts && tm < M.Tl) ? c + L * idt : c;
    }
    cap = M.rho * capp * (D * R(1.0 / 24.0));
}

// T += dt r / C in FP64 from T(H) of the stored state; the state keeps H(T_new)
template <class R> struct NodeApp;
template <> struct NodeApp<float> {
    static __device__ __forceinline__ void update(const Dev &d, const MatDev *mats, int64_t g, float r, float C,
                                                  uint32_t flag, float *Tn) {
        const MatDev &M = mats[flag & NODE_MAT_MASK];
        float2 *H = (float2 *)d.H;
        const float2 h = H[g];
        double T, fs;
        t_of_h(M, (double)h.x + (double)h.y, T, fs);
        const double Hn = h_of_t(M, T + M.dt * (double)r / (double)C);
        const float hi = (float)Hn;
        const float lo = (float)(Hn - (double)hi);
        H[g] = make_float2(hi, lo);
        t_of_h(M, (double)hi + (double)lo, T, fs);
        Tn[g] = (float)T;
        ((float *)d.fs)[g] = (float)fs;
    }
};
template <> struct NodeApp<double> {
    static __device__ __forceinline__ void update(const Dev &d, const MatDev *mats, int64_t g, double r, double C,
                                                  uint32_t flag, double *Tn) {
        const MatDev &M = mats[flag & NODE_MAT_MASK];
        double *H = (double *)d.H;
        double T, fs;
        t_of_h(M, H[g], T, fs);
        const double Hn = h_of_t(M, T + M.dt * r / C);
        H[g] = Hn;
        t_of_h(M, Hn, T, fs);
        Tn[g] = T;
        ((double *)d.fs)[g] = fs;
    }
};

// Element loop of one block: residual and capacitance of every element added to
// the LDS accumulators of its nodes.  UNIFORM: every element has material M;
// otherwise each element takes the material of its first node.  Returns true
// if a contribution fell outside the fixed-point range (or was not finite).
template <class R, bool UNIFORM, class ACC, class CACC>
__device__ __forceinline__ bool block_elements(const AppDev &a, const BlockInfo &bi, const typename VT<R>::V4 *s_x,
                                               ACC *s_acc, CACC *s_cap, const int32_t *s_mat, const AppMat *amats,
                                               const MatR<R> M) {
    using V4 = typename VT<R>::V4;
    const Dev &d = a.d;
    bool bad = false;
    step::ConnRaw<4> cur{};
    if ((int)threadIdx.x < bi.n_e) cur = step::conn_load<4>(d, (int64_t)bi.e_begin + threadIdx.x);
    for (int e = threadIdx.x; e < bi.n_e; e += blockDim.x) {
        step::ConnRaw<4> nxt{};
        if (e + (int)blockDim.x < bi.n_e) nxt = step::conn_load<4>(d, (int64_t)bi.e_begin + e + blockDim.x);
        int l[4];
        step::conn_ids<4>(cur, l);
        const int l0 = l[0], l1 = l[1], l2 = l[2], l3 = l[3];
        V4 p[4] = {s_x[l0], s_x[l1], s_x[l2], s_x[l3]};
        step::local_coords<4>(p, d.x_scale);
        R re[4], cap;
        tet_app<R>(p, UNIFORM ? M : mat_r(amats[s_mat[l0]], R(0)), re, cap);
        if constexpr (std::is_same<R, float>::value) {
            bad |= !(fabsf(re[1]) < d.fx_limit) || !(fabsf(re[2]) < d.fx_limit) || !(fabsf(re[3]) < d.fx_limit);
            bad |= !(cap < a.cx_limit);   // also catches NaN
            const long long q1 = fx_from(re[1], d.fx_scale), q2 = fx_from(re[2], d.fx_scale),
                            q3 = fx_from(re[3], d.fx_scale);
            const long long q0 = -(q1 + q2 + q3);
            // capacitances are positive and their node sums stay below 2^31: 32-bit sums
            const uint32_t qc = (uint32_t)fx_from(cap, a.cx_scale);
            atomicAdd((unsigned long long *)&s_acc[l0], (unsigned long long)q0);
            atomicAdd((unsigned long long *)&s_acc[l1], (unsigned long long)q1);
            atomicAdd((unsigned long long *)&s_acc[l2], (unsigned long long)q2);
            atomicAdd((unsigned long long *)&s_acc[l3], (unsigned long long)q3);
            atomicAdd(&s_cap[l0], qc);
            atomicAdd(&s_cap[l1], qc);
            atomicAdd(&s_cap[l2], qc);
            atomicAdd(&s_cap[l3], qc);
        } else {
            atomicAdd(&s_acc[l0], re[0]);
            atomicAdd(&s_acc[l1], re[1]);
            atomicAdd(&s_acc[l2], re[2]);
            atomicAdd(&s_acc[l3], re[3]);
            atomicAdd(&s_cap[l0], cap);
            atomicAdd(&s_cap[l1], cap);
            atomicAdd(&s_cap[l2], cap);
            atomicAdd(&s_cap[l3], cap);
        }
        cur = nxt;
    }
    return bad;
}

// element phase, one workgroup per element block (linear tetrahedra)
template <class R, bool LDS_TABLES>
__global__ __launch_bounds__(1024) void k_block_app(AppDev a, int parity) {
    using V4 = typename VT<R>::V4;
    using ACC = typename std::conditional<std::is_same<R, float>::value, long long, double>::type;
    // FP32: 32-bit fixed-point capacitance sums; FP64: double
    using CACC = typename std::conditional<std::is_same<R, float>::value, uint32_t, double>::type;
    const Dev &d = a.d;
    extern __shared__ __attribute__((aligned(32))) unsigned char smem[];
    __shared__ MatDev s_mats[LDS_MATS];
    __shared__ AppMat s_amats[LDS_MATS];
    __shared__ int s_bad;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const BlockInfo bi = d.blocks[b];
    const int nloc = bi.n_int + bi.n_sh;
    V4 *s_x = (V4 *)smem;                        // x, y, z, T per local node
    ACC *s_acc = (ACC *)(s_x + nloc);            // residual
    CACC *s_cap = (CACC *)(s_acc + nloc);        // lumped capacitance
    int32_t *s_mat = (int32_t *)(s_cap + nloc);  // material index
    const V4 *X = (const V4 *)d.node_x;
    const R *Tc = (const R *)d.T + parity * d.N;
    R *Tn = (R *)d.T + (1 - parity) * d.N;
    if (threadIdx.x == 0) s_bad = 0;
    if constexpr (LDS_TABLES) {
        stage_table(d.mats, d.n_mat, s_mats);
        stage_table(a.amats, d.n_mat, s_amats);
    }
    const MatDev *mats = LDS_TABLES ? s_mats : d.mats;
    const AppMat *amats = LDS_TABLES ? s_amats : a.amats;

    for (int l = threadIdx.x; l < nloc; l += blockDim.x) {
        const int64_t g = l < bi.n_int ? (int64_t)bi.int_base + l : (int64_t)d.sh_list[bi.sh_begin + (l - bi.n_int)];
        V4 x = X[g];
        s_mat[l] = (int32_t)x.w;
        x.w = Tc[g];
        s_x[l] = x;
        s_acc[l] = ACC(0);
        s_cap[l] = CACC(0);
    }
    __syncthreads();

    bool bad;
    if (bi.pad0 >= 0)   // one material in the whole block: its constants are read once
        bad = block_elements<R, true>(a, bi, s_x, s_acc, s_cap, s_mat, amats, mat_r(amats[bi.pad0], R(0)));
    else
        bad = block_elements<R, false>(a, bi, s_x, s_acc, s_cap, s_mat, amats, MatR<R>{});
    if (bad) s_bad = 1;
    __syncthreads();

    const bool poison = s_bad != 0;
    auto resid = [&](int l) -> R {
        R r;
        if constexpr (std::is_same<R, float>::value) r = fx_to(s_acc[l], d.fx_inv);
        else r = s_acc[l];
        return poison ? R(NAN) : r;
    };
    auto capv = [&](int l) -> R {
        if constexpr (std::is_same<R, float>::value) return (float)((double)s_cap[l] * a.cx_inv);
        else return s_cap[l];
    };
    for (int l = threadIdx.x; l < bi.n_int; l += blockDim.x) {
        const int64_t g = (int64_t)bi.int_base + l;
        NodeApp<R>::update(d, mats, g, resid(l), capv(l), d.flags[g], Tn);
    }
    R *P = (R *)d.partials;
    R *Pc = (R *)a.cap_partials;
    for (int l = threadIdx.x; l < bi.n_sh; l += blockDim.x) {
        const int32_t pos = d.sh_pos[bi.sh_begin + l];
        P[pos] = resid(bi.n_int + l);
        Pc[pos] = capv(bi.n_int + l);
    }
}

// node phase over the shared nodes: partial sums in block order, boundary terms, update
template <class R, bool LDS_TABLES>
__global__ __launch_bounds__(NODE_THREADS) void k_nodes_app(AppDev a, int parity) {
    const Dev &d = a.d;
    __shared__ MatDev s_mats[LDS_MATS];
    const int64_t count = d.N - d.n_private;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (LDS_TABLES) {
        stage_table(d.mats, d.n_mat, s_mats);
        __syncthreads();
    }
    const MatDev *mats = LDS_TABLES ? s_mats : d.mats;
    if (s >= count) return;
    const int64_t g = d.bc_first + s;
    const R *Tc = (const R *)d.T + parity * d.N;
    R *Tn = (R *)d.T + (1 - parity) * d.N;
    const uint32_t f = d.flags[g];
    const R *P = (const R *)d.partials;
    const R *Pc = (const R *)a.cap_partials;
    R r = step::combine_partials(d, P, s, f);
    R C = step::combine_partials(d, Pc, s, f);
    double q = 0.0;
    if (f & NODE_BC) q = boundary_terms<R>(d, s, Tc[g], Tc, r);
    if (f & NODE_FIXED) q -= (double)r;     // reaction of a fixed temperature
    else NodeApp<R>::update(d, mats, g, r, C, f, Tn);
    if (s < d.n_inflow) d.qnode[s] += q * mats[f & NODE_MAT_MASK].dt;
}

template <class R, bool LDS_TABLES>
hipError_t step_t(const AppDev &a, int parity, hipStream_t s, hipEvent_t *ev) {
    const Dev &d = a.d;
    // timed launches (eager) carry their own start and stop events
    const dim3 gb((unsigned)d.n_blocks), bb(d.threads);
    if (ev) hipExtLaunchKernelGGL((k_block_app<R, LDS_TABLES>), gb, bb, (uint32_t)d.lds_bytes, s, ev[0], ev[1], 0u, a, parity);
    else hipLaunchKernelGGL((k_block_app<R, LDS_TABLES>), gb, bb, d.lds_bytes, s, a, parity);
    const int64_t count = d.N - d.n_private;
    if (count > 0) {
        const dim3 g((unsigned)node_grid(count)), b(NODE_THREADS);
        if (ev) hipExtLaunchKernelGGL((k_nodes_app<R, LDS_TABLES>), g, b, 0u, s, ev[2], ev[3], 0u, a, parity);
        else hipLaunchKernelGGL((k_nodes_app<R, LDS_TABLES>), g, b, 0, s, a, parity);
    } else if (ev) {
        (void)hipEventRecord(ev[2], s);
        (void)hipEventRecord(ev[3], s);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t enqueue_step_apparent(const AppDev &a, int parity, hipStream_t s, hipEvent_t *ev) {
    const bool lds = a.d.n_mat <= LDS_MATS;
    if (a.d.prec == FEM_PREC_FP64) return lds ? step_t<double, true>(a, parity, s, ev) : step_t<double, false>(a, parity, s, ev);
    return lds ? step_t<float, true>(a, parity, s, ev) : step_t<float, false>(a, parity, s, ev);
}

hipError_t set_apparent_lds_limit(int prec, size_t bytes) {
    const void *f[2];
    if (prec == FEM_PREC_FP64) {
        f[0] = (const void *)k_block_app<double, true>;
        f[1] = (const void *)k_block_app<double, false>;
    } else {
        f[0] = (const void *)k_block_app<float, true>;
        f[1] = (const void *)k_block_app<float, false>;
    }
    for (const void *k : f) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace castfem
