// gfx950 kernels of the enthalpy step with temperature- and time-dependent
// properties, on the LDS-blocked layout.
//
//   element phase (k_block_var): as the enthalpy element kernel, with each
//     element's conductivity read from its material's k(T) table at the mean of
//     its nodal T^n;
//   node phase (k_nodes_var): per shared node the sum of partials, Robin terms,
//     interface links whose coefficient is scaled by h_T((T_i + T_j) / 2) and
//     h_t(t), the update; a fixed node takes T_D + shift(t + dt), and the change of
//     its enthalpy counts as boundary inflow.  The time of each T buffer lives in
//     device memory (two slots, one per parity, per scenario of a batch, each
//     advancing by its scenario's dt), so captured graphs of steps advance it
//     without host involvement.
#include "varprops.hpp"

#include <hip/hip_ext.h>

#include <type_traits>

#include "elem.hpp"
#include "step_common.hpp"

namespace castfem {
namespace {

using step::fx_from;
using step::fx_to;
using step::h_of_t;
using step::LDS_MATS;
using step::NodeH;
using step::stage_table;
using step::t_of_h;
using step::VT;
using step::xcd_remap;

__device__ __forceinline__ float mat_k(const MatDev &m, float) { return m.kf; }
__device__ __forceinline__ double mat_k(const MatDev &m, double) { return m.k; }

__device__ __forceinline__ const Tab<float> *tabs(const VarDev &v, float) { return v.tabs_f; }
__device__ __forceinline__ const Tab<double> *tabs(const VarDev &v, double) { return v.tabs_d; }

// linear between points, constant beyond the ends (n >= 1)
template <class R>
__device__ __forceinline__ R tab_eval(const Tab<R> &t, R x) {
    const int n = t.n;
    if (x <= t.x[0]) return t.y[0];
    if (x >= t.x[n - 1]) return t.y[n - 1];
    int j = 0;
    while (j + 2 < n && !(x < t.x[j + 1])) ++j;
    return t.y[j] + (t.y[j + 1] - t.y[j]) * (x - t.x[j]) / (t.x[j + 1] - t.x[j]);
}

// the scheduled temperature of shared slot s at time x: its row of values over
// the common times, linear in between, constant beyond the ends (as tab_eval)
__device__ __forceinline__ double sched_value(const VarDev &v, int64_t s, double x) {
    const int n = v.n_sched;
    const double *y = v.sched + s * n;
    if (x <= v.sched_t[0]) return y[0];
    if (x >= v.sched_t[n - 1]) return y[n - 1];
    int j = 0;
    while (j + 2 < n && !(x < v.sched_t[j + 1])) ++j;
    return y[j] + (y[j + 1] - y[j]) * (x - v.sched_t[j]) / (v.sched_t[j + 1] - v.sched_t[j]);
}

template <class R, int NEN>
__device__ __forceinline__ void elem_residual(const typename VT<R>::V4 *p, R k, R *r) {
    if constexpr (NEN == 4) {
        tet_residual<R>({p[0].x, p[0].y, p[0].z}, {p[1].x, p[1].y, p[1].z}, {p[2].x, p[2].y, p[2].z},
                        {p[3].x, p[3].y, p[3].z}, p[0].w, p[1].w, p[2].w, p[3].w, k, r[0], r[1], r[2], r[3]);
    } else {
        V3<R> x[8];
        R t[8];
        for (int a = 0; a < 8; ++a) {
            x[a] = {p[a].x, p[a].y, p[a].z};
            t[a] = p[a].w;
        }
        hex_residual<R>(x, t, k, r);
    }
}

// element phase, one workgroup per element block
template <class R, int NEN, bool LDS_TABLES>
__global__ __launch_bounds__(1024) void k_block_var(VarDev v, int parity) {
    using V4 = typename VT<R>::V4;
    using ACC = typename std::conditional<std::is_same<R, float>::value, long long, double>::type;
    const Dev &d = v.d;
    extern __shared__ __attribute__((aligned(32))) unsigned char smem[];
    __shared__ MatDev s_mats[LDS_MATS];
    __shared__ Tab<R> s_tabs[LDS_MATS];
    __shared__ int s_bad;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const BlockInfo bi = d.blocks[b];
    const int nloc = bi.n_int + bi.n_sh;
    V4 *s_x = (V4 *)smem;                        // x, y, z, T per local node
    ACC *s_acc = (ACC *)(s_x + nloc);            // residual accumulator
    int32_t *s_mat = (int32_t *)(s_acc + nloc);  // material index
    const V4 *X = (const V4 *)d.node_x;
    const R *Tc = (const R *)d.T + parity * d.N;
    R *Tn = (R *)d.T + (1 - parity) * d.N;
    if (threadIdx.x == 0) s_bad = 0;
    if constexpr (LDS_TABLES) {
        stage_table(d.mats, d.n_mat, s_mats);
        stage_table(tabs(v, R(0)), d.n_mat, s_tabs);
    }
    const MatDev *mats = LDS_TABLES ? s_mats : d.mats;
    const Tab<R> *ktab = LDS_TABLES ? s_tabs : tabs(v, R(0));

    for (int l = threadIdx.x; l < nloc; l += blockDim.x) {
        const int64_t g = l < bi.n_int ? (int64_t)bi.int_base + l : (int64_t)d.sh_list[bi.sh_begin + (l - bi.n_int)];
        const V4 x = X[g];
        s_mat[l] = (int32_t)x.w;
        s_x[l] = V4{x.x, x.y, x.z, Tc[g]};
        s_acc[l] = ACC(0);
    }
    __syncthreads();

    step::ConnRaw<NEN> cur{};
    if ((int)threadIdx.x < bi.n_e) cur = step::conn_load<NEN>(d, (int64_t)bi.e_begin + threadIdx.x);
    bool bad = false;
    for (int e = threadIdx.x; e < bi.n_e; e += blockDim.x) {
        step::ConnRaw<NEN> nxt{};
        if (e + (int)blockDim.x < bi.n_e) nxt = step::conn_load<NEN>(d, (int64_t)bi.e_begin + e + blockDim.x);
        int l[NEN];
        step::conn_ids<NEN>(cur, l);
        V4 p[NEN];
        for (int a = 0; a < NEN; ++a) p[a] = s_x[l[a]];
        // conductivity at the element's mean temperature
        const int m = s_mat[l[0]];
        R k = mat_k(mats[m], R(0));
        if (tab_given(ktab[m].n)) {
            R tsum = p[0].w;
            for (int a = 1; a < NEN; ++a) tsum += p[a].w;
            k = tab_eval(ktab[m], tsum * R(1.0 / NEN));
        }
        R re[NEN];
        step::local_units<NEN>(p);
        elem_residual<R, NEN>(p, k * d.x_scale, re);   // k per unit length of the element coordinates
        if constexpr (std::is_same<R, float>::value) {
            long long q[NEN];
            long long sum = 0;
            for (int a = 1; a < NEN; ++a) {
                bad |= !(fabsf(re[a]) < d.fx_limit);   // also catches NaN
                q[a] = fx_from(re[a], d.fx_scale);
                sum += q[a];
            }
            q[0] = -sum;
            for (int a = 0; a < NEN; ++a) atomicAdd((unsigned long long *)&s_acc[l[a]], (unsigned long long)q[a]);
        } else {
            for (int a = 0; a < NEN; ++a) atomicAdd(&s_acc[l[a]], re[a]);
        }
        cur = nxt;
    }
    if (bad) s_bad = 1;
    __syncthreads();

    const bool poison = s_bad != 0;
    auto resid = [&](int l) -> R {
        R r;
        if constexpr (std::is_same<R, float>::value) r = fx_to(s_acc[l], d.fx_inv);
        else r = s_acc[l];
        return poison ? R(NAN) : r;
    };
    // private nodes are free and have no boundary terms
    for (int l = threadIdx.x; l < bi.n_int; l += blockDim.x) {
        const int64_t g = (int64_t)bi.int_base + l;
        NodeH<R>::update(d, mats[d.flags[g] & NODE_MAT_MASK], g, resid(l), Tn);
    }
    R *P = (R *)d.partials;
    for (int l = threadIdx.x; l < bi.n_sh; l += blockDim.x) P[d.sh_pos[bi.sh_begin + l]] = resid(bi.n_int + l);
}

// node phase over the shared nodes
template <class R, bool LDS_TABLES>
__global__ __launch_bounds__(NODE_THREADS) void k_nodes_var(VarDev v, int parity) {
    using V2 = typename VT<R>::V2;
    const Dev &d = v.d;
    __shared__ MatDev s_mats[LDS_MATS];
    const int64_t count = d.N - d.n_private;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (LDS_TABLES) {
        stage_table(d.mats, d.n_mat, s_mats);
        __syncthreads();
    }
    const MatDev *mats = LDS_TABLES ? s_mats : d.mats;
    const int ns = v.n_scen;
    // thread s < n_scen advances the time of scenario s (by its own dt) in the
    // slot of the state this step writes
    if (s < ns) v.time[(1 - parity) * ns + s] = v.time[parity * ns + s] + d.mats[v.scen_mat[s]].dt;
    if (s >= count) return;
    const Tab<R> *gt = tabs(v, R(0)) + d.n_mat;
    const Tab<double> *gd = v.tabs_d + d.n_mat;
    const int64_t g = d.bc_first + s;
    const R *Tc = (const R *)d.T + parity * d.N;
    R *Tn = (R *)d.T + (1 - parity) * d.N;
    const uint32_t f = d.flags[g];
    const MatDev &M = mats[f & NODE_MAT_MASK];
    const double t = v.time[parity * ns + (ns > 1 ? v.mat_scen[f & NODE_MAT_MASK] : 0)];
    const double dt = M.dt;         // the node's scenario's step
    const R *P = (const R *)d.partials;
    R r = step::combine_partials(d, P, s, f);
    double q = 0.0;
    if (f & NODE_BC) {
        const R Ti = Tc[g];
        if (d.robin) {
            const V2 ab = ((const V2 *)d.robin)[s];
            const R fr = ab.x - ab.y * Ti;
            r += fr;
            q = (double)fr;
        }
        const R ft = tab_given(gt[TAB_H_OF_TIME].n) ? tab_eval(gt[TAB_H_OF_TIME], R(t)) : R(1);
        const bool by_T = tab_given(gt[TAB_H_OF_T].n);
        const int32_t l0 = d.link_ptr[s], l1 = d.link_ptr[s + 1];
        const R *w = (const R *)d.link_w;
        for (int32_t k = l0; k < l1; ++k) {
            const R Tj = Tc[d.link_node[k]];
            R fk = ft;
            if (by_T) fk = tab_eval(gt[TAB_H_OF_T], (Ti + Tj) / R(2)) * ft;
            r += w[k] * fk * (Tj - Ti);
        }
    }
    double qfix = 0.0;
    if (f & NODE_FIXED) {
        q -= (double)r;   // reaction of a fixed temperature
        const bool shifted = tab_given(gd[TAB_DIR_OF_TIME].n);
        if (shifted || v.n_sched) {
            // the prescribed temperature of the next state; its enthalpy change is inflow
            const double tn = t + dt;
            const double Tnew = (v.n_sched ? sched_value(v, s, tn) : v.T_fixed[g]) +
                                (shifted ? tab_eval(gd[TAB_DIR_OF_TIME], tn) : 0.0);
            const double Hn = h_of_t(M, Tnew);
            double Hold, Tchk, fs;
            if constexpr (std::is_same<R, float>::value) {
                const float2 h = ((const float2 *)d.H)[g];
                Hold = (double)h.x + (double)h.y;
                const float hi = (float)Hn;
                ((float2 *)d.H)[g] = make_float2(hi, (float)(Hn - (double)hi));
            } else {
                Hold = ((const double *)d.H)[g];
                ((double *)d.H)[g] = Hn;
            }
            t_of_h(M, Hn, Tchk, fs);
            Tn[g] = (R)Tnew;
            ((R *)d.fs)[g] = (R)fs;
            qfix = (Hn - Hold) / (double)((const R *)d.inv_m)[g];
        }
    } else {
        NodeH<R>::update(d, M, g, r, Tn);
    }
    if (s < d.n_inflow) d.qnode[s] += q * M.dt + qfix;
}

template <class R, int NEN, bool LDS_TABLES>
hipError_t step_t(const VarDev &v, int parity, hipStream_t s, hipEvent_t *ev) {
    const Dev &d = v.d;
    // timed launches (eager) carry their own start and stop events
    const dim3 gb((unsigned)d.n_blocks), bb(d.threads);
    if (ev) hipExtLaunchKernelGGL((k_block_var<R, NEN, LDS_TABLES>), gb, bb, (uint32_t)d.lds_bytes, s, ev[0], ev[1], 0u, v, parity);
    else hipLaunchKernelGGL((k_block_var<R, NEN, LDS_TABLES>), gb, bb, d.lds_bytes, s, v, parity);
    // launched even without shared nodes: its first n_scen threads advance the time
    const int64_t count = d.N - d.n_private;
    const dim3 g((unsigned)node_grid(std::max<int64_t>(count, v.n_scen))), b(NODE_THREADS);
    if (ev) hipExtLaunchKernelGGL((k_nodes_var<R, LDS_TABLES>), g, b, 0u, s, ev[2], ev[3], 0u, v, parity);
    else hipLaunchKernelGGL((k_nodes_var<R, LDS_TABLES>), g, b, 0, s, v, parity);
    return hipGetLastError();
}

template <class R, int NEN>
hipError_t step_nen(const VarDev &v, int parity, hipStream_t s, hipEvent_t *ev) {
    return v.d.n_mat <= LDS_MATS ? step_t<R, NEN, true>(v, parity, s, ev) : step_t<R, NEN, false>(v, parity, s, ev);
}

template <class R>
hipError_t set_limit(int nen, size_t bytes) {
    const void *f[2];
    if (nen == 4) {
        f[0] = (const void *)k_block_var<R, 4, true>;
        f[1] = (const void *)k_block_var<R, 4, false>;
    } else {
        f[0] = (const void *)k_block_var<R, 8, true>;
        f[1] = (const void *)k_block_var<R, 8, false>;
    }
    for (const void *k : f) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t enqueue_step_var(const VarDev &v, int parity, hipStream_t s, hipEvent_t *ev) {
    if (v.d.prec == FEM_PREC_FP64)
        return v.d.nen == 4 ? step_nen<double, 4>(v, parity, s, ev) : step_nen<double, 8>(v, parity, s, ev);
    return v.d.nen == 4 ? step_nen<float, 4>(v, parity, s, ev) : step_nen<float, 8>(v, parity, s, ev);
}

hipError_t set_var_lds_limit(int prec, int nen, size_t bytes) {
    return prec == FEM_PREC_FP64 ? set_limit<double>(nen, bytes) : set_limit<float>(nen, bytes);
}

}  // namespace castfem
