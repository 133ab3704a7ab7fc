// gfx950 kernels of the explicit casting step.
//
// One step is two launches:
//   element phase: the conduction residual r = -K T assembled element by
//     element (Eq. 15-18 of the paper).  Three ways to scatter it:
//       - LDS-blocked: a workgroup takes one element block (the cache block of
//         Sec. 4.2 with the private/shared node classes of Sec. 4.1), gathers
//         the block's node coordinates and temperatures into LDS, accumulates
//         the residual with LDS atomics, updates its private nodes in place and
//         writes one partial per shared node (the Eq. 19-22 exchange, on chip);
//       - global atomics into r[N];
//       - colour by colour with plain read-modify-write (no two elements of a
//         colour share a node).
//   node phase: per node (or per shared node in the blocked layout) the sum of
//     partials, the flux and interface terms (Eq. 4, Eq. 8, sister-face mean),
//     and the enthalpy update H += dt r / m (Eq. 14 in enthalpy form) with
//     T = T(H), fs = fs(H) (Eq. 11) in FP64; FP64 wavefront reductions of the
//     energy balance.
// FP32 state keeps the enthalpy as an FP32 (hi, lo) pair updated by an
// error-free two-sum; T(H) is evaluated in FP64 from hi + lo.
#include "kernels.hpp"

#include <hip/hip_ext.h>

#include <cfloat>
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "elem.hpp"
#include "step_common.hpp"

namespace castfem {
namespace {

using step::boundary_terms;
using step::fx_from;
using step::fx_to;
using step::LDS_MATS;
using step::NodeH;
using step::stage_table;
using step::t_of_h;
using step::VT;
using step::xcd_remap;

struct DiagAcc {
    double v[NDIAG];
    __device__ void init() {
        for (int k = 0; k < NDIAG; ++k) v[k] = 0.0;
        v[DG_TMIN] = DBL_MAX;
        v[DG_TMAX] = -DBL_MAX;
    }
};

// sum / min / max over the 64 lanes of a wavefront
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// workgroup reduction of the state diagnostics into d.diag[slot]
__device__ void reduce_diag(const Dev &d, DiagAcc &acc, int64_t slot) {
    __shared__ double part[16][NDIAG];
    for (int k = 0; k < NDIAG; ++k)
        acc.v[k] = k == DG_TMIN ? wave_min(acc.v[k]) : (k == DG_TMAX ? wave_max(acc.v[k]) : wave_sum(acc.v[k]));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int k = 0; k < NDIAG; ++k) part[wave][k] = acc.v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double out[NDIAG];
        for (int k = 0; k < NDIAG; ++k) out[k] = part[0][k];
        for (int w = 1; w < nw; ++w)
            for (int k = 0; k < NDIAG; ++k) {
                if (k == DG_TMIN) out[k] = fmin(out[k], part[w][k]);
                else if (k == DG_TMAX) out[k] = fmax(out[k], part[w][k]);
                else out[k] += part[w][k];
            }
        for (int k = 0; k < NDIAG; ++k) d.diag[slot * NDIAG + k] = out[k];
    }
}

// ------------------------------------------------------------ element math
template <class R, int NEN> struct Elem;

template <class R> struct Elem<R, 4> {
    using V4 = typename VT<R>::V4;
    static __device__ __forceinline__ void residual(const V4 *p, R k, R *r) {
        tet_residual<R>({p[0].x, p[0].y, p[0].z}, {p[1].x, p[1].y, p[1].z}, {p[2].x, p[2].y, p[2].z},
                        {p[3].x, p[3].y, p[3].z}, p[0].w, p[1].w, p[2].w, p[3].w, k, r[0], r[1], r[2], r[3]);
    }
};

template <class R> struct Elem<R, 8> {
    using V4 = typename VT<R>::V4;
    static __device__ __forceinline__ void residual(const V4 *p, R k, R *r) {
        V3<R> x[8];
        R t[8];
        for (int a = 0; a < 8; ++a) {
            x[a] = {p[a].x, p[a].y, p[a].z};
            t[a] = p[a].w;
        }
        hex_residual<R>(x, t, k, r);
    }
};

// ------------------------------------------------------------ kernels
// element phase, one thread per element, scatter into r[N] by global atomics
// (ATOMIC) or by plain read-modify-write within one colour
template <class R, int NEN, bool ATOMIC>
__global__ __launch_bounds__(256) void k_elems(Dev d, int parity, int64_t e0, int64_t e1) {
    using V4 = typename VT<R>::V4;
    const int64_t e = e0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= e1) return;
    const V4 *X = (const V4 *)d.node_x;
    const R *Tc = (const R *)d.T + parity * d.N;
    R *r = (R *)d.r;
    int32_t c[NEN];
    V4 p[NEN];
    for (int a = 0; a < NEN; ++a) c[a] = d.conn[e * NEN + a];
    for (int a = 0; a < NEN; ++a) p[a] = X[c[a]];
    const R k = p[0].w * d.x_scale;     // conductivity of the element's material, per unit length
    for (int a = 0; a < NEN; ++a) p[a].w = Tc[c[a]];
    step::local_units<NEN>(p);
    R re[NEN];
    Elem<R, NEN>::residual(p, k, re);
    for (int a = 0; a < NEN; ++a) {
        if (ATOMIC) atomicAdd(&r[c[a]], re[a]);
        else r[c[a]] += re[a];
    }
}

// Fixed-point residual accumulation (FP32 state).  LDS floating-point atomic
// adds are slow on gfx950 while 64-bit integer adds run at close to full LDS
// rate, so each element contribution r is rounded to the integer q = r * 2^S
// (|q| < 2^51, scale chosen on the host from a bound on every node's element
// sums) and added with an integer atomic (step::fx_from).  Integer sums do not
// depend on the order of the additions, so the blocked path is bitwise
// reproducible, and the four contributions of an element sum to exactly zero.

// nodes per thread and pass of the gather and of the private-node update
constexpr int GATHER_U = 4;
constexpr int UPDATE_U = 2;

// element phase of the blocked layout, one workgroup per element block
template <class R, int NEN, bool LDS_TABLES>
__global__ __launch_bounds__(1024) void k_block(Dev d, int parity) {
    using V4 = typename VT<R>::V4;
    // FP32: 64-bit fixed-point accumulators; FP64: double accumulators
    using ACC = typename std::conditional<std::is_same<R, float>::value, long long, double>::type;
    extern __shared__ __attribute__((aligned(32))) unsigned char smem[];
    __shared__ MatDev s_mats[LDS_MATS];
    __shared__ int s_bad;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const BlockInfo bi = d.blocks[b];
    const int nloc = bi.n_int + bi.n_sh;
    // nloc + 1 slots each: slot nloc is the gather's spare
    V4 *s_x = (V4 *)smem;                       // x, y, z, T per local node
    ACC *s_acc = (ACC *)(s_x + nloc + 1);       // residual accumulator
    R *s_k = (R *)(s_acc + nloc + 1);           // conductivity of the node's material
    const V4 *X = (const V4 *)d.node_x;
    const R *Tc = (const R *)d.T + parity * d.N;
    R *Tn = (R *)d.T + (1 - parity) * d.N;
    if (threadIdx.x == 0) s_bad = 0;
    // material rows in LDS (visible after the next barrier): the whole table when
    // it has at most LDS_MATS rows, else the block's window of rows (a block of a
    // batch holds the few materials of one scenario; bi.pad1 < 0: no window)
    if constexpr (LDS_TABLES) stage_table(d.mats, d.n_mat, s_mats);
    else if (bi.pad1 >= 0) stage_table(d.mats + bi.pad1, min(LDS_MATS, d.n_mat - bi.pad1), s_mats);

    // gather: private nodes are a contiguous range, shared nodes a list;
    // node_x holds x, y, z and the conductivity of the node's material.
    // GATHER_U nodes per thread and pass, with no condition inside a pass, so
    // that their loads are in flight together: first the shared-node indices,
    // then every coordinate and temperature.  Lanes past the block load valid
    // entries (the shared list ends with one padding entry) and write the spare
    // LDS slot nloc, which nothing reads.
    const int32_t *shl = d.sh_list + bi.sh_begin;
    for (int l0 = threadIdx.x; l0 < nloc; l0 += GATHER_U * blockDim.x) {
        int32_t sv[GATHER_U];
#pragma unroll
        for (int u = 0; u < GATHER_U; ++u) sv[u] = shl[min(max(l0 + u * (int)blockDim.x - bi.n_int, 0), bi.n_sh)];
        V4 x[GATHER_U];
        R t[GATHER_U];
#pragma unroll
        for (int u = 0; u < GATHER_U; ++u) {
            const int l = l0 + u * (int)blockDim.x;
            const int64_t g = l < bi.n_int ? (int64_t)bi.int_base + l : (int64_t)sv[u];
            x[u] = X[g];
            t[u] = Tc[g];
        }
#pragma unroll
        for (int u = 0; u < GATHER_U; ++u) {
            const int w = min(l0 + u * (int)blockDim.x, nloc);
            s_k[w] = x[u].w;
            V4 v;
            v.x = x[u].x;
            v.y = x[u].y;
            v.z = x[u].z;
            v.w = t[u];
            s_x[w] = v;
            s_acc[w] = ACC(0);
        }
    }
    __syncthreads();

    // element residuals accumulated in LDS; the next element's connectivity
    // is loaded one iteration ahead
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
        const R k = s_k[l[0]] * d.x_scale;   // per unit length of the element coordinates
        step::local_units<NEN>(p);
        R re[NEN];
        Elem<R, NEN>::residual(p, k, re);
        if constexpr (std::is_same<R, float>::value) {
            long long q[NEN];
            long long sum = 0;
            for (int a = 1; a < NEN; ++a) {
                bad |= !(fabsf(re[a]) < d.fx_limit);   // also catches NaN
                q[a] = fx_from(re[a], d.fx_scale);
                sum += q[a];
            }
            q[0] = -sum;
            for (int a = 0; a < NEN; ++a)
                atomicAdd((unsigned long long *)&s_acc[l[a]], (unsigned long long)q[a]);
        } else {
            for (int a = 0; a < NEN; ++a) atomicAdd(&s_acc[l[a]], re[a]);
        }
        cur = nxt;
    }
    // matched interface pairs of the block (Eq. 8 with the sister face's mean as
    // ambient): node p of face a receives w (sum of face b's T - 3 T_p) and node
    // q of face b the converse; the six sum to zero, exactly in fixed point
    for (int v = threadIdx.x; v < bi.n_v; v += blockDim.x) {
        const int64_t gv = (int64_t)bi.v_begin + v;
        const uint32_t *vc = (const uint32_t *)(d.vconn + 6 * gv);
        const uint32_t c0 = vc[0], c1 = vc[1], c2 = vc[2];
        const int l[6] = {(int)(c0 & 0xFFFF), (int)(c0 >> 16), (int)(c1 & 0xFFFF),
                          (int)(c1 >> 16), (int)(c2 & 0xFFFF), (int)(c2 >> 16)};
        const R w = ((const R *)d.vw)[gv];
        R T[6];
        for (int a = 0; a < 6; ++a) T[a] = s_x[l[a]].w;
        const R sa = (T[0] + T[1]) + T[2], sb = (T[3] + T[4]) + T[5];
        R re[6];
        for (int a = 0; a < 3; ++a) {
            re[a] = w * (sb - R(3) * T[a]);
            re[3 + a] = w * (sa - R(3) * T[3 + a]);
        }
        if constexpr (std::is_same<R, float>::value) {
            long long q[6];
            long long sum = 0;
            for (int a = 1; a < 6; ++a) {
                bad |= !(fabsf(re[a]) < d.fx_limit);
                q[a] = fx_from(re[a], d.fx_scale);
                sum += q[a];
            }
            q[0] = -sum;
            for (int a = 0; a < 6; ++a)
                atomicAdd((unsigned long long *)&s_acc[l[a]], (unsigned long long)q[a]);
        } else {
            for (int a = 0; a < 6; ++a) atomicAdd(&s_acc[l[a]], re[a]);
        }
    }
    if (bad) s_bad = 1;
    __syncthreads();

    // private nodes are complete and free (fixed nodes are always shared):
    // update them in place; a contribution outside the fixed-point range
    // poisons the block so the run reports non-finite values
    const bool poison = s_bad != 0;
    auto resid = [&](int l) -> R {
        R r;
        if constexpr (std::is_same<R, float>::value) r = fx_to(s_acc[l], d.fx_inv);
        else r = s_acc[l];
        return poison ? R(NAN) : r;
    };
    // UPDATE_U private nodes per thread and pass, their loads issued together
    // before the first update; the last nodes of a thread go one by one.  Material
    // m is row m - m0 of `mats` (LDS rows, or the global table with m0 = 0).
    auto update_private = [&](const MatDev *mats, int m0) {
        int l = threadIdx.x;
        for (; l + (UPDATE_U - 1) * (int)blockDim.x < bi.n_int; l += UPDATE_U * blockDim.x) {
            uint32_t f[UPDATE_U];
            typename NodeH<R>::Pre pre[UPDATE_U];
#pragma unroll
            for (int u = 0; u < UPDATE_U; ++u) {
                const int64_t g = (int64_t)bi.int_base + l + u * (int)blockDim.x;
                f[u] = d.flags[g];
                pre[u] = NodeH<R>::load(d, g);
            }
#pragma unroll
            for (int u = 0; u < UPDATE_U; ++u) {
                const int lu = l + u * (int)blockDim.x;
                NodeH<R>::store(d, mats[(int)(f[u] & NODE_MAT_MASK) - m0], (int64_t)bi.int_base + lu, pre[u],
                                resid(lu), Tn);
            }
        }
        for (; l < bi.n_int; l += blockDim.x) {
            const int64_t g = (int64_t)bi.int_base + l;
            NodeH<R>::update(d, mats[(int)(d.flags[g] & NODE_MAT_MASK) - m0], g, resid(l), Tn);
        }
    };
    if (LDS_TABLES) update_private(s_mats, 0);
    else if (bi.pad1 >= 0) update_private(s_mats, bi.pad1);
    else update_private(d.mats, 0);
    // one partial per shared node, stored where the combine reads it
    R *P = (R *)d.partials;
    for (int l = threadIdx.x; l < bi.n_sh; l += blockDim.x) P[d.sh_pos[bi.sh_begin + l]] = resid(bi.n_int + l);
}

// node phase: all nodes (COMBINE = false: residual from r[N], which is reset)
// or the shared nodes of the blocked layout (COMBINE = true: sum of the node's
// partials in block order).  The first n_inflow slots may carry boundary inflow
// (Robin faces, reactions of fixed temperatures); each of them accumulates its
// own FP64 sum of dt * inflow, so no reduction runs per step and the total does
// not depend on the schedule.  A thread first loads its word of the material
// table and then all of its node's data, so that the table's wait before the
// barrier leaves the node loads in flight.
template <class R, bool COMBINE, bool LDS_TABLES>
__global__ __launch_bounds__(NODE_THREADS) void k_nodes(Dev d, int parity) {
    __shared__ MatDev s_mats[LDS_MATS];
    static_assert(LDS_MATS * sizeof(MatDev) / 4 <= NODE_THREADS, "one table word per thread");
    const int64_t count = COMBINE ? d.N - d.n_private : d.N;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = s < count;
    const int64_t g = d.bc_first + (live ? s : 0);
    // material rows in LDS: the whole table, or this workgroup's window of
    // LDS_MATS rows from m0 (m0 < 0: no window, rows read from global memory)
    const int m0 = LDS_TABLES ? 0 : (d.node_win ? d.node_win[blockIdx.x] : -1);
    const bool staged = LDS_TABLES || m0 >= 0;
    const int words = staged ? min(LDS_MATS, d.n_mat - m0) * (int)(sizeof(MatDev) / 4) : 0;
    uint32_t tw = 0;
    if ((int)threadIdx.x < words) tw = ((const uint32_t *)(d.mats + m0))[threadIdx.x];
    uint32_t f = 0;
    R r = R(0);
    typename NodeH<R>::Pre pre{};
    int32_t l0 = 0, l1 = 0;         // this slot's interface links (loaded with the rest)
    if (live) {
        f = d.flags[g];
        pre = NodeH<R>::load(d, g);
        l0 = d.link_ptr[s];
        l1 = d.link_ptr[s + 1];
        if (COMBINE) r = step::partial_slots(d, (const R *)d.partials, s);
        else r = ((const R *)d.r)[g];
    }
    if (staged) {           // uniform over the workgroup
        if ((int)threadIdx.x < words) ((uint32_t *)s_mats)[threadIdx.x] = tw;
        __syncthreads();
    }
    if (!live) return;
    const R *Tc = (const R *)d.T + parity * d.N;
    R *Tn = (R *)d.T + (1 - parity) * d.N;
    if (COMBINE) r = step::partial_extras(d, (const R *)d.partials, s, f, r);
    else ((R *)d.r)[g] = R(0);
    double q = 0.0;
    if (f & NODE_BC) q = boundary_terms<R>(d, s, Tc[g], Tc, r, l0, l1);
    auto finish = [&](const MatDev &M) {
        if (f & NODE_FIXED) q -= (double)r;     // reaction of a fixed temperature
        else NodeH<R>::store(d, M, g, pre, r, Tn);
        if (s < d.n_inflow) d.qnode[s] += q * M.dt;
    };
    const int m = (int)(f & NODE_MAT_MASK);
    if (staged) finish(s_mats[m - m0]);
    else finish(d.mats[m]);
}

// state diagnostics on demand: one workgroup per single-scenario node segment
// (E, latent heat still to release, T range, liquid and non-finite counts)
template <class R>
__global__ __launch_bounds__(NODE_THREADS) void k_state(Dev d, int parity) {
    DiagAcc acc;
    acc.init();
    const int32_t n0 = d.seg_begin[blockIdx.x], n1 = d.seg_begin[blockIdx.x + 1];
    // four nodes per thread per pass, their loads issued together
    constexpr int U = 4;
    for (int64_t i0 = n0 + (int64_t)threadIdx.x; i0 < n1; i0 += U * (int64_t)blockDim.x) {
        uint32_t f[U];
        double H[U], m[U], T[U];
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + u * (int64_t)blockDim.x;
            const int64_t j = i < n1 ? i : i0;            // a valid node, not counted below
            f[u] = d.flags[j];
            if constexpr (std::is_same<R, float>::value) {
                const float2 h = ((const float2 *)d.H)[j];
                H[u] = (double)h.x + (double)h.y;
            } else {
                H[u] = ((const double *)d.H)[j];
            }
            m[u] = 1.0 / (double)((const R *)d.inv_m)[j];
            T[u] = (double)((const R *)d.T)[parity * d.N + j];
        }
        for (int u = 0; u < U; ++u) {
            if (i0 + u * (int64_t)blockDim.x >= n1) break;
            const MatDev &M = d.mats[f[u] & NODE_MAT_MASK];
            double Th, fs;
            t_of_h(M, H[u], Th, fs);
            acc.v[DG_E] += m[u] * H[u];
            acc.v[DG_LAT] += m[u] * M.L * (1.0 - fs);
            acc.v[DG_TMIN] = fmin(acc.v[DG_TMIN], T[u]);
            acc.v[DG_TMAX] = fmax(acc.v[DG_TMAX], T[u]);
            acc.v[DG_NLIQ] += (M.latent && fs < 1.0) ? 1.0 : 0.0;
            acc.v[DG_NONFIN] += isfinite(H[u]) ? 0.0 : 1.0;
        }
    }
    reduce_diag(d, acc, blockIdx.x);
}

// plain copy, four 16-byte words in flight per thread
__global__ __launch_bounds__(256) void k_copy(float4 *__restrict__ dst, const float4 *__restrict__ src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], e = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = e;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// copy with non-temporal loads and stores (the data is not kept in the caches
// for a later reader), four 16-byte words in flight per thread: the ceiling of
// streaming HBM bandwidth on this device
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_nt(v4f *__restrict__ dst, const v4f *__restrict__ src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4f a = __builtin_nontemporal_load(src + i);
        const v4f b = __builtin_nontemporal_load(src + i + stride);
        const v4f c = __builtin_nontemporal_load(src + i + 2 * stride);
        const v4f e = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(e, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// the read-back of one check: integer check counts, per-segment diagnostics and
// per-node inflow sums gathered into one page-locked host buffer that the
// device writes directly (each part at a 16-byte aligned offset)
__global__ __launch_bounds__(256) void k_stage(int32_t *__restrict__ dst_chk, const int32_t *__restrict__ chk,
                                               int64_t n_chk, double *__restrict__ dst_dg,
                                               const double *__restrict__ dg, int64_t n_dg,
                                               double *__restrict__ dst_qn, const double *__restrict__ qn,
                                               int64_t n_qn) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < n_chk; i += stride) dst_chk[i] = chk[i];
    for (int64_t i = t; i < n_dg; i += stride) dst_dg[i] = dg[i];
    for (int64_t i = t; i < n_qn; i += stride) dst_qn[i] = qn[i];
}

template <class R, int NEN, bool LDS_TABLES>
hipError_t step_t(const Dev &d, int parity, hipStream_t s, hipEvent_t *ev) {
    const bool blocked = d.scatter == FEM_SCATTER_LDS_BLOCKED;
    if (ev && !blocked) (void)hipEventRecord(ev[0], s);
    if (blocked) {
        // timed launches (eager) carry their own start and stop events
        if (ev)
            hipExtLaunchKernelGGL((k_block<R, NEN, LDS_TABLES>), dim3((unsigned)d.n_blocks), dim3(d.threads),
                                  (uint32_t)d.lds_bytes, s, ev[0], ev[1], 0u, d, parity);
        else
            hipLaunchKernelGGL((k_block<R, NEN, LDS_TABLES>), dim3((unsigned)d.n_blocks), dim3(d.threads),
                               d.lds_bytes, s, d, parity);
    } else if (d.scatter == FEM_SCATTER_GLOBAL_ATOMIC) {
        if (d.E > 0)
            hipLaunchKernelGGL((k_elems<R, NEN, true>), dim3((unsigned)((d.E + 255) / 256)), dim3(256), 0, s, d,
                               parity, (int64_t)0, d.E);
    } else {
        for (int c = 0; c < d.n_colors; ++c) {
            const int64_t e0 = d.color_ptr_host[c], e1 = d.color_ptr_host[c + 1];
            if (e1 > e0)
                hipLaunchKernelGGL((k_elems<R, NEN, false>), dim3((unsigned)((e1 - e0 + 255) / 256)), dim3(256), 0, s,
                                   d, parity, e0, e1);
        }
    }
    if (ev && !blocked) (void)hipEventRecord(ev[1], s);
    const int64_t count = blocked ? d.N - d.n_private : d.N;
    if (count > 0) {
        const dim3 g((unsigned)node_grid(count)), b(NODE_THREADS);
        if (ev) {
            if (blocked) hipExtLaunchKernelGGL((k_nodes<R, true, LDS_TABLES>), g, b, 0u, s, ev[2], ev[3], 0u, d, parity);
            else hipExtLaunchKernelGGL((k_nodes<R, false, LDS_TABLES>), g, b, 0u, s, ev[2], ev[3], 0u, d, parity);
        } else {
            if (blocked) hipLaunchKernelGGL((k_nodes<R, true, LDS_TABLES>), g, b, 0, s, d, parity);
            else hipLaunchKernelGGL((k_nodes<R, false, LDS_TABLES>), g, b, 0, s, d, parity);
        }
    } else if (ev) {
        (void)hipEventRecord(ev[2], s);
        (void)hipEventRecord(ev[3], s);
    }
    return hipGetLastError();
}

// material tables of at most LDS_MATS rows are read from LDS, larger ones (a
// batch) from global memory, each in its own instantiation
template <class R, int NEN>
hipError_t step_nen(const Dev &d, int parity, hipStream_t s, hipEvent_t *ev) {
    return d.n_mat <= LDS_MATS ? step_t<R, NEN, true>(d, parity, s, ev) : step_t<R, NEN, false>(d, parity, s, ev);
}

template <class R, int NEN>
hipError_t set_limit(size_t bytes) {
    for (const void *k : {(const void *)k_block<R, NEN, true>, (const void *)k_block<R, NEN, false>}) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t enqueue_step(const Dev &d, int parity, hipStream_t s, hipEvent_t *ev) {
    if (d.prec == FEM_PREC_FP64) return d.nen == 4 ? step_nen<double, 4>(d, parity, s, ev) : step_nen<double, 8>(d, parity, s, ev);
    return d.nen == 4 ? step_nen<float, 4>(d, parity, s, ev) : step_nen<float, 8>(d, parity, s, ev);
}

hipError_t enqueue_state_diag(const Dev &d, int parity, hipStream_t s) {
    const unsigned grid = (unsigned)d.n_seg;
    if (d.prec == FEM_PREC_FP64) hipLaunchKernelGGL((k_state<double>), dim3(grid), dim3(NODE_THREADS), 0, s, d, parity);
    else hipLaunchKernelGGL((k_state<float>), dim3(grid), dim3(NODE_THREADS), 0, s, d, parity);
    return hipGetLastError();
}

hipError_t set_block_lds_limit(int prec, int nen, size_t bytes) {
    if (prec == FEM_PREC_FP64) return nen == 4 ? set_limit<double, 4>(bytes) : set_limit<double, 8>(bytes);
    return nen == 4 ? set_limit<float, 4>(bytes) : set_limit<float, 8>(bytes);
}

hipError_t enqueue_stage(int32_t *dst_chk, const int32_t *chk, int64_t n_chk, double *dst_dg, const double *dg,
                         int64_t n_dg, double *dst_qn, const double *qn, int64_t n_qn, hipStream_t s) {
    const int64_t n = std::max(n_chk, std::max(n_dg, n_qn));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
    hipLaunchKernelGGL(k_stage, dim3(grid), dim3(256), 0, s, dst_chk, chk, n_chk, dst_dg, dg, n_dg, dst_qn, qn, n_qn);
    return hipGetLastError();
}

hipError_t enqueue_copy(void *dst, const void *src, int64_t n16, hipStream_t s) {
    const int64_t want = (n16 + 4 * 256 - 1) / (4 * 256);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 256 * 32));
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, (float4 *)dst, (const float4 *)src, n16);
    return hipGetLastError();
}

hipError_t enqueue_copy_nt(void *dst, const void *src, int64_t n16, hipStream_t s) {
    const int64_t want = (n16 + 4 * 256 - 1) / (4 * 256);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 32768));
    hipLaunchKernelGGL(k_copy_nt, dim3(grid), dim3(256), 0, s, (v4f *)dst, (const v4f *)src, n16);
    return hipGetLastError();
}

// ------------------------------------------------------------ allocation-free stepping
// The partial residuals of fem_step_no_alloc live in this file-scope device
// array: every GPU the library runs on holds its own copy until the process
// ends, and every call on that GPU shares it.  Host code never uses the
// array's name as an address; scratch_address() resolves it once per device.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

__global__ __launch_bounds__(256) void k_zero(uint4 *__restrict__ p, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_set_dt(MatDev *m, int n, double dt) {
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        m[q].dt = dt;
        m[q].dtf = (float)dt;
    }
}

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void *scratch_ptrs[MAX_DEVICES] = {};

}  // namespace

hipError_t scratch_address(int device, void **out) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptrs[device]) {
        // the device must be current: each GPU has its own copy of the array
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptrs[device] = p;
    }
    *out = scratch_ptrs[device];
    return hipSuccess;
}

hipError_t enqueue_zero(void *p, int64_t bytes, hipStream_t s) {
    const int64_t n16 = (bytes + 15) / 16;
    if (n16 == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n16 + 255) / 256, 4096));
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, (uint4 *)p, n16);
    return hipGetLastError();
}

hipError_t enqueue_set_dt(MatDev *mats, int n, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(64), 0, s, mats, n, dt);
    return hipGetLastError();
}

}  // namespace castfem
