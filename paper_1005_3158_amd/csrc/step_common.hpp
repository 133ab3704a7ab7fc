// Device helpers shared by the step variants of apparent.hip and varprops.hip:
// the same constructions as in the enthalpy kernels of kernels.hip, which keep
// their own copies so that they stay byte-for-byte as profiled.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace castfem {
namespace step {

template <class R> struct VT;
template <> struct VT<float> { using V4 = float4; using V2 = float2; };
template <> struct VT<double> { using V4 = double4; using V2 = double2; };

// contiguous ranges of logical blocks per XCD (workgroups are dispatched
// round-robin over the 8 XCDs), so that neighbouring blocks share an L2
__device__ __forceinline__ int xcd_remap(int w, int n) {
    const int x = w & 7, i = w >> 3;
    const int q = n >> 3, rem = n & 7;
    return x * q + min(x, rem) + i;
}

// round(r * scale) as a two's-complement integer via the 1.5 * 2^52 shift
__device__ __forceinline__ long long fx_from(float r, double scale) {
    const double magic = 6755399441055744.0;
    const double x = __builtin_fma((double)r, scale, magic);
    return __double_as_longlong(x) - __double_as_longlong(magic);
}
__device__ __forceinline__ float fx_to(long long q, double inv_scale) { return (float)((double)q * inv_scale); }

// error-free two-sum of (hi, inc) carried into lo, then renormalised
__device__ __forceinline__ float2 kahan_add(float2 h, float inc) {
#pragma clang fp contract(off)
    float s = h.x + inc;
    float bp = s - h.x;
    float e = (h.x - (s - bp)) + (inc - bp);
    float lo = h.y + e;
    float hi = s + lo;
    lo = lo - (hi - s);
    return make_float2(hi, lo);
}

// enthalpy relation (Eq. 11, linear latent release) and its inverse
__device__ __forceinline__ void t_of_h(const MatDev &M, double H, double &T, double &fs) {
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
__device__ __forceinline__ double h_of_t(const MatDev &M, double T) {
    double g = 0.0;
    if (M.latent && T > M.Ts) g = T >= M.Tl ? 1.0 : (T - M.Ts) / (M.Tl - M.Ts);
    return M.c * T + M.L * g;
}

// Enthalpy update of a free node g with residual r: H += dt r / m (FP32: two-sum
// into the (hi, lo) pair), then T and f_s from H in FP64.
template <class R> struct NodeH;
template <> struct NodeH<float> {
    static __device__ __forceinline__ void update(const Dev &d, const MatDev &M, int64_t g, float r, float *Tn) {
        float2 *H = (float2 *)d.H;
        const float im = ((const float *)d.inv_m)[g];
        float inc;
        {
#pragma clang fp contract(off)
            inc = r * (M.dtf * im);
        }
        const float2 h = kahan_add(H[g], inc);
        H[g] = h;
        double T, fs;
        t_of_h(M, (double)h.x + (double)h.y, T, fs);
        Tn[g] = (float)T;
        ((float *)d.fs)[g] = (float)fs;
    }
};
template <> struct NodeH<double> {
    static __device__ __forceinline__ void update(const Dev &d, const MatDev &M, int64_t g, double r, double *Tn) {
        double *H = (double *)d.H;
        const double im = ((const double *)d.inv_m)[g];
        const double h = H[g] + r * (M.dt * im);
        H[g] = h;
        double T, fs;
        t_of_h(M, h, T, fs);
        Tn[g] = T;
        ((double *)d.fs)[g] = fs;
    }
};

// Robin and interface terms of boundary slot s for a node at temperature Ti:
// adds them to r and returns the Robin inflow
template <class R>
__device__ __forceinline__ double boundary_terms(const Dev &d, int64_t s, R Ti, const R *Tc, R &r) {
    using V2 = typename VT<R>::V2;
    double q = 0.0;
    if (d.robin) {
        const V2 ab = ((const V2 *)d.robin)[s];
        const R f = ab.x - ab.y * Ti;
        r += f;
        q = (double)f;
    }
    const int32_t l0 = d.link_ptr[s], l1 = d.link_ptr[s + 1];
    const R *w = (const R *)d.link_w;
    for (int32_t k = l0; k < l1; ++k) r += w[k] * (Tc[d.link_node[k]] - Ti);
    return q;
}

// material tables of at most LDS_MATS rows are read from LDS, larger ones from
// global memory; kernels are instantiated for each case so that every table
// access compiles to LDS or global loads (a pointer that may be either would
// compile to the slower flat loads)
constexpr int LDS_MATS = 8;

// copy a small table into LDS (visible after the caller's next barrier)
template <class M>
__device__ __forceinline__ void stage_table(const M *src, int n, M *dst) {
    static_assert(sizeof(M) % 4 == 0, "table rows are whole words");
    const int words = n * (int)(sizeof(M) / 4);
    for (int w = threadIdx.x; w < words; w += blockDim.x) ((uint32_t *)dst)[w] = ((const uint32_t *)src)[w];
}

}  // namespace step
}  // namespace castfem
