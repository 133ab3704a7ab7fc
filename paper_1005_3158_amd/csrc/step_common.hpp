// Device helpers shared by the step variants of apparent.hip and varprops.hip:
// the same constructions as in the enthalpy kernels of kernels.hip, which keep
// their own copies so that they stay byte-for-byte as profiled.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace castfem {
namespace step {

// Local ids of element e (global element index) of the blocked layout: raw
// words loaded ahead of their use (x, y, z; w = which tet of a packed pair, or
// 2 for 16-bit ids), then decoded.
template <int NEN>
struct ConnRaw {
    uint32_t x, y, z, w;
};
template <int NEN>
__device__ __forceinline__ ConnRaw<NEN> conn_load(const Dev &d, int64_t e) {
    if constexpr (NEN == 4) {
        if (d.conn12) {
            const uint3 v = ((const uint3 *)d.lconn)[e >> 1];
            return {v.x, v.y, v.z, (uint32_t)(e & 1)};
        }
        const uint2 v = ((const uint2 *)d.lconn)[e];
        return {v.x, v.y, 0u, 2u};
    } else {
        const uint4 v = ((const uint4 *)d.lconn)[e];
        return {v.x, v.y, v.z, v.w};
    }
}
template <int NEN>
__device__ __forceinline__ void conn_ids(const ConnRaw<NEN> &c, int *l) {
    if constexpr (NEN == 4) {
        if (c.w == 2u) {
            l[0] = c.x & 0xFFFF;
            l[1] = c.x >> 16;
            l[2] = c.y & 0xFFFF;
            l[3] = c.y >> 16;
        } else {
            const uint64_t v = c.w ? (((uint64_t)c.z << 16) | (c.y >> 16)) : (((uint64_t)c.y << 32) | c.x);
            for (int a = 0; a < 4; ++a) l[a] = (int)((v >> (12 * a)) & 0xFFFu);
        }
    } else {
        const uint32_t w[4] = {c.x, c.y, c.z, c.w};
        for (int a = 0; a < 4; ++a) {
            l[2 * a] = w[a] & 0xFFFF;
            l[2 * a + 1] = w[a] >> 16;
        }
    }
}

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

// Node coordinates of the FP32 kernels are fixed-point integers carried in
// the float bits of x, y and z (Dev::x_scale metres per unit, a power of two
// chosen so that no element spans 2^24 units or more).  An element takes them
// relative to its node 0: integer differences are exact, and so is their
// conversion to float, so every edge carries the fixed-point resolution
// (about 1e-7 of a typical edge) instead of the FP32 rounding of absolute
// coordinates (about 1e-5 of an edge on a 128^3 grid of the domain, a
// systematic error of the conduction operator).  The element formulas depend
// on coordinate differences only.
//   local_units: coordinates in units.  The residual -K^e T^e of a linear
//     element scales with length, so the caller multiplies the conductivity
//     by x_scale instead of every coordinate.
//   local_coords: coordinates in metres (for formulas with volumes).
// FP64 coordinates are plain metres (x_scale = 1) and stay as they are.
template <int NEN>
__device__ __forceinline__ void local_units(float4 *p) {
    const int x0 = __float_as_int(p[0].x), y0 = __float_as_int(p[0].y), z0 = __float_as_int(p[0].z);
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
        p[a].x = (float)(__float_as_int(p[a].x) - x0);
        p[a].y = (float)(__float_as_int(p[a].y) - y0);
        p[a].z = (float)(__float_as_int(p[a].z) - z0);
    }
}
template <int NEN>
__device__ __forceinline__ void local_units(double4 *) {}
template <int NEN>
__device__ __forceinline__ void local_coords(float4 *p, float scale) {
    local_units<NEN>(p);
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
        p[a].x *= scale;
        p[a].y *= scale;
        p[a].z *= scale;
    }
}
template <int NEN>
__device__ __forceinline__ void local_coords(double4 *, float) {}

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
// into the (hi, lo) pair), then T and f_s from H in FP64.  update() does it in
// one go; load() and store() split it, so that a thread can issue the loads of
// several nodes before it waits for the first.
template <class R> struct NodeH;
template <> struct NodeH<float> {
    struct Pre {
        float2 h;
        float im;
    };
    static __device__ __forceinline__ Pre load(const Dev &d, int64_t g) {
        return Pre{((const float2 *)d.H)[g], ((const float *)d.inv_m)[g]};
    }
    static __device__ __forceinline__ void store(const Dev &d, const MatDev &M, int64_t g, const Pre &p, float r,
                                                 float *Tn) {
        float inc;
        {
#pragma clang fp contract(off)
            inc = r * (M.dtf * p.im);
        }
        const float2 h = kahan_add(p.h, inc);
        ((float2 *)d.H)[g] = h;
        double T, fs;
        t_of_h(M, (double)h.x + (double)h.y, T, fs);
        Tn[g] = (float)T;
        ((float *)d.fs)[g] = (float)fs;
    }
    static __device__ __forceinline__ void update(const Dev &d, const MatDev &M, int64_t g, float r, float *Tn) {
        store(d, M, g, load(d, g), r, Tn);
    }
};
template <> struct NodeH<double> {
    struct Pre {
        double h;
        double im;
    };
    static __device__ __forceinline__ Pre load(const Dev &d, int64_t g) {
        return Pre{((const double *)d.H)[g], ((const double *)d.inv_m)[g]};
    }
    static __device__ __forceinline__ void store(const Dev &d, const MatDev &M, int64_t g, const Pre &p, double r,
                                                 double *Tn) {
        const double h = p.h + r * (M.dt * p.im);
        ((double *)d.H)[g] = h;
        double T, fs;
        t_of_h(M, h, T, fs);
        Tn[g] = T;
        ((double *)d.fs)[g] = fs;
    }
    static __device__ __forceinline__ void update(const Dev &d, const MatDev &M, int64_t g, double r, double *Tn) {
        store(d, M, g, load(d, g), r, Tn);
    }
};

// Robin and interface terms of boundary slot s for a node at temperature Ti:
// adds them to r and returns the Robin inflow
template <class R>
__device__ __forceinline__ double boundary_terms(const Dev &d, int64_t s, R Ti, const R *Tc, R &r, int32_t l0,
                                                 int32_t l1) {
    using V2 = typename VT<R>::V2;
    double q = 0.0;
    if (d.robin) {
        const V2 ab = ((const V2 *)d.robin)[s];
        const R f = ab.x - ab.y * Ti;
        r += f;
        q = (double)f;
    }
    const R *w = (const R *)d.link_w;
    for (int32_t k = l0; k < l1; ++k) r += w[k] * (Tc[d.link_node[k]] - Ti);
    return q;
}
// the same, with the slot's link range [link_ptr[s], link_ptr[s + 1]) read here
template <class R>
__device__ __forceinline__ double boundary_terms(const Dev &d, int64_t s, R Ti, const R *Tc, R &r) {
    return boundary_terms<R>(d, s, Ti, Tc, r, d.link_ptr[s], d.link_ptr[s + 1]);
}

// Sum of the residual partials of the blocked layout's shared node s (slot s of
// the node kernels) with flags f: the PARTIAL_SLOTS slot-major partials (zero
// where the node is in fewer blocks), then, for a node flagged NODE_XTRA, the
// rest from its list; left to right in block order.  The slot loads depend on
// s only, so they issue together with the node's other loads.
template <class R>
__device__ __forceinline__ R partial_slots(const Dev &d, const R *P, int64_t s) {
    const int64_t nsh = d.N - d.n_private;
    R p[PARTIAL_SLOTS];
#pragma unroll
    for (int j = 0; j < PARTIAL_SLOTS; ++j) p[j] = P[j * nsh + s];
    R r = p[0];
#pragma unroll
    for (int j = 1; j < PARTIAL_SLOTS; ++j) r += p[j];
    return r;
}
template <class R>
__device__ __forceinline__ R partial_extras(const Dev &d, const R *P, int64_t s, uint32_t f, R r) {
    if (f & NODE_XTRA) {
        const R *X = P + PARTIAL_SLOTS * (d.N - d.n_private);
        const int32_t k0 = d.comb_ptr[s], k1 = d.comb_ptr[s + 1];
        for (int32_t k = k0; k < k1; ++k) r += X[k];
    }
    return r;
}
template <class R>
__device__ __forceinline__ R combine_partials(const Dev &d, const R *P, int64_t s, uint32_t f) {
    return partial_extras(d, P, s, f, partial_slots(d, P, s));
}

// material tables of at most LDS_MATS rows are read from LDS, larger ones from
// global memory; kernels are instantiated for each case so that every table
// access compiles to LDS or global loads (a pointer that may be either would
// compile to the slower flat loads)
constexpr int LDS_MATS = MAT_WINDOW;

// copy a small table into LDS (visible after the caller's next barrier)
template <class M>
__device__ __forceinline__ void stage_table(const M *src, int n, M *dst) {
    static_assert(sizeof(M) % 4 == 0, "table rows are whole words");
    const int words = n * (int)(sizeof(M) / 4);
    for (int w = threadIdx.x; w < words; w += blockDim.x) ((uint32_t *)dst)[w] = ((const uint32_t *)src)[w];
}

}  // namespace step
}  // namespace castfem
