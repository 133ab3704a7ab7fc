// Element formulas of the Galerkin conduction operator (Sec. 3 of the paper,
// Eq. 9 and the element-by-element assembly of Eq. 15-18), written once for
// the host preprocessing (lumping, stability bound) and the gfx950 kernels.
//
// Linear tetrahedron with edges d_j = x_j - x_0 (j = 1..3): the gradients of
// the barycentric shape functions are grad N_j = c_j / D with
//   c_1 = d_2 x d_3, c_2 = d_3 x d_1, c_3 = d_1 x d_2, D = d_1 . c_1 = 6 V,
// and grad N_0 = -(grad N_1 + grad N_2 + grad N_3).  With
//   G = sum_j (T_j - T_0) c_j  (= D grad T),
// the element residual -K^e T^e is r_j = -k / (6 D) c_j . G and r_0 = -(r_1 + r_2 + r_3).
//
// Trilinear hexahedron: 2x2x2 Gauss-Legendre, r_a = -sum_q k |J_q| grad N_a . grad T.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

#define CF_HD __host__ __device__ __forceinline__

namespace castfem {

template <class R>
struct V3 {
    R x, y, z;
};

template <class R>
CF_HD V3<R> sub3(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R>
CF_HD V3<R> cross3(V3<R> a, V3<R> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class R>
CF_HD R dot3(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// reciprocal: one hardware reciprocal (1 ulp) for FP32 on the device, exact
// division otherwise
CF_HD float recip(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
CF_HD double recip(double x) { return 1.0 / x; }

// 6 * signed volume of a tetrahedron
template <class R>
CF_HD R tet_six_vol(V3<R> x0, V3<R> x1, V3<R> x2, V3<R> x3) {
    V3<R> d1 = sub3(x1, x0), d2 = sub3(x2, x0), d3 = sub3(x3, x0);
    return dot3(d1, cross3(d2, d3));
}

// element residual r = -K^e T^e of a linear tetrahedron
template <class R>
CF_HD void tet_residual(V3<R> x0, V3<R> x1, V3<R> x2, V3<R> x3, R t0, R t1, R t2, R t3, R k,
                        R &r0, R &r1, R &r2, R &r3) {
    V3<R> d1 = sub3(x1, x0), d2 = sub3(x2, x0), d3 = sub3(x3, x0);
    V3<R> c1 = cross3(d2, d3), c2 = cross3(d3, d1), c3 = cross3(d1, d2);
    R D = dot3(d1, c1);
    R a1 = t1 - t0, a2 = t2 - t0, a3 = t3 - t0;
    V3<R> G = {a1 * c1.x + a2 * c2.x + a3 * c3.x, a1 * c1.y + a2 * c2.y + a3 * c3.y,
               a1 * c1.z + a2 * c2.z + a3 * c3.z};
    R s = -k * recip(R(6) * D);
    r1 = s * dot3(c1, G);
    r2 = s * dot3(c2, G);
    r3 = s * dot3(c3, G);
    r0 = -(r1 + r2 + r3);
}

// full 4x4 conduction matrix of a linear tetrahedron (host preprocessing)
template <class R>
CF_HD void tet_ke(V3<R> x0, V3<R> x1, V3<R> x2, V3<R> x3, R k, R Ke[4][4]) {
    V3<R> d1 = sub3(x1, x0), d2 = sub3(x2, x0), d3 = sub3(x3, x0);
    V3<R> c[4];
    c[1] = cross3(d2, d3);
    c[2] = cross3(d3, d1);
    c[3] = cross3(d1, d2);
    c[0] = {-(c[1].x + c[2].x + c[3].x), -(c[1].y + c[2].y + c[3].y), -(c[1].z + c[2].z + c[3].z)};
    R D = dot3(d1, c[1]);
    R s = k / (R(6) * D);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) Ke[a][b] = s * dot3(c[a], c[b]);
}

// reference-cube sign of hex node a along axis i, node order (0,0,0) (1,0,0)
// (1,1,0) (0,1,0) then the same on the top face
CF_HD int hex_sign(int a, int i) {
    // bit patterns: x: 0110 0110, y: 0011 0011, z: 0000 1111 (node 0 = lowest bit)
    const int mask = i == 0 ? 0x66 : (i == 1 ? 0xCC : 0xF0);
    return ((mask >> a) & 1) ? 1 : -1;
}

// reference derivative dN_a/dxi_i at the Gauss point q (signs of q as for nodes)
template <class R>
CF_HD R hex_dN(int a, int i, int q) {
    const R g = R(0.57735026918962576451);  // 1/sqrt(3)
    R f[3];
    for (int j = 0; j < 3; ++j) f[j] = R(1) + R(hex_sign(a, j)) * R(hex_sign(q, j)) * g;
    R v = R(0.125) * R(hex_sign(a, i));
    for (int j = 0; j < 3; ++j)
        if (j != i) v *= f[j];
    return v;
}

template <class R>
CF_HD R hex_N(int a, int q) {
    const R g = R(0.57735026918962576451);
    R v = R(0.125);
    for (int j = 0; j < 3; ++j) v *= R(1) + R(hex_sign(a, j)) * R(hex_sign(q, j)) * g;
    return v;
}

// Jacobian J[i][j] = d x_j / d xi_i at Gauss point q, its inverse and determinant
template <class R>
CF_HD R hex_jac(const V3<R> *x, int q, R Ji[3][3]) {
    R J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int a = 0; a < 8; ++a) {
        for (int i = 0; i < 3; ++i) {
            R d = hex_dN<R>(a, i, q);
            J[i][0] += d * x[a].x;
            J[i][1] += d * x[a].y;
            J[i][2] += d * x[a].z;
        }
    }
    V3<R> r0 = {J[0][0], J[0][1], J[0][2]}, r1 = {J[1][0], J[1][1], J[1][2]}, r2 = {J[2][0], J[2][1], J[2][2]};
    V3<R> k0 = cross3(r1, r2), k1 = cross3(r2, r0), k2 = cross3(r0, r1);
    R det = dot3(r0, k0);
    R id = R(1) / det;
    // inverse of a matrix with rows r0, r1, r2 has columns k0, k1, k2 / det
    Ji[0][0] = k0.x * id; Ji[0][1] = k1.x * id; Ji[0][2] = k2.x * id;
    Ji[1][0] = k0.y * id; Ji[1][1] = k1.y * id; Ji[1][2] = k2.y * id;
    Ji[2][0] = k0.z * id; Ji[2][1] = k1.z * id; Ji[2][2] = k2.z * id;
    return det;
}

// element residual r = -K^e T^e of a trilinear hexahedron
template <class R>
CF_HD void hex_residual(const V3<R> *x, const R *t, R k, R *r) {
    for (int a = 0; a < 8; ++a) r[a] = R(0);
    for (int q = 0; q < 8; ++q) {
        R Ji[3][3];
        R det = hex_jac<R>(x, q, Ji);
        V3<R> g[8];
        V3<R> gT = {0, 0, 0};
        for (int a = 0; a < 8; ++a) {
            R d0 = hex_dN<R>(a, 0, q), d1 = hex_dN<R>(a, 1, q), d2 = hex_dN<R>(a, 2, q);
            g[a] = {Ji[0][0] * d0 + Ji[0][1] * d1 + Ji[0][2] * d2,
                    Ji[1][0] * d0 + Ji[1][1] * d1 + Ji[1][2] * d2,
                    Ji[2][0] * d0 + Ji[2][1] * d1 + Ji[2][2] * d2};
            gT.x += t[a] * g[a].x;
            gT.y += t[a] * g[a].y;
            gT.z += t[a] * g[a].z;
        }
        R w = -k * det;
        for (int a = 0; a < 8; ++a) r[a] += w * dot3(g[a], gT);
    }
}

// full 8x8 conduction matrix and lumped weights rho int N_a dV of a hexahedron
// (host preprocessing); returns the smallest Jacobian determinant
template <class R>
CF_HD R hex_ke_mass(const V3<R> *x, R k, R rho, R Ke[8][8], R m[8]) {
    R mindet = R(1e300);
    for (int a = 0; a < 8; ++a) {
        m[a] = 0;
        for (int b = 0; b < 8; ++b) Ke[a][b] = 0;
    }
    for (int q = 0; q < 8; ++q) {
        R Ji[3][3];
        R det = hex_jac<R>(x, q, Ji);
        if (det < mindet) mindet = det;
        V3<R> g[8];
        for (int a = 0; a < 8; ++a) {
            R d0 = hex_dN<R>(a, 0, q), d1 = hex_dN<R>(a, 1, q), d2 = hex_dN<R>(a, 2, q);
            g[a] = {Ji[0][0] * d0 + Ji[0][1] * d1 + Ji[0][2] * d2,
                    Ji[1][0] * d0 + Ji[1][1] * d1 + Ji[1][2] * d2,
                    Ji[2][0] * d0 + Ji[2][1] * d1 + Ji[2][2] * d2};
            m[a] += rho * hex_N<R>(a, q) * det;
        }
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) Ke[a][b] += k * det * dot3(g[a], g[b]);
    }
    return mindet;
}

}  // namespace castfem
