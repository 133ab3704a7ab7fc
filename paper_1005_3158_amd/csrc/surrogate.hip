// gfx950 kernels of the message-passing surrogate: features, BF16 MFMA
// products (forward, data gradient, weight gradient), mean-neighbour
// aggregation and its transpose, output layer and loss, Adam.
#include "surrogate.hpp"

#include <algorithm>

#include "kernels.hpp"

namespace castfem {
namespace sur {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(bf16 b) { return __uint_as_float((uint32_t)b << 16); }

// round to nearest even (NaN stays NaN)
__device__ __forceinline__ bf16 f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16)((u >> 16) | 0x40u);
    return (bf16)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ s4 load_s4(const bf16 *p) {
    const uint2 v = *(const uint2 *)p;
    s4 r;
    r[0] = (short)(v.x & 0xffff);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xffff);
    r[3] = (short)(v.y >> 16);
    return r;
}

// enthalpy relation of the node's material (as in the explicit step)
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

// ---------------------------------------------------------------- features
// Row r = q N + i holds node i of state slot q; the slot is sample idx[q]
// (q without a list), read at offset sample * stride of H0 / H1 / H2 / Ht,
// three consecutive explicit states and the state `horizon` steps after H0.
// the features, base, implied increment, scale (and target, with Ht) of row r
// (node i) from its three enthalpies
__device__ __forceinline__ void feature_row(const SurDev &s, int64_t r, int64_t i, double h0, double h1, double h2,
                                            const float *Ht_at) {
    const MatDev &M = ((const MatDev *)s.mats)[s.flags[i] & NODE_MAT_MASK];
    const double rate = h2 - h1, acc = (h2 - h1) - (h1 - h0);
    double T2, fs2;
    t_of_h(M, h2, T2, fs2);
    const float4 co = ((const float4 *)s.coef)[i];
    const double c = M.c, dt = M.dt, m = (double)s.horizon - 2.0, qm = 0.5 * m * (m + 1.0);
    // activity over the window and the kinks within reach of it
    const double span = fabs(m * rate) + fabs(qm * acc);
    const double sa = span + c * EPS_T;
    const bool free = !(s.flags[i] & NODE_FIXED);
    const bool near = fabs(h2 - M.Hl) < REACH * span || fabs(h2 - M.Hs) < REACH * span;
    const bool mu = free && M.latent && near;
    float x[NFEAT];
    x[0] = (float)((T2 - T_REF) / T_SCALE);
    x[1] = (float)fs2;
    x[2] = M.latent ? 1.0f : 0.0f;
    x[3] = (float)(co.x * dt);
    x[4] = (float)(co.y * dt);
    x[5] = (float)(co.z * dt);
    x[6] = (float)(m * rate / sa);
    x[7] = (float)(qm * acc / sa);
    x[8] = 1.0f;
    x[9] = (float)(log(sa / c) / 8.0);
    x[10] = M.latent ? (float)(fmin(fmax((h2 - M.Hl) / sa, -4.0), 4.0) / 4.0) : 0.0f;
    x[11] = M.latent ? (float)(fmin(fmax((h2 - M.Hs) / sa, -4.0), 4.0) / 4.0) : 0.0f;
    uint32_t w[KIN / 2];
    for (int k = 0; k < KIN / 2; ++k) {
        const float lo = 2 * k < NFEAT ? x[2 * k] : 0.0f, hi = 2 * k + 1 < NFEAT ? x[2 * k + 1] : 0.0f;
        w[k] = (uint32_t)f2bf(lo) | ((uint32_t)f2bf(hi) << 16);
    }
    uint4 *out = (uint4 *)(s.X + r * KIN);
    out[0] = make_uint4(w[0], w[1], w[2], w[3]);
    out[1] = make_uint4(w[4], w[5], w[6], w[7]);
    // linear extrapolation through H1, H2, or quadratic through H0, H1, H2
    s.base[r] = s.quadratic ? h2 + m * rate + qm * acc : h2 + m * rate;
    // the increment of the step after the horizon that the extrapolation implies
    if (r < s.N) s.rext[r] = s.quadratic ? rate + (m + 1.0) * acc : rate;
    s.scale[r] = mu ? (float)sa : 0.0f;
    if (Ht_at) {
        if (s.loss_mode == LOSS_T) {
            double Tt, fst;
            t_of_h(M, (double)*Ht_at, Tt, fst);
            s.target[r] = (float)Tt;
        } else {
            s.target[r] = (float)(((double)*Ht_at - s.base[r]) / sa);   // LOSS_H, LOSS_HUBER
        }
    }
}

template <class HT>
__global__ __launch_bounds__(256) void k_features(SurDev s, const HT *H0, const HT *H1, const HT *H2, const float *Ht,
                                                  int64_t stride, const int32_t *idx, int64_t slots) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= slots * s.N) return;
    const int64_t q = r / s.N, i = r - q * s.N;
    const int64_t at = (idx ? (int64_t)idx[q] : q) * stride + i;
    feature_row(s, r, i, (double)H0[at], (double)H1[at], (double)H2[at], Ht ? Ht + at : nullptr);
}

// One state of the solver: H2 is the solver's current state, read here and kept
// (FP64 copy in s.H2, the raw FP32 pairs, the node inflow sums) for a rejected
// jump to return to; H0 and H1 are earlier FP64 copies.
template <class R>
__global__ __launch_bounds__(256) void k_features_live(SurDev s, Dev d, const double *H0, const double *H1,
                                                       double *keep_qnode) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (keep_qnode && i < d.n_inflow) keep_qnode[i] = d.qnode[i];
    if (i >= s.N) return;
    double h2;
    if constexpr (sizeof(R) == 8) {
        h2 = ((const double *)d.H)[i];
    } else {
        const float2 v = ((const float2 *)d.H)[i];
        h2 = (double)v.x + (double)v.y;
        if (s.H2_pair) s.H2_pair[i] = v;
    }
    s.H2[i] = h2;
    feature_row(s, i, i, H0[i], H1[i], h2, nullptr);
}

// ---------------------------------------------------------------- products
// C[R x NOUT] = A[R x K] B[K x NOUT], B given transposed (Bt: NOUT x K, row-major).
// One wavefront computes 16 rows; MFMA operands follow the 16x16x16 layout:
// lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16], D[4(l/16)+j][l%16].
// MODE 0: z = C + bias -> Zout, h = relu(z) -> Hout
// MODE 1: z = C + bias -> Zout, h = Hprev + relu(z) -> Hout
// MODE 2: C -> Cout (FP32)
template <int NOUT, int MODE>
__global__ __launch_bounds__(256) void k_gemm(const bf16 *__restrict__ A, int lda, int K, const bf16 *__restrict__ Bt,
                                              const float *__restrict__ bias, int64_t R, bf16 *Zout,
                                              const bf16 *Hprev, int ldhp, bf16 *Hout, int ldh, float *Cout, int ldc) {
    constexpr int NT = NOUT / 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int ar = lane & 15, kq = (lane >> 4) * 4;
    const int64_t arow = row0 + ar;
    f4 acc[NT];
    float bcol[NT];                     // the epilogue's bias, loaded with the operands
    for (int t = 0; t < NT; ++t) {
        acc[t] = f4{0.f, 0.f, 0.f, 0.f};
        bcol[t] = MODE == 2 ? 0.f : bias[t * 16 + ar];
    }
    for (int k0 = 0; k0 < K; k0 += 16) {
        s4 a = {0, 0, 0, 0};
        if (arow < R) a = load_s4(A + arow * lda + k0 + kq);
        for (int t = 0; t < NT; ++t) {
            const s4 b = load_s4(Bt + (int64_t)(t * 16 + ar) * K + k0 + kq);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
    for (int t = 0; t < NT; ++t) {
        const int col = t * 16 + ar;
        for (int j = 0; j < 4; ++j) {
            const int64_t row = row0 + kq + j;
            if (row >= R) continue;
            const float v = acc[t][j];
            if constexpr (MODE == 2) {
                Cout[row * ldc + col] = v;
            } else {
                const float z = v + bcol[t];
                if (Zout) Zout[row * NOUT + col] = f2bf(z);
                const float act = z > 0.f ? z : 0.f;
                const float h = MODE == 0 ? act : bf2f(Hprev[row * ldhp + col]) + act;
                Hout[row * ldh + col] = f2bf(h);
            }
        }
    }
}

// partial weight and bias gradients of one workgroup's GRAD_ROWS rows:
// P[wg][f][c] = sum_r A[r][f] B[r][c] (A: R x KA, row stride lda; B: R x 64)
// and Pb[wg][c] = sum_r B[r][c].  The rows are the MFMA K dimension, so 64-row
// chunks of A and B are staged transposed in LDS: the four consecutive rows a
// lane needs are then one 8-byte LDS read.  Wave w owns columns 16w..16w+15.
template <int KA>
__global__ __launch_bounds__(256) void k_wgrad(const bf16 *__restrict__ A, int lda, const bf16 *__restrict__ B,
                                               int64_t R, float *__restrict__ P, float *__restrict__ Pb) {
    constexpr int FT = KA / 16, CH = 64, LDR = CH + 8;
    __shared__ __align__(16) bf16 At[KA][LDR];
    __shared__ __align__(16) bf16 Bt[WIDTH][LDR];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int mi = lane & 15, kq = (lane >> 4) * 4;
    f4 acc[FT];
    for (int ft = 0; ft < FT; ++ft) acc[ft] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const int64_t r_begin = (int64_t)blockIdx.x * GRAD_ROWS;
    const int64_t r_end = std::min<int64_t>(R, r_begin + GRAD_ROWS);
    for (int64_t r0 = r_begin; r0 < r_end; r0 += CH) {
        constexpr int AV = KA / 8;   // 16-byte vectors per row of A
        for (int v = t; v < CH * AV; v += 256) {
            const int rr = v / AV, f8 = (v % AV) * 8;
            const int64_t r = r0 + rr;
            uint4 w = make_uint4(0, 0, 0, 0);
            if (r < r_end) w = *(const uint4 *)(A + r * lda + f8);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
            for (int k = 0; k < 4; ++k) {
                At[f8 + 2 * k][rr] = (bf16)(ws[k] & 0xffffu);
                At[f8 + 2 * k + 1][rr] = (bf16)(ws[k] >> 16);
            }
        }
        for (int v = t; v < CH * (WIDTH / 8); v += 256) {
            const int rr = v / (WIDTH / 8), c8 = (v % (WIDTH / 8)) * 8;
            const int64_t r = r0 + rr;
            uint4 w = make_uint4(0, 0, 0, 0);
            if (r < r_end) w = *(const uint4 *)(B + r * WIDTH + c8);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
            for (int k = 0; k < 4; ++k) {
                Bt[c8 + 2 * k][rr] = (bf16)(ws[k] & 0xffffu);
                Bt[c8 + 2 * k + 1][rr] = (bf16)(ws[k] >> 16);
            }
        }
        __syncthreads();
        for (int kk = 0; kk < CH; kk += 16) {
            const s4 b = *(const s4 *)&Bt[wave * 16 + mi][kk + kq];
            for (int j = 0; j < 4; ++j) bsum += bf2f((bf16)b[j]);
            for (int ft = 0; ft < FT; ++ft) {
                const s4 a = *(const s4 *)&At[ft * 16 + mi][kk + kq];
                acc[ft] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[ft], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float *out = P + (int64_t)blockIdx.x * KA * WIDTH;
    for (int ft = 0; ft < FT; ++ft)
        for (int j = 0; j < 4; ++j) out[(ft * 16 + kq + j) * WIDTH + wave * 16 + mi] = acc[ft][j];
    bsum += __shfl_down(bsum, 32, 64);
    bsum += __shfl_down(bsum, 16, 64);
    if (lane < 16) Pb[(int64_t)blockIdx.x * WIDTH + wave * 16 + mi] = bsum;
}

// Deterministic sum of the workgroup partials P[b][k] (b < nblk, partials `per`
// floats apart) into out[k], k < keep, in two passes: groups of PARTIAL_GROUP
// partials in order into P2[g][k], then the groups in order.

__global__ void k_reduce_groups(const float *__restrict__ P, int64_t nblk, int64_t per, int keep,
                                float *__restrict__ P2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= keep) return;
    const int64_t b0 = (int64_t)blockIdx.y * PARTIAL_GROUP, b1 = std::min<int64_t>(nblk, b0 + PARTIAL_GROUP);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int64_t b = b0;
    for (; b + 4 <= b1; b += 4) {
        a0 += P[b * per + k];
        a1 += P[(b + 1) * per + k];
        a2 += P[(b + 2) * per + k];
        a3 += P[(b + 3) * per + k];
    }
    for (; b < b1; ++b) a0 += P[b * per + k];
    P2[(int64_t)blockIdx.y * keep + k] = (a0 + a1) + (a2 + a3);
}

__global__ void k_reduce_final(const float *__restrict__ P2, int64_t ngroups, int keep, float *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= keep) return;
    float s = 0.f;
    for (int64_t g = 0; g < ngroups; ++g) s += P2[g * keep + k];
    out[k] = s;
}

// ---------------------------------------------------------------- graph
// One message-passing layer for 32 rows per workgroup: h_{l-1} of the rows and
// the mean of h_{l-1} over their mesh neighbours (one 8-channel task per
// thread, eight neighbours in flight) are put side by side in LDS with W_l^T,
// then [h, a] W_l runs on MFMA: wave w takes rows 16 (w & 1).. and output
// columns 32 (w >> 1)...  Epilogue: z = . + b_l (kept in Z[l] when store),
// h_l = h_{l-1} + relu(z) into U[l+1] (or H_last); the last layer also forms
// y = h_L . w_out + b_out.  With store the mean is also written into the
// second half of U[l] (the weight gradient reads it).
// Rows per workgroup: 32 for large row counts (training batches: the weights
// are staged once per 32 rows), 16 for a single small mesh (inference on a few
// thousand rows: twice the workgroups, so that every compute unit gathers)
constexpr int LAYER_ROWS = 32;
constexpr int LAYER_ROWS_SMALL = 16;
constexpr int64_t LAYER_SMALL_MAX = 16384;   // row counts up to this take the 16-row form

template <int ROWS>
__global__ __launch_bounds__(256) void k_layer(SurDev s, int l, int64_t R, int store) {
    static_assert(ROWS == 16 || ROWS == 32, "16 or 32 rows per workgroup");
    constexpr int LDU = 2 * WIDTH + 8;
    constexpr int TPR = 256 / ROWS;          // threads per row in the gather
    constexpr int CH = WIDTH / TPR;          // channels per thread: 8 (one 16-byte word) or 4
    constexpr int NW = CH / 2;               // 32-bit words per thread
    constexpr int NT = ROWS / 16 == 2 ? 2 : 1;   // 16-column output tiles per wave
    __shared__ __align__(16) bf16 Ut[ROWS][LDU];
    __shared__ __align__(16) bf16 Wt[WIDTH][LDU];      // W_l^T, row n holds W_l[:, n]
    __shared__ float ypart[4][ROWS];
    const bf16 *__restrict__ U = s.U[l];
    const int t = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * ROWS;
    // W_l^T: all four 16-byte pieces of this thread in flight at once, stored to
    // LDS only after the neighbour loads below have been issued
    constexpr int WPIECES = WIDTH * (2 * WIDTH / 8) / 256;
    uint4 wv[WPIECES];
    for (int j = 0; j < WPIECES; ++j) {
        const int v = t + 256 * j;
        wv[j] = *(const uint4 *)(s.wt[l] + (v / (2 * WIDTH / 8)) * 2 * WIDTH + (v % (2 * WIDTH / 8)) * 8);
    }
    auto load_w = [&](const bf16 *p, uint32_t *w) {
        if constexpr (NW == 4) {
            const uint4 v = *(const uint4 *)p;
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else {
            const uint2 v = *(const uint2 *)p;
            w[0] = v.x; w[1] = v.y;
        }
    };
    auto store_w = [&](bf16 *p, const uint32_t *w) {
        if constexpr (NW == 4) *(uint4 *)p = make_uint4(w[0], w[1], w[2], w[3]);
        else *(uint2 *)p = make_uint2(w[0], w[1]);
    };
    {
        const int rr = t / TPR, cc = (t % TPR) * CH;
        const int64_t r = row0 + rr;
        uint32_t own[NW] = {}, mean[NW] = {};
        if (r < R) {
            load_w(U + r * 2 * WIDTH + cc, own);
            const int64_t i = r % s.N, base = r - i;
            float acc[CH] = {};
            const int32_t q0 = s.nbr_ptr[i], q1 = s.nbr_ptr[i + 1];
            // eight neighbour rows in flight (more in flight measured no faster on
            // small graphs and, with the registers they take, slower on large ones)
            int32_t q = q0;
            for (; q + 8 <= q1; q += 8) {
                uint32_t w[8][NW];
                for (int u = 0; u < 8; ++u) load_w(U + (base + s.nbr[q + u]) * 2 * WIDTH + cc, w[u]);
                for (int u = 0; u < 8; ++u)
                    for (int k = 0; k < NW; ++k) {
                        acc[2 * k] += bf2f((bf16)(w[u][k] & 0xffffu));
                        acc[2 * k + 1] += bf2f((bf16)(w[u][k] >> 16));
                    }
            }
            for (; q < q1; ++q) {
                uint32_t w[NW];
                load_w(U + (base + s.nbr[q]) * 2 * WIDTH + cc, w);
                for (int k = 0; k < NW; ++k) {
                    acc[2 * k] += bf2f((bf16)(w[k] & 0xffffu));
                    acc[2 * k + 1] += bf2f((bf16)(w[k] >> 16));
                }
            }
            // the mean as a correctly rounded division of the exact FP32 sum (the BF16
            // neighbour values add exactly), so that its BF16 rounding matches that of
            // the exact mean; a product with a rounded 1/deg lands on the other side of
            // a rounding tie, which the repeated values of a mesh make frequent
            const float dg = (float)(q1 - q0);
            for (int k = 0; k < NW; ++k) {
                const float m0 = q1 > q0 ? acc[2 * k] / dg : 0.f, m1 = q1 > q0 ? acc[2 * k + 1] / dg : 0.f;
                mean[k] = (uint32_t)f2bf(m0) | ((uint32_t)f2bf(m1) << 16);
            }
            if (store) store_w(s.U[l] + r * 2 * WIDTH + WIDTH + cc, mean);
        }
        store_w(&Ut[rr][cc], own);
        store_w(&Ut[rr][WIDTH + cc], mean);
    }
    for (int j = 0; j < WPIECES; ++j) {
        const int v = t + 256 * j;
        *(uint4 *)&Wt[v / (2 * WIDTH / 8)][(v % (2 * WIDTH / 8)) * 8] = wv[j];
    }
    __syncthreads();
    constexpr int K = 2 * WIDTH;
    const int wave = t >> 6, lane = t & 63;
    const int ar = lane & 15, kq = (lane >> 4) * 4;
    // 32 rows: wave w takes row tile w & 1 and column tiles 2 (w >> 1), +1;
    // 16 rows: one row tile, wave w takes column tile w
    const int rt = NT == 2 ? (wave & 1) : 0, nt0 = NT == 2 ? (wave >> 1) * 2 : wave;
    f4 acc[NT];
    for (int n = 0; n < NT; ++n) acc[n] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        const s4 a = *(const s4 *)&Ut[rt * 16 + ar][k0 + kq];
        for (int n = 0; n < NT; ++n) {
            const s4 b = *(const s4 *)&Wt[(nt0 + n) * 16 + ar][k0 + kq];
            acc[n] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[n], 0, 0, 0);
        }
    }
    const float *bias = s.params + s.pl.b[l];
    const bool last = l + 1 == s.layers;
    bf16 *hout = last ? s.HL : s.U[l + 1];
    const int ldh = last ? WIDTH : 2 * WIDTH;
    const float *wo = s.params + s.pl.w_out;
    float yp[4] = {0.f, 0.f, 0.f, 0.f};   // last layer: this lane's part of y for rows kq + j
    for (int n = 0; n < NT; ++n) {
        const int col = (nt0 + n) * 16 + ar;
        for (int j = 0; j < 4; ++j) {
            const int rr = rt * 16 + kq + j;
            const int64_t row = row0 + rr;
            const float z = acc[n][j] + bias[col];
            const bf16 hb = f2bf(bf2f(Ut[rr][col]) + (z > 0.f ? z : 0.f));
            yp[j] += bf2f(hb) * wo[col];
            if (row >= R) continue;
            if (store) s.Z[l][row * WIDTH + col] = f2bf(z);
            hout[row * ldh + col] = hb;
        }
    }
    if (last) {
        // y = h_L . w_out + b_out: the 16 lanes holding a row, then the waves holding its columns
        for (int j = 0; j < 4; ++j)
            for (int off = 8; off > 0; off >>= 1) yp[j] += __shfl_xor(yp[j], off, 16);
        constexpr int PARTS = NT == 2 ? 2 : 4;   // waves sharing a row tile
        const int part = NT == 2 ? (wave >> 1) : wave;
        if (ar == 0)
            for (int j = 0; j < 4; ++j) ypart[part][rt * 16 + kq + j] = yp[j];
        __syncthreads();
        if (t < ROWS) {
            const int64_t row = row0 + t;
            float y = 0.f;
            for (int q = 0; q < PARTS; ++q) y += ypart[q][t];
            if (row < R) s.y[row] = y + s.params[s.pl.b_out];
        }
    }
}

// dH[j] += dU[j][:WIDTH] + sum over neighbours i of dU[i][WIDTH:] / deg_i  (transpose of
// the mean; the graph is symmetric).  Sixteen threads per row, four channels each.
__global__ __launch_bounds__(256) void k_aggT(SurDev s, const float *dU, float *dH, int64_t R) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t >> 4;
    const int c4 = (int)(t & 15) * 4;
    if (r >= R) return;
    const int64_t j = r % s.N, base = r - j;
    float4 acc = *(const float4 *)(dH + r * WIDTH + c4);
    const float4 own = *(const float4 *)(dU + r * 2 * WIDTH + c4);
    acc.x += own.x;
    acc.y += own.y;
    acc.z += own.z;
    acc.w += own.w;
    const int32_t q0 = s.nbr_ptr[j], q1 = s.nbr_ptr[j + 1];
    int32_t q = q0;
    for (; q + 4 <= q1; q += 4) {
        float4 v[4];
        float w[4];
        for (int u = 0; u < 4; ++u) {
            const int64_t i = s.nbr[q + u];
            v[u] = *(const float4 *)(dU + (base + i) * 2 * WIDTH + WIDTH + c4);
            w[u] = s.inv_deg[i];
        }
        for (int u = 0; u < 4; ++u) {
            acc.x += v[u].x * w[u];
            acc.y += v[u].y * w[u];
            acc.z += v[u].z * w[u];
            acc.w += v[u].w * w[u];
        }
    }
    for (; q < q1; ++q) {
        const int64_t i = s.nbr[q];
        const float4 v = *(const float4 *)(dU + (base + i) * 2 * WIDTH + WIDTH + c4);
        const float w = s.inv_deg[i];
        acc.x += v.x * w;
        acc.y += v.y * w;
        acc.z += v.z * w;
        acc.w += v.w * w;
    }
    *(float4 *)(dH + r * WIDTH + c4) = acc;
}

// dZ = dH where z > 0, else 0 (BF16)
__global__ __launch_bounds__(256) void k_relu_back(const float *dH, const bf16 *Z, bf16 *dZ, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dZ[k] = bf2f(Z[k]) > 0.f ? f2bf(dH[k]) : (bf16)0;
}

// ---------------------------------------------------------------- energy-neutral correction
// weighted (forward): seg_part[q][g] = (sum w_i v_i, sum w_i) over the nodes i
// of segment g, w_i = m_i mu_i s_i (coef.w times scale); otherwise (backward)
// the plain sum of v in the first slot
__global__ __launch_bounds__(256) void k_seg_sum(SurDev s, const float *v, int weighted) {
    __shared__ double part[2][4];
    const int64_t g = blockIdx.x, q = blockIdx.y;
    const int32_t b = s.seg_begin[g], e = s.seg_begin[g + 1];
    double acc = 0.0, accw = 0.0;
    // four nodes per thread per pass, their loads issued together
    constexpr int U = 4;
    for (int32_t i0 = b + (int32_t)threadIdx.x; i0 < e; i0 += U * (int32_t)blockDim.x) {
        float vv[U], cw[U], sc[U];
        for (int u = 0; u < U; ++u) {
            const int32_t i = i0 + u * (int32_t)blockDim.x;
            const int32_t j = i < e ? i : i0;              // a valid node, not counted below
            vv[u] = v[q * s.N + j];
            cw[u] = weighted ? ((const float4 *)s.coef)[j].w : 1.0f;
            sc[u] = weighted ? s.scale[q * s.N + j] : 1.0f;
        }
        for (int u = 0; u < U; ++u) {
            if (i0 + u * (int32_t)blockDim.x >= e) break;
            if (weighted) {
                const double w = (double)cw[u] * (double)sc[u];
                acc += w * (double)vv[u];
                accw += w;
            } else {
                acc += (double)vv[u];
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_down(acc, off, 64);
        accw += __shfl_down(accw, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = acc;
        part[1][threadIdx.x >> 6] = accw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *o = s.seg_part + 2 * (q * s.n_seg + g);
        o[0] = ((part[0][0] + part[0][1]) + part[0][2]) + part[0][3];
        o[1] = ((part[1][0] + part[1][1]) + part[1][2]) + part[1][3];
    }
}

// the segment partials of every scenario summed in segment order; weighted:
// scen_sum[q][c] = (sum w y / sum w, sum w) (0 for the mean where nothing is
// masked), otherwise the first slot alone takes the plain sum
__global__ void k_scen_sum(SurDev s, int64_t slots, int weighted) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= slots * s.n_scen) return;
    const int64_t q = t / s.n_scen, c = t - q * s.n_scen;
    double acc = 0.0, accw = 0.0;
    for (int32_t k = s.scen_seg_ptr[c]; k < s.scen_seg_ptr[c + 1]; ++k) {
        const double *p = s.seg_part + 2 * (q * s.n_seg + s.scen_seg[k]);
        acc += p[0];
        accw += p[1];
    }
    if (weighted) {
        s.scen_sum[2 * t] = accw > 0.0 ? acc / accw : 0.0;
        s.scen_sum[2 * t + 1] = accw;
    } else {
        s.scen_sum[2 * t] = acc;
    }
}

// forward: y_i -= the weighted mean of y over the node's scenario (sum_i w_i y_i becomes 0)
__global__ __launch_bounds__(256) void k_proj_fwd(SurDev s, int64_t R) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const int64_t q = r / s.N, i = r - q * s.N;
    s.y[r] = (float)((double)s.y[r] - s.scen_sum[2 * (q * s.n_scen + s.scen[i])]);
}

// backward: with g = dL/dy (in y), dL/dy_raw_k = g_k - (w_k / sum w) sum_i g_i into dy,
// and dH = dy_raw w_out.  Sixteen threads per row, four channels each.
__global__ __launch_bounds__(256) void k_proj_bwd(SurDev s, int64_t R) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t >> 4;
    const int c4 = (int)(t & 15) * 4;
    if (r >= R) return;
    const int64_t q = r / s.N, i = r - q * s.N;
    float dy = s.y[r];
    if (s.project) {
        const double *ss = s.scen_sum + 2 * (q * s.n_scen + s.scen[i]);
        const double w = ss[1] > 0.0 ? (double)((const float4 *)s.coef)[i].w * (double)s.scale[r] / ss[1] : 0.0;
        dy = (float)((double)s.y[r] - w * ss[0]);
    }
    if (c4 == 0) s.dy[r] = dy;
    const float4 wo = *(const float4 *)(s.params + s.pl.w_out + c4);
    *(float4 *)(s.dH + r * WIDTH + c4) = make_float4(dy * wo.x, dy * wo.y, dy * wo.z, dy * wo.w);
}

// per row: error e and dL/dy of the loss sum_r e_r^2 / R, with y the projected output.
// LOSS_H: e = y - t.  LOSS_T: e = (T(base + scale y) - T_t) / DT_SCALE, with the
// slope of the branch of T(H) the prediction lies on.  LOSS_HUBER: e = y - t,
// e^2 replaced by delta (2|e| - delta) beyond |e| = delta.
// Writes the per-workgroup loss partial and dL/dy (into y).
__global__ __launch_bounds__(256) void k_loss(SurDev s, int64_t R) {
    __shared__ double part[4];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (r < R) {
        float dy;
        if (s.loss_mode == LOSS_T) {
            const MatDev &M = ((const MatDev *)s.mats)[s.flags[r % s.N] & NODE_MAT_MASK];
            const double Hp = s.base[r] + (double)s.scale[r] * (double)s.y[r];
            double Tp, fsp;
            t_of_h(M, Hp, Tp, fsp);
            const double dTdH = (!M.latent || Hp <= M.Hs || Hp >= M.Hl) ? M.inv_c : M.slope;
            const double e = (Tp - (double)s.target[r]) / DT_SCALE;
            e2 = e * e;
            dy = (float)(2.0 * e / (double)R * dTdH * (double)s.scale[r] / DT_SCALE);
        } else if (!(s.scale[r] > 0.f)) {
            dy = 0.f;                                  // unmasked: the extrapolation stands
        } else if (s.loss_mode == LOSS_HUBER) {
            const float e = s.y[r] - s.target[r], a = fabsf(e);
            e2 = a <= HUBER_DELTA ? (double)e * (double)e : (double)HUBER_DELTA * (2.0 * (double)a - (double)HUBER_DELTA);
            dy = 2.f * fminf(fmaxf(e, -HUBER_DELTA), HUBER_DELTA) / (float)R;
        } else {
            const float e = s.y[r] - s.target[r];
            e2 = (double)e * (double)e;
            dy = 2.f * e / (float)R;
        }
        s.y[r] = dy;
    }
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_down(e2, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) s.loss_part[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
}

// partials of dw_out = sum_r HL[r] dy[r] and db_out = sum_r dy[r] (dy of the unprojected output)
__global__ __launch_bounds__(256) void k_out_grad(SurDev s, int64_t R, float *P) {
    __shared__ float part[4][WIDTH + 1];
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t r_begin = (int64_t)blockIdx.x * GRAD_ROWS;
    const int64_t r_end = std::min<int64_t>(R, r_begin + GRAD_ROWS);
    float acc = 0.f, accb = 0.f;
    for (int64_t r = r_begin + q; r < r_end; r += 4) {
        const float dy = s.dy[r];
        acc += bf2f(s.HL[r * WIDTH + c]) * dy;
        if (c == 0) accb += dy;
    }
    part[q][c] = acc;
    if (c == 0) part[q][WIDTH] = accb;
    __syncthreads();
    if (q == 0) {
        P[(int64_t)blockIdx.x * (WIDTH + 1) + c] = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
        if (c == 0)
            P[(int64_t)blockIdx.x * (WIDTH + 1) + WIDTH] =
                ((part[0][WIDTH] + part[1][WIDTH]) + part[2][WIDTH]) + part[3][WIDTH];
    }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void k_refresh(SurDev s) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const float *p = s.params;
    if (t < WIDTH * KIN) {                                  // W_in^T, zero-padded
        const int c = t / KIN, f = t % KIN;
        s.wt_in[t] = f < NFEAT ? f2bf(p[s.pl.w_in + f * WIDTH + c]) : (bf16)0;
    }
    for (int l = 0; l < s.layers; ++l) {
        if (t < 2 * WIDTH * WIDTH) {
            const int c = t / (2 * WIDTH), k = t % (2 * WIDTH);   // wt[l][c][k] = W_l[k][c]
            s.wt[l][t] = f2bf(p[s.pl.w[l] + k * WIDTH + c]);
            s.wr[l][t] = f2bf(p[s.pl.w[l] + t]);                 // row-major copy
        }
    }
}

__global__ void k_apply(SurDev s, int64_t R, double *H) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) H[r] = s.base[r] + (double)s.scale[r] * (double)s.y[r];
}

// ---------------------------------------------------------------- solver state
// the state's enthalpy into out; with keep, also the node inflow sums into keep
// (the state a rejected jump returns to)
template <class OUT>
__global__ __launch_bounds__(256) void k_state_out(Dev d, OUT *out, double *keep, float2 *pair_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (keep && i < d.n_inflow) keep[i] = d.qnode[i];
    if (i >= d.N) return;
    double h;
    if (d.prec == FEM_PREC_FP64) {
        h = ((const double *)d.H)[i];
    } else {
        const float2 v = ((const float2 *)d.H)[i];
        h = (double)v.x + (double)v.y;
        if (pair_out) pair_out[i] = v;
    }
    out[i] = (OUT)h;
}

// H of a free node := Hn (FP32: hi/lo split of the FP64 value), with T and fs
template <class R>
__device__ __forceinline__ void set_node(const Dev &d, int64_t i, const MatDev &M, double Hn, R *Tc) {
    double T, fs;
    t_of_h(M, Hn, T, fs);
    if constexpr (sizeof(R) == 8) {
        ((double *)d.H)[i] = Hn;
    } else {
        const float hi = (float)Hn;
        ((float2 *)d.H)[i] = make_float2(hi, (float)(Hn - (double)hi));
    }
    Tc[i] = (R)T;
    ((R *)d.fs)[i] = (R)fs;
}

template <class R>
__global__ __launch_bounds__(256) void k_write_jump(SurDev s, Dev d, int parity, float fs_tol) {
    __shared__ int cnt[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i < d.N) {
        const uint32_t f = d.flags[i];
        if (f & NODE_FIXED) {
            s.Hn[i] = s.H2[i];
        } else {
            const MatDev &M = d.mats[f & NODE_MAT_MASK];
            const double ybar = s.project ? s.scen_sum[2 * s.scen[i]] : 0.0;
            const double Hn = s.base[i] + (double)s.scale[i] * ((double)s.y[i] - ybar);
            s.Hn[i] = Hn;
            set_node<R>(d, i, M, Hn, (R *)d.T + parity * d.N);
            if (M.latent) {
                double T0, fs0, T1, fs1;
                t_of_h(M, s.H2[i], T0, fs0);
                t_of_h(M, Hn, T1, fs1);
                bad = (fs1 < fs0 - (double)fs_tol || !(Hn == Hn)) ? 1 : 0;
            } else {
                bad = !(Hn == Hn) ? 1 : 0;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = bad;
    __syncthreads();
    if (threadIdx.x == 0) s.check[blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

template <class R>
__global__ __launch_bounds__(256) void k_restore(SurDev s, Dev d, int parity, const double *kept_qnode) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kept_qnode && i < d.n_inflow) d.qnode[i] = kept_qnode[i];
    if (i >= d.N) return;
    const uint32_t f = d.flags[i];
    if (f & NODE_FIXED) return;
    const MatDev &M = d.mats[f & NODE_MAT_MASK];
    if (sizeof(R) == 4 && s.H2_pair) {
        // the saved pair itself, with T and f_s evaluated as the step does
        const float2 v = s.H2_pair[i];
        ((float2 *)d.H)[i] = v;
        double T, fs;
        t_of_h(M, (double)v.x + (double)v.y, T, fs);
        ((R *)d.T)[parity * d.N + i] = (R)T;
        ((R *)d.fs)[i] = (R)fs;
    } else {
        set_node<R>(d, i, M, s.H2[i], (R *)d.T + parity * d.N);
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_verify(SurDev s, Dev d, float tol) {
    __shared__ int cnt[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (i < d.N) {
        const uint32_t f = d.flags[i];
        if (!(f & NODE_FIXED)) {
            const MatDev &M = d.mats[f & NODE_MAT_MASK];
            double H;
            if constexpr (sizeof(R) == 8) {
                H = ((const double *)d.H)[i];
            } else {
                const float2 v = ((const float2 *)d.H)[i];
                H = (double)v.x + (double)v.y;
            }
            const double Hp = s.Hn[i];
            const double dTdH = (!M.latent || Hp <= M.Hs || Hp >= M.Hl) ? M.inv_c : M.slope;
            const double dev = dTdH * fabs((H - Hp) - s.rext[i]);
            bad = (dev > (double)tol || !(dev == dev)) ? 1 : 0;
        }
    }
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = bad;
    __syncthreads();
    if (threadIdx.x == 0) s.check[check_blocks(d.N) + blockIdx.x] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

inline unsigned grid_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t features(const SurDev &s, const void *H0, const void *H1, const void *H2, int h_is_double,
                    const float *Ht, int64_t stride, const int32_t *idx, int64_t slots, hipStream_t st) {
    const unsigned g = grid_for(slots * s.N, 256);
    if (h_is_double)
        hipLaunchKernelGGL(k_features<double>, dim3(g), dim3(256), 0, st, s, (const double *)H0, (const double *)H1,
                           (const double *)H2, Ht, stride, idx, slots);
    else
        hipLaunchKernelGGL(k_features<float>, dim3(g), dim3(256), 0, st, s, (const float *)H0, (const float *)H1,
                           (const float *)H2, Ht, stride, idx, slots);
    return hipGetLastError();
}

hipError_t features_live(const SurDev &s, const Dev &d, const double *H0, const double *H1, double *keep_qnode,
                         hipStream_t st) {
    const int64_t n = keep_qnode ? std::max<int64_t>(s.N, d.n_inflow) : s.N;
    if (d.prec == FEM_PREC_FP64)
        hipLaunchKernelGGL(k_features_live<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, s, d, H0, H1, keep_qnode);
    else
        hipLaunchKernelGGL(k_features_live<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, s, d, H0, H1, keep_qnode);
    return hipGetLastError();
}

hipError_t forward(const SurDev &s, int64_t R, int store, int project, hipStream_t st) {
    const unsigned g = grid_for(R, 64);
    // encoder into the first half of U_0
    hipLaunchKernelGGL((k_gemm<WIDTH, 0>), dim3(g), dim3(256), 0, st, s.X, KIN, KIN, s.wt_in,
                       s.params + s.pl.b_in, R, store ? s.Zin : (bf16 *)nullptr, (const bf16 *)nullptr, 0, s.U[0],
                       2 * WIDTH, (float *)nullptr, 0);
    if (R <= LAYER_SMALL_MAX) {
        const unsigned gl = grid_for(R, LAYER_ROWS_SMALL);
        for (int l = 0; l < s.layers; ++l)
            hipLaunchKernelGGL(k_layer<LAYER_ROWS_SMALL>, dim3(gl), dim3(256), 0, st, s, l, R, store);
    } else {
        const unsigned gl = grid_for(R, LAYER_ROWS);
        for (int l = 0; l < s.layers; ++l)
            hipLaunchKernelGGL(k_layer<LAYER_ROWS>, dim3(gl), dim3(256), 0, st, s, l, R, store);
    }
    if (!s.project) return hipGetLastError();
    const int64_t slots = R / s.N;
    hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)s.n_seg, (unsigned)slots), dim3(256), 0, st, s, (const float *)s.y, 1);
    hipLaunchKernelGGL(k_scen_sum, dim3(grid_for(slots * s.n_scen, 256)), dim3(256), 0, st, s, slots, 1);
    if (project) hipLaunchKernelGGL(k_proj_fwd, dim3(grid_for(R, 256)), dim3(256), 0, st, s, R);
    return hipGetLastError();
}

hipError_t loss_and_dy(const SurDev &s, int64_t R, hipStream_t st) {
    hipLaunchKernelGGL(k_loss, dim3(grid_for(R, 256)), dim3(256), 0, st, s, R);
    const int64_t slots = R / s.N;
    if (s.project) {
        hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)s.n_seg, (unsigned)slots), dim3(256), 0, st, s, (const float *)s.y, 0);
        hipLaunchKernelGGL(k_scen_sum, dim3(grid_for(slots * s.n_scen, 256)), dim3(256), 0, st, s, slots, 0);
    }
    hipLaunchKernelGGL(k_proj_bwd, dim3(grid_for(R * 16, 256)), dim3(256), 0, st, s, R);
    return hipGetLastError();
}

// deterministic two-pass sum of nblk workgroup partials into out[0..keep)
static void reduce_partials(const SurDev &s, const float *P, int64_t nblk, int64_t per, int keep, float *out,
                            hipStream_t st) {
    const int64_t ng = (nblk + PARTIAL_GROUP - 1) / PARTIAL_GROUP;
    hipLaunchKernelGGL(k_reduce_groups, dim3(grid_for(keep, 256), (unsigned)ng), dim3(256), 0, st, P, nblk, per, keep,
                       s.partials2);
    hipLaunchKernelGGL(k_reduce_final, dim3(grid_for(keep, 256)), dim3(256), 0, st, (const float *)s.partials2, ng,
                       keep, out);
}

hipError_t backward(const SurDev &s, int64_t R, hipStream_t st) {
    const int64_t nb = (R + GRAD_ROWS - 1) / GRAD_ROWS;
    float *P = s.partials;                                             // nb x 2 WIDTH x WIDTH
    float *Pb = s.partials + s.n_partial_blocks * 2 * WIDTH * WIDTH;   // nb x WIDTH
    // output layer
    hipLaunchKernelGGL(k_out_grad, dim3((unsigned)nb), dim3(256), 0, st, s, R, P);
    reduce_partials(s, P, nb, WIDTH + 1, WIDTH + 1, s.grads + s.pl.w_out, st);
    for (int l = s.layers - 1; l >= 0; --l) {
        hipLaunchKernelGGL(k_relu_back, dim3(grid_for(R * WIDTH, 256)), dim3(256), 0, st, s.dH, s.Z[l], s.dZ,
                           R * WIDTH);
        hipLaunchKernelGGL((k_wgrad<2 * WIDTH>), dim3((unsigned)nb), dim3(256), 0, st, s.U[l], 2 * WIDTH, s.dZ, R, P, Pb);
        reduce_partials(s, P, nb, 2 * WIDTH * WIDTH, 2 * WIDTH * WIDTH, s.grads + s.pl.w[l], st);
        reduce_partials(s, Pb, nb, WIDTH, WIDTH, s.grads + s.pl.b[l], st);
        hipLaunchKernelGGL((k_gemm<2 * WIDTH, 2>), dim3(grid_for(R, 64)), dim3(256), 0, st, s.dZ, WIDTH, WIDTH,
                           s.wr[l], (const float *)nullptr, R, (bf16 *)nullptr, (const bf16 *)nullptr, 0,
                           (bf16 *)nullptr, 0, s.dU, 2 * WIDTH);
        hipLaunchKernelGGL(k_aggT, dim3(grid_for(R * 16, 256)), dim3(256), 0, st, s, s.dU, s.dH, R);
    }
    // encoder
    hipLaunchKernelGGL(k_relu_back, dim3(grid_for(R * WIDTH, 256)), dim3(256), 0, st, s.dH, s.Zin, s.dZ, R * WIDTH);
    hipLaunchKernelGGL((k_wgrad<KIN>), dim3((unsigned)nb), dim3(256), 0, st, s.X, KIN, s.dZ, R, P, Pb);
    reduce_partials(s, P, nb, KIN * WIDTH, NFEAT * WIDTH, s.grads + s.pl.w_in, st);
    reduce_partials(s, Pb, nb, WIDTH, WIDTH, s.grads + s.pl.b_in, st);
    return hipGetLastError();
}

hipError_t adam(const SurDev &s, float lr, float b1, float b2, float eps, int step, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(s.pl.total, 256)), dim3(256), 0, st, s.params, s.grads, s.adam_m,
                       s.adam_v, s.pl.total, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t refresh_bf16(const SurDev &s, hipStream_t st) {
    hipLaunchKernelGGL(k_refresh, dim3(grid_for(2 * WIDTH * WIDTH, 256)), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t apply(const SurDev &s, int64_t R, double *H_out, hipStream_t st) {
    hipLaunchKernelGGL(k_apply, dim3(grid_for(R, 256)), dim3(256), 0, st, s, R, H_out);
    return hipGetLastError();
}

hipError_t state_to_f64(const Dev &d, double *out, double *keep_qnode, hipStream_t st, float2 *pair_out) {
    const int64_t n = keep_qnode ? std::max<int64_t>(d.N, d.n_inflow) : d.N;
    hipLaunchKernelGGL(k_state_out<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, d, out, keep_qnode, pair_out);
    return hipGetLastError();
}

hipError_t state_to_f32(const Dev &d, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_state_out<float>, dim3(grid_for(d.N, 256)), dim3(256), 0, st, d, out, (double *)nullptr,
                       (float2 *)nullptr);
    return hipGetLastError();
}

hipError_t write_jump(const SurDev &s, const Dev &d, int parity, float fs_tol, hipStream_t st) {
    const dim3 g((unsigned)check_blocks(d.N));
    if (d.prec == FEM_PREC_FP64)
        hipLaunchKernelGGL(k_write_jump<double>, g, dim3(256), 0, st, s, d, parity, fs_tol);
    else
        hipLaunchKernelGGL(k_write_jump<float>, g, dim3(256), 0, st, s, d, parity, fs_tol);
    return hipGetLastError();
}

hipError_t verify_jump(const SurDev &s, const Dev &d, float tol, hipStream_t st) {
    const dim3 g((unsigned)check_blocks(d.N));
    if (d.prec == FEM_PREC_FP64) hipLaunchKernelGGL(k_verify<double>, g, dim3(256), 0, st, s, d, tol);
    else hipLaunchKernelGGL(k_verify<float>, g, dim3(256), 0, st, s, d, tol);
    return hipGetLastError();
}

hipError_t restore_h2(const SurDev &s, const Dev &d, int parity, const double *kept_qnode, hipStream_t st) {
    const int64_t n = kept_qnode ? std::max<int64_t>(d.N, d.n_inflow) : d.N;
    const dim3 g((unsigned)grid_for(n, 256));
    if (d.prec == FEM_PREC_FP64)
        hipLaunchKernelGGL(k_restore<double>, g, dim3(256), 0, st, s, d, parity, kept_qnode);
    else
        hipLaunchKernelGGL(k_restore<float>, g, dim3(256), 0, st, s, d, parity, kept_qnode);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace castfem
