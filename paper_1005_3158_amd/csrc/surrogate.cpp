// C interface of the learned surrogate: device buffers, parameters, training
// on device-resident solver states, prediction, and the accelerated advance
// that checks every jump in FP64 and falls back to plain explicit steps.
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "surrogate.hpp"

using namespace castfem;
using namespace castfem::sur;

namespace {

enum SBuf {
    S_NBR_PTR, S_NBR, S_INV_DEG, S_COEF, S_PARAMS, S_GRADS, S_ADAM_M, S_ADAM_V, S_WBF, S_X, S_ZIN, S_U, S_Z,
    S_HL, S_Y, S_BASE, S_SCALE, S_TARGET, S_DH, S_DZ, S_DU, S_PARTIALS, S_LOSS, S_IDX, S_PARTIALS2, S_DY, S_H0, S_H1, S_H2, S_HN, S_REXT, S_QSAVE, S_CHECK,
    S_SCEN, S_SCEN_SEG_PTR, S_SCEN_SEG, S_SEG_PART, S_SCEN_SUM, S_H2_PAIR, S_COUNT
};
const char *const SBUF_NAMES[S_COUNT] = {"nbr_ptr", "nbr", "inv_deg", "coef", "params", "grads", "adam_m",
                                         "adam_v", "weights_bf16", "X", "Z_in", "U", "Z", "H_last", "y",
                                         "base", "scale", "target", "dH", "dZ", "dU", "partials", "loss_part",
                                         "sample_idx", "partials2", "dy", "H0", "H1", "H2", "H_pred", "r_ext", "q_saved", "check", "scenario",
                                         "scen_seg_ptr", "scen_seg", "seg_part", "scen_sum", "H2_pair"};

// counter-based generator (SplitMix64 of seed and counter) for the
// initial parameters and the sample shuffles
inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
inline double unit(uint64_t seed, uint64_t stream, uint64_t k) {
    return ((mix64(mix64(seed ^ (stream * 0xD1B54A32D192ED03ull)) + k) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
inline double normal(uint64_t seed, uint64_t stream, uint64_t k) {   // Box-Muller
    const double u1 = unit(seed, stream, 2 * k), u2 = unit(seed, stream, 2 * k + 1);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

}  // namespace

struct fem_sur {
    fem_ctx *ctx = nullptr;
    fem_sur_options opt{};
    int64_t N = 0, rows = 0, nnz = 0, nb = 0;
    ParamLayout pl;
    std::vector<int32_t> nbr_ptr, nbr;
    std::vector<float> inv_deg, coef;
    std::vector<int32_t> scen, scen_seg_ptr, scen_seg;
    int64_t n_seg = 0, n_scen = 1;
    int64_t sizes[S_COUNT] = {};
    void *ptr[S_COUNT] = {};
    bool bound = false;
    SurDev d;
    int adam_t = 0;
    // captured graphs of the accelerated advance, per starting T parity: a
    // jump chunk from a fresh state, a jump chunk continuing after a kept
    // jump, and the horizon - 2 fallback steps
    hipGraph_t graph[3][2] = {};
    hipGraphExec_t exec[3][2] = {};
    float graph_fs_tol = -1.0f, graph_verify_tol = -1.0f;
    ~fem_sur() {
        for (auto &row : exec)
            for (hipGraphExec_t &e : row)
                if (e) (void)hipGraphExecDestroy(e);
        for (auto &row : graph)
            for (hipGraph_t &g : row)
                if (g) (void)hipGraphDestroy(g);
    }
};

namespace {

int64_t aligned(int64_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

void sur_sizes(fem_sur *s) {
    const int64_t N = s->N, R = s->rows, W = WIDTH, L = s->opt.layers, P = s->pl.total;
    const bool tr = s->opt.train != 0;
    int64_t *z = s->sizes;
    std::fill(z, z + S_COUNT, 0);
    z[S_NBR_PTR] = (N + 1) * 4;
    z[S_NBR] = s->nnz * 4;
    z[S_INV_DEG] = N * 4;
    z[S_COEF] = N * 16;
    z[S_PARAMS] = P * 4;
    z[S_WBF] = (W * KIN + L * 2 * (2 * W * W)) * 2;
    z[S_X] = R * KIN * 2;
    z[S_ZIN] = R * W * 2;
    z[S_U] = L * R * 2 * W * 2;
    z[S_Z] = L * R * W * 2;
    z[S_HL] = R * W * 2;
    z[S_Y] = R * 4;
    z[S_BASE] = R * 8;
    z[S_SCALE] = R * 4;
    z[S_H0] = N * 8;
    z[S_H1] = N * 8;
    z[S_H2] = N * 8;
    z[S_HN] = N * 8;
    z[S_REXT] = N * 8;
    z[S_QSAVE] = s->ctx->L().n_inflow * 8;
    // FP32 state: the raw (hi, lo) enthalpy pairs at H2, so that a rejected jump
    // returns to exactly that state (hi + lo can need more than the 53 bits of
    // the FP64 copy in H2)
    z[S_H2_PAIR] = s->ctx->opt.precision == FEM_PREC_FP64 ? 0 : N * 8;
    z[S_CHECK] = 2 * check_blocks(N) * 4;
    z[S_SCEN] = N * 4;
    z[S_SCEN_SEG_PTR] = (s->n_scen + 1) * 4;
    z[S_SCEN_SEG] = s->n_seg * 4;
    z[S_SEG_PART] = (int64_t)s->opt.max_samples * s->n_seg * 16;
    z[S_SCEN_SUM] = (int64_t)s->opt.max_samples * s->n_scen * 16;
    if (tr) {
        z[S_GRADS] = P * 4;
        z[S_ADAM_M] = P * 4;
        z[S_ADAM_V] = P * 4;
        z[S_TARGET] = R * 4;
        z[S_DH] = R * W * 4;
        z[S_DZ] = R * W * 2;
        z[S_DU] = R * 2 * W * 4;
        z[S_PARTIALS] = s->nb * (2 * W * W + W) * 4;
        z[S_LOSS] = ((R + 255) / 256) * 8;
        z[S_IDX] = (int64_t)s->opt.max_samples * 4;
        z[S_PARTIALS2] = ((s->nb + PARTIAL_GROUP - 1) / PARTIAL_GROUP) * (2 * W * W) * 4;
        z[S_DY] = R * 4;
    }
}

// mesh neighbours (nodes sharing an element) in device numbering, as CSR
void build_graph(fem_sur *s) {
    const Layout &L = s->ctx->L();
    const int64_t N = L.N, E = L.E;
    const int nen = L.nen;
    std::vector<int64_t> cnt(N + 1, 0);
    for (int64_t k = 0; k < E * nen; ++k) ++cnt[L.conn[k] + 1];
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    std::vector<int64_t> inc(E * nen);
    {
        std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
        for (int64_t k = 0; k < E * nen; ++k) inc[at[L.conn[k]]++] = k / nen;
    }
    std::vector<std::vector<int32_t>> nb(N);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < N; ++i) {
        std::vector<int32_t> &v = nb[i];
        for (int64_t q = cnt[i]; q < cnt[i + 1]; ++q)
            for (int a = 0; a < nen; ++a) {
                const int32_t j = L.conn[inc[q] * nen + a];
                if (j != i) v.push_back(j);
            }
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    s->nbr_ptr.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) s->nbr_ptr[i + 1] = s->nbr_ptr[i] + (int32_t)nb[i].size();
    s->nnz = s->nbr_ptr[N];
    s->nbr.resize(s->nnz);
    s->inv_deg.resize(N);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        std::copy(nb[i].begin(), nb[i].end(), s->nbr.begin() + s->nbr_ptr[i]);
        s->inv_deg[i] = nb[i].empty() ? 0.0f : 1.0f / (float)nb[i].size();
    }
}

// per-node strengths over m_i c_i (Robin, interface, conduction), the scenario
// of every node and its lumped mass over the sum of its scenario's free nodes
// (the mass part of the projection weight m_i mu_i s_i)
void build_coef(fem_sur *s) {
    const fem_ctx *c = s->ctx;
    const Layout &L = c->L();
    const Base &b = c->base;
    const int32_t ns = c->prob.n_scen;
    s->coef.assign(L.N * 4, 0.0f);
    s->scen.assign(L.N, 0);
    std::vector<double> tot(ns, 0.0);
    for (int64_t g = 0; g < L.N; ++g) {
        const int32_t o = L.iperm[g];
        const double mc = b.m[o] * c->prob.mats[b.nmat[o]].c;
        double wl = 0.0;
        for (int32_t k = b.lptr[o]; k < b.lptr[o + 1]; ++k) wl += b.lw[k];
        s->coef[4 * g + 0] = (float)(b.robin_b[o] / mc);
        s->coef[4 * g + 1] = (float)(2.0 * wl / mc);
        s->coef[4 * g + 2] = (float)(b.kabs[o] / mc);
        s->scen[g] = c->prob.scen_of_mat(b.nmat[o]);
        if (!(L.nflag[g] & NODE_FIXED)) tot[s->scen[g]] += b.m[o];
    }
    for (int64_t g = 0; g < L.N; ++g) {
        const double t = tot[s->scen[g]];
        s->coef[4 * g + 3] = (L.nflag[g] & NODE_FIXED) || !(t > 0) ? 0.0f : (float)(b.m[L.iperm[g]] / t);
    }
    // segments of every scenario (the context's single-scenario node segments)
    s->n_seg = (int64_t)L.seg_scen.size();
    s->n_scen = ns;
    s->scen_seg_ptr.assign(ns + 1, 0);
    for (int32_t sc : L.seg_scen) ++s->scen_seg_ptr[sc + 1];
    for (int32_t k = 0; k < ns; ++k) s->scen_seg_ptr[k + 1] += s->scen_seg_ptr[k];
    s->scen_seg.resize(s->n_seg);
    std::vector<int32_t> at(s->scen_seg_ptr.begin(), s->scen_seg_ptr.end() - 1);
    for (int64_t g = 0; g < s->n_seg; ++g) s->scen_seg[at[L.seg_scen[g]]++] = (int32_t)g;
}

void init_params(fem_sur *s, std::vector<float> &p) {
    const ParamLayout &pl = s->pl;
    const uint64_t seed = s->opt.seed;
    p.assign(pl.total, 0.0f);
    const double s_in = std::sqrt(2.0 / NFEAT), s_l = std::sqrt(1.0 / (2 * WIDTH));
    for (int64_t k = 0; k < NFEAT * WIDTH; ++k) p[pl.w_in + k] = (float)(s_in * normal(seed, 1, k));
    for (int l = 0; l < pl.layers; ++l)
        for (int64_t k = 0; k < 2 * WIDTH * WIDTH; ++k) p[pl.w[l] + k] = (float)(s_l * normal(seed, 2 + l, k));
    // w_out = 0, b_out = 0: an untrained network predicts the extrapolation itself
}

void fill_surdev(fem_sur *s) {
    SurDev &d = s->d;
    fem_ctx *c = s->ctx;
    const int64_t R = s->rows, W = WIDTH;
    d = SurDev{};
    d.N = s->N;
    d.layers = s->opt.layers;
    d.horizon = s->opt.horizon;
    d.loss_mode = s->opt.loss;
    d.project = s->opt.no_projection ? 0 : 1;
    d.quadratic = s->opt.extrapolation == FEM_SUR_EXTRAP_QUADRATIC ? 1 : 0;
    d.pl = s->pl;
    d.nbr_ptr = (const int32_t *)s->ptr[S_NBR_PTR];
    d.nbr = (const int32_t *)s->ptr[S_NBR];
    d.inv_deg = (const float *)s->ptr[S_INV_DEG];
    d.coef = (const float *)s->ptr[S_COEF];
    d.flags = (const uint32_t *)c->ptr[B_FLAGS];
    d.mats = c->ptr[B_MATS];
    d.params = (float *)s->ptr[S_PARAMS];
    d.grads = (float *)s->ptr[S_GRADS];
    d.adam_m = (float *)s->ptr[S_ADAM_M];
    d.adam_v = (float *)s->ptr[S_ADAM_V];
    bf16 *wb = (bf16 *)s->ptr[S_WBF];
    d.wt_in = wb;
    wb += W * KIN;
    for (int l = 0; l < d.layers; ++l) {
        d.wt[l] = wb;
        wb += 2 * W * W;
        d.wr[l] = wb;
        wb += 2 * W * W;
    }
    d.rows = R;
    d.X = (bf16 *)s->ptr[S_X];
    d.Zin = (bf16 *)s->ptr[S_ZIN];
    for (int l = 0; l < d.layers; ++l) {
        d.U[l] = (bf16 *)s->ptr[S_U] + l * R * 2 * W;
        d.Z[l] = (bf16 *)s->ptr[S_Z] + l * R * W;
    }
    d.HL = (bf16 *)s->ptr[S_HL];
    d.y = (float *)s->ptr[S_Y];
    d.base = (double *)s->ptr[S_BASE];
    d.scale = (float *)s->ptr[S_SCALE];
    d.target = (float *)s->ptr[S_TARGET];
    d.dH = (float *)s->ptr[S_DH];
    d.dZ = (bf16 *)s->ptr[S_DZ];
    d.dU = (float *)s->ptr[S_DU];
    d.partials = (float *)s->ptr[S_PARTIALS];
    d.partials2 = (float *)s->ptr[S_PARTIALS2];
    d.dy = (float *)s->ptr[S_DY];
    d.n_partial_blocks = s->nb;
    d.loss_part = (double *)s->ptr[S_LOSS];
    d.H0 = (double *)s->ptr[S_H0];
    d.H1 = (double *)s->ptr[S_H1];
    d.H2 = (double *)s->ptr[S_H2];
    d.H2_pair = (float2 *)s->ptr[S_H2_PAIR];
    d.Hn = (double *)s->ptr[S_HN];
    d.rext = (double *)s->ptr[S_REXT];
    d.check = (int32_t *)s->ptr[S_CHECK];
    d.scen = (const int32_t *)s->ptr[S_SCEN];
    d.seg_begin = (const int32_t *)c->ptr[B_SEG];
    d.n_seg = s->n_seg;
    d.n_scen = s->n_scen;
    d.scen_seg_ptr = (const int32_t *)s->ptr[S_SCEN_SEG_PTR];
    d.scen_seg = (const int32_t *)s->ptr[S_SCEN_SEG];
    d.seg_part = (double *)s->ptr[S_SEG_PART];
    d.scen_sum = (double *)s->ptr[S_SCEN_SUM];
}

void need_bound(const fem_sur *s) {
    if (!s->bound) throw PrepError{FEM_E_STATE, "call fem_sur_bind_buffers first"};
}
void need_train(const fem_sur *s) {
    need_bound(s);
    if (!s->opt.train) throw PrepError{FEM_E_STATE, "the surrogate was created without training buffers"};
}
void check_slots(const fem_sur *s, int64_t slots) {
    if (slots < 1 || slots > s->opt.max_samples)
        throw PrepError{FEM_E_INVALID_ARG, "between 1 and max_samples states per call"};
}

void upload_params(fem_sur *s, const float *p) {
    HIPCHECK(hipMemcpyAsync(s->ptr[S_PARAMS], p, s->pl.total * 4, hipMemcpyHostToDevice, s->ctx->stream));
    HIPCHECK(refresh_bf16(s->d, s->ctx->stream));
    HIPCHECK(hipStreamSynchronize(s->ctx->stream));
}

// one forward and backward pass over `slots` states; loss partials left on the device
void pass(fem_sur *s, const float *H0, const float *H1, const float *H2, const float *Ht, int64_t stride,
          const int32_t *idx, int64_t slots) {
    hipStream_t st = s->ctx->stream;
    const int64_t R = slots * s->N;
    HIPCHECK(features(s->d, H0, H1, H2, 0, Ht, stride, idx, slots, st));
    HIPCHECK(forward(s->d, R, 1, 1, st));
    HIPCHECK(loss_and_dy(s->d, R, st));
    HIPCHECK(backward(s->d, R, st));
}

double loss_of(fem_sur *s, int64_t R) {
    const int64_t nl = (R + 255) / 256;
    std::vector<double> lp(nl);
    HIPCHECK(hipMemcpyAsync(lp.data(), s->ptr[S_LOSS], nl * 8, hipMemcpyDeviceToHost, s->ctx->stream));
    HIPCHECK(hipStreamSynchronize(s->ctx->stream));
    double sum = 0.0;
    for (double v : lp) sum += v;
    return sum / (double)R;
}

enum ChunkKind { CHUNK_FRESH = 0, CHUNK_FALLBACK = 1, CHUNK_CONT = 2 };

// work of one jump chunk from T parity p.
// Fresh (the state is H^n): H0 = H^n, step, H1, step, H2.  Continued (the
// previous jump was kept, the state is H^{n+1} and s.Hn holds H^n): H0 = s.Hn,
// H1 = the state, step, H2.  Then inference, the jump written into the state
// with its f_s check, one explicit step from the prediction and its
// verification, and the state diagnostics of the result.
void enqueue_jump(fem_sur *s, int p, bool cont, float fs_tol, float verify_tol) {
    fem_ctx *c = s->ctx;
    hipStream_t st = c->stream;
    int q = p;
    if (!cont) {
        HIPCHECK(state_to_f64(c->dev, s->d.H0, nullptr, st));
        HIPCHECK(enqueue_step(c->dev, q, st, nullptr));
        q ^= 1;
    }
    HIPCHECK(state_to_f64(c->dev, s->d.H1, nullptr, st));
    HIPCHECK(enqueue_step(c->dev, q, st, nullptr));
    q ^= 1;
    // features from the state H2 itself, which the same kernel keeps (with the
    // inflow sums at H2) for a fallback to start from
    HIPCHECK(features_live(s->d, c->dev, cont ? s->d.Hn : s->d.H0, s->d.H1,
                           c->L().n_inflow ? (double *)s->ptr[S_QSAVE] : nullptr, st));
    HIPCHECK(forward(s->d, s->N, 0, 0, st));
    HIPCHECK(write_jump(s->d, c->dev, q, fs_tol, st));
    HIPCHECK(enqueue_step(c->dev, q, st, nullptr));
    q ^= 1;
    HIPCHECK(verify_jump(s->d, c->dev, verify_tol, st));
    HIPCHECK(enqueue_state_diag(c->dev, q, st));
}

// the fallback of a rejected jump: back to H2 (T parity p), then horizon - 2 explicit steps
void enqueue_fallback(fem_sur *s, int p) {
    fem_ctx *c = s->ctx;
    HIPCHECK(restore_h2(s->d, c->dev, p, c->L().n_inflow ? (const double *)s->ptr[S_QSAVE] : nullptr, c->stream));
    for (int k = 0; k < s->opt.horizon - 2; ++k) HIPCHECK(enqueue_step(c->dev, p ^ (k & 1), c->stream, nullptr));
}

void drop_graph(fem_sur *s, int what, int p) {
    if (s->exec[what][p]) HIPCHECK(hipGraphExecDestroy(s->exec[what][p]));
    if (s->graph[what][p]) HIPCHECK(hipGraphDestroy(s->graph[what][p]));
    s->exec[what][p] = nullptr;
    s->graph[what][p] = nullptr;
}

// run a chunk of kind `what` from parity p through a graph captured on first use
void run_chunk(fem_sur *s, int what, int p, float fs_tol, float verify_tol) {
    fem_ctx *c = s->ctx;
    c->diag_fresh = false;
    auto enqueue = [&] {
        if (what == CHUNK_FALLBACK) enqueue_fallback(s, p);
        else enqueue_jump(s, p, what == CHUNK_CONT, fs_tol, verify_tol);
    };
    if (!c->stream) {                       // the null stream cannot be captured
        enqueue();
        return;
    }
    if (fs_tol != s->graph_fs_tol || verify_tol != s->graph_verify_tol) {   // tolerances are kernel arguments
        for (int q = 0; q < 2; ++q) {
            drop_graph(s, CHUNK_FRESH, q);
            drop_graph(s, CHUNK_CONT, q);
        }
        s->graph_fs_tol = fs_tol;
        s->graph_verify_tol = verify_tol;
    }
    if (!s->exec[what][p]) {
        HIPCHECK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        std::string err;
        try {
            enqueue();
        } catch (const PrepError &e) {
            err = e.msg;
        }
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (!err.empty()) {
            if (g) (void)hipGraphDestroy(g);
            throw PrepError{FEM_E_HIP, err};
        }
        HIPCHECK(e2);
        s->graph[what][p] = g;
        HIPCHECK(hipGraphInstantiate(&s->exec[what][p], g, nullptr, nullptr, 0));
    }
    HIPCHECK(hipGraphLaunch(s->exec[what][p], c->stream));
}

// page-locked staging of the per-chunk read-back (check counts, state
// diagnostics, inflow sums), written by one device kernel: one launch and one
// stream synchronisation per check
struct Staging {
    void *p = nullptr;
    char *dev = nullptr;                  // the same memory as the device addresses it
    size_t n_chk = 0, n_dg = 0, n_qn = 0; // element counts
    size_t off_dg = 0, off_qn = 0;        // 16-byte aligned byte offsets
    Staging(size_t chk_count, size_t dg_count, size_t qn_count) : n_chk(chk_count), n_dg(dg_count), n_qn(qn_count) {
        auto up16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
        off_dg = up16(n_chk * 4);
        off_qn = off_dg + up16(n_dg * 8);
        const size_t bytes = std::max<size_t>(off_qn + up16(n_qn * 8), 64);
        HIPCHECK(hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocCoherent));
        void *d = nullptr;
        const hipError_t e = hipHostGetDevicePointer(&d, p, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(p);
            p = nullptr;
            HIPCHECK(e);
        }
        dev = (char *)d;
    }
    ~Staging() {
        if (p) (void)hipHostFree(p);
    }
    const int32_t *chk() const { return (const int32_t *)p; }
    const double *dg() const { return (const double *)((const char *)p + off_dg); }
    const double *qn() const { return (const double *)((const char *)p + off_qn); }
};

// enqueue the staging of the state diagnostics and inflow sums of ctx (and the
// check counts of s, if any)
void stage_copies(fem_ctx *ctx, fem_sur *s, Staging &sg) {
    const bool chk = s && sg.n_chk;
    HIPCHECK(enqueue_stage((int32_t *)sg.dev, chk ? (const int32_t *)s->ptr[S_CHECK] : nullptr, chk ? sg.n_chk : 0,
                           (double *)(sg.dev + sg.off_dg), (const double *)ctx->ptr[B_DIAG], sg.n_dg,
                           (double *)(sg.dev + sg.off_qn), (const double *)ctx->ptr[B_QNODE], sg.n_qn, ctx->stream));
}

// after a stream sync: the per-scenario energy reports from the staged values
void staged_energy(fem_ctx *ctx, Staging &sg, std::vector<double> &dg, std::vector<double> &qn,
                   fem_energy_report *er) {
    dg.assign(sg.dg(), sg.dg() + sg.n_dg);
    qn.assign(sg.qn(), sg.qn() + sg.n_qn);
    energy_reduce(ctx, dg, qn, er);
}

// FP32 parameters into the surrogate (BF16 copies refreshed), Adam moments cleared
void set_params(fem_sur *s, const float *host, int64_t n) {
    need_bound(s);
    if (n != s->pl.total) throw PrepError{FEM_E_INVALID_ARG, "parameter count mismatch"};
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(host[k])) throw PrepError{FEM_E_INVALID_ARG, "parameters must be finite"};
    upload_params(s, host);
    s->adam_t = 0;
    if (s->opt.train) {
        HIPCHECK(hipMemsetAsync(s->ptr[S_ADAM_M], 0, s->sizes[S_ADAM_M], s->ctx->stream));
        HIPCHECK(hipMemsetAsync(s->ptr[S_ADAM_V], 0, s->sizes[S_ADAM_V], s->ctx->stream));
        HIPCHECK(hipStreamSynchronize(s->ctx->stream));
    }
}

// parameter file: this header, then n_params FP32 values (host byte order)
struct ParamFileHeader {
    char magic[8];
    int32_t width, layers, horizon, extrapolation;
    int64_t n_params;
};
ParamFileHeader file_header(const fem_sur *s) {
    ParamFileHeader h{};
    std::memcpy(h.magic, "CASTSUR1", 8);
    h.width = s->opt.width;
    h.layers = s->opt.layers;
    h.horizon = s->opt.horizon;
    h.extrapolation = s->opt.extrapolation;
    h.n_params = s->pl.total;
    return h;
}

}  // namespace

extern "C" {

int fem_sur_create(fem_sur **out, fem_ctx *ctx, const fem_sur_options *o) {
    if (!out || !ctx || !o) return set_err(FEM_E_INVALID_ARG, "null argument");
    *out = nullptr;
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (ctx->apparent()) throw PrepError{FEM_E_UNSUPPORTED, "the surrogate runs on the enthalpy form only"};
        if (ctx->variable()) throw PrepError{FEM_E_UNSUPPORTED, "the surrogate needs constant properties"};
        if (o->width != WIDTH) throw PrepError{FEM_E_UNSUPPORTED, "width must be 64"};
        if (o->layers < 1 || o->layers > MAX_LAYERS) throw PrepError{FEM_E_INVALID_ARG, "layers must be 1..4"};
        if (o->horizon < 3) throw PrepError{FEM_E_INVALID_ARG, "horizon must be >= 3"};
        if (o->max_samples < 1 || o->max_samples > 65535) throw PrepError{FEM_E_INVALID_ARG, "max_samples must be 1..65535"};
        if (o->loss != FEM_SUR_LOSS_H && o->loss != FEM_SUR_LOSS_T && o->loss != FEM_SUR_LOSS_HUBER)
            throw PrepError{FEM_E_INVALID_ARG, "unknown loss"};
        if (o->extrapolation != FEM_SUR_EXTRAP_LINEAR && o->extrapolation != FEM_SUR_EXTRAP_QUADRATIC)
            throw PrepError{FEM_E_INVALID_ARG, "unknown extrapolation"};
        for (int32_t r : o->reserved)
            if (r) throw PrepError{FEM_E_INVALID_ARG, "reserved fields must be zero"};
        if ((int64_t)o->max_samples * ctx->L().N > (int64_t)1 << 31)
            throw PrepError{FEM_E_INVALID_ARG, "max_samples * n_nodes must stay below 2^31 rows"};
        fem_sur *s = new fem_sur;
        s->ctx = ctx;
        s->opt = *o;
        s->N = ctx->L().N;
        s->rows = (int64_t)o->max_samples * s->N;
        s->nb = (s->rows + GRAD_ROWS - 1) / GRAD_ROWS;
        s->pl.build(o->layers);
        try {
            build_graph(s);
            build_coef(s);
            sur_sizes(s);
        } catch (...) {
            delete s;
            throw;
        }
        *out = s;
    });
}

int fem_sur_destroy(fem_sur *s) {
    delete s;
    return FEM_OK;
}

int fem_sur_query_buffers(const fem_sur *s, fem_buffer_desc *d, int32_t *n) {
    if (!s || !n) return set_err(FEM_E_INVALID_ARG, "null argument");
    if (!d) {
        *n = S_COUNT;
        return FEM_OK;
    }
    if (*n < S_COUNT) return set_err(FEM_E_INVALID_ARG, "descriptor array too small");
    for (int k = 0; k < S_COUNT; ++k) {
        std::memset(&d[k], 0, sizeof(fem_buffer_desc));
        std::strncpy(d[k].name, SBUF_NAMES[k], sizeof(d[k].name) - 1);
        d[k].bytes = s->sizes[k] ? aligned(s->sizes[k]) : 0;
        d[k].alignment = ALIGN;
    }
    *n = S_COUNT;
    return FEM_OK;
}

int fem_sur_bind_buffers(fem_sur *s, void *const *dev_ptrs, int32_t n) {
    if (!s || !dev_ptrs) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        if (n != S_COUNT) throw PrepError{FEM_E_INVALID_ARG, "expected " + std::to_string(S_COUNT) + " buffers"};
        for (int k = 0; k < S_COUNT; ++k) {
            if (s->sizes[k] && !dev_ptrs[k]) throw PrepError{FEM_E_INVALID_ARG, std::string("buffer ") + SBUF_NAMES[k] + " is null"};
            if ((uintptr_t)dev_ptrs[k] % ALIGN) throw PrepError{FEM_E_INVALID_ARG, std::string("buffer ") + SBUF_NAMES[k] + " is misaligned"};
            s->ptr[k] = s->sizes[k] ? dev_ptrs[k] : nullptr;
        }
        fill_surdev(s);
        hipStream_t st = s->ctx->stream;
        HIPCHECK(hipMemcpyAsync(s->ptr[S_NBR_PTR], s->nbr_ptr.data(), s->sizes[S_NBR_PTR], hipMemcpyHostToDevice, st));
        if (s->nnz) HIPCHECK(hipMemcpyAsync(s->ptr[S_NBR], s->nbr.data(), s->sizes[S_NBR], hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(s->ptr[S_INV_DEG], s->inv_deg.data(), s->sizes[S_INV_DEG], hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(s->ptr[S_COEF], s->coef.data(), s->sizes[S_COEF], hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(s->ptr[S_SCEN], s->scen.data(), s->sizes[S_SCEN], hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(s->ptr[S_SCEN_SEG_PTR], s->scen_seg_ptr.data(), s->sizes[S_SCEN_SEG_PTR],
                                hipMemcpyHostToDevice, st));
        HIPCHECK(hipMemcpyAsync(s->ptr[S_SCEN_SEG], s->scen_seg.data(), s->sizes[S_SCEN_SEG], hipMemcpyHostToDevice, st));
        if (s->opt.train) {
            HIPCHECK(hipMemsetAsync(s->ptr[S_ADAM_M], 0, s->sizes[S_ADAM_M], st));
            HIPCHECK(hipMemsetAsync(s->ptr[S_ADAM_V], 0, s->sizes[S_ADAM_V], st));
        }
        std::vector<float> p;
        init_params(s, p);
        s->bound = true;
        s->adam_t = 0;
        upload_params(s, p.data());
    });
}

int fem_sur_n_params(const fem_sur *s, int64_t *n) {
    if (!s || !n) return set_err(FEM_E_INVALID_ARG, "null argument");
    *n = s->pl.total;
    return FEM_OK;
}

int fem_sur_get_params(fem_sur *s, float *host, int64_t n) {
    if (!s || !host) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_bound(s);
        if (n != s->pl.total) throw PrepError{FEM_E_INVALID_ARG, "parameter count mismatch"};
        HIPCHECK(hipMemcpyAsync(host, s->ptr[S_PARAMS], n * 4, hipMemcpyDeviceToHost, s->ctx->stream));
        HIPCHECK(hipStreamSynchronize(s->ctx->stream));
    });
}

int fem_sur_set_params(fem_sur *s, const float *host, int64_t n) {
    if (!s || !host) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] { set_params(s, host, n); });
}

int fem_sur_save(fem_sur *s, const char *path) {
    if (!s || !path) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_bound(s);
        std::vector<float> p(s->pl.total);
        HIPCHECK(hipMemcpyAsync(p.data(), s->ptr[S_PARAMS], p.size() * 4, hipMemcpyDeviceToHost, s->ctx->stream));
        HIPCHECK(hipStreamSynchronize(s->ctx->stream));
        const ParamFileHeader h = file_header(s);
        FILE *f = std::fopen(path, "wb");
        if (!f) throw PrepError{FEM_E_INVALID_ARG, std::string("cannot open ") + path + " for writing"};
        const bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(p.data(), 4, p.size(), f) == p.size();
        if (std::fclose(f) != 0 || !ok) throw PrepError{FEM_E_INVALID_ARG, std::string("cannot write ") + path};
    });
}

int fem_sur_load(fem_sur *s, const char *path) {
    if (!s || !path) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_bound(s);
        FILE *f = std::fopen(path, "rb");
        if (!f) throw PrepError{FEM_E_INVALID_ARG, std::string("cannot open ") + path};
        ParamFileHeader h{};
        std::vector<float> p;
        bool ok = std::fread(&h, sizeof(h), 1, f) == 1;
        const ParamFileHeader want = file_header(s);
        const bool same = ok && std::memcmp(h.magic, want.magic, sizeof(h.magic)) == 0 && h.width == want.width &&
                          h.layers == want.layers && h.horizon == want.horizon &&
                          h.extrapolation == want.extrapolation && h.n_params == want.n_params;
        if (same) {
            p.resize(h.n_params);
            ok = std::fread(p.data(), 4, p.size(), f) == p.size() && std::fgetc(f) == EOF;
        }
        std::fclose(f);
        if (!same) throw PrepError{FEM_E_INVALID_ARG, std::string(path) + ": not parameters of a surrogate of this shape"};
        if (!ok) throw PrepError{FEM_E_INVALID_ARG, std::string(path) + ": truncated or oversized parameter file"};
        set_params(s, p.data(), (int64_t)p.size());
    });
}

int fem_sur_features(fem_sur *s, const float *H0, const float *H1, const float *H2, int64_t stride, int64_t slots,
                     float *X_host) {
    if (!s || !H0 || !H1 || !H2 || !X_host) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_bound(s);
        check_slots(s, slots);
        const int64_t R = slots * s->N;
        HIPCHECK(features(s->d, H0, H1, H2, 0, nullptr, stride, nullptr, slots, s->ctx->stream));
        std::vector<bf16> x(R * KIN);
        HIPCHECK(hipMemcpyAsync(x.data(), s->ptr[S_X], R * KIN * 2, hipMemcpyDeviceToHost, s->ctx->stream));
        HIPCHECK(hipStreamSynchronize(s->ctx->stream));
        for (int64_t r = 0; r < R; ++r)
            for (int k = 0; k < NFEAT; ++k) {
                const uint32_t u = (uint32_t)x[r * KIN + k] << 16;
                float f;
                std::memcpy(&f, &u, 4);
                X_host[r * NFEAT + k] = f;
            }
    });
}

int fem_sur_loss_grad(fem_sur *s, const float *H0, const float *H1, const float *H2, const float *Ht, int64_t stride,
                      int64_t slots, double *loss, float *grad_host) {
    if (!s || !H0 || !H1 || !H2 || !Ht || !loss || !grad_host) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_train(s);
        check_slots(s, slots);
        pass(s, H0, H1, H2, Ht, stride, nullptr, slots);
        HIPCHECK(hipMemcpyAsync(grad_host, s->ptr[S_GRADS], s->pl.total * 4, hipMemcpyDeviceToHost, s->ctx->stream));
        *loss = loss_of(s, slots * s->N);
    });
}

int fem_sur_train(fem_sur *s, const float *H0, const float *H1, const float *H2, const float *Ht, int64_t stride,
                  int64_t n_samples, int32_t batch, int32_t epochs, float lr, float lr_final, uint64_t seed,
                  double *loss_per_epoch) {
    if (!s || !H0 || !H1 || !H2 || !Ht) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_train(s);
        check_slots(s, batch);
        if (n_samples < 1 || epochs < 0 || !(lr > 0) || !(lr_final > 0))
            throw PrepError{FEM_E_INVALID_ARG, "need n_samples >= 1, epochs >= 0 and positive rates"};
        if (n_samples > INT32_MAX) throw PrepError{FEM_E_INVALID_ARG, "too many samples"};
        hipStream_t st = s->ctx->stream;
        const int64_t per_epoch = (n_samples + batch - 1) / batch;
        const int64_t total = per_epoch * epochs;
        int64_t it = 0;
        std::vector<int32_t> perm(n_samples);
        for (int32_t e = 0; e < epochs; ++e) {
            // shuffle: sort by a counter-based key (seed, epoch, sample)
            std::vector<uint64_t> key(n_samples);
            for (int64_t k = 0; k < n_samples; ++k) key[k] = mix64(mix64(seed + 0x632BE59BD9B4E019ull * (e + 1)) ^ (uint64_t)k);
            std::iota(perm.begin(), perm.end(), 0);
            std::sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
            double lsum = 0.0;
            int64_t lrows = 0;
            for (int64_t b0 = 0; b0 < n_samples; b0 += batch) {
                const int64_t slots = std::min<int64_t>(batch, n_samples - b0);
                HIPCHECK(hipMemcpyAsync(s->ptr[S_IDX], perm.data() + b0, slots * 4, hipMemcpyHostToDevice, st));
                pass(s, H0, H1, H2, Ht, stride, (const int32_t *)s->ptr[S_IDX], slots);
                // cosine decay from lr to lr_final over all iterations
                const double fr = total > 1 ? (double)it / (double)(total - 1) : 0.0;
                const float rate = (float)(lr_final + 0.5 * (lr - lr_final) * (1.0 + std::cos(3.141592653589793 * fr)));
                HIPCHECK(adam(s->d, rate, 0.9f, 0.999f, 1e-8f, ++s->adam_t, st));
                HIPCHECK(refresh_bf16(s->d, st));
                lsum += loss_of(s, slots * s->N) * (double)(slots * s->N);
                lrows += slots * s->N;
                ++it;
            }
            if (loss_per_epoch) loss_per_epoch[e] = lsum / (double)lrows;
        }
        HIPCHECK(hipStreamSynchronize(st));
    });
}

int fem_sur_predict(fem_sur *s, const float *H0, const float *H1, const float *H2, int64_t stride, int64_t slots,
                    double *H_out) {
    if (!s || !H0 || !H1 || !H2 || !H_out) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_bound(s);
        check_slots(s, slots);
        hipStream_t st = s->ctx->stream;
        const int64_t R = slots * s->N;
        HIPCHECK(features(s->d, H0, H1, H2, 0, nullptr, stride, nullptr, slots, st));
        HIPCHECK(forward(s->d, R, 0, 1, st));
        HIPCHECK(apply(s->d, R, H_out, st));
        HIPCHECK(hipStreamSynchronize(st));
    });
}

int fem_snapshot_H(fem_ctx *ctx, float *H_dev) {
    if (!ctx || !H_dev) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        HIPCHECK(state_to_f32(ctx->dev, H_dev, ctx->stream));
    });
}

int fem_sur_generate(fem_sur *s, const double *dt_per_scenario, int64_t n_chunks, int32_t jump_every, float *S_dev) {
    if (!s || !dt_per_scenario || !S_dev) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        need_bound(s);
        fem_ctx *ctx = s->ctx;
        if (n_chunks < 0 || jump_every < 0) throw PrepError{FEM_E_INVALID_ARG, "need n_chunks >= 0 and jump_every >= 0"};
        const int32_t ns = ctx->prob.n_scen;
        std::vector<double> dt(dt_per_scenario, dt_per_scenario + ns);
        for (int32_t sc = 0; sc < ns; ++sc) {
            if (!(dt[sc] > 0) || !std::isfinite(dt[sc])) throw PrepError{FEM_E_INVALID_ARG, "every dt must be > 0"};
            if (dt[sc] > ctx->base.dt_scen[sc] && !ctx->opt.allow_unstable)
                throw PrepError{FEM_E_UNSTABLE, "dt of scenario " + std::to_string(sc) + " above its stability bound"};
        }
        set_dt_scen(ctx, dt);
        hipStream_t st = ctx->stream;
        const int64_t N = s->N, H = s->opt.horizon;
        auto clock = [&](int64_t n) {
            ctx->steps += n;
            for (int32_t sc = 0; sc < ns; ++sc) ctx->time_s[sc] += dt[sc] * (double)n;
        };
        for (int64_t k = 0; k < n_chunks; ++k) {
            float *S = S_dev + k * 4 * N;
            HIPCHECK(state_to_f32(ctx->dev, S, st));
            HIPCHECK(state_to_f64(ctx->dev, s->d.H0, nullptr, st));
            run_steps(ctx, 1);
            HIPCHECK(state_to_f32(ctx->dev, S + N, st));
            HIPCHECK(state_to_f64(ctx->dev, s->d.H1, nullptr, st));
            run_steps(ctx, 1);
            HIPCHECK(state_to_f32(ctx->dev, S + 2 * N, st));
            HIPCHECK(state_to_f64(ctx->dev, s->d.H2, nullptr, st, s->d.H2_pair));
            run_steps(ctx, H - 2);
            HIPCHECK(state_to_f32(ctx->dev, S + 3 * N, st));
            clock(H);
            if (jump_every > 0 && k % jump_every == jump_every - 1) {
                // continue from the network's jump instead of the explicit state
                const int p = ctx->parity ^ (int)((H - 2) & 1);   // T parity at H2
                ctx->diag_fresh = false;
                HIPCHECK(restore_h2(s->d, ctx->dev, p, nullptr, st));
                ctx->parity = p;
                HIPCHECK(features(s->d, s->d.H0, s->d.H1, s->d.H2, 1, nullptr, N, nullptr, 1, st));
                HIPCHECK(forward(s->d, N, 0, 0, st));
                HIPCHECK(write_jump(s->d, ctx->dev, p, 1.0f, st));
            }
        }
        HIPCHECK(hipStreamSynchronize(st));
    });
}

int fem_advance(fem_ctx *ctx, fem_sur *s, const double *dt_per_scenario, int64_t max_steps, int32_t until_solid,
                double energy_tol, double fs_tol, double verify_tol, fem_advance_report *rep) {
    if (!ctx || !dt_per_scenario || !rep) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        const auto t0 = std::chrono::steady_clock::now();
        check_bound(ctx, ST_BOUND);
        if (s) {
            need_bound(s);
            if (s->ctx != ctx) throw PrepError{FEM_E_INVALID_ARG, "the surrogate belongs to another context"};
        }
        if (max_steps < 0 || !(energy_tol > 0) || !(fs_tol >= 0) || !(verify_tol > 0))
            throw PrepError{FEM_E_INVALID_ARG, "need max_steps >= 0, energy_tol > 0, fs_tol >= 0, verify_tol > 0"};
        const int32_t ns = ctx->prob.n_scen;
        std::vector<double> dt(dt_per_scenario, dt_per_scenario + ns);
        for (int32_t sc = 0; sc < ns; ++sc) {
            if (!(dt[sc] > 0) || !std::isfinite(dt[sc])) throw PrepError{FEM_E_INVALID_ARG, "every dt must be > 0"};
            if (dt[sc] > ctx->base.dt_scen[sc] && !ctx->opt.allow_unstable)
                throw PrepError{FEM_E_UNSTABLE, "dt of scenario " + std::to_string(sc) + " above its stability bound"};
        }
        set_dt_scen(ctx, dt);
        std::memset(rep, 0, sizeof(*rep));
        const int64_t H = s ? s->opt.horizon : GRAPH_STEPS;
        hipStream_t st = ctx->stream;
        std::vector<fem_energy_report> er(ns);
        energy_scenarios(ctx, er.data());
        auto all_solid = [&] {
            for (const fem_energy_report &r : er)
                if (r.n_liquid) return false;
            return true;
        };
        auto advance_clock = [&](int64_t n) {
            ctx->steps += n;
            for (int32_t sc = 0; sc < ns; ++sc) ctx->time_s[sc] += dt[sc] * (double)n;
            rep->steps += n;
        };
        std::vector<double> E_prev(ns), Q_prev(ns);
        for (int32_t sc = 0; sc < ns; ++sc) {
            E_prev[sc] = er[sc].E;
            Q_prev[sc] = er[sc].Q_cum;
        }
        const int64_t nchk = check_blocks(ctx->L().N);
        std::vector<double> dg, qn;
        Staging sg(s ? 2 * nchk : 0, ctx->L().seg_scen.size() * NDIAG, ctx->L().n_inflow);
        // plain chunk: steps, diagnostics, one read-back
        auto plain_chunk = [&](int64_t n) {
            run_steps(ctx, n);
            HIPCHECK(enqueue_state_diag(ctx->dev, ctx->parity, st));
            stage_copies(ctx, nullptr, sg);
            HIPCHECK(hipStreamSynchronize(st));
            staged_energy(ctx, sg, dg, qn, er.data());
        };
        bool cont = false;     // the last jump was kept: the state is one step past it, s->d.Hn holds it
        while (!(until_solid && all_solid()) && rep->steps + ((s && !cont) ? H + 1 : H) <= max_steps) {
            if (!s) {
                plain_chunk(H);
                advance_clock(H);
                rep->plain_steps += H;
                continue;
            }
            // explicit steps to H0, H1, H2 (one of them is already done after a kept
            // jump), the network's jump over H - 2 steps, one explicit step from it
            const int p = ctx->parity;
            const int n_plain = cont ? 2 : 3;
            const int p_h2 = cont ? p ^ 1 : p;           // T parity of the state H2
            run_chunk(s, cont ? CHUNK_CONT : CHUNK_FRESH, p, (float)fs_tol, (float)verify_tol);
            ctx->parity = p ^ (n_plain & 1);
            rep->plain_steps += n_plain;
            stage_copies(ctx, s, sg);
            HIPCHECK(hipStreamSynchronize(st));
            staged_energy(ctx, sg, dg, qn, er.data());
            const int32_t *chk = sg.chk();
            int64_t bad_fs = 0, bad_verify = 0;
            for (int64_t k = 0; k < nchk; ++k) {
                bad_fs += chk[k];
                bad_verify += chk[nchk + k];
            }
            bool ok = true;
            if (bad_fs) {
                ok = false;
                ++rep->rejected_fs;
            } else if (bad_verify) {
                ok = false;
                ++rep->rejected_verify;
            }
            // FP64 energy gate: the energy change since the last check against the
            // inflow of the explicit steps in between (exact, per node) plus their
            // mean rate over the H - 2 jumped steps, which they bracket
            std::vector<double> est(ns), res(ns);
            for (int32_t sc = 0; sc < ns && ok; ++sc) {
                const fem_energy_report &r = er[sc];
                const double q_plain = r.Q_cum - Q_prev[sc];
                est[sc] = (double)(H - 2) * q_plain / (double)n_plain;
                res[sc] = std::fabs((r.E - E_prev[sc]) - (q_plain + est[sc])) / std::fabs(E_prev[sc] - ctx->Eref_s[sc]);
                if (r.nonfinite || !(res[sc] <= energy_tol)) {
                    ok = false;
                    ++rep->rejected_energy;
                }
            }
            if (ok) {
                for (int32_t sc = 0; sc < ns; ++sc) {
                    ctx->Qx_s[sc] += est[sc];
                    E_prev[sc] = er[sc].E;
                    Q_prev[sc] = er[sc].Q_cum + est[sc];
                    er[sc].Q_cum += est[sc];
                    rep->max_residual = std::max(rep->max_residual, res[sc]);
                }
                advance_clock(cont ? H : H + 1);
                ++rep->jumps_accepted;
                cont = true;
            } else {
                run_chunk(s, CHUNK_FALLBACK, p_h2, (float)fs_tol, (float)verify_tol);
                ctx->parity = p_h2 ^ (int)((H - 2) & 1);
                advance_clock(cont ? H - 1 : H);
                rep->plain_steps += H - 2;
                ++rep->jumps_rejected;
                HIPCHECK(enqueue_state_diag(ctx->dev, ctx->parity, st));
                stage_copies(ctx, nullptr, sg);
                HIPCHECK(hipStreamSynchronize(st));
                staged_energy(ctx, sg, dg, qn, er.data());
                for (int32_t sc = 0; sc < ns; ++sc) {
                    E_prev[sc] = er[sc].E;
                    Q_prev[sc] = er[sc].Q_cum;
                }
                cont = false;
            }
        }
        HIPCHECK(hipStreamSynchronize(st));
        rep->solid = all_solid() ? 1 : 0;
        rep->wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    });
}

}  // extern "C"
