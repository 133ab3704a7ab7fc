// C interface of the casting step (include/castfem.h).
#include "ctx.hpp"

#include <numeric>

namespace castfem {

namespace {
thread_local std::string g_err;
}

int set_err(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

const char *last_error() { return g_err.c_str(); }

}  // namespace castfem

namespace castfem {

int64_t rup(int64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// byte sizes of every buffer for one layout
void layout_sizes(const fem_ctx *c, const Layout &L, int64_t *sz) {
    const int64_t R = (int64_t)c->rsize();
    const int64_t N = L.N, E = L.E;
    const bool blocked = c->opt.scatter == FEM_SCATTER_LDS_BLOCKED;
    for (int b = 0; b < B_COUNT; ++b) sz[b] = 0;
    sz[B_NODE_X] = N * 4 * R;
    sz[B_T] = 2 * N * R;
    sz[B_H] = N * 8;
    sz[B_INV_M] = N * R;
    sz[B_FS] = N * R;
    sz[B_MATS] = (int64_t)c->prob.mats.size() * (int64_t)sizeof(MatDev);
    if (!blocked) {
        sz[B_CONN] = E * L.nen * 4;
        sz[B_R] = N * R;
    } else {
        const int64_t np = (int64_t)L.sh_list.size();
        sz[B_LCONN] = L.lconn12.empty() ? E * L.nen * 2 : (int64_t)L.lconn12.size() * 4;
        sz[B_VCONN] = (int64_t)L.vconn.size() * 2;
        sz[B_VW] = (int64_t)L.vw.size() * R;
        sz[B_BLOCKS] = (int64_t)L.blocks.size() * (int64_t)sizeof(BlockInfo);
        sz[B_SH_LIST] = (np + 1) * 4;   // one padding entry: the gather's clamped loads
        sz[B_PARTIALS] = L.n_partial_slots * R;
        sz[B_COMB_PTR] = (N - L.n_private + 1) * 4;
        sz[B_SH_POS] = np * 4;
        // windows of the material table for the node kernel's workgroups (large tables only)
        if ((int64_t)c->prob.mats.size() > MAT_WINDOW) sz[B_NODE_WIN] = node_grid(N - L.n_private) * 4;
        if (c->apparent()) {
            sz[B_CAP_PARTIALS] = L.n_partial_slots * R;
            sz[B_APP_MATS] = (int64_t)c->prob.mats.size() * (int64_t)sizeof(AppMat);
        }
        if (c->variable()) {
            sz[B_VAR_TABS_F] = (int64_t)c->vtabs.size() * (int64_t)sizeof(Tab<float>);
            sz[B_VAR_TABS_D] = (int64_t)c->vtabs.size() * (int64_t)sizeof(Tab<double>);
            sz[B_T_FIXED] = N * 8;
            sz[B_TIME] = 16 * (int64_t)c->prob.n_scen;
            sz[B_VAR_SCEN] = ((int64_t)c->prob.mats.size() + c->prob.n_scen) * 4;
            sz[B_SCHED] = L.n_inflow * (int64_t)c->sched_t.size() * 8;
        }
    }
    sz[B_ROBIN] = (int64_t)L.robin_a.size() * 2 * R;
    sz[B_LINK_PTR] = (L.n_bc_slots + 1) * 4;
    sz[B_LINK_NODE] = (int64_t)L.link_node.size() * 4;
    sz[B_LINK_W] = (int64_t)L.link_w.size() * R;
    const int64_t nseg = (int64_t)L.seg_scen.size();
    sz[B_DIAG] = nseg * NDIAG * 8;
    sz[B_QNODE] = L.n_inflow * 8;
    sz[B_SEG] = (nseg + 1) * 4;
    sz[B_FLAGS] = N * 4;
}

template <class T>
void h2d(fem_ctx *c, int b, const T *src, int64_t bytes) {
    if (bytes == 0) return;
    if (bytes > c->sizes[b]) throw PrepError{FEM_E_INVALID_ARG, std::string("internal: buffer too small: ") + BUF_NAMES[b]};
    HIPCHECK(hipMemcpyAsync(c->ptr[b], src, bytes, hipMemcpyHostToDevice, c->stream));
}

template <class R>
void upload_layout_t(fem_ctx *c, const Layout &L) {
    using V4 = typename std::conditional<sizeof(R) == 4, float4, double4>::type;
    const int64_t N = L.N;
    std::vector<V4> nx(N);
    std::vector<R> im(N), T2(2 * N), fs(N);
    std::vector<uint8_t> H(N * 8);
    c->E0 = c->Eref = c->lat0 = 0;
    c->E0_s.assign(c->prob.n_scen, 0.0);
    c->Eref_s.assign(c->prob.n_scen, 0.0);
    c->tmin0 = INFINITY;
    c->tmax0 = -INFINITY;
    c->nliq0 = 0;
    // FP32: coordinates as fixed-point integers (in the float bits) of a
    // power-of-two unit that maps the bounding box into [0, 2^30] and keeps
    // every element's extent below 2^24 units (exact in FP32, and element
    // formulas evaluated in units stay far from FP32 overflow)
    double lo[3] = {INFINITY, INFINITY, INFINITY}, ext = 0.0, span = 0.0;
    for (int64_t n = 0; n < N; ++n)
        for (int a = 0; a < 3; ++a) lo[a] = std::min(lo[a], L.xyz[3 * n + a]);
    for (int64_t n = 0; n < N; ++n)
        for (int a = 0; a < 3; ++a) ext = std::max(ext, L.xyz[3 * n + a] - lo[a]);
    for (int64_t e = 0; e < L.E; ++e)
        for (int a = 0; a < 3; ++a) {
            double mn = INFINITY, mx = -INFINITY;
            for (int j = 0; j < L.nen; ++j) {
                const double x = L.xyz[3 * (int64_t)L.conn[e * L.nen + j] + a];
                mn = std::min(mn, x);
                mx = std::max(mx, x);
            }
            span = std::max(span, mx - mn);
        }
    const double unit = std::ldexp(1.0, (int)std::ceil(std::log2(std::max(
                                            {ext / 1073741824.0, span / 8388608.0, 1e-30}))));
    c->x_scale = sizeof(R) == 4 ? (float)unit : 1.0f;
    for (int64_t n = 0; n < N; ++n) {
        const uint32_t f = L.nflag[n];
        V4 v;
        if constexpr (sizeof(R) == 4) {
            int32_t q[3];
            for (int a = 0; a < 3; ++a) q[a] = (int32_t)std::llround((L.xyz[3 * n + a] - lo[a]) / unit);
            std::memcpy(&v.x, &q[0], 4);
            std::memcpy(&v.y, &q[1], 4);
            std::memcpy(&v.z, &q[2], 4);
        } else {
            v.x = (R)L.xyz[3 * n];
            v.y = (R)L.xyz[3 * n + 1];
            v.z = (R)L.xyz[3 * n + 2];
        }
        // conductivity of the node's material; the apparent-capacity kernel
        // takes the material index instead
        v.w = c->mat_in_node_x() ? (R)(f & NODE_MAT_MASK) : (R)c->prob.mats[f & NODE_MAT_MASK].k;
        nx[n] = v;
        im[n] = (R)(1.0 / L.m[n]);
        const fem_material &mat = c->prob.mats[f & NODE_MAT_MASK];
        const MatDev &M = c->mats_host[f & NODE_MAT_MASK];
        // a fixed node starts at T_D + shift(0)
        const double T_start = (f & NODE_FIXED) ? L.T_init[n] + c->dir_shift(0.0) : L.T_init[n];
        const double h0 = h_of_t(mat, T_start);
        double hd;
        if (sizeof(R) == 4) {
            float hi = (float)h0;
            float lo = (float)(h0 - (double)hi);
            std::memcpy(&H[8 * n], &hi, 4);
            std::memcpy(&H[8 * n + 4], &lo, 4);
            hd = (double)hi + (double)lo;
        } else {
            std::memcpy(&H[8 * n], &h0, 8);
            hd = h0;
        }
        double T, f_s;
        t_of_h(M, hd, T, f_s);
        if (f & NODE_FIXED) T = T_start;
        T2[n] = T2[N + n] = (R)T;
        fs[n] = (R)f_s;
        const double m = 1.0 / (double)im[n];
        const int32_t sc = c->prob.scen_of_mat((int32_t)(f & NODE_MAT_MASK));
        c->E0_s[sc] += m * hd;
        c->Eref_s[sc] += m * h_of_t(mat, 25.0);
        c->E0 += m * hd;
        c->Eref += m * h_of_t(mat, 25.0);
        c->lat0 += m * mat.L * (1.0 - f_s);
        c->tmin0 = std::min(c->tmin0, (double)T2[n]);
        c->tmax0 = std::max(c->tmax0, (double)T2[n]);
        if (mat.L > 0 && f_s < 1.0) c->nliq0++;
    }
    h2d(c, B_NODE_X, nx.data(), N * (int64_t)sizeof(V4));
    h2d(c, B_INV_M, im.data(), N * (int64_t)sizeof(R));
    h2d(c, B_H, H.data(), N * 8);
    h2d(c, B_T, T2.data(), 2 * N * (int64_t)sizeof(R));
    h2d(c, B_FS, fs.data(), N * (int64_t)sizeof(R));
    h2d(c, B_FLAGS, L.nflag.data(), N * 4);
    std::vector<R> rob(L.robin_a.size() * 2), lw(L.link_w.size()), vw;
    std::vector<BlockInfo> blocks_app;
    std::vector<int32_t> node_win;
    for (size_t s = 0; s < L.robin_a.size(); ++s) {
        rob[2 * s] = (R)L.robin_a[s];
        rob[2 * s + 1] = (R)L.robin_b[s];
    }
    for (size_t s = 0; s < L.link_w.size(); ++s) lw[s] = (R)L.link_w[s];
    h2d(c, B_ROBIN, rob.data(), (int64_t)rob.size() * (int64_t)sizeof(R));
    h2d(c, B_LINK_PTR, L.link_ptr.data(), (int64_t)L.link_ptr.size() * 4);
    h2d(c, B_LINK_NODE, L.link_node.data(), (int64_t)L.link_node.size() * 4);
    h2d(c, B_LINK_W, lw.data(), (int64_t)lw.size() * (int64_t)sizeof(R));
    if (c->opt.scatter == FEM_SCATTER_LDS_BLOCKED) {
        if (L.lconn12.empty()) h2d(c, B_LCONN, L.lconn.data(), (int64_t)L.lconn.size() * 2);
        else h2d(c, B_LCONN, L.lconn12.data(), (int64_t)L.lconn12.size() * 4);
        if (!L.vw.empty()) {
            h2d(c, B_VCONN, L.vconn.data(), (int64_t)L.vconn.size() * 2);
            vw.resize(L.vw.size());
            for (size_t v = 0; v < L.vw.size(); ++v) vw[v] = (R)L.vw[v];
            h2d(c, B_VW, vw.data(), (int64_t)vw.size() * (int64_t)sizeof(R));
        }
        // per block: its one material or -1 (pad0; the apparent-capacity kernels
        // read the constants of a single-material block once), and the first row
        // of its window of MAT_WINDOW material rows or -1 if its materials span
        // more (pad1; the step kernels stage the window in LDS)
        blocks_app = L.blocks;
        for (BlockInfo &b : blocks_app) {
            int32_t lo = INT32_MAX, hi = -1;
            auto see = [&](int64_t g) {
                const int32_t q = (int32_t)(L.nflag[g] & NODE_MAT_MASK);
                lo = std::min(lo, q);
                hi = std::max(hi, q);
            };
            for (int32_t i = 0; i < b.n_int; ++i) see((int64_t)b.int_base + i);
            for (int32_t i = 0; i < b.n_sh; ++i) see(L.sh_list[b.sh_begin + i]);
            b.pad0 = (c->mat_in_node_x() && hi == lo) ? lo : -1;
            b.pad1 = (hi >= lo && hi - lo < MAT_WINDOW) ? lo : -1;
        }
        h2d(c, B_BLOCKS, blocks_app.data(), (int64_t)blocks_app.size() * (int64_t)sizeof(BlockInfo));
        if (c->sizes[B_NODE_WIN]) {
            const int64_t cnt = N - L.n_private, nw = node_grid(cnt);
            node_win.resize(nw);
            for (int64_t w = 0; w < nw; ++w) {
                int32_t lo = INT32_MAX, hi = -1;
                for (int64_t k = w * NODE_THREADS; k < std::min(cnt, (w + 1) * NODE_THREADS); ++k) {
                    const int32_t q = (int32_t)(L.nflag[L.bc_first + k] & NODE_MAT_MASK);
                    lo = std::min(lo, q);
                    hi = std::max(hi, q);
                }
                node_win[w] = (hi >= lo && hi - lo < MAT_WINDOW) ? lo : -1;
            }
            h2d(c, B_NODE_WIN, node_win.data(), nw * 4);
        }
        {
            std::vector<int32_t> shp(L.sh_list);
            shp.push_back(0);
            h2d(c, B_SH_LIST, shp.data(), (int64_t)shp.size() * 4);
            HIPCHECK(hipStreamSynchronize(c->stream));   // shp is a temporary
        }
        h2d(c, B_COMB_PTR, L.comb_ptr.data(), (int64_t)L.comb_ptr.size() * 4);
        // partial slots of a node's missing blocks are never written: zero them once
        HIPCHECK(hipMemsetAsync(c->ptr[B_PARTIALS], 0, (size_t)(L.n_partial_slots * sizeof(R)), c->stream));
        if (c->apparent())
            HIPCHECK(hipMemsetAsync(c->ptr[B_CAP_PARTIALS], 0, (size_t)(L.n_partial_slots * sizeof(R)), c->stream));
        h2d(c, B_SH_POS, L.sh_pos.data(), (int64_t)L.sh_pos.size() * 4);
    } else {
        h2d(c, B_CONN, L.conn.data(), (int64_t)L.conn.size() * 4);
        HIPCHECK(hipMemsetAsync(c->ptr[B_R], 0, N * sizeof(R), c->stream));
    }
    std::vector<AppMat> am;
    if (c->apparent()) {
        for (const fem_material &m : c->prob.mats) {
            AppMat a{};
            a.k = m.k;
            a.rho = m.rho;
            a.c = m.c;
            a.L = m.L;
            a.Ts = m.T_sol;
            a.Tl = m.T_liq;
            a.inv_dT = m.L > 0 ? 1.0 / (m.T_liq - m.T_sol) : 0.0;
            a.kf = (float)a.k;
            a.rhof = (float)a.rho;
            a.cf = (float)a.c;
            a.Lf = (float)a.L;
            a.Tsf = (float)a.Ts;
            a.Tlf = (float)a.Tl;
            a.inv_dTf = (float)a.inv_dT;
            am.push_back(a);
        }
        h2d(c, B_APP_MATS, am.data(), (int64_t)(am.size() * sizeof(AppMat)));
    }
    std::vector<Tab<float>> tf;
    std::vector<double> tfix, sched, t0;
    std::vector<int32_t> vscen;
    if (c->variable()) {
        for (const Tab<double> &t : c->vtabs) {
            Tab<float> u{};
            u.n = t.n;
            for (int j = 0; j < TAB_POINTS; ++j) {
                u.x[j] = (float)t.x[j];
                u.y[j] = (float)t.y[j];
            }
            tf.push_back(u);
        }
        h2d(c, B_VAR_TABS_F, tf.data(), (int64_t)(tf.size() * sizeof(Tab<float>)));
        h2d(c, B_VAR_TABS_D, c->vtabs.data(), (int64_t)(c->vtabs.size() * sizeof(Tab<double>)));
        tfix.assign(N, 0.0);
        for (int64_t n = 0; n < N; ++n)
            if (L.nflag[n] & NODE_FIXED) tfix[n] = L.T_init[n];
        h2d(c, B_T_FIXED, tfix.data(), N * 8);
        t0.assign(2 * (size_t)c->prob.n_scen, 0.0);
        h2d(c, B_TIME, t0.data(), (int64_t)t0.size() * 8);
        // the scenario of every material, then a material of every scenario (its dt)
        vscen.assign(c->prob.mats.size() + (size_t)c->prob.n_scen, -1);
        for (size_t m = 0; m < c->prob.mats.size(); ++m) {
            const int32_t sc = c->prob.scen_of_mat((int32_t)m);
            vscen[m] = sc;
            if (vscen[c->prob.mats.size() + sc] < 0) vscen[c->prob.mats.size() + sc] = (int32_t)m;
        }
        h2d(c, B_VAR_SCEN, vscen.data(), (int64_t)vscen.size() * 4);
        if (const int64_t K = (int64_t)c->sched_t.size()) {
            // the rows of the fixed nodes' schedules at their shared slots
            sched.assign(L.n_inflow * K, 0.0);
            for (size_t q = 0; q < c->prob.dir_nodes.size(); ++q) {
                const int64_t slot = (int64_t)L.perm[c->prob.dir_nodes[q]] - L.bc_first;
                if (slot < 0 || slot >= L.n_inflow) throw PrepError{FEM_E_INVALID_ARG, "fixed node outside the inflow slots"};
                std::copy(c->sched_T.begin() + q * K, c->sched_T.begin() + (q + 1) * K, sched.begin() + slot * K);
            }
            h2d(c, B_SCHED, sched.data(), L.n_inflow * K * 8);
        }
    }
    int64_t sz[B_COUNT];
    layout_sizes(c, L, sz);
    HIPCHECK(hipMemsetAsync(c->ptr[B_DIAG], 0, sz[B_DIAG], c->stream));
    if (sz[B_QNODE]) HIPCHECK(hipMemsetAsync(c->ptr[B_QNODE], 0, sz[B_QNODE], c->stream));
    h2d(c, B_SEG, L.seg_begin.data(), (int64_t)L.seg_begin.size() * 4);
    // the host vectors above must outlive the copies
    HIPCHECK(hipStreamSynchronize(c->stream));
}

void fill_dev(fem_ctx *c, const Candidate &cd) {
    const Layout &L = cd.L;
    Dev d;
    d.prec = c->opt.precision;
    d.nen = L.nen;
    d.scatter = c->opt.scatter;
    d.N = L.N;
    d.E = L.E;
    d.node_x = c->ptr[B_NODE_X];
    d.x_scale = c->x_scale;
    d.T = c->ptr[B_T];
    d.H = c->ptr[B_H];
    d.inv_m = c->ptr[B_INV_M];
    d.fs = c->ptr[B_FS];
    d.mats = (const MatDev *)c->ptr[B_MATS];
    d.conn = (const int32_t *)c->ptr[B_CONN];
    d.r = c->ptr[B_R];
    d.lconn = (const uint16_t *)c->ptr[B_LCONN];
    d.conn12 = L.lconn12.empty() ? 0 : 1;
    d.vconn = (const uint16_t *)c->ptr[B_VCONN];
    d.vw = c->ptr[B_VW];
    d.blocks = (const BlockInfo *)c->ptr[B_BLOCKS];
    d.sh_list = (const int32_t *)c->ptr[B_SH_LIST];
    d.partials = c->ptr[B_PARTIALS];
    d.node_win = (const int32_t *)c->ptr[B_NODE_WIN];
    d.comb_ptr = (const int32_t *)c->ptr[B_COMB_PTR];
    d.sh_pos = (const int32_t *)c->ptr[B_SH_POS];
    d.flags = (const uint32_t *)c->ptr[B_FLAGS];
    d.robin = L.robin_a.empty() ? nullptr : c->ptr[B_ROBIN];
    d.link_ptr = (const int32_t *)c->ptr[B_LINK_PTR];
    d.link_node = (const int32_t *)c->ptr[B_LINK_NODE];
    d.link_w = c->ptr[B_LINK_W];
    d.diag = (double *)c->ptr[B_DIAG];
    d.qnode = (double *)c->ptr[B_QNODE];
    d.seg_begin = (const int32_t *)c->ptr[B_SEG];
    d.n_seg = (int64_t)L.seg_scen.size();
    d.n_inflow = L.n_inflow;
    d.n_mat = (int32_t)c->prob.mats.size();
    d.n_private = L.n_private;
    d.n_blocks = (int64_t)L.blocks.size();
    d.n_bc_slots = L.n_bc_slots;
    d.bc_first = L.bc_first;
    d.threads = cd.threads;
    d.lds_bytes = block_lds_bytes(d.prec, L.max_local);
    d.n_colors = L.color_ptr.empty() ? 0 : (int)L.color_ptr.size() - 1;
    d.color_ptr_host = L.color_ptr.empty() ? nullptr : L.color_ptr.data();
    // fixed-point scale: a node's element sum is bounded by
    // sum_e sum_j |K^e_ij| times the temperature span; with a margin of 16 on
    // the span every partial sum stays below 2^50
    {
        const double bound = 16.0 * std::max(c->base.elem_abs_max, 1e-300) * c->base.T_span;
        const int S = std::min(80, (int)std::floor(std::log2(std::ldexp(1.0, 50) / bound)));
        d.fx_scale = std::ldexp(1.0, S);
        d.fx_inv = std::ldexp(1.0, -S);
        d.fx_limit = (float)std::ldexp(1.0, 50 - S);
    }
    c->dev = d;
    if (c->apparent()) {
        AppDev a;
        a.d = d;
        a.d.lds_bytes = (size_t)L.max_local * lds_per_node_apparent(d.prec);
        a.cap_partials = c->ptr[B_CAP_PARTIALS];
        a.amats = (const AppMat *)c->ptr[B_APP_MATS];
        // FP32 capacitance sums in 32-bit fixed point: every element share is
        // positive and each node's sum is at most cap_bound, so cap_bound * 2^S
        // <= 2^31 keeps every sum (with its rounding) below 2^32.  For a typical
        // node the quantisation is ~1e-7 of its capacitance (the bound exceeds a
        // node's sum by the Lemmon-ratio bound, ~10-100).
        const double bound = 2.0 * std::max(c->cap_bound, 1e-300);
        const int S = std::min(80, (int)std::floor(std::log2(std::ldexp(1.0, 32) / bound)));
        a.cx_scale = std::ldexp(1.0, S);
        a.cx_inv = std::ldexp(1.0, -S);
        a.cx_limit = (float)std::ldexp(1.0, 31 - S);
        c->app = a;
    }
    if (c->variable()) {
        VarDev v;
        v.d = d;
        v.tabs_f = (const Tab<float> *)c->ptr[B_VAR_TABS_F];
        v.tabs_d = (const Tab<double> *)c->ptr[B_VAR_TABS_D];
        v.T_fixed = (const double *)c->ptr[B_T_FIXED];
        v.time = (double *)c->ptr[B_TIME];
        v.n_scen = c->prob.n_scen;
        v.mat_scen = (const int32_t *)c->ptr[B_VAR_SCEN];
        v.scen_mat = v.mat_scen + c->prob.mats.size();
        v.n_sched = (int32_t)c->sched_t.size();
        if (v.n_sched) {
            v.sched = (const double *)c->ptr[B_SCHED];
            for (int k = 0; k < v.n_sched; ++k) v.sched_t[k] = c->sched_t[k];
        }
        c->vdev = v;
    }
}

hipError_t enqueue_ctx_step(const fem_ctx *c, int parity, hipStream_t s, hipEvent_t *ev) {
    if (c->apparent()) return enqueue_step_apparent(c->app, parity, s, ev);
    if (c->variable()) return enqueue_step_var(c->vdev, parity, s, ev);
    return enqueue_step(c->dev, parity, s, ev);
}

// Bound on the lumped apparent capacitance of any node: an element's Lemmon
// ratio |A W a| / |A a| (A = [c_1 c_2 c_3], W = diag of dH/dT over the nodal
// differences a) is at most max dH/dT times ||A|| ||A^-1||, and A^-1 = [d_j]^T / D;
// the Frobenius norms bound both.
double apparent_cap_bound(const Problem &p) {
    std::vector<double> acc(p.N, 0.0);
    for (int64_t e = 0; e < p.E; ++e) {
        const int32_t *cn = &p.conn[4 * e];
        const double *x0 = &p.xyz[3 * cn[0]];
        double d[3][3];
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) d[j][i] = p.xyz[3 * cn[j + 1] + i] - x0[i];
        auto cross = [](const double *a, const double *b, double *o) {
            o[0] = a[1] * b[2] - a[2] * b[1];
            o[1] = a[2] * b[0] - a[0] * b[2];
            o[2] = a[0] * b[1] - a[1] * b[0];
        };
        double cv[3][3];
        cross(d[1], d[2], cv[0]);
        cross(d[2], d[0], cv[1]);
        cross(d[0], d[1], cv[2]);
        const double D = d[0][0] * cv[0][0] + d[0][1] * cv[0][1] + d[0][2] * cv[0][2];
        double nc = 0, nd = 0;
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                nc += cv[j][i] * cv[j][i];
                nd += d[j][i] * d[j][i];
            }
        const fem_material &m = p.mats[p.emat[e]];
        const double wmax = m.c + (m.L > 0 ? m.L / (m.T_liq - m.T_sol) : 0.0);
        // rho * wmax * (||A|| ||A^-1||) * V / 4 with ||A^-1|| = sqrt(nd) / |D| and V / 4 = |D| / 24
        const double share = m.rho * wmax * std::sqrt(nc * nd) / 24.0;
        (void)D;
        for (int a = 0; a < 4; ++a) acc[cn[a]] += share;
    }
    double mx = 0;
    for (double v : acc) mx = std::max(mx, v);
    return mx;
}

}  // namespace castfem

double fem_ctx::dir_shift(double t) const {
    if (!variable()) return 0.0;
    const Tab<double> &sh = vtabs[prob.mats.size() + TAB_DIR_OF_TIME];
    return sh.n ? tab_eval_host(sh, t) : 0.0;
}

namespace castfem {

void reset_graph(fem_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

// time step of every scenario, written into the material table the kernels read
void set_dt_scen(fem_ctx *c, const std::vector<double> &dt) {
    if (dt == c->dt_s) return;
    for (size_t q = 0; q < c->prob.mats.size(); ++q)
        c->mats_host[q] = make_mat(c->prob.mats[q], dt[c->prob.scen_of_mat((int32_t)q)]);
    h2d(c, B_MATS, c->mats_host.data(), (int64_t)(c->mats_host.size() * sizeof(MatDev)));
    HIPCHECK(hipStreamSynchronize(c->stream));
    c->dt_s = dt;
}

void set_dt(fem_ctx *c, double dt) { set_dt_scen(c, std::vector<double>(c->prob.n_scen, dt)); }

void eager_steps(fem_ctx *c, int64_t n) {
    if (n > 0) c->diag_fresh = false;
    for (int64_t s = 0; s < n; ++s) {
        HIPCHECK(enqueue_ctx_step(c, c->parity, c->stream, nullptr));
        c->parity ^= 1;
    }
}

// capture GRAPH_STEPS steps (starting from T buffer 0) into the context's graph
void build_graph(fem_ctx *c) {
    HIPCHECK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int s = 0; s < GRAPH_STEPS && err == hipSuccess; ++s) err = enqueue_ctx_step(c, s & 1, c->stream, nullptr);
    // every GRAPH_STEPS steps the FP64 state reductions of the energy balance
    // (E, latent heat left, T range, liquid and non-finite counts per segment)
    if (err == hipSuccess) err = enqueue_state_diag(c->dev, 0, c->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    HIPCHECK(err);
    HIPCHECK(e2);
    c->graph = g;
    HIPCHECK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    // upload it now, so that its first launch does not pay for it
    HIPCHECK(hipGraphUpload(c->gexec, c->stream));
}

// n steps: whole graphs of GRAPH_STEPS steps, the rest eagerly.  The graph is
// built by the first call on a stream whatever its n (n = 0 included), so a
// short warm-up leaves it instantiated and later calls only launch it.
void run_steps(fem_ctx *c, int64_t n) {
    if (c->stream != nullptr && !c->gexec) build_graph(c);
    if (c->stream == nullptr || n < GRAPH_STEPS) {
        eager_steps(c, n);
        return;
    }
    if (c->parity == 1) {
        eager_steps(c, 1);
        --n;
    }
    for (int64_t r = 0; r < n / GRAPH_STEPS; ++r) HIPCHECK(hipGraphLaunch(c->gexec, c->stream));
    if (n >= GRAPH_STEPS) c->diag_fresh = true;
    eager_steps(c, n % GRAPH_STEPS);
}

void check_bound(fem_ctx *c, int fn_stage) {
    if (c->stage < fn_stage) throw PrepError{FEM_E_STATE, "call out of order: the context is not bound yet"};
}

void fill_report(const fem_ctx *c, fem_prep_report *rep) {
    std::memset(rep, 0, sizeof(*rep));
    const Layout &L = c->L();
    rep->n_nodes = L.N;
    rep->n_elems = L.E;
    rep->n_blocks = (int64_t)L.blocks.size();
    rep->n_shared = c->opt.scatter == FEM_SCATTER_LDS_BLOCKED ? L.N - L.n_private : 0;
    rep->n_partials = (int64_t)L.sh_list.size();
    rep->max_local_nodes = L.max_local;
    rep->block_threads = c->cands.empty() ? 0 : c->cands[c->chosen].threads;
    rep->n_colors = L.color_ptr.empty() ? 0 : (int64_t)L.color_ptr.size() - 1;
    rep->bandwidth_before = L.bw_before;
    rep->bandwidth_after = L.bw_after;
    rep->block_elems = L.block_elems;
    rep->shared_fraction = L.N ? (double)rep->n_shared / (double)L.N : 0.0;
    rep->dt_bound = c->base.dt_bound;
    rep->setup_seconds = c->setup_seconds;
    rep->contact_search_seconds = c->base.sister_seconds;
    rep->n_contact = (int64_t)c->base.sisters.size();
}

}  // namespace castfem

// =================================================================== C ABI
extern "C" {

const char *fem_last_error(void) { return castfem::last_error(); }

int fem_create(fem_ctx **out, const fem_options *opt) {
    if (!out) return set_err(FEM_E_INVALID_ARG, "out is null");
    return guarded([&] {
        fem_options o{};
        o.device = 0;
        o.precision = FEM_PREC_FP32_KAHAN;
        o.ordering = FEM_ORDER_HILBERT;
        o.scatter = FEM_SCATTER_LDS_BLOCKED;
        if (opt) o = *opt;
        if (o.precision != FEM_PREC_FP64 && o.precision != FEM_PREC_FP32_KAHAN)
            throw PrepError{FEM_E_INVALID_ARG, "unknown precision"};
        if (o.ordering < FEM_ORDER_NONE || o.ordering > FEM_ORDER_HILBERT) throw PrepError{FEM_E_INVALID_ARG, "unknown ordering"};
        if (o.scatter < FEM_SCATTER_GLOBAL_ATOMIC || o.scatter > FEM_SCATTER_COLORED)
            throw PrepError{FEM_E_INVALID_ARG, "unknown scatter"};
        if (o.block_elems < 0 || o.lds_bytes < 0 || o.threads < 0) throw PrepError{FEM_E_INVALID_ARG, "negative size option"};
        if (o.threads && (o.threads % 64 || o.threads > 1024)) throw PrepError{FEM_E_INVALID_ARG, "threads must be a multiple of 64 up to 1024"};
        if (o.latent_model != FEM_LATENT_ENTHALPY && o.latent_model != FEM_LATENT_APPARENT)
            throw PrepError{FEM_E_INVALID_ARG, "unknown latent-heat model"};
        for (int r : o.reserved)
            if (r) throw PrepError{FEM_E_INVALID_ARG, "reserved option fields must be zero"};
        fem_ctx *c = new fem_ctx();
        c->opt = o;
        *out = c;
    });
}

int fem_destroy(fem_ctx *ctx) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    reset_graph(ctx);
    delete ctx;
    return FEM_OK;
}

int fem_set_stream(fem_ctx *ctx, void *hip_stream) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    if (ctx->stream != (hipStream_t)hip_stream) reset_graph(ctx);
    ctx->stream = (hipStream_t)hip_stream;
    return FEM_OK;
}

int fem_upload_mesh(fem_ctx *ctx, int32_t elem_type, int64_t n_nodes, const double *xyz, int64_t n_elems,
                    const int32_t *conn, const int32_t *elem_mat) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "mesh must be uploaded before fem_finalize"};
        if (elem_type != FEM_TET4 && elem_type != FEM_HEX8) throw PrepError{FEM_E_INVALID_ARG, "elem_type must be 4 or 8"};
        if (n_nodes <= 0 || n_elems <= 0 || !xyz || !conn || !elem_mat) throw PrepError{FEM_E_INVALID_ARG, "empty mesh or null array"};
        if (n_nodes >= INT32_MAX || n_elems * elem_type >= INT32_MAX)
            throw PrepError{FEM_E_UNSUPPORTED, "mesh too large for 32-bit indices"};
        Problem p = ctx->prob;
        p.nen = elem_type;
        p.N = n_nodes;
        p.E = n_elems;
        p.xyz.assign(xyz, xyz + 3 * n_nodes);
        p.conn.assign(conn, conn + n_elems * elem_type);
        p.emat.assign(elem_mat, elem_mat + n_elems);
        for (int64_t i = 0; i < 3 * n_nodes; ++i)
            if (!std::isfinite(p.xyz[i])) throw PrepError{FEM_E_INVALID_ARG, "node coordinates must be finite"};
        if ((int64_t)p.T0.size() != n_nodes) p.T0.clear();
        ctx->prob = std::move(p);
        ctx->have_mesh = true;
    });
}

int fem_set_materials(fem_ctx *ctx, int32_t n_mat, const fem_material *m) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "materials must be set before fem_finalize"};
        if (n_mat <= 0 || n_mat > (int32_t)NODE_MAT_MASK || !m) throw PrepError{FEM_E_INVALID_ARG, "bad material table"};
        ctx->prob.mats.assign(m, m + n_mat);
    });
}

int fem_set_dirichlet(fem_ctx *ctx, int64_t n, const int32_t *node, const double *T_value) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "boundary sets must be given before fem_finalize"};
        if (n < 0 || (n > 0 && (!node || !T_value))) throw PrepError{FEM_E_INVALID_ARG, "bad fixed-temperature set"};
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(T_value[i])) throw PrepError{FEM_E_INVALID_ARG, "fixed temperature not finite"};
        ctx->prob.dir_nodes.assign(node, node + n);
        ctx->prob.dir_T.assign(T_value, T_value + n);
    });
}

int fem_set_flux_faces(fem_ctx *ctx, int64_t nf, int32_t nodes_per_face, const int32_t *face_nodes, const double *q,
                       const double *h, const double *T_inf) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "boundary sets must be given before fem_finalize"};
        if (nf < 0 || (nodes_per_face != 3 && nodes_per_face != 4)) throw PrepError{FEM_E_INVALID_ARG, "bad flux faces"};
        if (nf > 0 && (!face_nodes || !q || !h || !T_inf)) throw PrepError{FEM_E_INVALID_ARG, "null flux face array"};
        for (int64_t f = 0; f < nf; ++f)
            if (!std::isfinite(q[f]) || !std::isfinite(h[f]) || !std::isfinite(T_inf[f]) || h[f] < 0)
                throw PrepError{FEM_E_INVALID_ARG, "flux face values must be finite, h >= 0"};
        Problem &p = ctx->prob;
        p.npf = nodes_per_face;
        p.flux_faces.assign(face_nodes, face_nodes + nf * nodes_per_face);
        p.flux_q.assign(q, q + nf);
        p.flux_h.assign(h, h + nf);
        p.flux_Tinf.assign(T_inf, T_inf + nf);
    });
}

int fem_set_interface(fem_ctx *ctx, int64_t npairs, const int32_t *face_a, const int32_t *face_b, const double *h_i) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "interface must be given before fem_finalize"};
        if (npairs < 0 || (npairs > 0 && (!face_a || !face_b || !h_i))) throw PrepError{FEM_E_INVALID_ARG, "bad interface"};
        for (int64_t f = 0; f < npairs; ++f)
            if (!std::isfinite(h_i[f]) || h_i[f] < 0) throw PrepError{FEM_E_INVALID_ARG, "interface h must be finite, >= 0"};
        Problem &p = ctx->prob;
        p.if_a.assign(face_a, face_a + 3 * npairs);
        p.if_b.assign(face_b, face_b + 3 * npairs);
        p.if_h.assign(h_i, h_i + npairs);
    });
}

int fem_set_contact(fem_ctx *ctx, int64_t nf, const int32_t *face_nodes, const int32_t *side, const double *h) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "contact faces must be given before fem_finalize"};
        if (nf < 0 || (nf > 0 && (!face_nodes || !side || !h))) throw PrepError{FEM_E_INVALID_ARG, "bad contact faces"};
        if (nf >= INT32_MAX / 3) throw PrepError{FEM_E_UNSUPPORTED, "too many contact faces"};
        for (int64_t f = 0; f < nf; ++f) {
            if (!std::isfinite(h[f]) || h[f] < 0) throw PrepError{FEM_E_INVALID_ARG, "contact h must be finite, >= 0"};
            if (side[f] != 0 && side[f] != 1) throw PrepError{FEM_E_INVALID_ARG, "contact side must be 0 or 1"};
        }
        Problem &p = ctx->prob;
        p.contact_faces.assign(face_nodes, face_nodes + 3 * nf);
        p.contact_side.assign(side, side + nf);
        p.contact_h.assign(h, h + nf);
    });
}

int fem_get_sisters(const fem_ctx *ctx, int32_t *sister) {
    if (!ctx || !sister) return set_err(FEM_E_INVALID_ARG, "null argument");
    if (ctx->stage < ST_FINAL) return set_err(FEM_E_STATE, "call fem_finalize first");
    if (!ctx->base.sisters.empty()) std::memcpy(sister, ctx->base.sisters.data(), ctx->base.sisters.size() * sizeof(int32_t));
    return FEM_OK;
}

int fem_set_variable_properties(fem_ctx *ctx, int32_t n_mat, const fem_table *k_of_T, const fem_table *h_of_T,
                                const fem_table *h_of_t, const fem_table *dir_of_t) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "properties must be given before fem_finalize"};
        if (n_mat != (int32_t)ctx->prob.mats.size()) throw PrepError{FEM_E_INVALID_ARG, "n_mat must match the material table"};
        std::vector<Tab<double>> t(n_mat + TAB_GLOBAL);
        auto take = [&](const fem_table *src, Tab<double> &dst) {
            dst = Tab<double>{};
            if (!src || src->n == 0) return;
            if (src->n < 0 || src->n > TAB_POINTS) throw PrepError{FEM_E_INVALID_ARG, "a table holds 1 to 8 points"};
            for (int j = 0; j < src->n; ++j) {
                if (!std::isfinite(src->x[j]) || !std::isfinite(src->y[j]))
                    throw PrepError{FEM_E_INVALID_ARG, "table values must be finite"};
                if (j > 0 && !(src->x[j] > src->x[j - 1])) throw PrepError{FEM_E_INVALID_ARG, "table x must increase"};
                dst.x[j] = src->x[j];
                dst.y[j] = src->y[j];
            }
            dst.n = src->n;
        };
        for (int32_t q = 0; q < n_mat; ++q) {
            take(k_of_T ? &k_of_T[q] : nullptr, t[q]);
            for (int j = 0; j < t[q].n; ++j)
                if (!(t[q].y[j] > 0)) throw PrepError{FEM_E_INVALID_ARG, "conductivities must be positive"};
        }
        take(h_of_T, t[n_mat + TAB_H_OF_T]);
        take(h_of_t, t[n_mat + TAB_H_OF_TIME]);
        take(dir_of_t, t[n_mat + TAB_DIR_OF_TIME]);
        for (int g : {TAB_H_OF_T, TAB_H_OF_TIME})
            for (int j = 0; j < t[n_mat + g].n; ++j)
                if (t[n_mat + g].y[j] < 0) throw PrepError{FEM_E_INVALID_ARG, "interface factors must be >= 0"};
        ctx->vtabs = std::move(t);
    });
}

int fem_set_dirichlet_schedule(fem_ctx *ctx, int32_t n_times, const double *times, const double *values) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "the schedule must be given before fem_finalize"};
        const int64_t nd = (int64_t)ctx->prob.dir_nodes.size();
        if (nd == 0) throw PrepError{FEM_E_STATE, "no fixed-temperature nodes (fem_set_dirichlet first)"};
        if (n_times < 1 || n_times > TAB_POINTS) throw PrepError{FEM_E_INVALID_ARG, "a schedule holds 1 to 8 times"};
        if (!times || !values) throw PrepError{FEM_E_INVALID_ARG, "null schedule array"};
        for (int k = 0; k < n_times; ++k) {
            if (!std::isfinite(times[k])) throw PrepError{FEM_E_INVALID_ARG, "schedule times must be finite"};
            if (k > 0 && !(times[k] > times[k - 1])) throw PrepError{FEM_E_INVALID_ARG, "schedule times must increase"};
        }
        for (int64_t i = 0; i < nd * n_times; ++i)
            if (!std::isfinite(values[i])) throw PrepError{FEM_E_INVALID_ARG, "scheduled temperatures must be finite"};
        ctx->sched_t.assign(times, times + n_times);
        ctx->sched_T.assign(values, values + nd * n_times);
    });
}

int fem_set_initial_T(fem_ctx *ctx, const double *T0) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "initial field must be given before fem_finalize"};
        if (!ctx->have_mesh) throw PrepError{FEM_E_STATE, "upload the mesh first"};
        if (!T0) throw PrepError{FEM_E_INVALID_ARG, "T0 is null"};
        ctx->prob.T0.assign(T0, T0 + ctx->prob.N);
    });
}

int fem_finalize(fem_ctx *ctx, fem_prep_report *rep) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "already finalized"};
        if (!ctx->have_mesh) throw PrepError{FEM_E_STATE, "no mesh uploaded"};
        auto t0 = std::chrono::steady_clock::now();
        double sched_lo = INFINITY, sched_hi = -INFINITY;
        if (const size_t K = ctx->sched_t.size()) {
            // a node-by-node prescribed temperature: the context takes the
            // variable-property step, and every fixed node starts at f(x, 0)
            Problem &p = ctx->prob;
            if (ctx->sched_T.size() != p.dir_nodes.size() * K)
                throw PrepError{FEM_E_INVALID_ARG, "the schedule does not match the fixed-temperature set"};
            if (ctx->vtabs.empty()) ctx->vtabs.assign(p.mats.size() + TAB_GLOBAL, Tab<double>{});
            Tab<double> row{};
            row.n = (int32_t)K;
            for (size_t k = 0; k < K; ++k) row.x[k] = ctx->sched_t[k];
            for (size_t q = 0; q < p.dir_nodes.size(); ++q) {
                for (size_t k = 0; k < K; ++k) {
                    row.y[k] = ctx->sched_T[q * K + k];
                    sched_lo = std::min(sched_lo, row.y[k]);
                    sched_hi = std::max(sched_hi, row.y[k]);
                }
                p.dir_T[q] = tab_eval_host(row, 0.0);
            }
        }
        if (ctx->apparent()) {
            if (ctx->prob.nen != FEM_TET4) throw PrepError{FEM_E_UNSUPPORTED, "apparent capacity: linear tetrahedra only"};
            if (ctx->opt.scatter != FEM_SCATTER_LDS_BLOCKED)
                throw PrepError{FEM_E_UNSUPPORTED, "apparent capacity: LDS-blocked scatter only"};
            for (const fem_material &m : ctx->prob.mats)
                if (m.L > 0 && !(m.T_liq > m.T_sol))
                    throw PrepError{FEM_E_UNSUPPORTED, "apparent capacity needs T_liq > T_sol where L > 0"};
        }
        if (ctx->variable()) {
            if (ctx->opt.scatter != FEM_SCATTER_LDS_BLOCKED)
                throw PrepError{FEM_E_UNSUPPORTED, "variable properties: LDS-blocked scatter only"};
            if (ctx->apparent()) throw PrepError{FEM_E_UNSUPPORTED, "variable properties: enthalpy form only"};
            if ((int32_t)ctx->vtabs.size() != (int32_t)ctx->prob.mats.size() + TAB_GLOBAL)
                throw PrepError{FEM_E_INVALID_ARG, "variable properties: material count changed"};
        }
        Base base;
        prep_base(ctx->prob, base);
        if (ctx->variable()) {
            // stability bound and fixed-point range with every property at its largest value
            Problem pmax = ctx->prob;
            double hmax = 1.0;
            for (int g : {TAB_H_OF_T, TAB_H_OF_TIME}) hmax *= tab_max(ctx->vtabs[pmax.mats.size() + g], 1.0);
            for (size_t q = 0; q < pmax.mats.size(); ++q) pmax.mats[q].k = tab_max(ctx->vtabs[q], pmax.mats[q].k);
            for (double &h : pmax.if_h) h *= hmax;
            for (double &h : pmax.contact_h) h *= hmax;
            Base bmax;
            prep_base(pmax, bmax);
            base.dt_bound = bmax.dt_bound;
            base.dt_scen = bmax.dt_scen;
            base.elem_abs_max = bmax.elem_abs_max;
            const Tab<double> &sh = ctx->vtabs[pmax.mats.size() + TAB_DIR_OF_TIME];
            double smin = 0.0, smax = 0.0;
            for (int j = 0; j < sh.n; ++j) {
                smin = std::min(smin, sh.y[j]);
                smax = std::max(smax, sh.y[j]);
            }
            if (sched_hi >= sched_lo) {
                // the scheduled values join the span of the data (initial field, fixed and ambient temperatures)
                double lo = sched_lo, hi = sched_hi;
                for (double T : base.T_init) {
                    lo = std::min(lo, T);
                    hi = std::max(hi, T);
                }
                for (double T : ctx->prob.flux_Tinf) {
                    lo = std::min(lo, T);
                    hi = std::max(hi, T);
                }
                base.T_span = std::max(base.T_span, hi - lo);
            }
            base.T_span += smax - smin;
        }
        Ordering ord;
        prep_order(ctx->prob, base, ctx->opt.ordering, ord);
        std::vector<Candidate> cands;
        const size_t per = ctx->apparent() ? lds_per_node_apparent(ctx->opt.precision) : lds_per_node(ctx->opt.precision);
        const int thr = ctx->opt.threads ? ctx->opt.threads : 256;
        if (ctx->opt.scatter == FEM_SCATTER_LDS_BLOCKED && ctx->opt.block_elems == 0 && ctx->opt.lds_bytes == 0) {
            // autotune over block node sets (the paper's timed search over the block count);
            // small meshes also try small blocks, so that more compute units take part
            // (node cap, threads): larger blocks also with more threads, so that a
            // compute unit keeps its waves when fewer blocks fit its LDS
            std::vector<std::pair<int64_t, int>> tries;
            for (int64_t nodes : {128, 256, 512, 640, 768, 1024, 1536}) tries.push_back({nodes, thr});
            if (!ctx->opt.threads)
                for (const auto &t : {std::pair<int64_t, int>{1024, 512}, {2048, 1024}, {3072, 1024}})
                    tries.push_back(t);
            for (const auto &t : tries) {
                const int64_t nodes = t.first;
                if ((size_t)(nodes + 1) * per > MAX_BLOCK_LDS) continue;
                if (nodes < 512 && ctx->prob.N > 512 * 512) continue;
                Candidate c;
                c.o.ordering = ctx->opt.ordering;
                c.o.scatter = ctx->opt.scatter;
                c.o.max_local_nodes = nodes;
                c.o.block_elems = 1 << 20;
                c.threads = t.second;
                cands.push_back(std::move(c));
            }
        } else {
            Candidate c;
            c.o.ordering = ctx->opt.ordering;
            c.o.scatter = ctx->opt.scatter;
            const size_t lds = ctx->opt.lds_bytes ? (size_t)ctx->opt.lds_bytes : (size_t)65536;
            if (lds > MAX_BLOCK_LDS) throw PrepError{FEM_E_INVALID_ARG, "lds_bytes above the gfx950 limit"};
            c.o.max_local_nodes = std::min<int64_t>(65535, (int64_t)(lds / per));
            c.o.block_elems = ctx->opt.block_elems ? ctx->opt.block_elems : (1 << 20);
            c.threads = thr;
            cands.push_back(std::move(c));
        }
        // matched interface pairs become elements of the blocks in the enthalpy
        // step with constant properties (the other forms keep them as node links)
        for (Candidate &cd : cands) cd.o.interface_in_blocks = !ctx->apparent() && !ctx->variable();
        // candidate layouts are independent: build them concurrently
        std::vector<PrepError> errs(cands.size(), PrepError{FEM_OK, ""});
#pragma omp parallel for schedule(dynamic, 1)
        for (int q = 0; q < (int)cands.size(); ++q) {
            try {
                prep_layout(ctx->prob, base, cands[q].o, ord, cands[q].L);
            } catch (const PrepError &e) {
                errs[q] = e;
            } catch (const std::bad_alloc &) {
                errs[q] = PrepError{FEM_E_INVALID_ARG, "host allocation failed"};
            }
        }
        for (const PrepError &e : errs)
            if (e.code != FEM_OK) throw e;
        ctx->base = std::move(base);
        ctx->cands = std::move(cands);
        ctx->chosen = 0;
        for (int b = 0; b < B_COUNT; ++b) ctx->sizes[b] = 0;
        for (const Candidate &c : ctx->cands) {
            int64_t sz[B_COUNT];
            layout_sizes(ctx, c.L, sz);
            for (int b = 0; b < B_COUNT; ++b) ctx->sizes[b] = std::max(ctx->sizes[b], sz[b]);
        }
        ctx->cap_bound = ctx->apparent() ? apparent_cap_bound(ctx->prob) : 0.0;
        ctx->mats_host.resize(ctx->prob.mats.size());
        for (size_t q = 0; q < ctx->prob.mats.size(); ++q) ctx->mats_host[q] = make_mat(ctx->prob.mats[q], 0.0);
        ctx->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        ctx->stage = ST_FINAL;
        if (rep) fill_report(ctx, rep);
    });
}

int fem_get_report(const fem_ctx *ctx, fem_prep_report *rep) {
    if (!ctx || !rep) return set_err(FEM_E_INVALID_ARG, "null argument");
    if (ctx->stage < ST_FINAL) return set_err(FEM_E_STATE, "not finalized");
    fill_report(ctx, rep);
    return FEM_OK;
}

int fem_query_buffers(const fem_ctx *ctx, fem_buffer_desc *d, int32_t *n) {
    if (!ctx || !n) return set_err(FEM_E_INVALID_ARG, "null argument");
    if (ctx->stage < ST_FINAL) return set_err(FEM_E_STATE, "call fem_finalize first");
    if (!d) {
        *n = B_COUNT;
        return FEM_OK;
    }
    if (*n < B_COUNT) return set_err(FEM_E_INVALID_ARG, "descriptor array too short");
    for (int b = 0; b < B_COUNT; ++b) {
        std::memset(&d[b], 0, sizeof(fem_buffer_desc));
        std::strncpy(d[b].name, BUF_NAMES[b], sizeof(d[b].name) - 1);
        d[b].bytes = ctx->sizes[b] ? rup(ctx->sizes[b]) : 0;
        d[b].alignment = ALIGN;
    }
    *n = B_COUNT;
    return FEM_OK;
}

int fem_bind_buffers(fem_ctx *ctx, void *const *dev_ptrs, int32_t n) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_FINAL) throw PrepError{FEM_E_STATE, "call fem_finalize (once) before binding"};
        if (n != B_COUNT || !dev_ptrs) throw PrepError{FEM_E_INVALID_ARG, "wrong number of device buffers"};
        for (int b = 0; b < B_COUNT; ++b) {
            if (ctx->sizes[b] > 0 && !dev_ptrs[b]) throw PrepError{FEM_E_INVALID_ARG, std::string("null buffer ") + BUF_NAMES[b]};
            if ((uintptr_t)dev_ptrs[b] % ALIGN) throw PrepError{FEM_E_INVALID_ARG, std::string("misaligned buffer ") + BUF_NAMES[b]};
        }
        HIPCHECK(hipSetDevice(ctx->opt.device));
        for (int b = 0; b < B_COUNT; ++b) ctx->ptr[b] = ctx->sizes[b] ? dev_ptrs[b] : nullptr;
        reset_graph(ctx);
        ctx->diag_fresh = false;
        if (ctx->opt.scatter == FEM_SCATTER_LDS_BLOCKED) {
            hipDeviceProp_t prop;
            HIPCHECK(hipGetDeviceProperties(&prop, ctx->opt.device));
            size_t mx = 0;
            const size_t per = ctx->apparent() ? lds_per_node_apparent(ctx->opt.precision) : lds_per_node(ctx->opt.precision);
            for (const Candidate &c : ctx->cands) mx = std::max(mx, (size_t)(c.L.max_local + 1) * per);
            const size_t cap = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor : prop.sharedMemPerBlock;
            if (mx + 1024 > cap) throw PrepError{FEM_E_UNSUPPORTED, "block LDS footprint above the device limit"};
            if (ctx->apparent()) HIPCHECK(set_apparent_lds_limit(ctx->opt.precision, mx));
            else if (ctx->variable()) HIPCHECK(set_var_lds_limit(ctx->opt.precision, ctx->prob.nen, mx));
            else HIPCHECK(set_block_lds_limit(ctx->opt.precision, ctx->prob.nen, mx));
        }
        ctx->dt_s.clear();
        if (ctx->cands.size() > 1) {
            // timed trial steps per candidate layout; keep the fastest
            const double dt = 0.5 * ctx->base.dt_bound;
            hipEvent_t e0, e1;
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
            // steps of one candidate from the initial state: eager, or (graphs) in
            // whole captured graphs of GRAPH_STEPS steps with their state
            // reductions, as fem_step runs them
            auto trial = [&](size_t q, int steps, bool graphs) {
                ctx->chosen = (int)q;
                if (ctx->opt.precision == FEM_PREC_FP64) upload_layout_t<double>(ctx, ctx->cands[q].L);
                else upload_layout_t<float>(ctx, ctx->cands[q].L);
                fill_dev(ctx, ctx->cands[q]);
                set_dt(ctx, dt);
                ctx->parity = 0;
                graphs = graphs && ctx->stream != nullptr;
                if (graphs) {
                    reset_graph(ctx);
                    build_graph(ctx);
                    steps = std::max(1, steps / GRAPH_STEPS) * GRAPH_STEPS;
                    HIPCHECK(hipGraphLaunch(ctx->gexec, ctx->stream));
                } else {
                    eager_steps(ctx, 4);
                }
                HIPCHECK(hipEventRecord(e0, ctx->stream));
                if (graphs)
                    for (int r = 0; r < steps / GRAPH_STEPS; ++r) HIPCHECK(hipGraphLaunch(ctx->gexec, ctx->stream));
                else
                    eager_steps(ctx, steps);
                HIPCHECK(hipEventRecord(e1, ctx->stream));
                HIPCHECK(hipEventSynchronize(e1));
                if (graphs) reset_graph(ctx);
                float ms = 0;
                HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
                return ms / (double)steps;
            };
            for (size_t q = 0; q < ctx->cands.size(); ++q) ctx->cands[q].ms = trial(q, 20, false);
            // the three fastest again as the timed path runs, in captured graphs, over
            // at least 50 ms of steps: candidates within a few per cent of each other
            // are told apart by the second trial, not by the noise of the first
            std::vector<size_t> rank(ctx->cands.size());
            std::iota(rank.begin(), rank.end(), (size_t)0);
            std::sort(rank.begin(), rank.end(), [&](size_t a, size_t b) { return ctx->cands[a].ms < ctx->cands[b].ms; });
            const size_t finalists = std::min<size_t>(3, rank.size());
            for (size_t r = 0; r < finalists; ++r) {
                const double ms1 = ctx->cands[rank[r]].ms;
                const int n2 = (int)std::min(4000.0, std::max(64.0, 50.0 / std::max(ms1, 1e-3)));
                ctx->cands[rank[r]].ms = trial(rank[r], n2, true);
            }
            // a candidate outside the finalists keeps its eager time, which counts its
            // launch gaps: it cannot be picked over a finalist timed in graphs
            for (size_t r = finalists; r < rank.size(); ++r) ctx->cands[rank[r]].ms = 1e30;
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            int best = 0;
            for (size_t q = 1; q < ctx->cands.size(); ++q)
                if (ctx->cands[q].ms < ctx->cands[best].ms) best = (int)q;
            ctx->chosen = best;
        }
        if (ctx->opt.precision == FEM_PREC_FP64) upload_layout_t<double>(ctx, ctx->L());
        else upload_layout_t<float>(ctx, ctx->L());
        fill_dev(ctx, ctx->cands[ctx->chosen]);
        ctx->dt_s.clear();
        ctx->time_s.assign(ctx->prob.n_scen, 0.0);
        ctx->Qx_s.assign(ctx->prob.n_scen, 0.0);
        ctx->parity = 0;
        ctx->steps = 0;
        // drop the layouts that lost the trial
        Candidate keep = std::move(ctx->cands[ctx->chosen]);
        ctx->cands.clear();
        ctx->cands.push_back(std::move(keep));
        ctx->chosen = 0;
        fill_dev(ctx, ctx->cands[0]);
        // the whole material table on the device (dt = 0 until a step sets it):
        // fem_step_no_alloc updates only its time-step fields
        for (size_t q = 0; q < ctx->prob.mats.size(); ++q) ctx->mats_host[q] = make_mat(ctx->prob.mats[q], 0.0);
        h2d(ctx, B_MATS, ctx->mats_host.data(), (int64_t)(ctx->mats_host.size() * sizeof(MatDev)));
        HIPCHECK(hipStreamSynchronize(ctx->stream));
        ctx->stage = ST_BOUND;
    });
}

int fem_stable_dt(const fem_ctx *ctx, double *dt) {
    if (!ctx || !dt) return set_err(FEM_E_INVALID_ARG, "null argument");
    if (ctx->stage < ST_FINAL) return set_err(FEM_E_STATE, "call fem_finalize first");
    *dt = ctx->base.dt_bound;
    return FEM_OK;
}

int fem_step(fem_ctx *ctx, double dt, int64_t n_steps) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (!(dt > 0) || !std::isfinite(dt) || n_steps < 0) throw PrepError{FEM_E_INVALID_ARG, "dt must be > 0 and n_steps >= 0"};
        if (dt > ctx->base.dt_bound && !ctx->opt.allow_unstable)
            throw PrepError{FEM_E_UNSTABLE, "dt " + std::to_string(dt) + " above the stability bound " + std::to_string(ctx->base.dt_bound)};
        set_dt(ctx, dt);
        run_steps(ctx, n_steps);
        ctx->steps += n_steps;
        for (double &t : ctx->time_s) t += dt * (double)n_steps;
    });
}

int fem_step_no_alloc(fem_ctx *ctx, double dt, int64_t n_steps) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (!(dt > 0) || !std::isfinite(dt) || n_steps < 0) throw PrepError{FEM_E_INVALID_ARG, "dt must be > 0 and n_steps >= 0"};
        if (dt > ctx->base.dt_bound && !ctx->opt.allow_unstable)
            throw PrepError{FEM_E_UNSTABLE, "dt " + std::to_string(dt) + " above the stability bound " + std::to_string(ctx->base.dt_bound)};
        if (ctx->apparent() || ctx->variable() || ctx->prob.n_scen != 1 || ctx->opt.scatter != FEM_SCATTER_LDS_BLOCKED)
            throw PrepError{FEM_E_UNSUPPORTED, "fem_step_no_alloc: enthalpy form, one scenario, LDS-blocked scatter"};
        const Layout &L = ctx->L();
        const int64_t bytes = L.n_partial_slots * (int64_t)ctx->rsize();
        if (bytes > SCRATCH_BYTES)
            throw PrepError{FEM_E_UNSUPPORTED, "fem_step_no_alloc: the mesh needs " + std::to_string(bytes) +
                                                   " bytes of partial residuals; the static scratch holds " +
                                                   std::to_string(SCRATCH_BYTES) + " (use fem_step)"};
        HIPCHECK(hipSetDevice(ctx->opt.device));
        void *sp = nullptr;
        HIPCHECK(scratch_address(ctx->opt.device, &sp));
        for (int b = 0; b < B_COUNT; ++b)
            if (ctx->ptr[b] && (char *)ctx->ptr[b] < (char *)sp + SCRATCH_BYTES && (char *)sp < (char *)ctx->ptr[b] + ctx->sizes[b])
                throw PrepError{FEM_E_HIP, std::string("internal: the static scratch overlaps buffer ") + BUF_NAMES[b]};
        // slots a shared node has no block for must read zero: clear the region
        // this mesh uses (the last call on this GPU, of any context, left its own)
        HIPCHECK(enqueue_zero(sp, bytes, ctx->stream));
        if (ctx->dt_s.size() != 1 || ctx->dt_s[0] != dt) {
            HIPCHECK(enqueue_set_dt((MatDev *)ctx->ptr[B_MATS], (int)ctx->prob.mats.size(), dt, ctx->stream));
            for (size_t q = 0; q < ctx->mats_host.size(); ++q) ctx->mats_host[q] = make_mat(ctx->prob.mats[q], dt);
            ctx->dt_s.assign(1, dt);
        }
        ctx->diag_fresh = false;
        Dev d = ctx->dev;
        d.partials = sp;
        for (int64_t k = 0; k < n_steps; ++k) {
            HIPCHECK(enqueue_step(d, ctx->parity, ctx->stream, nullptr));
            ctx->parity ^= 1;
        }
        ctx->steps += n_steps;
        for (double &t : ctx->time_s) t += dt * (double)n_steps;
    });
}

int fem_step_batch(fem_ctx *ctx, const double *dt_per_scenario, int64_t n_steps) {
    if (!ctx || !dt_per_scenario) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (n_steps < 0) throw PrepError{FEM_E_INVALID_ARG, "n_steps must be >= 0"};
        std::vector<double> dt(dt_per_scenario, dt_per_scenario + ctx->prob.n_scen);
        for (int32_t sc = 0; sc < ctx->prob.n_scen; ++sc) {
            if (!(dt[sc] > 0) || !std::isfinite(dt[sc])) throw PrepError{FEM_E_INVALID_ARG, "every dt must be > 0"};
            if (dt[sc] > ctx->base.dt_scen[sc] && !ctx->opt.allow_unstable)
                throw PrepError{FEM_E_UNSTABLE, "dt of scenario " + std::to_string(sc) + " above its stability bound"};
        }
        set_dt_scen(ctx, dt);
        run_steps(ctx, n_steps);
        ctx->steps += n_steps;
        for (int32_t sc = 0; sc < ctx->prob.n_scen; ++sc) ctx->time_s[sc] += dt[sc] * (double)n_steps;
    });
}

int fem_set_scenarios(fem_ctx *ctx, int32_t n_scen, const int32_t *material_scenario) {
    if (!ctx) return set_err(FEM_E_INVALID_ARG, "ctx is null");
    return guarded([&] {
        if (ctx->stage != ST_NEW) throw PrepError{FEM_E_STATE, "scenarios must be set before fem_finalize"};
        if (ctx->prob.mats.empty()) throw PrepError{FEM_E_STATE, "set the materials first"};
        if (n_scen < 1 || !material_scenario) throw PrepError{FEM_E_INVALID_ARG, "bad scenario table"};
        std::vector<int32_t> ms(material_scenario, material_scenario + ctx->prob.mats.size());
        std::vector<char> used(n_scen, 0);
        for (int32_t sc : ms) {
            if (sc < 0 || sc >= n_scen) throw PrepError{FEM_E_INVALID_ARG, "scenario id out of range"};
            used[sc] = 1;
        }
        for (char u : used)
            if (!u) throw PrepError{FEM_E_INVALID_ARG, "every scenario needs at least one material"};
        ctx->prob.n_scen = n_scen;
        ctx->prob.mat_scen = std::move(ms);
    });
}

int fem_stable_dt_scenarios(const fem_ctx *ctx, double *dt_bounds) {
    if (!ctx || !dt_bounds) return set_err(FEM_E_INVALID_ARG, "null argument");
    if (ctx->stage < ST_FINAL) return set_err(FEM_E_STATE, "call fem_finalize first");
    for (int32_t sc = 0; sc < ctx->prob.n_scen; ++sc) dt_bounds[sc] = ctx->base.dt_scen[sc];
    return FEM_OK;
}

}  // extern "C"

namespace {

template <class R>
void read_node_array(fem_ctx *c, const void *dev, double *out) {
    const Layout &L = c->L();
    std::vector<R> h(L.N);
    HIPCHECK(hipMemcpyAsync(h.data(), dev, L.N * sizeof(R), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < L.N; ++i) out[i] = (double)h[L.perm[i]];
}

const void *T_dev(fem_ctx *c) { return (const char *)c->ptr[B_T] + (size_t)c->parity * c->L().N * c->rsize(); }

}  // namespace

extern "C" {

int fem_read_T(fem_ctx *ctx, double *T_host) {
    if (!ctx || !T_host) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (ctx->opt.precision == FEM_PREC_FP64) read_node_array<double>(ctx, T_dev(ctx), T_host);
        else read_node_array<float>(ctx, T_dev(ctx), T_host);
    });
}

int fem_read_fs(fem_ctx *ctx, double *fs_host) {
    if (!ctx || !fs_host) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (ctx->opt.precision == FEM_PREC_FP64) read_node_array<double>(ctx, ctx->ptr[B_FS], fs_host);
        else read_node_array<float>(ctx, ctx->ptr[B_FS], fs_host);
    });
}

int fem_read_H(fem_ctx *ctx, double *H_host) {
    if (!ctx || !H_host) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        const Layout &L = ctx->L();
        std::vector<uint8_t> h(L.N * 8);
        HIPCHECK(hipMemcpyAsync(h.data(), ctx->ptr[B_H], L.N * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHECK(hipStreamSynchronize(ctx->stream));
        for (int64_t i = 0; i < L.N; ++i) {
            const int64_t n = L.perm[i];
            if (ctx->opt.precision == FEM_PREC_FP64) {
                std::memcpy(&H_host[i], &h[8 * n], 8);
            } else {
                float hi, lo;
                std::memcpy(&hi, &h[8 * n], 4);
                std::memcpy(&lo, &h[8 * n + 4], 4);
                H_host[i] = (double)hi + (double)lo;
            }
        }
    });
}

}  // extern "C"

namespace castfem {

// FP64 energy balance per scenario (reps[n_scen]): on-demand state reduction
// over single-scenario node segments plus the per-node inflow sums, all summed
// on the host in a fixed order
void energy_copies(fem_ctx *ctx, std::vector<double> &dg, std::vector<double> &qn) {
    const Layout &L = ctx->L();
    const int64_t S = (int64_t)L.seg_scen.size(), Q = L.n_inflow;
    dg.resize(S * NDIAG);
    qn.resize(Q);
    HIPCHECK(hipMemcpyAsync(dg.data(), ctx->ptr[B_DIAG], S * NDIAG * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (Q) HIPCHECK(hipMemcpyAsync(qn.data(), ctx->ptr[B_QNODE], Q * 8, hipMemcpyDeviceToHost, ctx->stream));
}

void energy_scenarios(fem_ctx *ctx, fem_energy_report *reps) {
    std::vector<double> dg, qn;
    if (!ctx->diag_fresh) HIPCHECK(enqueue_state_diag(ctx->dev, ctx->parity, ctx->stream));
    energy_copies(ctx, dg, qn);
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    HIPCHECK(hipGetLastError());
    energy_reduce(ctx, dg, qn, reps);
}

void energy_reduce(const fem_ctx *ctx, const std::vector<double> &dg, const std::vector<double> &qn,
                   fem_energy_report *reps) {
    const int32_t ns = ctx->prob.n_scen;
    const Layout &L = ctx->L();
    const int64_t S = (int64_t)L.seg_scen.size(), Q = L.n_inflow;
    for (int32_t sc = 0; sc < ns; ++sc) {
        std::memset(&reps[sc], 0, sizeof(fem_energy_report));
        reps[sc].E0 = ctx->E0_s[sc];
        reps[sc].T_min = INFINITY;
        reps[sc].T_max = -INFINITY;
        reps[sc].steps = ctx->steps;
        reps[sc].time = ctx->time_s[sc];
    }
    std::vector<double> nl(ns, 0.0), nf(ns, 0.0);
    for (int64_t g = 0; g < S; ++g) {
        fem_energy_report &r = reps[L.seg_scen[g]];
        const double *v = &dg[g * NDIAG];
        r.E += v[DG_E];
        r.latent += v[DG_LAT];
        r.T_min = std::min(r.T_min, v[DG_TMIN]);
        r.T_max = std::max(r.T_max, v[DG_TMAX]);
        nl[L.seg_scen[g]] += v[DG_NLIQ];
        nf[L.seg_scen[g]] += v[DG_NONFIN];
    }
    for (int64_t q = 0; q < Q; ++q)
        reps[ctx->prob.scen_of_mat((int32_t)(L.nflag[L.bc_first + q] & NODE_MAT_MASK))].Q_cum += qn[q];
    for (int32_t sc = 0; sc < ns; ++sc) {
        fem_energy_report &r = reps[sc];
        r.Q_cum += ctx->Qx_s[sc];
        r.n_liquid = (int64_t)nl[sc];
        r.nonfinite = (int64_t)nf[sc];
        r.residual = std::fabs(r.E - r.E0 - r.Q_cum) / std::fabs(r.E0 - ctx->Eref_s[sc]);
    }
}

}  // namespace castfem

extern "C" {

int fem_energy(fem_ctx *ctx, fem_energy_report *rep) {
    if (!ctx || !rep) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        std::vector<fem_energy_report> r(ctx->prob.n_scen);
        energy_scenarios(ctx, r.data());
        // the whole problem: sums over scenarios in order
        std::memset(rep, 0, sizeof(*rep));
        rep->T_min = INFINITY;
        rep->T_max = -INFINITY;
        double Eref = 0.0;
        for (int32_t sc = 0; sc < ctx->prob.n_scen; ++sc) {
            rep->E += r[sc].E;
            rep->E0 += r[sc].E0;
            rep->latent += r[sc].latent;
            rep->Q_cum += r[sc].Q_cum;
            rep->T_min = std::min(rep->T_min, r[sc].T_min);
            rep->T_max = std::max(rep->T_max, r[sc].T_max);
            rep->n_liquid += r[sc].n_liquid;
            rep->nonfinite += r[sc].nonfinite;
            rep->time = std::max(rep->time, r[sc].time);
            Eref += ctx->Eref_s[sc];
        }
        rep->steps = ctx->steps;
        rep->residual = std::fabs(rep->E - rep->E0 - rep->Q_cum) / std::fabs(rep->E0 - Eref);
        if (rep->nonfinite > 0 || !std::isfinite(rep->E))
            throw PrepError{FEM_E_NONFINITE, "the state holds non-finite enthalpy at " + std::to_string(rep->nonfinite) + " nodes"};
    });
}

int fem_energy_scenarios(fem_ctx *ctx, fem_energy_report *reps) {
    if (!ctx || !reps) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        energy_scenarios(ctx, reps);
        for (int32_t sc = 0; sc < ctx->prob.n_scen; ++sc)
            if (reps[sc].nonfinite > 0 || !std::isfinite(reps[sc].E))
                throw PrepError{FEM_E_NONFINITE, "scenario " + std::to_string(sc) + " holds non-finite enthalpy"};
    });
}

}  // extern "C"

namespace {

// Checkpoints hold every per-node array in input-node order (the numbering
// of fem_upload_mesh), so a state restores into any layout of the same
// problem: another ordering, block size or autotuner choice.  Layout: header,
// H (8 B per node: FP64, or the FP32 hi/lo pair), T of the current step and
// f_s (R per node), the inflow sums of the nodes carrying boundary inflow
// (FP64, in increasing input id), time and estimated jumped inflow per scenario.
struct CkptHeader {
    uint64_t magic, N, prec, n_inflow, n_scen;
    int64_t parity, steps;
};
constexpr uint64_t CKPT_MAGIC = 0x33504B434D454643ull;

int64_t ckpt_bytes(const fem_ctx *ctx) {
    const int64_t N = ctx->L().N, R = (int64_t)ctx->rsize();
    return (int64_t)sizeof(CkptHeader) + N * 8 + N * R + N * R + ctx->L().n_inflow * 8 + 2 * ctx->prob.n_scen * 8;
}

// inflow slots of the layout in increasing input id of their nodes
std::vector<int64_t> inflow_slots_by_input(const Layout &L) {
    std::vector<int64_t> q(L.n_inflow);
    for (int64_t k = 0; k < L.n_inflow; ++k) q[k] = k;
    std::sort(q.begin(), q.end(), [&](int64_t a, int64_t b) { return L.iperm[L.bc_first + a] < L.iperm[L.bc_first + b]; });
    return q;
}

// out[input i] = in[device perm[i]] for N items of `w` bytes (or the reverse)
void permute_items(const Layout &L, const char *in, char *out, int64_t w, bool to_input) {
    for (int64_t i = 0; i < L.N; ++i) {
        const int64_t dv = L.perm[i];
        if (to_input) std::memcpy(out + i * w, in + dv * w, w);
        else std::memcpy(out + dv * w, in + i * w, w);
    }
}

}  // namespace

extern "C" {

int fem_read_state(fem_ctx *ctx, void *buf, int64_t *bytes) {
    if (!ctx || !bytes) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        const Layout &L = ctx->L();
        const int64_t N = L.N, R = (int64_t)ctx->rsize(), Q = L.n_inflow;
        const int64_t need = ckpt_bytes(ctx);
        if (!buf) {
            *bytes = need;
            return;
        }
        if (*bytes < need) throw PrepError{FEM_E_INVALID_ARG, "checkpoint buffer too small"};
        std::vector<char> H(N * 8), T(N * R), fs(N * R);
        std::vector<double> qn(Q);
        HIPCHECK(hipMemcpyAsync(H.data(), ctx->ptr[B_H], N * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHECK(hipMemcpyAsync(T.data(), (char *)ctx->ptr[B_T] + ctx->parity * N * R, N * R, hipMemcpyDeviceToHost,
                                ctx->stream));
        HIPCHECK(hipMemcpyAsync(fs.data(), ctx->ptr[B_FS], N * R, hipMemcpyDeviceToHost, ctx->stream));
        if (Q) HIPCHECK(hipMemcpyAsync(qn.data(), ctx->ptr[B_QNODE], Q * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHECK(hipStreamSynchronize(ctx->stream));
        CkptHeader h{CKPT_MAGIC, (uint64_t)N, (uint64_t)ctx->opt.precision, (uint64_t)Q, (uint64_t)ctx->prob.n_scen,
                     ctx->parity, ctx->steps};
        char *p = (char *)buf;
        std::memcpy(p, &h, sizeof h);
        p += sizeof h;
        permute_items(L, H.data(), p, 8, true);
        p += N * 8;
        permute_items(L, T.data(), p, R, true);
        p += N * R;
        permute_items(L, fs.data(), p, R, true);
        p += N * R;
        const std::vector<int64_t> order = inflow_slots_by_input(L);
        for (int64_t k = 0; k < Q; ++k) std::memcpy(p + 8 * k, &qn[order[k]], 8);
        p += Q * 8;
        std::memcpy(p, ctx->time_s.data(), ctx->prob.n_scen * 8);
        p += ctx->prob.n_scen * 8;
        std::memcpy(p, ctx->Qx_s.data(), ctx->prob.n_scen * 8);
        *bytes = need;
    });
}

int fem_write_state(fem_ctx *ctx, const void *buf, int64_t bytes) {
    if (!ctx || !buf) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (ctx->variable()) throw PrepError{FEM_E_UNSUPPORTED, "checkpoints of time-dependent properties"};
        const Layout &L = ctx->L();
        const int64_t N = L.N, R = (int64_t)ctx->rsize(), Q = L.n_inflow;
        if (bytes < ckpt_bytes(ctx)) throw PrepError{FEM_E_INVALID_ARG, "checkpoint too small"};
        CkptHeader h;
        std::memcpy(&h, buf, sizeof h);
        if (h.magic != CKPT_MAGIC || h.N != (uint64_t)N || h.prec != (uint64_t)ctx->opt.precision ||
            h.n_inflow != (uint64_t)Q || h.n_scen != (uint64_t)ctx->prob.n_scen || (h.parity != 0 && h.parity != 1))
            throw PrepError{FEM_E_INVALID_ARG, "checkpoint does not match this context"};
        const char *p = (const char *)buf + sizeof h;
        std::vector<char> H(N * 8), T(N * R), fs(N * R);
        std::vector<double> qn(Q);
        permute_items(L, p, H.data(), 8, false);
        p += N * 8;
        permute_items(L, p, T.data(), R, false);
        p += N * R;
        permute_items(L, p, fs.data(), R, false);
        p += N * R;
        const std::vector<int64_t> order = inflow_slots_by_input(L);
        for (int64_t k = 0; k < Q; ++k) std::memcpy(&qn[order[k]], p + 8 * k, 8);
        p += Q * 8;
        std::vector<double> time_s(ctx->prob.n_scen), Qx_s(ctx->prob.n_scen);
        std::memcpy(time_s.data(), p, ctx->prob.n_scen * 8);
        p += ctx->prob.n_scen * 8;
        std::memcpy(Qx_s.data(), p, ctx->prob.n_scen * 8);
        const int par = (int)h.parity;
        ctx->diag_fresh = false;
        HIPCHECK(hipMemcpyAsync(ctx->ptr[B_H], H.data(), N * 8, hipMemcpyHostToDevice, ctx->stream));
        HIPCHECK(hipMemcpyAsync((char *)ctx->ptr[B_T] + par * N * R, T.data(), N * R, hipMemcpyHostToDevice,
                                ctx->stream));
        HIPCHECK(hipMemcpyAsync(ctx->ptr[B_FS], fs.data(), N * R, hipMemcpyHostToDevice, ctx->stream));
        if (Q) HIPCHECK(hipMemcpyAsync(ctx->ptr[B_QNODE], qn.data(), Q * 8, hipMemcpyHostToDevice, ctx->stream));
        HIPCHECK(hipStreamSynchronize(ctx->stream));
        ctx->time_s = time_s;
        ctx->Qx_s = Qx_s;
        ctx->parity = par;
        ctx->steps = h.steps;
    });
}

int fem_get_node_perm(const fem_ctx *ctx, int32_t *perm) {
    if (!ctx || !perm) return set_err(FEM_E_INVALID_ARG, "null argument");
    if (ctx->stage < ST_FINAL) return set_err(FEM_E_STATE, "call fem_finalize first");
    const Layout &L = ctx->L();
    std::memcpy(perm, L.perm.data(), L.N * sizeof(int32_t));
    return FEM_OK;
}

int fem_time_kernels(fem_ctx *ctx, double dt, int64_t n_steps, fem_kernel_times *out) {
    if (!ctx || !out) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        check_bound(ctx, ST_BOUND);
        if (n_steps <= 0 || n_steps > 100000) throw PrepError{FEM_E_INVALID_ARG, "n_steps must be in 1..100000"};
        if (!(dt > 0) || (dt > ctx->base.dt_bound && !ctx->opt.allow_unstable)) throw PrepError{FEM_E_UNSTABLE, "bad dt"};
        set_dt(ctx, dt);
        ctx->diag_fresh = false;
        std::vector<hipEvent_t> ev(4 * n_steps);
        for (auto &e : ev) HIPCHECK(hipEventCreate(&e));
        for (int64_t s = 0; s < n_steps; ++s) {
            HIPCHECK(enqueue_ctx_step(ctx, ctx->parity, ctx->stream, &ev[4 * s]));
            ctx->parity ^= 1;
        }
        HIPCHECK(hipEventSynchronize(ev.back()));
        double a = 0, b = 0;
        for (int64_t s = 0; s < n_steps; ++s) {
            float m1 = 0, m2 = 0;
            HIPCHECK(hipEventElapsedTime(&m1, ev[4 * s], ev[4 * s + 1]));
            HIPCHECK(hipEventElapsedTime(&m2, ev[4 * s + 2], ev[4 * s + 3]));
            a += m1;
            b += m2;
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
        ctx->steps += n_steps;
        for (double &t : ctx->time_s) t += dt * (double)n_steps;
        const Layout &L = ctx->L();
        const double R = (double)ctx->rsize();
        const double gather = 4.0 * R + 4.0;             // xyz + T read + flags
        // 1/m (enthalpy form only), H read+write, T and fs write
        const double update = (ctx->apparent() ? 0.0 : R) + 16.0 + 2.0 * R;
        const double elem = 4.0 * L.nen;                 // connectivity
        const bool blocked = ctx->opt.scatter == FEM_SCATTER_LDS_BLOCKED;
        const double upd_k1 = blocked ? (double)L.n_private : 0.0;
        std::memset(out, 0, sizeof(*out));
        out->launches_element = n_steps * (ctx->opt.scatter == FEM_SCATTER_COLORED ? (int64_t)ctx->dev.n_colors : 1);
        out->launches_combine = n_steps;
        out->ms_element = a / (double)n_steps;
        out->ms_combine = b / (double)n_steps;
        out->bytes_element = elem * (double)L.E + gather * (double)L.N + update * upd_k1;
        out->bytes_combine = update * ((double)L.N - upd_k1);
    });
}

namespace {
int timed_copy(fem_ctx *ctx, void *dst, const void *src, int64_t bytes, int32_t repeats, double *ms_per_copy,
               hipError_t (*copy)(void *, const void *, int64_t, hipStream_t)) {
    if (!ctx || !dst || !src || !ms_per_copy) return set_err(FEM_E_INVALID_ARG, "null argument");
    return guarded([&] {
        if (bytes <= 0 || bytes % 16 || repeats <= 0) throw PrepError{FEM_E_INVALID_ARG, "bytes must be a positive multiple of 16"};
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        HIPCHECK(copy(dst, src, bytes / 16, ctx->stream));
        HIPCHECK(hipEventRecord(e0, ctx->stream));
        for (int r = 0; r < repeats; ++r) HIPCHECK(copy(dst, src, bytes / 16, ctx->stream));
        HIPCHECK(hipEventRecord(e1, ctx->stream));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms_per_copy = ms / repeats;
    });
}
}  // namespace

int fem_copy_kernel(fem_ctx *ctx, void *dst, const void *src, int64_t bytes, int32_t repeats, double *ms_per_copy) {
    return timed_copy(ctx, dst, src, bytes, repeats, ms_per_copy, enqueue_copy);
}

int fem_copy_kernel_nt(fem_ctx *ctx, void *dst, const void *src, int64_t bytes, int32_t repeats, double *ms_per_copy) {
    return timed_copy(ctx, dst, src, bytes, repeats, ms_per_copy, enqueue_copy_nt);
}

}  // extern "C"
