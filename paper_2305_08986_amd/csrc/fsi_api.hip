// Host runtime and C ABI of the generalized-Stokes hot path: level hierarchy
// (Sec. 4: uniformly refined boxes), geometry/coefficient setup, the
// preconditioner setup, the monolithic block V-cycle with the smoother K_j of
// Sec. 4, FGMRES (Sec. 5, linear solver settings), HIP-graph capture of the
// V-cycle and the launch-variant autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fsi_common.h"

struct fsi_ctx {
    fsi::Context c;
};

namespace fsi {

fsi_status hip_fail(Context* ctx, hipError_t e, const char* what, const char* file, int line) {
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file, line);
    if (ctx) ctx->err = buf;
    return e == hipErrorOutOfMemory ? FSI_ERR_OOM : FSI_ERR_HIP;
}
fsi_status fail(Context* ctx, fsi_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

template <typename T>
static fsi_status dalloc(Context* ctx, T** p, int64_t n) {
    *p = nullptr;
    if (n <= 0) n = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)n);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(ctx, e, "hipMalloc", __FILE__, __LINE__);
    }
    ctx->allocations.push_back((void*)*p);
    return FSI_OK;
}

// release a buffer from dalloc (null is ignored); the caller makes sure no queued work
// still uses it
template <typename T>
static void dfree(Context* ctx, T** p) {
    if (!*p) return;
    auto& a = ctx->allocations;
    a.erase(std::remove(a.begin(), a.end(), (void*)*p), a.end());
    hipFree((void*)*p);
    *p = nullptr;
}

#define TRY(expr)                          \
    do {                                   \
        fsi_status st_ = (expr);           \
        if (st_ != FSI_OK) return st_;     \
    } while (0)

static int ilog2_exact(int r) {
    int l = 0;
    while ((1 << l) < r) ++l;
    return (1 << l) == r ? l : -1;
}

// ---------------------------------------------------------------- level construction
static fsi_status build_level(Context* ctx, Level& L, int dim, const int cells[3], const fsi_mesh_desc& m) {
    L.dim = dim;
    L.Q = dim == 3 ? 27 : 9;
    L.nc = 1;
    L.nvn = 1;
    L.np = 1;
    for (int d = 0; d < 3; ++d) {
        L.cells[d] = d < dim ? cells[d] : 1;
        L.vnodes[d] = d < dim ? 2 * cells[d] + 1 : 1;
        L.pnodes[d] = d < dim ? cells[d] + 1 : 1;
        L.nc *= L.cells[d];
        L.nvn *= L.vnodes[d];
        L.np *= L.pnodes[d];
    }
    L.nv = dim * L.nvn;
    L.nvert = L.np;
    L.dfaces = m.dirichlet_faces;
    const int NLOC = dim == 3 ? 27 : 9, NPL = dim == 3 ? 8 : 4;
    // wall mask of the velocity nodes
    L.h_dir_node.assign((size_t)L.nvn, 0);
    std::vector<int> dirn;
    for (int64_t n = 0; n < L.nvn; ++n) {
        int64_t r = n;
        bool w = false;
        for (int d = 0; d < dim; ++d) {
            const int i = (int)(r % L.vnodes[d]);
            r /= L.vnodes[d];
            if ((m.dirichlet_faces >> (2 * d)) & 1u) w |= (i == 0);
            if ((m.dirichlet_faces >> (2 * d + 1)) & 1u) w |= (i == L.vnodes[d] - 1);
        }
        L.h_dir_node[n] = w ? 1 : 0;
        if (w) dirn.push_back((int)n);
    }
    L.n_dir = (int64_t)dirn.size();
    // processing order: phases are the parity colours of (iy, iz); a phase holds
    // whole rows of cells along x (lexicographic), so one wavefront can own a row.
    // In 2D a row of cells is cut into segments of seg cells (seg = nx / 2^m, the
    // shortest such length of at least kSeg2D cells) and the segment's parity joins
    // the colour: four phases, and a wavefront owns one segment.  The 2D kernel walks
    // its row chunk by chunk with a dependent load chain per chunk, so short rows
    // (many wavefronts, one or two chunks each) hide the latency that one long row
    // per wavefront (nx / 21 chunks in sequence) cannot.
    const int nx = L.cells[0];
    int seg = nx;
    if (dim == 2) {
        constexpr int kSeg2D = 16;
        while (seg % 2 == 0 && seg / 2 >= kSeg2D) seg /= 2;
    }
    const bool split = seg < nx;
    L.ncolors = (1 << (dim - 1)) * (split ? 2 : 1);
    auto cell_coords = [&](int64_t c, int ci[3]) {
        int64_t r = c;
        ci[0] = ci[1] = ci[2] = 0;
        for (int d = 0; d < dim; ++d) {
            ci[d] = (int)(r % L.cells[d]);
            r /= L.cells[d];
        }
    };
    auto phase_of = [&](const int ci[3]) {
        int col = 0;
        for (int d = 1; d < dim; ++d) col |= (ci[d] & 1) << (d - 1);
        if (split) col |= ((ci[0] / seg) & 1) << (dim - 1);
        return col;
    };
    const int nph = L.nphases();
    const int cpw = dim == 3 ? Shape<3>::CPW : Shape<2>::CPW;
    const int nchunk = (seg + cpw - 1) / cpw;
    std::vector<int> col2lex((size_t)L.nc), lex2col((size_t)L.nc);
    // rows (segments) of each phase (lexicographic in the row index)
    std::vector<std::vector<int64_t>> rows((size_t)nph);
    for (int64_t c = 0; c < L.nc; c += seg) {
        int ci[3];
        cell_coords(c, ci);
        rows[phase_of(ci)].push_back(c);      // lex index of the row's first cell
    }
    // inside a phase, cells are numbered row by row (x fastest)
    L.phase_off.assign((size_t)nph + 1, 0);
    int64_t k = 0;
    for (int p = 0; p < nph; ++p) {
        L.phase_off[p] = k;
        for (int64_t r : rows[p])
            for (int ix = 0; ix < seg; ++ix) {
                col2lex[k] = (int)(r + ix);
                lex2col[r + ix] = (int)k;
                ++k;
            }
    }
    L.phase_off[nph] = k;
    // dispatch order of the single atomic launch (3D): slot g takes natural row g (iy
    // fastest), stored at its phase-major row
    const int64_t nrow = L.nc / seg;
    std::vector<int> atom_rows((size_t)nrow);
    {
        int64_t sr = 0;
        for (int p = 0; p < nph; ++p)
            for (int64_t r : rows[p]) atom_rows[(size_t)(r / seg)] = (int)sr++;
    }
    L.geo.nx = seg;
    L.geo.nchunks = nchunk;
    L.geo.cpw = cpw;
    L.geo.nt = dim == 3 ? Shape<3>::NT : Shape<2>::NT;
    L.geo.nchk = nrow * nchunk;
    std::vector<int> vmap((size_t)L.nc * NLOC), pmap((size_t)L.nc * NPL);
    std::vector<uint4> info((size_t)L.nc);
    // first/last touch of a shared node: compare the phase of every other cell containing it
    // x-neighbours in the same row (segment) are summed in the wavefront before the
    // write, so only y/z neighbours and the x-neighbours across a segment boundary
    // decide first/last touch
    auto touch_bits = [&](const int ci[3], const int li[3], int hi_index, bool& first, bool& last) {
        int dirs[3], nd = 0;
        if (split) {
            if (li[0] == 0 && ci[0] > 0 && ci[0] % seg == 0) dirs[nd++] = -1;
            else if (li[0] == hi_index && ci[0] < nx - 1 && (ci[0] + 1) % seg == 0) dirs[nd++] = 1;
        }
        for (int d = 1; d < dim; ++d) {
            if (li[d] == 0 && ci[d] > 0) dirs[nd++] = -(d + 1);
            else if (li[d] == hi_index && ci[d] < L.cells[d] - 1) dirs[nd++] = d + 1;
        }
        const int me = phase_of(ci);
        first = last = true;
        for (int m = 1; m < (1 << nd); ++m) {
            int nb[3] = {ci[0], ci[1], ci[2]};
            for (int b = 0; b < nd; ++b)
                if (m & (1 << b)) {
                    const int d = dirs[b] < 0 ? -dirs[b] - 1 : dirs[b] - 1;
                    nb[d] += dirs[b] < 0 ? -1 : 1;
                }
            const int ph = phase_of(nb);
            if (ph < me) first = false;
            if (ph > me) last = false;
        }
    };
    for (int64_t k = 0; k < L.nc; ++k) {
        int ci[3];
        cell_coords(col2lex[k], ci);
        uint4 inf = {0u, 0u, 0u, 0u};
        for (int n = 0; n < NLOC; ++n) {
            const int li[3] = {n % 3, (n / 3) % 3, n / 9};
            int64_t node = 0, st = 1;
            for (int d = 0; d < dim; ++d) {
                node += (int64_t)(2 * ci[d] + li[d]) * st;
                st *= L.vnodes[d];
            }
            vmap[k * NLOC + n] = (int)node;
            if (L.h_dir_node[node]) inf.x |= 1u << n;
            bool f, l;
            touch_bits(ci, li, 2, f, l);
            if (f) inf.y |= 1u << n;
            if (l) inf.w |= 1u << n;
        }
        for (int n = 0; n < NPL; ++n) {
            const int li[3] = {n & 1, (n >> 1) & 1, (n >> 2) & 1};
            int64_t node = 0, st = 1;
            for (int d = 0; d < dim; ++d) {
                node += (int64_t)(ci[d] + li[d]) * st;
                st *= L.pnodes[d];
            }
            pmap[k * NPL + n] = (int)node;
            bool f, l;
            touch_bits(ci, li, 1, f, l);
            if (f) inf.z |= 1u << n;
            if (l) inf.z |= 1u << (16 + n);
        }
        info[k] = inf;
    }
    TRY(dalloc(ctx, &L.d_col2lex, L.nc));
    TRY(dalloc(ctx, &L.d_lex2col, L.nc));
    TRY(dalloc(ctx, &L.d_vmap, L.nc * NLOC));
    TRY(dalloc(ctx, &L.d_atom_rows, nrow));
    TRY(dalloc(ctx, &L.d_pmap, L.nc * NPL));
    TRY(dalloc(ctx, &L.d_info, L.nc));
    TRY(dalloc(ctx, &L.d_wall, L.nvn));
    TRY(dalloc(ctx, &L.d_dir_nodes, std::max<int64_t>(1, L.n_dir)));
    FSI_HIP_TRY(hipMemcpy(L.d_col2lex, col2lex.data(), sizeof(int) * L.nc, hipMemcpyHostToDevice));
    FSI_HIP_TRY(hipMemcpy(L.d_lex2col, lex2col.data(), sizeof(int) * L.nc, hipMemcpyHostToDevice));
    FSI_HIP_TRY(hipMemcpy(L.d_vmap, vmap.data(), sizeof(int) * vmap.size(), hipMemcpyHostToDevice));
    FSI_HIP_TRY(hipMemcpy(L.d_atom_rows, atom_rows.data(), sizeof(int) * atom_rows.size(), hipMemcpyHostToDevice));
    FSI_HIP_TRY(hipMemcpy(L.d_pmap, pmap.data(), sizeof(int) * pmap.size(), hipMemcpyHostToDevice));
    FSI_HIP_TRY(hipMemcpy(L.d_info, info.data(), sizeof(uint4) * info.size(), hipMemcpyHostToDevice));
    FSI_HIP_TRY(hipMemcpy(L.d_wall, L.h_dir_node.data(), (size_t)L.nvn, hipMemcpyHostToDevice));
    if (L.n_dir > 0)
        FSI_HIP_TRY(hipMemcpy(L.d_dir_nodes, dirn.data(), sizeof(int) * dirn.size(), hipMemcpyHostToDevice));
    // geometry and coefficient storage
    const int64_t P = L.plane();
    TRY(dalloc(ctx, &L.d_K64, (int64_t)dim * dim * P));
    TRY(dalloc(ctx, &L.d_cw64, P));
    TRY(dalloc(ctx, &L.d_cv64, 2 * P));
    TRY(dalloc(ctx, &L.d_K32, (int64_t)dim * dim * P));
    TRY(dalloc(ctx, &L.d_cv32, 2 * P));
    TRY(dalloc(ctx, &L.d_cq32, 2 * P));
    TRY(dalloc(ctx, &L.d_Ks64, (int64_t)dim * dim * P));
    TRY(dalloc(ctx, &L.d_Ks32, (int64_t)dim * dim * P));
    TRY(dalloc(ctx, &L.d_vd32, L.np));
    TRY(dalloc(ctx, &L.d_cq64, 2 * P));
    TRY(dalloc(ctx, &L.d_vd64, L.np));
    for (int d = 0; d < dim; ++d) L.h[d] = m.extent[d] / L.cells[d];
    TRY(dalloc(ctx, &L.d_dAinv64, L.nv));
    TRY(dalloc(ctx, &L.d_dAinv32, L.nv));
    TRY(dalloc(ctx, &L.d_dSinv, L.np));
    return FSI_OK;
}

template <typename T> static std::vector<LevelWork<T>>& works(Context* c);
template <> std::vector<LevelWork<double>>& works<double>(Context* c) { return c->w64; }
template <> std::vector<LevelWork<float>>& works<float>(Context* c) { return c->w32; }
template <typename T> static const T* Kp(const Level& L);
template <> const double* Kp<double>(const Level& L) { return L.d_K64; }
template <> const float* Kp<float>(const Level& L) { return L.d_K32; }
// geometry planes a cell-kernel mode reads: A alone (and with the Chebyshev epilogue)
// reads sqrt(cvisc) K, the other modes K
static bool scaled_mode(int mode) { return mode == OP_A || mode == (OP_A | OP_CHEB); }
template <typename T> static const T* Kmode(const Level& L, int mode);
template <> const double* Kmode<double>(const Level& L, int mode) { return scaled_mode(mode) ? L.d_Ks64 : L.d_K64; }
template <> const float* Kmode<float>(const Level& L, int mode) { return scaled_mode(mode) ? L.d_Ks32 : L.d_K32; }
template <typename T> static const T* CVp(const Level& L);
template <> const double* CVp<double>(const Level& L) { return L.d_cv64; }
template <> const float* CVp<float>(const Level& L) { return L.d_cv32; }
template <typename T> static const T* DAp(const Level& L);
template <> const double* DAp<double>(const Level& L) { return L.d_dAinv64; }
template <> const float* DAp<float>(const Level& L) { return L.d_dAinv32; }
template <typename T> static constexpr int prec_index();
template <> constexpr int prec_index<double>() { return 0; }
template <> constexpr int prec_index<float>() { return 1; }

template <typename T>
static fsi_status alloc_work(Context* ctx) {
    auto& W = works<T>(ctx);
    if (!W.empty()) return FSI_OK;
    W.resize(ctx->nlev);
    for (int j = 0; j < ctx->nlev; ++j) {
        const Level& L = ctx->lv[j];
        LevelWork<T>& w = W[j];
        TRY(dalloc(ctx, &w.f_u, L.nv));
        TRY(dalloc(ctx, &w.x_u, L.nv));
        TRY(dalloc(ctx, &w.r_u, L.nv));
        TRY(dalloc(ctx, &w.w_u, L.nv));
        TRY(dalloc(ctx, &w.v_u, L.nv));
        TRY(dalloc(ctx, &w.cd_u, L.nv));
        TRY(dalloc(ctx, &w.cax_u, L.nv));
        TRY(dalloc(ctx, &w.tu, L.nv));
        TRY(dalloc(ctx, &w.f_p, L.np));
        TRY(dalloc(ctx, &w.x_p, L.np));
        TRY(dalloc(ctx, &w.r_p, L.np));
        TRY(dalloc(ctx, &w.t_p, L.np));
        TRY(dalloc(ctx, &w.z_p, L.np));
        TRY(dalloc(ctx, &w.b_p, L.np));
        TRY(dalloc(ctx, &w.s_p, L.np));
        TRY(dalloc(ctx, &w.dots, 4));
        TRY(dalloc(ctx, &w.partials, 2 * kReduceBlocks));
    }
    return FSI_OK;
}

static int variant_of(const Context* ctx, int prec, int level, int mode) {
    if (!ctx->prm.tuned) return 0;
    const auto& v = ctx->tune_variant[prec];
    const size_t k = (size_t)level * kTuneClasses + tune_class(mode);
    return k < v.size() ? v[k] : 0;
}

// the parameters that change what a captured graph launches
static int path_key(const Context* ctx) {
    return (ctx->prm.fused ? 1 : 0) | (ctx->prm.tuned ? 2 : 0) | (ctx->prm.vertex_geometry << 2) |
           (ctx->prm.corrector ? 16 : 0) | (ctx->prm.atomics ? 32 : 0);
}

// the single atomic launch serves a class on this level: on 3D levels with fixed cells only A
// has the kernel that reads the fixed nodes' wall mask (the other classes keep the phases)
static bool atomic_ok(const Level& L, int mode) { return !(L.dim == 3 && L.fixed_nodes) || mode == OP_A; }

// the solver's velocity block: A, or in the corrector mode A + N + S
static int solver_mode(const Context* ctx, int mode) {
    return (ctx->prm.corrector && (mode & OP_A)) ? (mode | OP_CONV) : mode;
}

// ---------------------------------------------------------------- operators
template <typename T>
static void op_apply(Context* ctx, int j, int mode, const T* u, const double* p, T* v, double* q, hipStream_t s) {
    // every output entry is written by its first touching cell (no clearing pass);
    // wall rows: identity for A, zero for B^T alone
    const Level& L = ctx->lv[j];
    const int am = !(ctx->prm.tuned && ctx->prm.atomics) ? -1
                   : (mode & OP_CONV) ? ctx->atom_conv[prec_index<T>()][(size_t)j]
                                      : ctx->atom_of(prec_index<T>(), j, mode);
    if (am >= 0 && atomic_ok(L, mode)) {
        launch_cell_atomic<T>(L, mode, am, Kmode<T>(L, mode), CVp<T>(L), u, p, v, q, s);   // wall rows included
        return;
    }
    launch_cell_all<T>(L, mode, variant_of(ctx, prec_index<T>(), j, mode), Kmode<T>(L, mode), CVp<T>(L), u, p, v, q,
                       s);
    if (mode & OP_A) launch_dirichlet_copy<T>(L, u, v, s);
    else if (mode & OP_BT) launch_dirichlet_zero<T>(L, v, s);
}

// Chebyshev smoother Cheb(A, diag A, k_A) from a zero initial guess: k_A - 1 applications of A
template <typename T>
static void cheb(Context* ctx, int j, const T* r, T* x, hipStream_t s) {
    const Level& L = ctx->lv[j];
    LevelWork<T>& W = works<T>(ctx)[j];
    const double theta = 0.5 * (L.hi + L.lo), delta = 0.5 * (L.hi - L.lo);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    launch_cheb_init<T>(DAp<T>(L), r, x, 1.0 / theta, L.nv, s);
    for (int i = 1; i < ctx->prm.k_A; ++i) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        const double c1 = rn * rho, c2 = 2.0 * rn / delta;
        // the first direction is the first iterate; the last step needs no direction
        const bool first = i == 1, store_d = i + 1 < ctx->prm.k_A;
        if (ctx->prm.fused && !ctx->prm.corrector && (!ctx->prm.tuned || ctx->fuse_cheb[prec_index<T>()][j])) {
            // the update happens at each node's last touch
            launch_cell_cheb_all<T>(L, variant_of(ctx, prec_index<T>(), j, OP_A | OP_CHEB), Kmode<T>(L, OP_A | OP_CHEB),
                                    CVp<T>(L), x, W.cd_u, r, DAp<T>(L), W.cax_u, c1, c2, first, store_d, s);
            launch_dirichlet_cheb<T>(L, x, W.cd_u, r, DAp<T>(L), c1, c2, first, store_d, s);
        } else {
            op_apply<T>(ctx, j, solver_mode(ctx, OP_A), x, nullptr, W.cax_u, nullptr, s);
            launch_cheb_step<T>(DAp<T>(L), r, W.cax_u, x, W.cd_u, c1, c2, first, store_d, L.nv, s);
        }
        rho = rn;
    }
}

// one step of the block smoother K_j (Sec. 4): w = Ah^{-1} r_u; z = D_S^{-1}(B w - r_p);
// v = Ah^{-1} B^T z; y = B v; beta = <y,z>/<y,D_S^{-1}y> (one MINRES step, k_S = 1);
// increment (w - beta v, beta z).  Ah^{-1} is linear, so Ah^{-1} B^T (beta z) = beta v.
template <typename T>
static void smoother(Context* ctx, int j, const T* r_u, const double* r_p, T* x_u, double* x_p, bool first,
                     hipStream_t s) {
    const Level& L = ctx->lv[j];
    LevelWork<T>& W = works<T>(ctx)[j];
    cheb<T>(ctx, j, r_u, W.w_u, s);
    op_apply<T>(ctx, j, OP_B, W.w_u, nullptr, nullptr, W.t_p, s);
    if (ctx->prm.corrector) {
        // ChebBiCGStab(1, 1): one right-preconditioned BiCGStab iteration from zero on
        // S y = b, b = B w - r_p, P = D_S^{-1}; Ah^{-1} B^T y = alpha t1 + omega t2 by
        // linearity.  t2 lives in W.r_u, free once w is formed.
        T* t1 = W.v_u;
        T* t2 = W.r_u;
        launch_bicg_start(L.d_dSinv, W.t_p, r_p, W.b_p, W.z_p, L.np, s);           // b, p
        op_apply<T>(ctx, j, OP_BT, nullptr, W.z_p, W.tu, nullptr, s);
        cheb<T>(ctx, j, W.tu, t1, s);
        op_apply<T>(ctx, j, OP_B, t1, nullptr, nullptr, W.t_p, s);                  // v = S p
        launch_dot<double>(W.b_p, W.b_p, L.np, W.partials, W.dots, s);
        launch_dot<double>(W.b_p, W.t_p, L.np, W.partials, W.dots + 1, s);
        launch_bicg_mid(L.d_dSinv, W.dots, W.t_p, W.b_p, W.s_p, L.np, s);          // s, q
        op_apply<T>(ctx, j, OP_BT, nullptr, W.s_p, W.tu, nullptr, s);
        cheb<T>(ctx, j, W.tu, t2, s);
        op_apply<T>(ctx, j, OP_B, t2, nullptr, nullptr, W.t_p, s);                  // t = S q
        launch_dot<double>(W.t_p, W.b_p, L.np, W.partials, W.dots + 2, s);
        launch_dot<double>(W.t_p, W.t_p, L.np, W.partials, W.dots + 3, s);
        launch_bicg_update<T>(W.w_u, t1, t2, W.z_p, W.s_p, W.dots, x_u, x_p, L.nv, L.np, first, s);
        return;
    }
    launch_schur_z(L.d_dSinv, W.t_p, r_p, W.z_p, L.np, s);
    op_apply<T>(ctx, j, OP_BT, nullptr, W.z_p, W.tu, nullptr, s);
    cheb<T>(ctx, j, W.tu, W.v_u, s);
    op_apply<T>(ctx, j, OP_B, W.v_u, nullptr, nullptr, W.t_p, s);
    launch_schur_dots(W.t_p, W.z_p, L.d_dSinv, W.partials, W.dots, L.np, s);
    launch_smoother_update<T>(W.w_u, W.v_u, W.z_p, W.dots, x_u, x_p, L.nv, L.np, first, s);
}

// the residual of level j in precision pi is formed in the cell kernel's last-touch epilogue
static bool res_epilogue(const Context* ctx, int pi, int j) {
    return ctx->prm.fused && !ctx->prm.corrector && (!ctx->prm.tuned || ctx->fuse_res[pi][j]);
}

// r = f - M x on level j (into W.r_u, W.r_p)
template <typename T>
static void residual(Context* ctx, int j, hipStream_t s) {
    const Level& L = ctx->lv[j];
    LevelWork<T>& W = works<T>(ctx)[j];
    if (res_epilogue(ctx, prec_index<T>(), j)) {
        launch_cell_res_all<T>(L, variant_of(ctx, prec_index<T>(), j, OP_A | OP_BT | OP_B | OP_RES), Kp<T>(L),
                               CVp<T>(L), W.x_u, W.x_p, W.f_u,
                               W.f_p, W.r_u, W.r_p, s);
        launch_dirichlet_res<T>(L, W.f_u, W.x_u, W.r_u, s);
        return;
    }
    op_apply<T>(ctx, j, solver_mode(ctx, OP_A | OP_BT | OP_B), W.x_u, W.x_p, W.r_u, W.r_p, s);
    launch_sub<T>(W.f_u, W.r_u, W.r_u, L.nv, s);
    launch_sub<double>(W.f_p, W.r_p, W.r_p, L.np, s);
}

// V-cycle on level j from a zero initial guess: W[j].f -> W[j].x
template <typename T>
static void vcycle_level(Context* ctx, int j, hipStream_t s) {
    LevelWork<T>& W = works<T>(ctx)[j];
    if (j == 0) {
        launch_coarse_apply<T>(ctx->coarse, ctx->lv[0], W.f_u, W.f_p, W.x_u, W.x_p, s);
        return;
    }
    const int m = ctx->prm.m;
    for (int st = 0; st < m; ++st) {
        if (st == 0) {
            smoother<T>(ctx, j, W.f_u, W.f_p, W.x_u, W.x_p, true, s);
        } else {
            residual<T>(ctx, j, s);
            smoother<T>(ctx, j, W.r_u, W.r_p, W.x_u, W.x_p, false, s);
        }
    }
    if (m == 0) {
        launch_fill<T>(W.x_u, T(0), ctx->lv[j].nv, s);
        launch_fill<double>(W.x_p, 0.0, ctx->lv[j].np, s);
    }
    LevelWork<T>& C = works<T>(ctx)[j - 1];
    // FP64 transfer scratch: the level's FP64 smoother work vectors, free here in
    // either precision (one V-cycle runs at a time on the context's stream)
    LevelWork<double>& S = ctx->w64[j];
    if (ctx->prm.fused && !res_epilogue(ctx, prec_index<T>(), j)) {
        // residual fused into the restriction: M x into W.r, the first pass restricts f - M x
        op_apply<T>(ctx, j, solver_mode(ctx, OP_A | OP_BT | OP_B), W.x_u, W.x_p, W.r_u, W.r_p, s);
        launch_restrict<T>(ctx->lv[j], ctx->lv[j - 1], W.f_u, W.f_p, C.f_u, C.f_p, S.w_u, S.v_u, s, W.r_u, W.r_p);
    } else {
        residual<T>(ctx, j, s);
        launch_restrict<T>(ctx->lv[j], ctx->lv[j - 1], W.r_u, W.r_p, C.f_u, C.f_p, S.w_u, S.v_u, s);
    }
    vcycle_level<T>(ctx, j - 1, s);
    launch_prolongate_add<T>(ctx->lv[j], ctx->lv[j - 1], C.x_u, C.x_p, W.x_u, W.x_p, S.w_u, S.v_u, s);
    for (int st = 0; st < m; ++st) {
        residual<T>(ctx, j, s);
        smoother<T>(ctx, j, W.r_u, W.r_p, W.x_u, W.x_p, false, s);
    }
}

// one preconditioner application in precision T: ctx->vc_in -> ctx->vc_out (FP64 buffers)
template <typename T>
static void vcycle_body(Context* ctx, hipStream_t s) {
    const int J = ctx->nlev - 1;
    const Level& L = ctx->lv[J];
    LevelWork<T>& W = works<T>(ctx)[J];
    launch_cast<T, double>(W.f_u, ctx->vc_in_u, L.nv, s);
    launch_cast<double, double>(W.f_p, ctx->vc_in_p, L.np, s);
    vcycle_level<T>(ctx, J, s);
    launch_cast<double, T>(ctx->vc_out_u, W.x_u, L.nv, s);
    launch_cast<double, double>(ctx->vc_out_p, W.x_p, L.np, s);
}

static fsi_status capture_graphs(Context* ctx);

static fsi_status run_vcycle(Context* ctx, hipStream_t s) {
    const int pi = ctx->prm.precision == FSI_PREC_MIXED ? 1 : 0;
    const int key = path_key(ctx);
    if (ctx->prm.use_graph && ctx->graph_valid[pi] && ctx->graph_key != key) TRY(capture_graphs(ctx));
    if (ctx->prm.use_graph && ctx->graph_valid[pi]) {
        FSI_HIP_TRY(hipGraphLaunch(ctx->graph[pi], s));
    } else if (pi == 1) {
        vcycle_body<float>(ctx, s);
    } else {
        vcycle_body<double>(ctx, s);
    }
    return FSI_OK;
}

static fsi_status capture_graphs(Context* ctx) {
    for (int pi = 0; pi < 2; ++pi) {
        // the extension graphs hold launch shapes too: recaptured at their next use
        if (ctx->ext_graph_valid[pi]) {
            hipGraphExecDestroy(ctx->ext_graph[pi]);
            ctx->ext_graph_valid[pi] = false;
        }
        if (ctx->graph_valid[pi]) {
            hipGraphExecDestroy(ctx->graph[pi]);
            ctx->graph_valid[pi] = false;
        }
    }
    // one graph per precision, so switching precision needs no new setup
    hipStream_t cs;
    FSI_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    for (int pi = 0; pi < 2; ++pi) {
        hipGraph_t g;
        FSI_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        if (pi == 1) vcycle_body<float>(ctx, cs);
        else vcycle_body<double>(ctx, cs);
        FSI_HIP_TRY(hipStreamEndCapture(cs, &g));
        FSI_HIP_TRY(hipGraphInstantiate(&ctx->graph[pi], g, nullptr, nullptr, 0));
        hipGraphDestroy(g);
        ctx->graph_valid[pi] = true;
    }
    hipStreamDestroy(cs);
    ctx->graph_key = path_key(ctx);
    return FSI_OK;
}

// ---------------------------------------------------------------- setup pieces
static fsi_status sync_flag(Context* ctx, fsi_status st, const char* msg) {
    FSI_HIP_TRY(hipMemcpyAsync(ctx->h_flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    FSI_HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (*ctx->h_flag != 0) return fail(ctx, st, msg);
    return FSI_OK;
}

static fsi_status read_scalars(Context* ctx, const double* d, int n, double* h) {
    FSI_HIP_TRY(hipMemcpyAsync(ctx->h_dbl, d, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
    FSI_HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < n; ++i) h[i] = ctx->h_dbl[i];
    return FSI_OK;
}

static fsi_status dot64(Context* ctx, const double* x, const double* y, int64_t n, double* out) {
    launch_dot<double>(x, y, n, ctx->d_scratch, ctx->d_scratch + 2 * kReduceBlocks, ctx->stream);
    return read_scalars(ctx, ctx->d_scratch + 2 * kReduceBlocks, 1, out);
}

// largest eigenvalue of the symmetric tridiagonal (alpha, beta) by Sturm bisection
static double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
    const int n = (int)a.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto count_below = [&](double x) {   // number of eigenvalues < x
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < n; ++i) {
            const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
            d = (a[i] - x) - (i > 0 ? bb / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= n) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

static fsi_status lanczos(Context* ctx, int j) {
    Level& L = ctx->lv[j];
    hipStream_t s = ctx->stream;
    LevelWork<double>& W = ctx->w64[j];
    // reuse work vectors: sA = sqrt(dAinv) in W.w_u, v in W.v_u, vprev in W.cd_u, w in W.cax_u, tmp in W.tu
    double *sA = W.w_u, *v = W.v_u, *vp = W.cd_u, *w = W.cax_u, *tmp = W.tu;
    launch_vsqrt(L.d_dAinv64, sA, L.nv, s);
    launch_lanczos_start(L, v, s);
    launch_fill<double>(vp, 0.0, L.nv, s);
    double nrm;
    TRY(dot64(ctx, v, v, L.nv, &nrm));
    nrm = std::sqrt(nrm);
    if (!(nrm > 0)) return fail(ctx, FSI_ERR_BREAKDOWN, "Lanczos start vector vanishes");
    launch_scale_host(1.0 / nrm, v, v, L.nv, s);
    std::vector<double> al, be;
    double beta = 0.0;
    for (int it = 0; it < ctx->prm.n_eig; ++it) {
        launch_mul(sA, v, tmp, L.nv, s);
        op_apply<double>(ctx, j, solver_mode(ctx, OP_A), tmp, nullptr, w, nullptr, s);
        launch_mul(sA, w, w, L.nv, s);
        double alpha;
        TRY(dot64(ctx, w, v, L.nv, &alpha));
        launch_axpy_host(-alpha, v, w, L.nv, s);
        if (it > 0) launch_axpy_host(-beta, vp, w, L.nv, s);
        al.push_back(alpha);
        double bn;
        TRY(dot64(ctx, w, w, L.nv, &bn));
        bn = std::sqrt(bn);
        if (it == ctx->prm.n_eig - 1 || !(bn > 1e-300)) break;
        be.push_back(bn);
        std::swap(vp, v);            // vprev <- v
        launch_scale_host(1.0 / bn, w, v, L.nv, s);   // v <- w / beta
        beta = bn;
    }
    L.lam = tridiag_max_eig(al, be);
    L.hi = ctx->prm.cheb_upper * L.lam;
    L.lo = L.hi / ctx->prm.cheb_ratio;
    return FSI_OK;
}

static fsi_status setup_coarse(Context* ctx) {
    Level& L = ctx->lv[0];
    Coarse& C = ctx->coarse;
    hipStream_t s = ctx->stream;
    std::vector<int> vrow((size_t)L.nv, -1), uidx;
    int64_t nf = 0;
    for (int a = 0; a < L.dim; ++a)
        for (int64_t n = 0; n < L.nvn; ++n)
            if (!L.h_dir_node[n]) {
                vrow[a * L.nvn + n] = (int)nf++;
                uidx.push_back((int)(a * L.nvn + n));
            }
    const int64_t n = nf + L.np;
    if (C.n != n) {
        C.n = n;
        C.nfree_u = nf;
        TRY(dalloc(ctx, &C.d_uidx, std::max<int64_t>(1, nf)));
        TRY(dalloc(ctx, &C.d_inv64, n * n));
        TRY(dalloc(ctx, &C.d_inv32, n * n));
        TRY(dalloc(ctx, &C.d_xin64, n));
        TRY(dalloc(ctx, &C.d_xout64, n));
        TRY(dalloc(ctx, &C.d_xin32, n));
        TRY(dalloc(ctx, &C.d_xout32, n));
        TRY(dalloc(ctx, &C.d_vrow, L.nv));
        TRY(dalloc(ctx, &C.d_piv, 2 * n));
        TRY(dalloc(ctx, &C.d_col, n));
        TRY(dalloc(ctx, &C.d_tmp, n * n));
    }
    if (nf > 0)
        FSI_HIP_TRY(hipMemcpyAsync(C.d_uidx, uidx.data(), sizeof(int) * nf, hipMemcpyHostToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(C.d_vrow, vrow.data(), sizeof(int) * L.nv, hipMemcpyHostToDevice, s));
    launch_fill<double>(C.d_inv64, 0.0, n * n, s);
    launch_coarse_assemble_impl(L, L.d_K64, L.d_cv64, C.d_vrow, nf, C.d_inv64, n, s, ctx->prm.corrector != 0);
    launch_fill<int>(ctx->d_flag, 0, 1, s);
    launch_gj(C.d_inv64, n, C.d_piv, C.d_piv + n, C.d_col, C.d_tmp, ctx->d_flag, s);
    launch_cast<float, double>(C.d_inv32, C.d_inv64, n * n, s);
    // synchronises the stream, so the host vectors above outlive their copies
    ctx->coarse_block_ok = true;
    if (ctx->has_fixed) {
        // fixed cells can leave pressure nodes with no free velocity dof around them: the
        // block matrix is then singular, and only the extension (velocity-only coarse
        // solve) is available on the context
        FSI_HIP_TRY(hipMemcpyAsync(ctx->h_flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        FSI_HIP_TRY(hipStreamSynchronize(s));
        ctx->coarse_block_ok = *ctx->h_flag == 0;
        return FSI_OK;
    }
    return sync_flag(ctx, FSI_ERR_BREAKDOWN, "singular coarse-level matrix");
}

static fsi_status check_level(Context* ctx, int level) {
    if (level < 0 || level >= ctx->nlev) return fail(ctx, FSI_ERR_ARG, "level out of range");
    return FSI_OK;
}

static fsi_status invalidate(Context* ctx) {
    ctx->setup_done = false;
    ctx->ext_ready = false;
    for (int pi = 0; pi < 2; ++pi) {
        if (ctx->graph_valid[pi]) {
            hipGraphExecDestroy(ctx->graph[pi]);
            ctx->graph_valid[pi] = false;
        }
        if (ctx->ext_graph_valid[pi]) {
            hipGraphExecDestroy(ctx->ext_graph[pi]);
            ctx->ext_graph_valid[pi] = false;
        }
    }
    return FSI_OK;
}

// ---------------------------------------------------------------- FGMRES
static fsi_status ensure_krylov(Context* ctx, int restart) {
    Krylov& K = ctx->kr;
    const Level& L = ctx->lv[ctx->nlev - 1];
    const int64_t n = L.nv + L.np;
    if (K.restart >= restart && K.n == n) return FSI_OK;
    // superseded buffers are released (no queued work uses them: every solve synchronises)
    FSI_HIP_TRY(hipStreamSynchronize(ctx->stream));
    dfree(ctx, &K.V);
    dfree(ctx, &K.Z);
    dfree(ctx, &K.w);
    dfree(ctx, &K.r);
    dfree(ctx, &K.x);
    dfree(ctx, &K.g);
    dfree(ctx, &K.h);
    dfree(ctx, &K.partials);
    K.restart = 0;
    K.n = 0;
    TRY(dalloc(ctx, &K.V, (int64_t)(restart + 1) * n));
    TRY(dalloc(ctx, &K.Z, (int64_t)restart * n));
    TRY(dalloc(ctx, &K.w, n));
    TRY(dalloc(ctx, &K.r, n));
    TRY(dalloc(ctx, &K.x, n));
    TRY(dalloc(ctx, &K.g, n));
    TRY(dalloc(ctx, &K.h, 2 * (restart + 2)));
    TRY(dalloc(ctx, &K.partials, std::max<int64_t>(std::max<int64_t>(1024 * (int64_t)(restart + 2), 4096),
                                                   2 * kReduceBlocks)));
    if (K.h_host) hipHostFree(K.h_host);
    K.h_host = nullptr;
    FSI_HIP_TRY(hipHostMalloc((void**)&K.h_host, sizeof(double) * 3 * (restart + 2)));
    K.restart = restart;
    K.n = n;
    return FSI_OK;
}

// y = M x on the finest level for combined vectors [u | p]
static void stokes_combined(Context* ctx, const double* x, double* y, hipStream_t s) {
    const int J = ctx->nlev - 1;
    const Level& L = ctx->lv[J];
    op_apply<double>(ctx, J, solver_mode(ctx, OP_A | OP_BT | OP_B), x, x + L.nv, y, y + L.nv, s);
}

static fsi_status precond_combined(Context* ctx, const double* r, double* z, hipStream_t s) {
    const Level& L = ctx->lv[ctx->nlev - 1];
    FSI_HIP_TRY(hipMemcpyAsync(ctx->vc_in_u, r, sizeof(double) * L.nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(ctx->vc_in_p, r + L.nv, sizeof(double) * L.np, hipMemcpyDeviceToDevice, s));
    TRY(run_vcycle(ctx, s));
    for (int c = 1; c < ctx->prm.n_cycles; ++c) {
        // z += V(r - M z)
        FSI_HIP_TRY(hipMemcpyAsync(z, ctx->vc_out_u, sizeof(double) * L.nv, hipMemcpyDeviceToDevice, s));
        FSI_HIP_TRY(hipMemcpyAsync(z + L.nv, ctx->vc_out_p, sizeof(double) * L.np, hipMemcpyDeviceToDevice, s));
        stokes_combined(ctx, z, ctx->vc_tmp, s);
        launch_sub_into(r, ctx->vc_tmp, ctx->vc_in_u, L.nv, s);
        launch_sub_into(r + L.nv, ctx->vc_tmp + L.nv, ctx->vc_in_p, L.np, s);
        TRY(run_vcycle(ctx, s));
        launch_axpy_host(1.0, z, ctx->vc_out_u, L.nv, s);
        launch_axpy_host(1.0, z + L.nv, ctx->vc_out_p, L.np, s);
    }
    FSI_HIP_TRY(hipMemcpyAsync(z, ctx->vc_out_u, sizeof(double) * L.nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(z + L.nv, ctx->vc_out_p, sizeof(double) * L.np, hipMemcpyDeviceToDevice, s));
    return FSI_OK;
}


// ---------------------------------------------------------------- unconstrained operator (boundary liftings)
// The finest level's operator with the Dirichlet rows and columns kept (the cell info with its
// wall bits cleared stands in for the level's own), in the phased launches: the single atomic
// launch derives its wall rows from the box faces, so it cannot serve here.
static fsi_status apply_unconstrained(Context* ctx, int mode, const double* u, const double* p, double* v,
                                      double* q, hipStream_t s) {
    Level& L = ctx->lv[ctx->nlev - 1];
    if (!ctx->d_info_free) TRY(dalloc(ctx, &ctx->d_info_free, L.nc));
    launch_clear_wall_bits(L.d_info, ctx->d_info_free, L.nc, s);
    uint4* own = L.d_info;
    L.d_info = ctx->d_info_free;
    launch_cell_all<double>(L, mode, 0, Kmode<double>(L, mode), L.d_cv64, u, p, v, q, s);
    L.d_info = own;
    return FSI_OK;
}

// ---------------------------------------------------------------- extension solve
// The pseudo-elastic extension of Sec. 2: u = g on the Dirichlet nodes and a(u, v) = 0
// for every v vanishing there, with a the context's A form (c_m = 0 and eta = mu_A / 2
// give (mu_A eps(u), eps(v))).  Classical matrix-free multigrid on A alone (Sec. 5,
// extension solver settings): Chebyshev(A, diag A, k_A) pre- and post-smoothing, the
// same transfers and a direct solve of the free velocity block on the coarsest level,
// inside flexible CG.

// velocity-only coarse inverse: the level-0 block matrix assembled once more into the
// set-up scratch, its free velocity block copied out and inverted
static fsi_status setup_coarse_u(Context* ctx) {
    Level& L = ctx->lv[0];
    Coarse& C = ctx->coarse;
    Coarse& U = ctx->coarse_u;
    hipStream_t s = ctx->stream;
    const int64_t n = C.n, nf = C.nfree_u;
    if (U.n != nf) {
        U.n = nf;
        U.nfree_u = nf;
        TRY(dalloc(ctx, &U.d_inv64, nf * nf));
        TRY(dalloc(ctx, &U.d_inv32, nf * nf));
        TRY(dalloc(ctx, &U.d_xin64, nf));
        TRY(dalloc(ctx, &U.d_xout64, nf));
        TRY(dalloc(ctx, &U.d_xin32, nf));
        TRY(dalloc(ctx, &U.d_xout32, nf));
    }
    U.d_uidx = C.d_uidx;
    if (nf == 0) return FSI_OK;
    launch_fill<double>(C.d_tmp, 0.0, n * n, s);
    launch_coarse_assemble_impl(L, L.d_K64, L.d_cv64, C.d_vrow, nf, C.d_tmp, n, s);
    FSI_HIP_TRY(hipMemcpy2DAsync(U.d_inv64, sizeof(double) * nf, C.d_tmp, sizeof(double) * n, sizeof(double) * nf,
                                 nf, hipMemcpyDeviceToDevice, s));
    launch_fill<int>(ctx->d_flag, 0, 1, s);
    launch_gj(U.d_inv64, nf, C.d_piv, C.d_piv + nf, C.d_col, C.d_tmp, ctx->d_flag, s);
    launch_cast<float, double>(U.d_inv32, U.d_inv64, nf * nf, s);
    return sync_flag(ctx, FSI_ERR_BREAKDOWN, "singular coarse-level velocity block");
}

// W.r_u = W.f_u - A W.x_u
template <typename T>
static void ext_residual(Context* ctx, int j, hipStream_t s) {
    LevelWork<T>& W = works<T>(ctx)[j];
    op_apply<T>(ctx, j, OP_A, W.x_u, nullptr, W.tu, nullptr, s);
    launch_sub<T>(W.f_u, W.tu, W.r_u, ctx->lv[j].nv, s);
}

// one V-cycle from a zero guess on level j: W.f_u -> W.x_u (velocity only)
template <typename T>
static void ext_vcycle_level(Context* ctx, int j, hipStream_t s) {
    LevelWork<T>& W = works<T>(ctx)[j];
    const Level& L = ctx->lv[j];
    if (j == 0) {
        launch_coarse_apply_u<T>(ctx->coarse_u, L, W.f_u, W.x_u, s);
        return;
    }
    cheb<T>(ctx, j, W.f_u, W.x_u, s);          // pre-smoothing from zero
    LevelWork<T>& C = works<T>(ctx)[j - 1];
    LevelWork<double>& S = ctx->w64[j];         // FP64 transfer scratch, free here
    if (ctx->prm.fused) {
        // residual fused into the restriction: A x into W.tu, the first pass restricts f - A x
        op_apply<T>(ctx, j, OP_A, W.x_u, nullptr, W.tu, nullptr, s);
        launch_restrict<T>(L, ctx->lv[j - 1], W.f_u, nullptr, C.f_u, nullptr, S.w_u, S.v_u, s, W.tu, nullptr);
    } else {
        ext_residual<T>(ctx, j, s);
        launch_restrict<T>(L, ctx->lv[j - 1], W.r_u, nullptr, C.f_u, nullptr, S.w_u, S.v_u, s);
    }
    ext_vcycle_level<T>(ctx, j - 1, s);
    launch_prolongate_add<T>(L, ctx->lv[j - 1], C.x_u, nullptr, W.x_u, nullptr, S.w_u, S.v_u, s);
    ext_residual<T>(ctx, j, s);                 // post-smoothing
    cheb<T>(ctx, j, W.r_u, W.w_u, s);
    launch_add<T>(W.x_u, W.w_u, L.nv, s);
}

// z = V(r) on the finest level, FP64 in and out
template <typename T>
static void ext_precondition(Context* ctx, const double* r, double* z, hipStream_t s) {
    const int J = ctx->nlev - 1;
    LevelWork<T>& W = works<T>(ctx)[J];
    const int64_t nv = ctx->lv[J].nv;
    launch_cast<T, double>(W.f_u, r, nv, s);
    ext_vcycle_level<T>(ctx, J, s);
    launch_cast<double, T>(z, W.x_u, nv, s);
}

// the extension preconditioner on the fixed CG buffers r -> z: captured once per
// precision and launch configuration (fused, tuned, vertex geometry), then replayed
static fsi_status ext_run_precond(Context* ctx, const double* r, double* z, hipStream_t s) {
    const int pi = ctx->prm.precision == FSI_PREC_MIXED ? 1 : 0;
    if (!ctx->prm.use_graph) {
        if (pi) ext_precondition<float>(ctx, r, z, s);
        else ext_precondition<double>(ctx, r, z, s);
        return FSI_OK;
    }
    const int key = path_key(ctx);
    if (!ctx->ext_graph_valid[pi] || ctx->ext_graph_key[pi] != key) {
        if (ctx->ext_graph_valid[pi]) {
            hipGraphExecDestroy(ctx->ext_graph[pi]);
            ctx->ext_graph_valid[pi] = false;
        }
        hipStream_t cs;
        FSI_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g;
        FSI_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        if (pi) ext_precondition<float>(ctx, r, z, cs);
        else ext_precondition<double>(ctx, r, z, cs);
        FSI_HIP_TRY(hipStreamEndCapture(cs, &g));
        FSI_HIP_TRY(hipGraphInstantiate(&ctx->ext_graph[pi], g, nullptr, nullptr, 0));
        hipGraphDestroy(g);
        hipStreamDestroy(cs);
        ctx->ext_graph_valid[pi] = true;
        ctx->ext_graph_key[pi] = key;
    }
    FSI_HIP_TRY(hipGraphLaunch(ctx->ext_graph[pi], s));
    return FSI_OK;
}

// ---------------------------------------------------------------- allocation-free FP32 Stokes apply
// Pressure staging of fsi_apply_stokes_f32_noalloc: the FP64 copy of p (first half)
// and the FP64 sums of q (second half), for levels of up to kNoAllocMaxP pressure
// nodes.  One copy per device, held until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: kernels receive the device address that
// hipGetSymbolAddress returned for the current device.
constexpr int64_t kNoAllocMaxP = int64_t(1) << 22;
static __device__ __align__(256) double scratch[2 * kNoAllocMaxP];

static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_addr;   // per device id; null until resolved

// the device address of `scratch` on the current device, resolved once per device
static double* scratch_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_addr[(size_t)dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_addr[(size_t)dev] = static_cast<double*>(ptr);
    }
    return g_scratch_addr[(size_t)dev];
}

}  // namespace fsi

using namespace fsi;

// ================================================================ C ABI
extern "C" {

void fsi_default_mg_params(fsi_mg_params* p) {
    if (!p) return;
    p->k_A = 4;
    p->m = 2;
    p->n_cycles = 1;
    p->k_S = 1;
    p->n_S = 1;
    p->cheb_upper = 1.2;
    p->cheb_ratio = 20.0;
    p->n_eig = 12;
    p->precision = FSI_PREC_FP64;
    p->use_graph = 1;
    p->fused = 1;
    p->tuned = 1;
    p->vertex_geometry = 0;   // measured slower than the stored values on MI355X
    p->corrector = 0;
    p->atomics = 1;
}

fsi_status fsi_create(fsi_ctx** out, const fsi_mesh_desc* m, void* hip_stream) {
    if (!out || !m) return FSI_ERR_ARG;
    *out = nullptr;
    if (m->dim != 2 && m->dim != 3) return FSI_ERR_ARG;
    int lev = -1;
    for (int d = 0; d < m->dim; ++d) {
        if (m->n_coarse[d] < 1 || m->n_fine[d] < 1 || m->n_fine[d] % m->n_coarse[d] != 0) return FSI_ERR_ARG;
        if (!(m->extent[d] > 0)) return FSI_ERR_ARG;
        const int l = ilog2_exact(m->n_fine[d] / m->n_coarse[d]);
        if (l < 0 || (lev >= 0 && l != lev)) return FSI_ERR_ARG;
        lev = l;
    }
    int64_t nvn = 1;
    for (int d = 0; d < m->dim; ++d) nvn *= 2 * (int64_t)m->n_fine[d] + 1;
    if (nvn * m->dim >= (int64_t)1 << 31) return FSI_ERR_ARG;   // 32-bit node indices
    fsi_ctx* h = new fsi_ctx();
    Context* ctx = &h->c;
    ctx->mesh = *m;
    ctx->nlev = lev + 1;
    fsi_default_mg_params(&ctx->prm);
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&ctx->stream) != hipSuccess) {
            delete h;
            return FSI_ERR_HIP;
        }
        ctx->own_stream = true;
    }
    ctx->lv.resize(ctx->nlev);
    fsi_status st = FSI_OK;
    for (int j = 0; j < ctx->nlev && st == FSI_OK; ++j) {
        int cells[3] = {1, 1, 1};
        for (int d = 0; d < m->dim; ++d) cells[d] = m->n_coarse[d] << j;
        st = build_level(ctx, ctx->lv[j], m->dim, cells, *m);
    }
    if (st == FSI_OK) st = dalloc(ctx, &ctx->d_scratch, 4 * kReduceBlocks + 64);
    // the allocation-free FP32 Stokes apply's staging array on this device
    if (st == FSI_OK) ctx->noalloc_scratch = scratch_address();
    if (st == FSI_OK) st = dalloc(ctx, &ctx->d_flag, 4);
    if (st == FSI_OK && hipHostMalloc((void**)&ctx->h_flag, sizeof(int) * 4) != hipSuccess) st = FSI_ERR_HIP;
    if (st == FSI_OK && hipHostMalloc((void**)&ctx->h_dbl, sizeof(double) * 64) != hipSuccess) st = FSI_ERR_HIP;
    for (int pi = 0; pi < 2; ++pi) {
        ctx->tune_variant[pi].assign((size_t)ctx->nlev * kTuneClasses, 0);
        ctx->tune_us[pi].assign((size_t)ctx->nlev * kTuneClasses, 0.0);
        ctx->fuse_cheb[pi].assign(ctx->nlev, 1);
        ctx->fuse_res[pi].assign(ctx->nlev, 1);
        ctx->atom[pi].assign((size_t)ctx->nlev * kTuneClasses, -1);
        ctx->atom_conv[pi].assign((size_t)ctx->nlev, -1);
    }
    if (st != FSI_OK) {
        fsi_destroy(h);
        return st;
    }
    *out = h;
    return FSI_OK;
}

void fsi_destroy(fsi_ctx* h) {
    if (!h) return;
    Context* ctx = &h->c;
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    for (int pi = 0; pi < 2; ++pi) {
        if (ctx->graph_valid[pi]) hipGraphExecDestroy(ctx->graph[pi]);
        if (ctx->ext_graph_valid[pi]) hipGraphExecDestroy(ctx->ext_graph[pi]);
    }
    for (void* p : ctx->allocations) hipFree(p);
    if (ctx->h_flag) hipHostFree(ctx->h_flag);
    if (ctx->h_dbl) hipHostFree(ctx->h_dbl);
    if (ctx->kr.h_host) hipHostFree(ctx->kr.h_host);
    if (ctx->own_stream) hipStreamDestroy(ctx->stream);
    delete h;
}

const char* fsi_last_error(const fsi_ctx* h) { return h ? h->c.err.c_str() : "null context"; }

fsi_status fsi_get_num_levels(const fsi_ctx* h, int* n) {
    if (!h || !n) return FSI_ERR_ARG;
    *n = h->c.nlev;
    return FSI_OK;
}

fsi_status fsi_get_sizes(const fsi_ctx* h, int level, fsi_sizes* s) {
    if (!h || !s) return FSI_ERR_ARG;
    if (level < 0 || level >= h->c.nlev) return FSI_ERR_ARG;
    const Level& L = h->c.lv[level];
    s->n_cells = L.nc;
    s->n_vel_nodes = L.nvn;
    s->n_vel = L.nv;
    s->n_p = L.np;
    s->n_qp = L.Q;
    s->n_vert = L.nvert;
    for (int d = 0; d < 3; ++d) {
        s->cells[d] = L.cells[d];
        s->vel_nodes[d] = L.vnodes[d];
        s->p_nodes[d] = L.pnodes[d];
    }
    return FSI_OK;
}

fsi_status fsi_set_jacobians(fsi_ctx* h, int level, const double* J) {
    if (!h || !J) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(check_level(ctx, level));
    Level& L = ctx->lv[level];
    invalidate(ctx);
    launch_fill<int>(ctx->d_flag, 0, 1, ctx->stream);
    launch_geometry(L, J, L.d_K64, L.d_cw64, L.d_K32, ctx->d_flag, ctx->stream);
    L.geo_set = false;
    L.coef_set = false;
    L.vgeo_avail = L.vgeo = L.vgeo64 = false;   // arbitrary per-point Jacobians: stored geometry only
    TRY(sync_flag(ctx, FSI_ERR_INVERTED_CELL, "det J <= 0 (or not finite) at a quadrature point"));
    L.geo_set = true;
    L.conv_set = false;   // beta = K v° follows the geometry
    return FSI_OK;
}

fsi_status fsi_set_displacement(fsi_ctx* h, const double* disp) {
    if (!h || !disp) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    invalidate(ctx);
    const int J = ctx->nlev - 1;
    const Level& F = ctx->lv[J];
    launch_fill<int>(ctx->d_flag, 0, 1, ctx->stream);
    for (int j = 0; j <= J; ++j) {
        Level& L = ctx->lv[j];
        double hh[3];
        for (int d = 0; d < L.dim; ++d) hh[d] = ctx->mesh.extent[d] / L.cells[d];
        launch_geometry_from_disp(L, disp, 1 << (J - j), F.pnodes, hh, L.d_K64, L.d_cw64, L.d_K32, ctx->d_flag,
                                    ctx->stream);
        launch_vertex_disp(L, disp, 1 << (J - j), F.pnodes, L.d_vd32, L.d_vd64, ctx->stream);
        L.geo_set = false;
        L.coef_set = false;
        L.vgeo_avail = L.dim == 3;
        L.vgeo = L.vgeo_avail && (ctx->prm.vertex_geometry & 1);
        L.vgeo64 = L.vgeo_avail && (ctx->prm.vertex_geometry & 2);
    }
    TRY(sync_flag(ctx, FSI_ERR_INVERTED_CELL, "det J <= 0 (or not finite) at a quadrature point"));
    for (int j = 0; j <= J; ++j) {
        ctx->lv[j].geo_set = true;
        ctx->lv[j].conv_set = false;   // beta = K v° follows the geometry
    }
    return FSI_OK;
}

fsi_status fsi_set_coefficients(fsi_ctx* h, int level, const double* c_mass, const double* eta) {
    if (!h || !c_mass || !eta) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(check_level(ctx, level));
    Level& L = ctx->lv[level];
    if (!L.geo_set) return fail(ctx, FSI_ERR_STATE, "set_coefficients before the level's geometry");
    invalidate(ctx);
    launch_fill<int>(ctx->d_flag, 0, 1, ctx->stream);
    launch_coefficients(L, c_mass, eta, L.d_cw64, L.d_cv64, L.d_cv32, L.d_cq32, L.d_cq64, L.d_K64, L.d_Ks64, L.d_Ks32,
                        ctx->d_flag, ctx->stream);
    L.coef_set = false;
    TRY(sync_flag(ctx, FSI_ERR_NONFINITE, "coefficient not finite (or negative viscosity)"));
    L.coef_set = true;
    return FSI_OK;
}

fsi_status fsi_set_mg_params(fsi_ctx* h, const fsi_mg_params* p) {
    if (!h || !p) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    if (p->k_A < 1 || p->m < 0 || p->n_cycles < 1 || p->k_S != 1 || p->n_S != 1 || !(p->cheb_upper > 0) ||
        !(p->cheb_ratio > 1) || p->n_eig < 1 || (p->precision != FSI_PREC_FP64 && p->precision != FSI_PREC_MIXED) ||
        (p->corrector != 0 && p->corrector != 1) || (p->atomics != 0 && p->atomics != 1) ||
        p->vertex_geometry < 0 || p->vertex_geometry > 3)
        return fail(ctx, FSI_ERR_ARG, "invalid multigrid parameters (only k_S = n_S = 1 are implemented)");
    const fsi_mg_params& o = ctx->prm;
    // precision and graph use select among already prepared paths; the rest changes the setup
    const bool same = o.k_A == p->k_A && o.m == p->m && o.n_cycles == p->n_cycles && o.cheb_upper == p->cheb_upper &&
                      o.cheb_ratio == p->cheb_ratio && o.n_eig == p->n_eig && o.corrector == p->corrector;
    ctx->prm = *p;
    for (Level& L : ctx->lv) {
        L.vgeo = L.vgeo_avail && (p->vertex_geometry & 1);
        L.vgeo64 = L.vgeo_avail && (p->vertex_geometry & 2);
    }
    if (!same) invalidate(ctx);
    return FSI_OK;
}

fsi_status fsi_setup(fsi_ctx* h) {
    if (!h) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    invalidate(ctx);
    for (int j = 0; j < ctx->nlev; ++j)
        if (!ctx->lv[j].geo_set || !ctx->lv[j].coef_set)
            return fail(ctx, FSI_ERR_STATE, "setup needs geometry and coefficients on every level");
    if (ctx->prm.corrector)
        for (int j = 0; j < ctx->nlev; ++j)
            if (!ctx->lv[j].conv_set)
                return fail(ctx, FSI_ERR_STATE, "corrector mode needs fsi_set_convection on every level");
    TRY(alloc_work<double>(ctx));
    TRY(alloc_work<float>(ctx));
    const int J = ctx->nlev - 1;
    const Level& F = ctx->lv[J];
    if (!ctx->vc_in_u) {
        TRY(dalloc(ctx, &ctx->vc_in_u, F.nv));
        TRY(dalloc(ctx, &ctx->vc_in_p, F.np));
        TRY(dalloc(ctx, &ctx->vc_out_u, F.nv));
        TRY(dalloc(ctx, &ctx->vc_out_p, F.np));
        TRY(dalloc(ctx, &ctx->vc_tmp, F.nv + F.np));
    }
    hipStream_t s = ctx->stream;
    for (int j = 0; j < ctx->nlev; ++j) {
        Level& L = ctx->lv[j];
        double* diag = ctx->w64[j].r_u;   // scratch
        launch_fill<double>(diag, 0.0, L.nv, s);
        launch_diagA(L, L.d_K64, L.d_cv64, diag, s, ctx->prm.corrector != 0);
        launch_diagA_finish(L, diag, L.d_dAinv64, L.d_dAinv32, s);
        double n2;
        TRY(dot64(ctx, diag, diag, L.nv, &n2));
        L.diagA_norm = std::sqrt(n2);
        launch_diagS_impl(L, L.d_wall, L.d_K64, L.d_dAinv64, L.d_dSinv, s);
        // ||diag S|| from its inverse
        double* tmp = ctx->w64[j].t_p;
        launch_recip(L.d_dSinv, tmp, L.np, s);
        TRY(dot64(ctx, tmp, tmp, L.np, &n2));
        L.diagS_norm = std::sqrt(n2);
        TRY(lanczos(ctx, j));
    }
    TRY(setup_coarse(ctx));
    FSI_HIP_TRY(hipStreamSynchronize(s));
    TRY(capture_graphs(ctx));
    ctx->setup_done = true;
    return FSI_OK;
}

fsi_status fsi_get_level_info(const fsi_ctx* h, int level, fsi_level_info* info) {
    if (!h || !info) return FSI_ERR_ARG;
    const Context* ctx = &h->c;
    if (level < 0 || level >= ctx->nlev) return FSI_ERR_ARG;
    if (!ctx->setup_done) return FSI_ERR_STATE;
    const Level& L = ctx->lv[level];
    info->lambda_max = L.lam;
    info->cheb_lo = L.lo;
    info->cheb_hi = L.hi;
    info->diagA_norm2 = L.diagA_norm;
    info->diagS_norm2 = L.diagS_norm;
    info->coarse_n = level == 0 ? ctx->coarse.n : 0;
    return FSI_OK;
}

static fsi_status apply_check(Context* ctx, int level, bool need_coef) {
    TRY(check_level(ctx, level));
    const Level& L = ctx->lv[level];
    if (!L.geo_set) return fail(ctx, FSI_ERR_STATE, "apply before the level's geometry");
    if (need_coef && !L.coef_set) return fail(ctx, FSI_ERR_STATE, "apply before the level's coefficients");
    return FSI_OK;
}

fsi_status fsi_apply_A(fsi_ctx* h, int level, const double* u, double* v) {
    if (!h || !u || !v) return FSI_ERR_ARG;
    TRY(apply_check(&h->c, level, true));
    op_apply<double>(&h->c, level, OP_A, u, nullptr, v, nullptr, h->c.stream);
    return FSI_OK;
}
fsi_status fsi_apply_B(fsi_ctx* h, int level, const double* u, double* q) {
    if (!h || !u || !q) return FSI_ERR_ARG;
    TRY(apply_check(&h->c, level, false));
    op_apply<double>(&h->c, level, OP_B, u, nullptr, nullptr, q, h->c.stream);
    return FSI_OK;
}
fsi_status fsi_apply_BT(fsi_ctx* h, int level, const double* p, double* v) {
    if (!h || !p || !v) return FSI_ERR_ARG;
    TRY(apply_check(&h->c, level, false));
    op_apply<double>(&h->c, level, OP_BT, nullptr, p, v, nullptr, h->c.stream);
    return FSI_OK;
}
fsi_status fsi_apply_stokes(fsi_ctx* h, int level, const double* u, const double* p, double* v, double* q) {
    if (!h || !u || !p || !v || !q) return FSI_ERR_ARG;
    TRY(apply_check(&h->c, level, true));
    op_apply<double>(&h->c, level, OP_A | OP_BT | OP_B, u, p, v, q, h->c.stream);
    return FSI_OK;
}

// FP32 twins: pressure is carried in FP64 inside the kernels; cast at the boundary
static fsi_status p_scratch(Context* ctx, int level, double** a, double** b) {
    TRY(alloc_work<double>(ctx));
    *a = ctx->w64[level].z_p;
    *b = ctx->w64[level].t_p;
    return FSI_OK;
}
fsi_status fsi_apply_A_f32(fsi_ctx* h, int level, const float* u, float* v) {
    if (!h || !u || !v) return FSI_ERR_ARG;
    TRY(apply_check(&h->c, level, true));
    op_apply<float>(&h->c, level, OP_A, u, nullptr, v, nullptr, h->c.stream);
    return FSI_OK;
}
fsi_status fsi_apply_B_f32(fsi_ctx* h, int level, const float* u, float* q) {
    if (!h || !u || !q) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(apply_check(ctx, level, false));
    double *a, *b;
    TRY(p_scratch(ctx, level, &a, &b));
    op_apply<float>(ctx, level, OP_B, u, nullptr, nullptr, b, ctx->stream);
    launch_cast<float, double>(q, b, ctx->lv[level].np, ctx->stream);
    return FSI_OK;
}
fsi_status fsi_apply_BT_f32(fsi_ctx* h, int level, const float* p, float* v) {
    if (!h || !p || !v) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(apply_check(ctx, level, false));
    double *a, *b;
    TRY(p_scratch(ctx, level, &a, &b));
    launch_cast<double, float>(a, p, ctx->lv[level].np, ctx->stream);
    op_apply<float>(ctx, level, OP_BT, nullptr, a, v, nullptr, ctx->stream);
    return FSI_OK;
}
fsi_status fsi_apply_stokes_f32(fsi_ctx* h, int level, const float* u, const float* p, float* v, float* q) {
    if (!h || !u || !p || !v || !q) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(apply_check(ctx, level, true));
    double *a, *b;
    TRY(p_scratch(ctx, level, &a, &b));
    launch_cast<double, float>(a, p, ctx->lv[level].np, ctx->stream);
    op_apply<float>(ctx, level, OP_A | OP_BT | OP_B, u, a, v, b, ctx->stream);
    launch_cast<float, double>(q, b, ctx->lv[level].np, ctx->stream);
    return FSI_OK;
}

fsi_status fsi_apply_stokes_f32_noalloc(fsi_ctx* h, int level, const float* u, const float* p, float* v,
                                        float* q) {
    if (!h || !u || !p || !v || !q) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(check_level(ctx, level));
    const Level& L = ctx->lv[level];
    if (L.np > kNoAllocMaxP)
        return fail(ctx, FSI_ERR_ARG, "fsi_apply_stokes_f32_noalloc: the level has " + std::to_string(L.np) +
                                          " pressure nodes, more than the staging limit of " +
                                          std::to_string(kNoAllocMaxP));
    if (!ctx->noalloc_scratch)
        return fail(ctx, FSI_ERR_HIP, "fsi_apply_stokes_f32_noalloc: no device address for the staging array");
    TRY(apply_check(ctx, level, true));
    // the same kernels as fsi_apply_stokes_f32; the outputs of the pressure sums are
    // written in full by the apply (first-touch stores, or the atomic form's zeroing)
    double* a = ctx->noalloc_scratch;
    double* b = ctx->noalloc_scratch + kNoAllocMaxP;
    launch_cast<double, float>(a, p, L.np, ctx->stream);
    op_apply<float>(ctx, level, OP_A | OP_BT | OP_B, u, a, v, b, ctx->stream);
    launch_cast<float, double>(q, b, L.np, ctx->stream);
    return FSI_OK;
}

fsi_status fsi_set_convection(fsi_ctx* h, int level, const double* vconv, const double* r, double rho) {
    if (!h || !vconv || !r) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(check_level(ctx, level));
    Level& L = ctx->lv[level];
    if (!(rho >= 0.0) || !std::isfinite(rho)) return fail(ctx, FSI_ERR_ARG, "fsi_set_convection: rho must be >= 0");
    if (!L.geo_set) return fail(ctx, FSI_ERR_STATE, "fsi_set_convection before the level's geometry");
    const int64_t P = L.plane();
    if (!L.d_cb64) {
        TRY(dalloc(ctx, &L.d_cb64, 3 * P));   // dim planes used
        TRY(dalloc(ctx, &L.d_cs64, P));
        TRY(dalloc(ctx, &L.d_cb32, 3 * P));
        TRY(dalloc(ctx, &L.d_cs32, P));
    }
    launch_fill<int>(ctx->d_flag, 0, 1, ctx->stream);
    launch_convection(L, vconv, r, L.d_cb64, L.d_cs64, L.d_cb32, L.d_cs32, ctx->d_flag, ctx->stream);
    L.conv_set = false;
    TRY(sync_flag(ctx, FSI_ERR_NONFINITE, "convective velocity or streamline parameter not finite, or r < 0"));
    L.rho = rho;
    L.conv_set = true;
    return FSI_OK;
}

static fsi_status conv_check(Context* ctx, int level) {
    TRY(apply_check(ctx, level, true));
    if (!ctx->lv[level].conv_set) return fail(ctx, FSI_ERR_STATE, "corrector apply before fsi_set_convection");
    return FSI_OK;
}

fsi_status fsi_apply_corrector(fsi_ctx* h, int level, const double* u, const double* p, double* v, double* q) {
    if (!h || !u || !p || !v || !q) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(conv_check(ctx, level));
    op_apply<double>(ctx, level, OP_A | OP_BT | OP_B | OP_CONV, u, p, v, q, ctx->stream);
    return FSI_OK;
}

fsi_status fsi_apply_corrector_f32(fsi_ctx* h, int level, const float* u, const float* p, float* v, float* q) {
    if (!h || !u || !p || !v || !q) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(conv_check(ctx, level));
    double *a, *b;
    TRY(p_scratch(ctx, level, &a, &b));
    launch_cast<double, float>(a, p, ctx->lv[level].np, ctx->stream);
    op_apply<float>(ctx, level, OP_A | OP_BT | OP_B | OP_CONV, u, a, v, b, ctx->stream);
    launch_cast<float, double>(q, b, ctx->lv[level].np, ctx->stream);
    return FSI_OK;
}

fsi_status fsi_vcycle(fsi_ctx* h, const double* r_u, const double* r_p, double* z_u, double* z_p) {
    if (!h || !r_u || !r_p || !z_u || !z_p) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    if (!ctx->setup_done) return fail(ctx, FSI_ERR_STATE, "vcycle before setup");
    if (!ctx->coarse_block_ok)
        return fail(ctx, FSI_ERR_STATE, "singular coarse block matrix (fixed cells): extension solves only");
    const Level& L = ctx->lv[ctx->nlev - 1];
    hipStream_t s = ctx->stream;
    // combined staging through the Krylov-independent IO buffers
    FSI_HIP_TRY(hipMemcpyAsync(ctx->vc_in_u, r_u, sizeof(double) * L.nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(ctx->vc_in_p, r_p, sizeof(double) * L.np, hipMemcpyDeviceToDevice, s));
    if (ctx->prm.n_cycles == 1) {
        TRY(run_vcycle(ctx, s));
        FSI_HIP_TRY(hipMemcpyAsync(z_u, ctx->vc_out_u, sizeof(double) * L.nv, hipMemcpyDeviceToDevice, s));
        FSI_HIP_TRY(hipMemcpyAsync(z_p, ctx->vc_out_p, sizeof(double) * L.np, hipMemcpyDeviceToDevice, s));
        return FSI_OK;
    }
    TRY(ensure_krylov(ctx, std::max(ctx->kr.restart, 1)));
    double* r = ctx->kr.r;
    double* z = ctx->kr.w;
    FSI_HIP_TRY(hipMemcpyAsync(r, r_u, sizeof(double) * L.nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(r + L.nv, r_p, sizeof(double) * L.np, hipMemcpyDeviceToDevice, s));
    TRY(precond_combined(ctx, r, z, s));
    FSI_HIP_TRY(hipMemcpyAsync(z_u, z, sizeof(double) * L.nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(z_p, z + L.nv, sizeof(double) * L.np, hipMemcpyDeviceToDevice, s));
    return FSI_OK;
}

fsi_status fsi_solve(fsi_ctx* h, const double* g_u, const double* g_p, double* u, double* p,
                     const fsi_solve_opts* o, fsi_solve_info* info) {
    if (!h || !g_u || !g_p || !u || !p || !o) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    if (!ctx->setup_done) return fail(ctx, FSI_ERR_STATE, "solve before setup");
    if (!ctx->coarse_block_ok)
        return fail(ctx, FSI_ERR_STATE, "singular coarse block matrix (fixed cells): extension solves only");
    if (o->restart < 1 || o->max_iter < 0 || !(o->rtol >= 0) || o->reorth < 0 || o->reorth > 2)
        return fail(ctx, FSI_ERR_ARG, "invalid solve options");
    const auto t0 = std::chrono::steady_clock::now();
    TRY(ensure_krylov(ctx, o->restart));
    Krylov& K = ctx->kr;
    const Level& L = ctx->lv[ctx->nlev - 1];
    const int64_t n = K.n, nv = L.nv, np = L.np;
    hipStream_t s = ctx->stream;
    FSI_HIP_TRY(hipMemcpyAsync(K.g, g_u, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(K.g + nv, g_p, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(K.x, u, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(K.x + nv, p, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
    launch_fill<int>(ctx->d_flag, 0, 1, s);
    launch_nonfinite(K.g, n, ctx->d_flag, s);
    launch_nonfinite(K.x, n, ctx->d_flag, s);
    TRY(sync_flag(ctx, FSI_ERR_NONFINITE, "right-hand side or initial guess not finite"));
    double gn2;
    TRY(dot64(ctx, K.g, K.g, n, &gn2));
    const double gnorm = std::sqrt(gn2);
    int hist_n = 0;
    auto push_hist = [&](double v) {
        if (info && info->res_history && hist_n < o->max_iter + 1) info->res_history[hist_n] = v;
        ++hist_n;
    };
    if (gnorm == 0.0) {
        launch_fill<double>(u, 0.0, nv, s);
        launch_fill<double>(p, 0.0, np, s);
        FSI_HIP_TRY(hipStreamSynchronize(s));
        if (info) {
            info->iters = 0;
            info->final_rel_res = 0.0;
            info->n_hist = 0;
            info->time_ms = 0.0;
        }
        return FSI_OK;
    }
    stokes_combined(ctx, K.x, K.w, s);
    launch_sub_into(K.g, K.w, K.r, n, s);
    double b2;
    TRY(dot64(ctx, K.r, K.r, n, &b2));
    double beta = std::sqrt(b2);
    push_hist(beta / gnorm);
    int it = 0, reorth = 0;
    const int R = o->restart;
    std::vector<double> H((size_t)(R + 1) * R), cs(R), sn(R), sv(R + 1), y(R);
    fsi_status status = FSI_OK;
    while (beta / gnorm > o->rtol && it < o->max_iter) {
        if (!std::isfinite(beta)) {
            status = fail(ctx, FSI_ERR_NONFINITE, "non-finite residual in FGMRES");
            break;
        }
        launch_scale_host(1.0 / beta, K.r, K.V, n, s);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(sv.begin(), sv.end(), 0.0);
        sv[0] = beta;
        int kused = 0;
        bool done = false;
        for (int k = 0; k < R; ++k) {
            double* Vk = K.V + (int64_t)k * n;
            double* Zk = K.Z + (int64_t)k * n;
            TRY(precond_combined(ctx, Vk, Zk, s));
            stokes_combined(ctx, Zk, K.w, s);
            // classical Gram-Schmidt as batched passes over the basis
            // h[0..k] = V^T w and h[k+1] = ||w||^2 in one sweep; the projection
            // returns ||w||^2 after it in h[R+1]
            launch_multi_dot(K.V, n, k + 1, K.w, n, K.partials, K.h, s, true);
            launch_multi_axpy_norm(K.V, n, k + 1, K.h, -1.0, K.w, n, K.partials, K.h + (R + 1), s);
            FSI_HIP_TRY(hipMemcpyAsync(K.h_host, K.h, sizeof(double) * (R + 2), hipMemcpyDeviceToHost, s));
            FSI_HIP_TRY(hipStreamSynchronize(s));
            for (int i = 0; i <= k; ++i) H[(size_t)i * R + k] = K.h_host[i];
            double after = K.h_host[R + 1];
            // second pass: never (reorth 0), when the DGKS test flags cancellation
            // (reorth 1), or always (reorth 2)
            if (o->reorth == 2 || (o->reorth == 1 && after < 0.5 * K.h_host[k + 1])) {
                launch_multi_dot(K.V, n, k + 1, K.w, n, K.partials, K.h + (R + 2), s);
                launch_multi_axpy_norm(K.V, n, k + 1, K.h + (R + 2), -1.0, K.w, n, K.partials, K.h + (R + 1), s);
                FSI_HIP_TRY(hipMemcpyAsync(K.h_host, K.h, sizeof(double) * 2 * (R + 2), hipMemcpyDeviceToHost, s));
                FSI_HIP_TRY(hipStreamSynchronize(s));
                for (int i = 0; i <= k; ++i) H[(size_t)i * R + k] += K.h_host[(R + 2) + i];
                after = K.h_host[R + 1];
                ++reorth;
            }
            const double hnext = std::sqrt(after);
            H[(size_t)(k + 1) * R + k] = hnext;
            for (int i = 0; i < k; ++i) {
                const double a = H[(size_t)i * R + k], b = H[(size_t)(i + 1) * R + k];
                H[(size_t)i * R + k] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * R + k] = -sn[i] * a + cs[i] * b;
            }
            const double a = H[(size_t)k * R + k], b = H[(size_t)(k + 1) * R + k];
            const double den = std::hypot(a, b);
            if (!(den > 0) || !std::isfinite(den)) {
                status = fail(ctx, FSI_ERR_BREAKDOWN, "FGMRES breakdown (zero or non-finite Hessenberg column)");
                done = true;
                break;
            }
            cs[k] = a / den;
            sn[k] = b / den;
            H[(size_t)k * R + k] = den;
            H[(size_t)(k + 1) * R + k] = 0.0;
            sv[k + 1] = -sn[k] * sv[k];
            sv[k] = cs[k] * sv[k];
            ++it;
            kused = k + 1;
            push_hist(std::fabs(sv[k + 1]) / gnorm);
            if (std::fabs(sv[k + 1]) / gnorm <= o->rtol || it >= o->max_iter || hnext == 0.0) break;
            launch_scale_host(1.0 / hnext, K.w, K.V + (int64_t)(k + 1) * n, n, s);
        }
        if (kused > 0) {
            for (int i = kused - 1; i >= 0; --i) {
                double acc = sv[i];
                for (int jj = i + 1; jj < kused; ++jj) acc -= H[(size_t)i * R + jj] * y[jj];
                y[i] = acc / H[(size_t)i * R + i];
            }
            double* yh = K.h_host + 2 * (R + 2);
            for (int i = 0; i < kused; ++i) yh[i] = y[i];
            FSI_HIP_TRY(hipMemcpyAsync(K.h, yh, sizeof(double) * kused, hipMemcpyHostToDevice, s));
            launch_multi_axpy(K.Z, n, kused, K.h, 1.0, K.x, n, s);
        }
        stokes_combined(ctx, K.x, K.w, s);
        launch_sub_into(K.g, K.w, K.r, n, s);
        TRY(dot64(ctx, K.r, K.r, n, &b2));
        beta = std::sqrt(b2);
        if (done) break;
    }
    FSI_HIP_TRY(hipMemcpyAsync(u, K.x, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipMemcpyAsync(p, K.x + nv, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
    FSI_HIP_TRY(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (getenv("FSI_SOLVE_VERBOSE"))
        fprintf(stderr, "[fsi solve] %d iterations, %d reorthogonalisations, %.1f ms\n", it, reorth, ms);
    if (info) {
        info->iters = it;
        info->final_rel_res = beta / gnorm;
        info->time_ms = ms;
        info->n_hist = std::min(hist_n, o->max_iter + 1);
    }
    if (status != FSI_OK) return status;
    if (!std::isfinite(beta)) return fail(ctx, FSI_ERR_NONFINITE, "non-finite final residual");
    return beta / gnorm <= o->rtol ? FSI_OK : FSI_NOT_CONVERGED;
}

// one processing phase of a level operator on the level's work vectors (timing and
// tuning only: the fused Chebyshev mode runs with c1 = c2 = 0, so it leaves x as is)
static void launch_phase_on_work(Context* ctx, int prec, int j, int mode, int var, int ph, hipStream_t s) {
    const Level& L = ctx->lv[j];
    if (prec == 0) {
        LevelWork<double>& W = ctx->w64[j];
        if (mode == (OP_A | OP_CHEB))
            launch_cell_cheb<double>(L, var, ph, L.d_Ks64, L.d_cv64, W.w_u, W.cd_u, W.f_u, L.d_dAinv64, W.cax_u, 0.0,
                                     0.0, false, true, s);
        else if (mode == (OP_A | OP_BT | OP_B | OP_RES))
            launch_cell_res<double>(L, var, ph, L.d_K64, L.d_cv64, W.x_u, W.x_p, W.f_u, W.f_p, W.r_u, W.r_p, s);
        else
            launch_cell<double>(L, mode, var, ph, Kmode<double>(L, mode), L.d_cv64, W.x_u, W.x_p, W.r_u, W.r_p, s);
    } else {
        LevelWork<float>& W = ctx->w32[j];
        if (mode == (OP_A | OP_CHEB))
            launch_cell_cheb<float>(L, var, ph, L.d_Ks32, L.d_cv32, W.w_u, W.cd_u, W.f_u, L.d_dAinv32, W.cax_u, 0.0,
                                    0.0, false, true, s);
        else if (mode == (OP_A | OP_BT | OP_B | OP_RES))
            launch_cell_res<float>(L, var, ph, L.d_K32, L.d_cv32, W.x_u, W.x_p, W.f_u, W.f_p, W.r_u, W.r_p, s);
        else
            launch_cell<float>(L, mode, var, ph, Kmode<float>(L, mode), L.d_cv32, W.x_u, W.x_p, W.r_u, W.r_p, s);
    }
}

// the single atomic launch of an unfused level operator on the level's work vectors
// (timing and tuning only)
static void launch_atomic_on_work(Context* ctx, int prec, int j, int mode, int shape, hipStream_t s) {
    const Level& L = ctx->lv[j];
    if (prec == 0) {
        LevelWork<double>& W = ctx->w64[j];
        launch_cell_atomic<double>(L, mode, shape, Kmode<double>(L, mode), L.d_cv64, W.x_u, W.x_p, W.r_u, W.r_p, s);
    } else {
        LevelWork<float>& W = ctx->w32[j];
        launch_cell_atomic<float>(L, mode, shape, Kmode<float>(L, mode), CVp<float>(L), W.x_u, W.x_p, W.r_u, W.r_p, s);
    }
}

fsi_status fsi_solve_extension(fsi_ctx* h, const double* g, double* u, const fsi_solve_opts* o,
                               fsi_solve_info* info) {
    if (!h || !g || !u || !o) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    if (!ctx->setup_done) return fail(ctx, FSI_ERR_STATE, "extension solve before setup");
    if (o->max_iter < 0 || !(o->rtol >= 0)) return fail(ctx, FSI_ERR_ARG, "invalid solve options");
    if (ctx->prm.corrector) return fail(ctx, FSI_ERR_ARG, "the extension solve is not a corrector-mode problem");
    const int J = ctx->nlev - 1;
    Level& L = ctx->lv[J];
    const int64_t nv = L.nv;
    hipStream_t s = ctx->stream;
    if (!ctx->ext_ready) {
        TRY(setup_coarse_u(ctx));
        if (!ctx->ext_buf) TRY(dalloc(ctx, &ctx->ext_buf, 8 * nv));
        ctx->ext_ready = true;
    }
    const auto t0 = std::chrono::steady_clock::now();
    double* b = ctx->ext_buf;
    double* x = b + nv;
    double* r = x + nv;
    double* z = r + nv;
    double* zo = z + nv;
    double* pd = zo + nv;
    double* q = pd + nv;
    double* gw = q + nv;
    // boundary data on the walls (gw) and the interior initial guess (x, walls zero)
    launch_fill<double>(gw, 0.0, nv, s);
    launch_dirichlet_copy<double>(L, g, gw, s);
    FSI_HIP_TRY(hipMemcpyAsync(x, u, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
    launch_dirichlet_zero<double>(L, x, s);
    launch_fill<int>(ctx->d_flag, 0, 1, s);
    launch_nonfinite(gw, nv, ctx->d_flag, s);
    launch_nonfinite(x, nv, ctx->d_flag, s);
    TRY(sync_flag(ctx, FSI_ERR_NONFINITE, "boundary data or initial guess not finite"));
    // lifting: b = -(A gw) on the interior rows, with the unconstrained operator (wall
    // columns kept)
    TRY(apply_unconstrained(ctx, OP_A, gw, nullptr, q, nullptr, s));
    launch_scale_host(-1.0, q, b, nv, s);
    launch_dirichlet_zero<double>(L, b, s);
    double bn2;
    TRY(dot64(ctx, b, b, nv, &bn2));
    const double bnorm = std::sqrt(bn2);
    int hist_n = 0;
    auto push_hist = [&](double v) {
        if (info && info->res_history && hist_n < o->max_iter + 1) info->res_history[hist_n] = v;
        ++hist_n;
    };
    auto finish = [&](int it, double rel, fsi_status st) -> fsi_status {
        // u = x on the interior, g on the walls
        FSI_HIP_TRY(hipMemcpyAsync(u, x, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
        launch_dirichlet_copy<double>(L, gw, u, s);
        FSI_HIP_TRY(hipStreamSynchronize(s));
        if (info) {
            info->iters = it;
            info->final_rel_res = rel;
            info->n_hist = std::min(hist_n, o->max_iter + 1);
            info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        return st;
    };
    if (bnorm == 0.0) {   // zero boundary data: the extension vanishes
        launch_fill<double>(x, 0.0, nv, s);
        return finish(0, 0.0, FSI_OK);
    }
    op_apply<double>(ctx, J, OP_A, x, nullptr, q, nullptr, s);
    launch_sub<double>(b, q, r, nv, s);
    launch_dirichlet_zero<double>(L, r, s);
    double rr;
    TRY(dot64(ctx, r, r, nv, &rr));
    double rel = std::sqrt(rr) / bnorm;
    push_hist(rel);
    int it = 0;
    fsi_status status = FSI_OK;
    if (rel > o->rtol && o->max_iter > 0) {
        TRY(ext_run_precond(ctx, r, z, s));
        double rz;
        TRY(dot64(ctx, r, z, nv, &rz));
        FSI_HIP_TRY(hipMemcpyAsync(pd, z, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
        while (rel > o->rtol && it < o->max_iter) {
            op_apply<double>(ctx, J, OP_A, pd, nullptr, q, nullptr, s);
            double pq;
            TRY(dot64(ctx, pd, q, nv, &pq));
            if (!(pq > 0.0) || !std::isfinite(pq)) {
                status = fail(ctx, FSI_ERR_BREAKDOWN, "CG breakdown in the extension solve");
                break;
            }
            const double alpha = rz / pq;
            launch_axpy_host(alpha, pd, x, nv, s);
            launch_axpy_host(-alpha, q, r, nv, s);
            TRY(dot64(ctx, r, r, nv, &rr));
            rel = std::sqrt(rr) / bnorm;
            ++it;
            push_hist(rel);
            if (rel <= o->rtol) break;
            // flexible (Polak-Ribiere) beta: the preconditioner may vary between calls;
            // the preconditioner always writes the same buffer (the captured graph's)
            FSI_HIP_TRY(hipMemcpyAsync(zo, z, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
            TRY(ext_run_precond(ctx, r, z, s));
            double rz_new, rzo;
            TRY(dot64(ctx, r, z, nv, &rz_new));
            TRY(dot64(ctx, r, zo, nv, &rzo));
            const double beta = (rz_new - rzo) / rz;
            rz = rz_new;
            launch_xpby_host(z, beta, pd, nv, s);
        }
    }
    if (status != FSI_OK) return status;
    // true residual at exit
    op_apply<double>(ctx, J, OP_A, x, nullptr, q, nullptr, s);
    launch_sub<double>(b, q, r, nv, s);
    launch_dirichlet_zero<double>(L, r, s);
    TRY(dot64(ctx, r, r, nv, &rr));
    rel = std::sqrt(rr) / bnorm;
    return finish(it, rel, rel <= o->rtol ? FSI_OK : FSI_NOT_CONVERGED);
}

// ---------------------------------------------------------------- fixed nodes (extension on the fluid part)
fsi_status fsi_set_fixed_cells(fsi_ctx* h, const uint8_t* fixed) {
    if (!h || !fixed) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    if (ctx->setup_done) return fail(ctx, FSI_ERR_STATE, "fsi_set_fixed_cells after fsi_setup");
    if (ctx->has_fixed) return fail(ctx, FSI_ERR_STATE, "fsi_set_fixed_cells called twice");
    const int J = ctx->nlev - 1;
    Level& F = ctx->lv[J];
    const int dim = F.dim, NLOC = dim == 3 ? 27 : 9;
    // nodes of the fixed cells on the finest level
    std::vector<uint8_t> fm((size_t)F.nvn, 0);
    for (int64_t c = 0; c < F.nc; ++c) {
        if (!fixed[c]) continue;
        const int64_t cx = c % F.cells[0], cy = (c / F.cells[0]) % F.cells[1], cz = c / ((int64_t)F.cells[0] * F.cells[1]);
        for (int n = 0; n < NLOC; ++n) {
            const int lx = n % 3, ly = (n / 3) % 3, lz = n / 9;
            fm[(size_t)((2 * cx + lx) + F.vnodes[0] * ((2 * cy + ly) + (int64_t)F.vnodes[1] * (2 * cz + lz)))] = 1;
        }
    }
    hipStream_t s = ctx->stream;
    FSI_HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j <= J; ++j) {
        Level& L = ctx->lv[j];
        const int64_t st = int64_t(1) << (J - j);
        bool changed = false;
        for (int64_t n = 0; n < L.nvn; ++n) {
            const int64_t ix = n % L.vnodes[0], iy = (n / L.vnodes[0]) % L.vnodes[1],
                          iz = n / ((int64_t)L.vnodes[0] * L.vnodes[1]);
            const int64_t fn = st * ix + F.vnodes[0] * (st * iy + (int64_t)F.vnodes[1] * st * iz);
            if (fm[(size_t)fn] && !L.h_dir_node[(size_t)n]) {
                L.h_dir_node[(size_t)n] = 1;
                changed = true;
            }
        }
        if (!changed) continue;
        std::vector<int> dirn;
        for (int64_t n = 0; n < L.nvn; ++n)
            if (L.h_dir_node[(size_t)n]) dirn.push_back((int)n);
        dfree(ctx, &L.d_dir_nodes);
        TRY(dalloc(ctx, &L.d_dir_nodes, (int64_t)dirn.size()));
        L.n_dir = (int64_t)dirn.size();
        FSI_HIP_TRY(hipMemcpy(L.d_dir_nodes, dirn.data(), sizeof(int) * dirn.size(), hipMemcpyHostToDevice));
        FSI_HIP_TRY(hipMemcpy(L.d_wall, L.h_dir_node.data(), (size_t)L.nvn, hipMemcpyHostToDevice));
        L.fixed_nodes = true;
        // wall bits of the cell info (processing order; vmap gives each local node's node)
        std::vector<int> vmap((size_t)L.nc * NLOC);
        std::vector<uint4> info((size_t)L.nc);
        FSI_HIP_TRY(hipMemcpy(vmap.data(), L.d_vmap, sizeof(int) * vmap.size(), hipMemcpyDeviceToHost));
        FSI_HIP_TRY(hipMemcpy(info.data(), L.d_info, sizeof(uint4) * info.size(), hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < L.nc; ++k)
            for (int n = 0; n < NLOC; ++n)
                if (L.h_dir_node[(size_t)vmap[(size_t)(k * NLOC + n)]]) info[(size_t)k].x |= 1u << n;
        FSI_HIP_TRY(hipMemcpy(L.d_info, info.data(), sizeof(uint4) * info.size(), hipMemcpyHostToDevice));
    }
    TRY(dalloc(ctx, &F.d_fixed, F.nvn));
    FSI_HIP_TRY(hipMemcpy(F.d_fixed, fm.data(), (size_t)F.nvn, hipMemcpyHostToDevice));
    for (int pi = 0; pi < 2; ++pi) {
        std::fill(ctx->atom[pi].begin(), ctx->atom[pi].end(), (int8_t)-1);
        std::fill(ctx->atom_conv[pi].begin(), ctx->atom_conv[pi].end(), (int8_t)-1);
    }
    ctx->has_fixed = true;
    return FSI_OK;
}

fsi_status fsi_fixed_values(fsi_ctx* h, const double* v, double* g) {
    if (!h || !v || !g) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    if (!ctx->has_fixed) return fail(ctx, FSI_ERR_STATE, "fsi_fixed_values without fsi_set_fixed_cells");
    const Level& F = ctx->lv[ctx->nlev - 1];
    launch_fixed_values(F, F.d_fixed, v, g, ctx->stream);
    return FSI_OK;
}

// ---------------------------------------------------------------- time step (Algorithm 1)
struct Bdf {
    double gamma, a1, a2;
};
static fsi_status gcsi_check(Context* ctx, const fsi_gcsi_params* p, Bdf* b) {
    if (!p) return FSI_ERR_ARG;
    if (p->k != 1 && p->k != 2) return fail(ctx, FSI_ERR_ARG, "BDF order k must be 1 or 2");
    auto fin = [](double x) { return std::isfinite(x); };
    if (!(p->tau > 0) || !fin(p->tau) || !(p->rho_f >= 0) || !fin(p->rho_f) || !(p->rho_s >= 0) || !fin(p->rho_s) ||
        !(p->eta_f > 0) || !fin(p->eta_f) || !(p->mu_s >= 0) || !fin(p->mu_s) || std::isnan(p->eta_V) ||
        !fin(p->body[0]) || !fin(p->body[1]) || (ctx->lv[0].dim == 3 && !fin(p->body[2])))
        return fail(ctx, FSI_ERR_ARG, "invalid time-step parameters");
    // BDF stencil of Sec. 3.1 (alpha_0 = 1)
    if (p->k == 1) *b = {1.0, -1.0, 0.0};
    else *b = {2.0 / 3.0, -4.0 / 3.0, 1.0 / 3.0};
    return FSI_OK;
}

fsi_status fsi_gcsi_displacement(fsi_ctx* h, const fsi_gcsi_params* prm, const double* w, const double* u1,
                                 const double* u2, double* u_out, double* disp_out) {
    if (!h || !w || !u1 || (!u_out && !disp_out)) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    Bdf b;
    TRY(gcsi_check(ctx, prm, &b));
    if (prm->k == 2 && !u2) return fail(ctx, FSI_ERR_ARG, "k = 2 needs u^{n-2}");
    const Level& F = ctx->lv[ctx->nlev - 1];
    launch_gcsi_displacement(F, w, u1, prm->k == 2 ? u2 : nullptr, b.gamma * prm->tau, b.a1, b.a2, u_out, disp_out,
                             ctx->stream);
    return FSI_OK;
}

static fsi_status gcsi_scratch(Context* ctx) {
    const Level& F = ctx->lv[ctx->nlev - 1];
    if (!ctx->gcsi_tmp) TRY(dalloc(ctx, &ctx->gcsi_tmp, (F.dim + 1) * F.nc * F.Q));
    return FSI_OK;
}

fsi_status fsi_gcsi_set_coefficients(fsi_ctx* h, const fsi_gcsi_params* prm, const uint8_t* const* solid_q) {
    if (!h || !solid_q) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    Bdf b;
    TRY(gcsi_check(ctx, prm, &b));
    for (int j = 0; j < ctx->nlev; ++j)
        if (!solid_q[j]) return fail(ctx, FSI_ERR_ARG, "fsi_gcsi_set_coefficients: null solid indicator");
    TRY(gcsi_scratch(ctx));
    const double gt = b.gamma * prm->tau;
    for (int j = 0; j < ctx->nlev; ++j) {
        Level& L = ctx->lv[j];
        const int64_t n = L.nc * L.Q;
        if (!L.d_gcsi_eta) TRY(dalloc(ctx, &L.d_gcsi_eta, n));
        launch_gcsi_coefficients(solid_q[j], prm->rho_f / gt, prm->rho_s / gt, prm->eta_f, gt * prm->mu_s,
                                 ctx->gcsi_tmp, L.d_gcsi_eta, n, ctx->stream);
        TRY(fsi_set_coefficients(h, j, ctx->gcsi_tmp, L.d_gcsi_eta));
    }
    ctx->gcsi_rho_f = prm->rho_f;
    return FSI_OK;
}

fsi_status fsi_gcsi_rhs(fsi_ctx* h, const fsi_gcsi_params* prm, int mode, const uint8_t* solid_q,
                        const double* disp, const double* u_hash, const double* u1, const double* u2,
                        const double* v1, const double* v2, const double* w1, const double* w2, double* g_u,
                        double* g_p) {
    if (!h || !solid_q || !disp || !u_hash || !u1 || !v1 || !g_u || !g_p) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    Bdf b;
    TRY(gcsi_check(ctx, prm, &b));
    if (mode != FSI_GCSI_PREDICTOR && mode != FSI_GCSI_CORRECTOR) return fail(ctx, FSI_ERR_ARG, "mode must be P or C");
    const bool k2 = prm->k == 2, pred = mode == FSI_GCSI_PREDICTOR;
    if (k2 && (!u2 || !v2)) return fail(ctx, FSI_ERR_ARG, "k = 2 needs the fields at n-2");
    if (pred && (!w1 || (k2 && !w2))) return fail(ctx, FSI_ERR_ARG, "the predictor needs the mesh velocities");
    const Level& F = ctx->lv[ctx->nlev - 1];
    GcsiRhsArgs a{};
    a.nx = F.cells[0];
    a.ny = F.cells[1];
    a.nz = F.cells[2];
    a.vnx = F.vnodes[0];
    a.vny = F.vnodes[1];
    a.pnx = F.pnodes[0];
    a.pny = F.pnodes[1];
    a.nvn = F.nvn;
    a.nvert = F.nvert;
    for (int d = 0; d < 3; ++d) a.h[d] = F.h[d];
    a.disp = disp;
    a.solid = solid_q;
    a.wall = F.d_wall;
    a.uh = u_hash;
    a.u1 = u1;
    a.u2 = k2 ? u2 : nullptr;
    a.v1 = v1;
    a.v2 = k2 ? v2 : nullptr;
    a.w1 = pred ? w1 : nullptr;
    a.w2 = (pred && k2) ? w2 : nullptr;
    a.a1 = b.a1;
    a.a2 = b.a2;
    a.gt = b.gamma * prm->tau;
    a.rho_f = prm->rho_f;
    a.rho_s = prm->rho_s;
    a.mu_s = prm->mu_s;
    a.inv_etaV = (prm->eta_V > 0 && std::isfinite(prm->eta_V)) ? 1.0 / prm->eta_V : 0.0;
    for (int d = 0; d < 3; ++d) a.body[d] = prm->body[d];
    a.predictor = pred ? 1 : 0;
    a.g_u = g_u;
    a.g_p = g_p;
    launch_fill<double>(g_u, 0.0, F.nv, ctx->stream);
    launch_fill<double>(g_p, 0.0, F.np, ctx->stream);
    launch_gcsi_rhs(a, F.dim, F.nc, ctx->stream);
    return FSI_OK;
}

fsi_status fsi_gcsi_set_convection(fsi_ctx* h, const fsi_gcsi_params* prm, const double* v_hash,
                                   const double* w_hash) {
    if (!h || !v_hash || !w_hash) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    Bdf b;
    TRY(gcsi_check(ctx, prm, &b));
    const int J = ctx->nlev - 1;
    for (int j = 0; j <= J; ++j)
        if (!ctx->lv[j].d_gcsi_eta || !ctx->lv[j].coef_set)
            return fail(ctx, FSI_ERR_STATE, "fsi_gcsi_set_convection before fsi_gcsi_set_coefficients");
    TRY(gcsi_scratch(ctx));
    const Level& F = ctx->lv[J];
    for (int j = 0; j <= J; ++j) {
        const Level& L = ctx->lv[j];
        double* vconv = ctx->gcsi_tmp;
        double* r = vconv + (int64_t)L.dim * L.nc * L.Q;
        launch_gcsi_convection(L, F, v_hash, w_hash, L.d_gcsi_eta, 1 << (J - j), vconv, r, ctx->stream);
        TRY(fsi_set_convection(h, j, vconv, r, prm->rho_f));
    }
    return FSI_OK;
}

fsi_status fsi_lift_dirichlet(fsi_ctx* h, const double* d, double* g_u, double* g_p) {
    if (!h || !d || !g_u || !g_p) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    const int J = ctx->nlev - 1;
    TRY(apply_check(ctx, J, true));
    Level& L = ctx->lv[J];
    const bool conv = ctx->prm.corrector != 0;
    if (conv && !L.conv_set) return fail(ctx, FSI_ERR_STATE, "corrector lifting before fsi_set_convection");
    hipStream_t s = ctx->stream;
    if (!ctx->lift_buf) TRY(dalloc(ctx, &ctx->lift_buf, 2 * L.nv + 2 * L.np));
    double* gw = ctx->lift_buf;
    double* qu = gw + L.nv;
    double* zp = qu + L.nv;
    double* qp = zp + L.np;
    launch_fill<double>(gw, 0.0, L.nv, s);
    launch_dirichlet_copy<double>(L, d, gw, s);
    launch_fill<int>(ctx->d_flag, 0, 1, s);
    launch_nonfinite(gw, L.nv, ctx->d_flag, s);
    TRY(sync_flag(ctx, FSI_ERR_NONFINITE, "Dirichlet data not finite"));
    launch_fill<double>(zp, 0.0, L.np, s);
    // [q_u; q_p] = [A (+ N + S); B] gw with the constrained columns kept
    TRY(apply_unconstrained(ctx, conv ? (OP_A | OP_BT | OP_B | OP_CONV) : (OP_A | OP_BT | OP_B), gw, zp, qu, qp, s));
    launch_axpy_host(-1.0, qu, g_u, L.nv, s);
    launch_dirichlet_copy<double>(L, d, g_u, s);
    launch_axpy_host(-1.0, qp, g_p, L.np, s);
    return FSI_OK;
}

fsi_status fsi_autotune(fsi_ctx* h) {
    if (!h) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    for (int j = 0; j < ctx->nlev; ++j)
        if (!ctx->lv[j].geo_set || !ctx->lv[j].coef_set)
            return fail(ctx, FSI_ERR_STATE, "autotune needs geometry and coefficients on every level");
    TRY(alloc_work<double>(ctx));
    TRY(alloc_work<float>(ctx));
    hipStream_t s = ctx->stream;
    hipEvent_t e0, e1;
    FSI_HIP_TRY(hipEventCreate(&e0));
    FSI_HIP_TRY(hipEventCreate(&e1));
    for (int pi = 0; pi < 2; ++pi)
        for (int j = 0; j < ctx->nlev; ++j)
            for (int cls = 0; cls < kTuneClasses; ++cls) {
                const int mode = kTuneModes[cls];
                double best = 1e300;
                int bestv = 0;
                for (int var = 0; var < kNumVariants; ++var) {
                    const int reps = 3;
                    for (int r = 0; r <= reps; ++r) {
                        if (r == 1) FSI_HIP_TRY(hipEventRecord(e0, s));
                        for (int ph = 0; ph < ctx->lv[j].nphases(); ++ph)
                            launch_phase_on_work(ctx, pi, j, mode, var, ph, s);
                    }
                    FSI_HIP_TRY(hipEventRecord(e1, s));
                    FSI_HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0;
                    FSI_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    const double us = 1000.0 * ms / reps;
                    if (getenv("FSI_TUNE_VERBOSE"))
                        fprintf(stderr, "[fsi autotune] precision %d level %d mode %d variant %d: %.1f us\n", pi, j,
                                mode, var, us);
                    if (us < best) {
                        best = us;
                        bestv = var;
                    }
                }
                ctx->tune_variant[pi][(size_t)j * kTuneClasses + cls] = bestv;
                ctx->tune_us[pi][(size_t)j * kTuneClasses + cls] = best;
            }
    // per unfused class (A, Stokes, B, B^T): phased launches (tuned variant) against
    // the single atomic launch in either shape
    const int unfused[4] = {OP_A, OP_A | OP_BT | OP_B, OP_B, OP_BT};
    for (int pi = 0; pi < 2; ++pi)
        for (int j = 0; j < ctx->nlev; ++j)
            for (int m : unfused) {
                const size_t k = (size_t)j * kTuneClasses + tune_class(m);
                ctx->atom[pi][k] = -1;
                if (!atomic_ok(ctx->lv[j], m)) continue;
                double best = ctx->tune_us[pi][k];
                for (int shape = 0; shape < atom_shapes(ctx->lv[j].dim); ++shape) {
                    // large levels: more repetitions (the atomic shapes there differ by about 1%)
                    const int reps = ctx->lv[j].nc >= (int64_t(1) << 18) ? 10 : 3;
                    for (int r = 0; r <= reps; ++r) {
                        if (r == 1) FSI_HIP_TRY(hipEventRecord(e0, s));
                        launch_atomic_on_work(ctx, pi, j, m, shape, s);
                    }
                    FSI_HIP_TRY(hipEventRecord(e1, s));
                    FSI_HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0;
                    FSI_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    const double us = 1000.0 * ms / reps;
                    if (getenv("FSI_TUNE_VERBOSE"))
                        fprintf(stderr, "[fsi autotune] precision %d level %d mode %d: %.1f us phased / %.1f us atomic "
                                "(shape %d)\n", pi, j, m, ctx->tune_us[pi][k], us, shape);
                    if (us < best) {
                        best = us;
                        ctx->atom[pi][k] = (int8_t)shape;
                    }
                }
                ctx->tune_us[pi][k] = best;   // the time of the chosen form
            }
    // the corrector terms (A + N + S, alone and in the Stokes apply) on levels where they are
    // set: phased launches of the tuned variant against the single atomic launch
    for (int pi = 0; pi < 2; ++pi)
        for (int j = 0; j < ctx->nlev; ++j) {
            ctx->atom_conv[pi][(size_t)j] = -1;
            const Level& L = ctx->lv[j];
            if (!L.conv_set || !atomic_ok(L, OP_A | OP_CONV)) continue;
            const int m = OP_A | OP_CONV;
            double best = 1e300;
            for (int shape = -1; shape < atom_shapes(L.dim); ++shape) {
                const int reps = L.nc >= (int64_t(1) << 18) ? 10 : 3;
                for (int r = 0; r <= reps; ++r) {
                    if (r == 1) FSI_HIP_TRY(hipEventRecord(e0, s));
                    if (shape < 0) {
                        for (int ph = 0; ph < L.nphases(); ++ph)
                            launch_phase_on_work(ctx, pi, j, m, variant_of(ctx, pi, j, m), ph, s);
                    } else {
                        launch_atomic_on_work(ctx, pi, j, m, shape, s);
                    }
                }
                FSI_HIP_TRY(hipEventRecord(e1, s));
                FSI_HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                FSI_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                const double us = 1000.0 * ms / reps;
                if (getenv("FSI_TUNE_VERBOSE"))
                    fprintf(stderr, "[fsi autotune] precision %d level %d corrector A: %.1f us (%s %d)\n", pi, j, us,
                            shape < 0 ? "phased" : "atomic shape", shape);
                if (us < best) {
                    best = us;
                    ctx->atom_conv[pi][(size_t)j] = (int8_t)shape;
                }
            }
        }
    // fused epilogues against operator + separate vector kernel, each with its tuned variant
    auto timed = [&](auto&& body, double* us) -> fsi_status {
        body();
        FSI_HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) body();
        FSI_HIP_TRY(hipEventRecord(e1, s));
        FSI_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        FSI_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        *us = 1000.0 * ms / 3;
        return FSI_OK;
    };
    for (int pi = 0; pi < 2; ++pi)
        for (int j = 0; j < ctx->nlev; ++j) {
            const Level& L = ctx->lv[j];
            auto var = [&](int mode) { return ctx->tune_variant[pi][(size_t)j * kTuneClasses + tune_class(mode)]; };
            auto all = [&](int mode) {
                const bool epilogue = (mode & (OP_CHEB | OP_RES)) != 0;
                if (!epilogue && ctx->atom_of(pi, j, mode) >= 0) {
                    launch_atomic_on_work(ctx, pi, j, mode, ctx->atom_of(pi, j, mode), s);
                    return;
                }
                for (int ph = 0; ph < L.nphases(); ++ph) launch_phase_on_work(ctx, pi, j, mode, var(mode), ph, s);
            };
            double sep_c = 0, fus_c = 0, sep_r = 0, fus_r = 0;
            if (pi == 0) {
                LevelWork<double>& W = ctx->w64[j];
                TRY(timed([&] { all(OP_A); launch_cheb_step<double>(L.d_dAinv64, W.f_u, W.cax_u, W.w_u, W.cd_u, 0.0, 0.0, false, true, L.nv, s); }, &sep_c));
                TRY(timed([&] { all(OP_A | OP_CHEB); launch_dirichlet_cheb<double>(L, W.w_u, W.cd_u, W.f_u, L.d_dAinv64, 0.0, 0.0, false, true, s); }, &fus_c));
                TRY(timed([&] { all(OP_A | OP_BT | OP_B); launch_dirichlet_copy<double>(L, W.x_u, W.r_u, s);
                                launch_sub<double>(W.f_u, W.r_u, W.r_u, L.nv, s); launch_sub<double>(W.f_p, W.r_p, W.r_p, L.np, s); }, &sep_r));
                TRY(timed([&] { all(OP_A | OP_BT | OP_B | OP_RES); launch_dirichlet_res<double>(L, W.f_u, W.x_u, W.r_u, s); }, &fus_r));
            } else {
                LevelWork<float>& W = ctx->w32[j];
                TRY(timed([&] { all(OP_A); launch_cheb_step<float>(L.d_dAinv32, W.f_u, W.cax_u, W.w_u, W.cd_u, 0.0, 0.0, false, true, L.nv, s); }, &sep_c));
                TRY(timed([&] { all(OP_A | OP_CHEB); launch_dirichlet_cheb<float>(L, W.w_u, W.cd_u, W.f_u, L.d_dAinv32, 0.0, 0.0, false, true, s); }, &fus_c));
                TRY(timed([&] { all(OP_A | OP_BT | OP_B); launch_dirichlet_copy<float>(L, W.x_u, W.r_u, s);
                                launch_sub<float>(W.f_u, W.r_u, W.r_u, L.nv, s); launch_sub<double>(W.f_p, W.r_p, W.r_p, L.np, s); }, &sep_r));
                TRY(timed([&] { all(OP_A | OP_BT | OP_B | OP_RES); launch_dirichlet_res<float>(L, W.f_u, W.x_u, W.r_u, s); }, &fus_r));
            }
            ctx->fuse_cheb[pi][j] = fus_c < sep_c ? 1 : 0;
            ctx->fuse_res[pi][j] = fus_r < sep_r ? 1 : 0;
            if (getenv("FSI_TUNE_VERBOSE"))
                fprintf(stderr, "[fsi autotune] precision %d level %d chebyshev step %.1f us separate / %.1f us fused; "
                        "residual %.1f us separate / %.1f us fused\n", pi, j, sep_c, fus_c, sep_r, fus_r);
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    // captured graphs hold the old launch shapes
    if (ctx->setup_done) TRY(capture_graphs(ctx));
    return FSI_OK;
}

fsi_status fsi_time_operator(fsi_ctx* h, int level, int precision, int mode, int reps, double* kernel_us,
                             double* op_us, int* n_launches) {
    const bool fused_mode = mode == (OP_A | OP_CHEB) || mode == (OP_A | OP_BT | OP_B | OP_RES);
    const bool conv_mode = mode == (OP_A | OP_CONV) || mode == (OP_A | OP_BT | OP_B | OP_CONV);
    if (!h || !kernel_us || !op_us || !n_launches || reps < 1 || (precision != 0 && precision != 1) ||
        ((mode < 1 || mode > 7) && !fused_mode && !conv_mode))
        return FSI_ERR_ARG;
    Context* ctx = &h->c;
    TRY(apply_check(ctx, level, (mode & OP_A) != 0));
    if (conv_mode) TRY(conv_check(ctx, level));
    TRY(alloc_work<double>(ctx));
    TRY(alloc_work<float>(ctx));
    const Level& L = ctx->lv[level];
    hipStream_t s = ctx->stream;
    // tuned levels where the autotuner chose the single atomic launch time that launch
    // (with the zeroing of its outputs) as one unit
    const int am = (ctx->prm.tuned && ctx->prm.atomics && !fused_mode && !conv_mode) ? ctx->atom_of(precision, level, mode) : -1;
    const bool atomic = am >= 0 && atomic_ok(L, mode);
    const int nph = atomic ? 1 : L.nphases();
    std::vector<hipEvent_t> ev((size_t)2 * nph + 2);
    for (auto& e : ev) FSI_HIP_TRY(hipEventCreate(&e));
    const int var = variant_of(ctx, precision, level, mode);
    auto nonempty = [&](int ph) { return atomic || L.phase_off[ph + 1] > L.phase_off[ph]; };
    constexpr int kWarmup = 3;
    std::vector<double> kt, ot;
    int launched = 0;
    for (int r = 0; r < kWarmup + reps; ++r) {
        FSI_HIP_TRY(hipEventRecord(ev[0], s));
        launched = 0;
        for (int ph = 0; ph < nph; ++ph) {
            FSI_HIP_TRY(hipEventRecord(ev[1 + 2 * ph], s));
            if (nonempty(ph)) ++launched;
            if (atomic) launch_atomic_on_work(ctx, precision, level, mode, am, s);
            else launch_phase_on_work(ctx, precision, level, mode, var, ph, s);
            FSI_HIP_TRY(hipEventRecord(ev[2 + 2 * ph], s));
        }
        if (atomic) {
            // the atomic launch's initialisation has set the wall rows
        } else if (precision == 0) {
            LevelWork<double>& W = ctx->w64[level];
            if (mode & OP_A) launch_dirichlet_copy<double>(L, W.x_u, W.r_u, s);
            else if (mode & OP_BT) launch_dirichlet_zero<double>(L, W.r_u, s);
        } else {
            LevelWork<float>& W = ctx->w32[level];
            if (mode & OP_A) launch_dirichlet_copy<float>(L, W.x_u, W.r_u, s);
            else if (mode & OP_BT) launch_dirichlet_zero<float>(L, W.r_u, s);
        }
        FSI_HIP_TRY(hipEventRecord(ev[2 * nph + 1], s));
        FSI_HIP_TRY(hipEventSynchronize(ev[2 * nph + 1]));
        if (r < kWarmup) continue;
        float ms;
        double ksum = 0.0;
        for (int ph = 0; ph < nph; ++ph) {
            if (!nonempty(ph)) continue;
            FSI_HIP_TRY(hipEventElapsedTime(&ms, ev[1 + 2 * ph], ev[2 + 2 * ph]));
            ksum += ms;
        }
        kt.push_back(ksum);
        FSI_HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[2 * nph + 1]));
        ot.push_back(ms);
    }
    for (auto& e : ev) hipEventDestroy(e);
    auto median = [](std::vector<double> v) {
        std::sort(v.begin(), v.end());
        const size_t m = v.size() / 2;
        return v.size() % 2 ? v[m] : 0.5 * (v[m - 1] + v[m]);
    };
    *kernel_us = 1000.0 * median(kt);
    *op_us = 1000.0 * median(ot);
    *n_launches = launched;
    return FSI_OK;
}

fsi_status fsi_set_tuning(fsi_ctx* h, int level, int precision, int variant) {
    if (!h) return FSI_ERR_ARG;
    Context* ctx = &h->c;
    if (level < 0 || level >= ctx->nlev || (precision != 0 && precision != 1) || variant < 0 ||
        variant >= kNumVariants + kAtomShapes)
        return fail(ctx, FSI_ERR_ARG, "fsi_set_tuning: level, precision or variant out of range");
    const bool atomic = variant >= kNumVariants;
    if (atomic && variant >= kNumVariants + atom_shapes(ctx->lv[level].dim))
        return fail(ctx, FSI_ERR_ARG, "fsi_set_tuning: 2D levels have two atomic shapes (variants 16, 17)");
    for (int c = 0; c < kTuneClasses; ++c)
        ctx->tune_variant[precision][(size_t)level * kTuneClasses + c] = atomic ? 0 : variant;
    for (int c = 0; c < kTuneClasses; ++c)
        ctx->atom[precision][(size_t)level * kTuneClasses + c] = atomic ? (int8_t)(variant - kNumVariants) : (int8_t)-1;
    ctx->atom_conv[precision][(size_t)level] = atomic ? (int8_t)(variant - kNumVariants) : (int8_t)-1;
    if (ctx->setup_done) TRY(capture_graphs(ctx));   // captured graphs hold the old launch shapes
    return FSI_OK;
}

fsi_status fsi_get_tuning(const fsi_ctx* h, int level, int precision, int* variant, double* best_us) {
    if (!h || !variant || !best_us) return FSI_ERR_ARG;
    const Context* ctx = &h->c;
    if (level < 0 || level >= ctx->nlev || (precision != 0 && precision != 1)) return FSI_ERR_ARG;
    const int am = ctx->atom[precision][(size_t)level * kTuneClasses];   // class A
    *variant = am >= 0 ? kNumVariants + am : ctx->tune_variant[precision][(size_t)level * kTuneClasses];   // class A
    *best_us = ctx->tune_us[precision][(size_t)level * kTuneClasses];
    return FSI_OK;
}

}  // extern "C"
