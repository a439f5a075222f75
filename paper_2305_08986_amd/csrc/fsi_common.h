// Shared definitions of the HIP library: 1D reference data, launch helpers,
// the level/context structures and the kernel-launcher prototypes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fsi.h"

namespace fsi {

// ---------------------------------------------------------------- 1D reference data
// Q2 Lagrange basis on the nodes {0, 1/2, 1} and Q1 basis on {0, 1}, evaluated at
// the 3-point Gauss-Legendre points {1/2 - s, 1/2, 1/2 + s}, s = sqrt(15)/10, on [0,1].
// With g0 = 1/2 - s:  N0(g0) = 3/10 + s, N1(g0) = 2/5, N2(g0) = 3/10 - s,
// N0'(g0) = -1 - 4s, N1'(g0) = 8s, N2'(g0) = 1 - 4s; the tables at g2 follow by symmetry.
constexpr double kS15 = 0.38729833462074168852;           // sqrt(15)/10
constexpr double kG0 = 0.5 - kS15, kG2 = 0.5 + kS15;
constexpr double kW0 = 5.0 / 18.0, kW1 = 8.0 / 18.0;

struct Tab {
    // S[q][n] = N_n(g_q), D[q][n] = N_n'(g_q), L[q][a] = Q1 basis a at g_q
    static constexpr double S[3][3] = {{0.3 + kS15, 0.4, 0.3 - kS15}, {0.0, 1.0, 0.0}, {0.3 - kS15, 0.4, 0.3 + kS15}};
    static constexpr double D[3][3] = {{-1.0 - 4.0 * kS15, 8.0 * kS15, 1.0 - 4.0 * kS15},
                                       {-1.0, 0.0, 1.0},
                                       {-1.0 + 4.0 * kS15, -8.0 * kS15, 1.0 + 4.0 * kS15}};
    static constexpr double L[3][2] = {{0.5 + kS15, 0.5 - kS15}, {0.5, 0.5}, {0.5 - kS15, 0.5 + kS15}};
    static constexpr double W[3] = {kW0, kW1, kW0};
};

// cell-kernel thread shapes: NT threads per cell (one per line of 3 points),
// CPW cells per 64-wide wavefront
template <int DIM> struct Shape;
template <> struct Shape<2> { static constexpr int NT = 3, CPW = 21, NLOC = 9, NPL = 4, Q = 9, NK = 4; };
template <> struct Shape<3> { static constexpr int NT = 9, CPW = 7, NLOC = 27, NPL = 8, Q = 27, NK = 9; };

// Geometry/coefficient layout: the cell kernels read, per wavefront chunk of CPW
// cells and per quadrature abscissa qx, the CPW * NT values (NT points (qy[, qz])
// per cell) of every plane as one aligned block of 64 slots (63 used), so that
// consecutive chunks never share a cache line.  Chunks are numbered row by row in
// processing order; col is the cell's processing-order index.
struct GeoLayout {
    int64_t nchk = 0;              // chunks on the level
    int nx = 1, nchunks = 1, cpw = 1, nt = 1;   // cells per row, chunks per row, CPW, NT
};
constexpr int kGeoSlots = 64;
__host__ __device__ inline int64_t geo_off(const GeoLayout& g, int qx, int64_t col, int t) {
    const int64_t row = col / g.nx;
    const int ix = (int)(col - row * g.nx);
    const int ch = ix / g.cpw, slot = ix - ch * g.cpw;
    return ((int64_t)qx * g.nchk + row * g.nchunks + ch) * kGeoSlots + slot * g.nt + t;
}

// operator mode bits of the cell kernel; OP_CHEB (with OP_A) and OP_RES (with
// OP_A | OP_BT | OP_B) replace the plain store at a node's last touch by a
// Chebyshev update of the iterate or by the residual f - M u
// OP_CONV (with OP_A, 3D) adds the corrector-mode terms: convection rho (grad u) v° and
// the streamline term r (v° . grad u)(v° . grad w)
// OP_ATOM: one launch over every phase, adding into zeroed outputs with atomics
// (small levels, where the four phase launches are latency-bound)
enum : int { OP_A = 1, OP_BT = 2, OP_B = 4, OP_CHEB = 8, OP_RES = 16, OP_CONV = 32, OP_ATOM = 64, OP_FIXW = 128 };
// OP_FIXW (3D, with OP_ATOM | OP_A only): the level has interior constrained nodes (fixed cells), whose
// wall bits come from the per-node mask instead of the box faces; a template bit, so that the
// other atomic kernels carry no test for it

// ---------------------------------------------------------------- error helpers
#define FSI_HIP_TRY(expr)                                                          \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            return ::fsi::hip_fail(ctx, e_, #expr, __FILE__, __LINE__);            \
        }                                                                          \
    } while (0)

struct Context;
fsi_status hip_fail(Context* ctx, hipError_t e, const char* what, const char* file, int line);
fsi_status fail(Context* ctx, fsi_status st, const std::string& msg);

// ---------------------------------------------------------------- device buffers
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
};

// ---------------------------------------------------------------- level data
struct Level {
    int dim = 0;
    int cells[3] = {1, 1, 1};
    int vnodes[3] = {1, 1, 1};
    int pnodes[3] = {1, 1, 1};
    int64_t nc = 0, nvn = 0, nv = 0, np = 0, nvert = 0;
    uint32_t dfaces = 0;           // Dirichlet face bits of the mesh (fsi_mesh_desc)
    int Q = 0;
    int ncolors = 0;
    // processing phases: the parity colours of the row index (iy[, iz]); cells
    // are stored phase-major as whole rows along x, phase p owning cells
    // [phase_off[p], phase_off[p+1])
    std::vector<int64_t> phase_off;
    int nphases() const { return ncolors; }

    // colour-ordered cell structure
    int* d_col2lex = nullptr;      // [nc]
    int* d_lex2col = nullptr;      // [nc]
    int* d_vmap = nullptr;         // [nc][NLOC] Q2 node of local node
    // single atomic launch (3D): phase-major row of each dispatch slot, in natural
    // (iy, iz) order, so that rows sharing node lines run at the same time and their
    // repeated touches of a line meet in the caches
    int* d_atom_rows = nullptr;    // [nc / nx]
    int* d_pmap = nullptr;         // [nc][NPL]  Q1 node / vertex of local vertex
    // per cell: x = wall bits of the local Q2 nodes, y = first-touch bits of the
    // local Q2 nodes, z = first-touch bits of the local vertices (bits 0..7) and
    // last-touch bits of the local vertices (bits 16..23), w = last-touch bits of
    // the local Q2 nodes (first/last in phase order)
    uint4* d_info = nullptr;
    uint8_t* d_wall = nullptr;     // [nvn] 1: velocity node on a wall
    int* d_dir_nodes = nullptr;    // wall nodes
    int64_t n_dir = 0;
    std::vector<uint8_t> h_dir_node;   // [nvn] host copy of the wall mask
    // fsi_set_fixed_cells: nodes of fixed cells (finest level; also in the wall mask)
    uint8_t* d_fixed = nullptr;
    // fsi_gcsi_set_coefficients: the viscosity per point ([nc][Q]) for the streamline law
    double* d_gcsi_eta = nullptr;

    // geometry and coefficients, internal layout [plane][qx][chunk][slot] (GeoLayout)
    double* d_K64 = nullptr;       // 9 (or 4) planes: det(J) w_q J^{-1}, entry (b,a) in plane b*dim+a
    double* d_cw64 = nullptr;      // det(J) w_q
    double* d_cv64 = nullptr;      // 2 planes: 2 eta/(det J w), c_m det J w
    float* d_K32 = nullptr;
    float* d_cv32 = nullptr;
    // sqrt(cvisc) K: with it the viscous flux of A alone is sym(grad-hat u K') K'^T,
    // so A reads 9 + 1 values per point instead of 9 + 2
    double* d_Ks64 = nullptr;
    float* d_Ks32 = nullptr;
    // FP32 geometry from vertices: level vertex displacement (x, y, z, 0) and per
    // point (2 eta, c_m) in the geometry layout; valid after fsi_set_displacement
    float4* d_vd32 = nullptr;
    float* d_cq32 = nullptr;
    // the same for the FP64 kernels: vertex displacement (x, y, z, 0) and (2 eta, c_m)
    double4* d_vd64 = nullptr;
    double* d_cq64 = nullptr;
    // corrector-mode terms per point in the geometry layout: beta = K v° (3 planes,
    // K = det(J) w J^{-1}) and sigma = r / (det J w) (1 plane); rho is the density
    double* d_cb64 = nullptr;
    double* d_cs64 = nullptr;
    float* d_cb32 = nullptr;
    float* d_cs32 = nullptr;
    bool conv_set = false;
    bool fixed_nodes = false;   // interior constrained nodes (fsi_set_fixed_cells) in d_wall
    double rho = 0.0;
    bool vgeo_avail = false;          // geometry came from vertex displacements (3D)
    bool vgeo = false;                // ... and the FP32 kernels use it
    bool vgeo64 = false;              // ... and the FP64 kernels use it
    double h[3] = {1.0, 1.0, 1.0};    // reference cell sizes
    bool geo_set = false, coef_set = false;

    // preconditioner data
    double* d_dAinv64 = nullptr;   // 1/diag(A) (1 on wall dofs)
    float* d_dAinv32 = nullptr;
    double* d_dSinv = nullptr;     // 1/diag(B diag(A)^{-1} B^T)
    double lam = 0, lo = 0, hi = 0;
    double diagA_norm = 0, diagS_norm = 0;

    GeoLayout geo;
    int64_t plane() const { return 3 * geo.nchk * kGeoSlots; }
};

// per-level work vectors of the V-cycle in one precision (T velocity, double pressure)
template <typename T>
struct LevelWork {
    T *f_u = nullptr, *x_u = nullptr, *r_u = nullptr, *w_u = nullptr, *v_u = nullptr;
    T *cd_u = nullptr, *cax_u = nullptr, *tu = nullptr;
    double *f_p = nullptr, *x_p = nullptr, *r_p = nullptr, *t_p = nullptr, *z_p = nullptr;
    double *b_p = nullptr, *s_p = nullptr;   // BiCGStab Schur step (corrector mode)
    double *dots = nullptr;        // [4] device scalars: <y,z>, <y, D_S^{-1} y> (MINRES) or
                                   // <b,b>, <b,v>, <t,s>, <t,t> (BiCGStab)
    double *partials = nullptr;    // reduction scratch
};

struct Coarse {
    int64_t n = 0;                 // free velocity dofs + pressure dofs
    int64_t nfree_u = 0;
    int* d_uidx = nullptr;         // [nfree_u] velocity dof index of free dof i
    double* d_inv64 = nullptr;     // [n][n] row-major inverse of M_0 restricted to free dofs
    float* d_inv32 = nullptr;
    double* d_xin64 = nullptr;     // gathered rhs
    double* d_xout64 = nullptr;
    float* d_xin32 = nullptr;
    float* d_xout32 = nullptr;
    // set-up scratch, kept for the next set-up: velocity dof -> free row, pivot rows and
    // column permutation (2n), pivot column, and the n x n permutation target
    int* d_vrow = nullptr;
    int* d_piv = nullptr;
    double* d_col = nullptr;
    double* d_tmp = nullptr;
};

struct Krylov {
    int restart = 0;
    int64_t n = 0;
    double* V = nullptr;           // [restart+1][n]
    double* Z = nullptr;           // [restart][n]
    double* w = nullptr;           // [n]
    double* r = nullptr;           // [n]
    double* x = nullptr;           // [n]
    double* g = nullptr;           // [n]
    double* h = nullptr;           // device [restart+2]
    double* partials = nullptr;
    double* h_host = nullptr;      // pinned host mirror
};

// cell-operator launch variants (wavefronts per workgroup, load kind, register cap)
constexpr int kNumVariants = 16;
// launch variants are tuned per operator class: A, A with the Chebyshev epilogue,
// Stokes, Stokes with the residual epilogue, B, B^T
constexpr int kTuneClasses = 6;
constexpr int kTuneModes[kTuneClasses] = {OP_A, OP_A | OP_CHEB, OP_A | OP_BT | OP_B, OP_A | OP_BT | OP_B | OP_RES,
                                          OP_B, OP_BT};
inline int tune_class(int mode) {
    for (int c = 0; c < kTuneClasses; ++c)
        if (kTuneModes[c] == mode) return c;
    return 2;   // A + B^T is timed as the Stokes class
}

struct Context {
    fsi_mesh_desc mesh{};
    int nlev = 0;
    std::vector<Level> lv;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    fsi_mg_params prm{};
    bool setup_done = false;

    std::vector<LevelWork<double>> w64;
    std::vector<LevelWork<float>> w32;
    Coarse coarse;
    Krylov kr;
    // extension solve: velocity-only coarse inverse (shares the free-dof list of
    // `coarse`), finest-level cell info without wall bits (the unconstrained operator
    // for the boundary lifting) and the CG vectors; built at the first extension solve
    // after a set-up
    Coarse coarse_u;
    bool ext_ready = false;
    uint4* d_info_free = nullptr;
    double* ext_buf = nullptr;     // 8 finest-level velocity vectors
    // the extension preconditioner (r -> z on fixed CG buffers) as a graph per precision
    hipGraphExec_t ext_graph[2] = {nullptr, nullptr};
    bool ext_graph_valid[2] = {false, false};
    int ext_graph_key[2] = {-1, -1};
    double* d_scratch = nullptr;   // general scratch (partials, flags)
    int* d_flag = nullptr;
    int* h_flag = nullptr;         // pinned
    double* h_dbl = nullptr;       // pinned [64]
    // top-level V-cycle IO buffers (FP64) for the graph path
    double *vc_in_u = nullptr, *vc_in_p = nullptr, *vc_out_u = nullptr, *vc_out_p = nullptr;
    double* vc_tmp = nullptr;      // [nv + np] residual of repeated V-cycles
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graph_valid[2] = {false, false};
    int graph_key = -1;            // (fused, tuned, vertex_geometry) the graphs were captured with
    // tuning: per level and precision, index into the launch-variant table
    std::vector<int> tune_variant[2];
    std::vector<double> tune_us[2];
    // per level and precision: use the fused Chebyshev / residual epilogue (when the
    // fused path is enabled); the autotuner keeps whichever it measured faster
    std::vector<uint8_t> fuse_cheb[2], fuse_res[2];
    // per level, operator class (as tune_variant) and precision: -1 phased launches;
    // 0 or 1 the single atomic launch (one or four wavefronts per row) of an unfused
    // class, where the autotuner measured it faster (results then vary in the last
    // bits from run to run)
    std::vector<int8_t> atom[2];
    // per level and precision: the same choice for the corrector classes (A + N + S, alone
    // and in the Stokes apply), measured by fsi_autotune where the terms are set
    std::vector<int8_t> atom_conv[2];
    int atom_of(int prec, int level, int mode) const {
        return atom[prec][(size_t)level * kTuneClasses + tune_class(mode)];
    }
    std::vector<void*> allocations;
    // device address of the file-scope pressure staging array of the allocation-free
    // FP32 Stokes apply on this context's device (resolved at create; null if that failed)
    double* noalloc_scratch = nullptr;
    // fsi_set_fixed_cells was called: interior Dirichlet nodes, so no single atomic launch
    // (it derives the wall rows from the faces)
    bool has_fixed = false;
    // the block coarse matrix could be inverted (false only with fixed cells)
    bool coarse_block_ok = true;
    // time-step scratch: [n_cells][27] x 4 doubles of the finest level
    double* gcsi_tmp = nullptr;
    double* lift_buf = nullptr;    // fsi_lift_dirichlet: 2 velocity + 2 pressure vectors
    double gcsi_rho_f = -1.0;   // fluid density of the last fsi_gcsi_set_coefficients
};

// ---------------------------------------------------------------- launchers (kernels_*.hip)
// cell operator on one colour range; mode = OP_* bits; variant selects the
// workgroup size (wavefronts per workgroup) and block->tile mapping.
template <typename T>
void launch_cell(const Level& L, int mode, int variant, int phase, const T* K, const T* cv,
                 const T* u, const double* p, T* v, double* q, hipStream_t s);
template <typename T>
void launch_cell_all(const Level& L, int mode, int variant, const T* K, const T* cv,
                     const T* u, const double* p, T* v, double* q, hipStream_t s);
// the same apply in one launch over all phases with atomic adds, wall rows included
// (modes A, B, B^T and A + B^T + B, and the corrector classes; 3D shapes 0 ..
// kAtomShapes - 1: one or four wavefronts per row, rows grouped along z by one, two or
// four, or one wavefront per half or quarter row; 2D shapes 0 .. kAtomShapes2D - 1: one or
// two wavefronts per workgroup)
constexpr int kAtomShapes = 7;
constexpr int kAtomShapes2D = 2;
inline int atom_shapes(int dim) { return dim == 3 ? kAtomShapes : kAtomShapes2D; }
template <typename T>
void launch_cell_atomic(const Level& L, int mode, int shape, const T* K, const T* cv,
                        const T* u, const double* p, T* v, double* q, hipStream_t s);
template <typename T>
void launch_cell_cheb(const Level& L, int variant, int phase, const T* K, const T* cv, T* x, T* d, const T* r,
                      const T* dinv, T* v, double c1, double c2, bool first, bool store_d, hipStream_t s);
template <typename T>
void launch_cell_res(const Level& L, int variant, int phase, const T* K, const T* cv, const T* u, const double* p,
                     const T* f_u, const double* f_p, T* r_u, double* r_p, hipStream_t s);
// one Chebyshev step fused into A x: at each node's last touch
// d = c1 d + c2 dinv (r - A x), x += d (first: d taken as x; d is stored only if
// store_d); v holds the
// partial sums of nodes touched by several phases.  Wall nodes are left alone.
template <typename T>
void launch_cell_cheb_all(const Level& L, int variant, const T* K, const T* cv, T* x, T* d, const T* r,
                          const T* dinv, T* v, double c1, double c2, bool first, bool store_d, hipStream_t s);
// residual fused into the Stokes apply: r_u = f_u - (A u + B^T p), r_p = f_p - B u,
// written at each node's last touch.  Wall nodes are left alone.
template <typename T>
void launch_cell_res_all(const Level& L, int variant, const T* K, const T* cv, const T* u, const double* p,
                         const T* f_u, const double* f_p, T* r_u, double* r_p, hipStream_t s);

void launch_geometry(const Level& L, const double* J, double* K, double* cw, float* K32, int* flag,
                     hipStream_t s);
void launch_geometry_from_disp(const Level& L, const double* disp_fine, int stride, const int* fine_pnodes,
                                 const double* h, double* K, double* cw, float* K32, int* flag, hipStream_t s);
void launch_coefficients(const Level& L, const double* cm, const double* eta, const double* cw,
                         double* cv64, float* cv32, float* cq32, double* cq64, const double* K64, double* Ks64,
                         float* Ks32, int* flag, hipStream_t s);
// level vertex displacement (FP32 float4 and FP64 double4) from the fine-level
// displacement by injection
void launch_vertex_disp(const Level& L, const double* disp_fine, int stride, const int* fine_pnodes,
                        float4* out32, double4* out64, hipStream_t s);
// conv: add the corrector-mode terms of the level (fsi_set_convection)
void launch_diagA(const Level& L, const double* K, const double* cv, double* diag, hipStream_t s, bool conv = false);
void launch_diagA_finish(const Level& L, double* diag, double* dinv64, float* dinv32, hipStream_t s);
void launch_diagS_impl(const Level& L, const uint8_t* d_wall, const double* K, const double* dAinv,
                       double* dSinv, hipStream_t s);
inline const uint8_t* level_wall_mask(const Level& L) { return L.d_wall; }

template <typename T>
void launch_fill(T* x, T val, int64_t n, hipStream_t s);
// outputs of the single atomic launch: v = 0 (all rows) and q = 0; v or q may be null
template <typename T>
void launch_atomic_init(const Level& L, T* v, double* q, hipStream_t s);
template <typename T>
void launch_dirichlet_copy(const Level& L, const T* u, T* v, hipStream_t s);   // v[wall] = u[wall]
template <typename T>
void launch_dirichlet_zero(const Level& L, T* v, hipStream_t s);
// wall rows of the fused epilogues (identity rows of A): the Chebyshev step with
// A x = x, and r = f - u
template <typename T>
void launch_dirichlet_cheb(const Level& L, T* x, T* d, const T* r, const T* dinv, double c1, double c2, bool first,
                           bool store_d, hipStream_t s);
template <typename T>
void launch_dirichlet_res(const Level& L, const T* f, const T* u, T* r, hipStream_t s);
template <typename TD, typename TS>
void launch_cast(TD* d, const TS* src, int64_t n, hipStream_t s);

// Chebyshev pieces: x = dinv*r*c0 (the first direction equals x and is not stored);
// d' = c1 d + c2 dinv (r - ax), x += d' (first: d taken as x; store_d: keep d')
template <typename T>
void launch_cheb_init(const T* dinv, const T* r, T* x, double c0, int64_t n, hipStream_t s);
template <typename T>
void launch_cheb_step(const T* dinv, const T* r, const T* ax, T* x, T* d, double c1, double c2, bool first,
                      bool store_d, int64_t n, hipStream_t s);
// r = f - a (velocity, type T) ; and pressure (double)
template <typename T>
void launch_sub(const T* f, const T* a, T* r, int64_t n, hipStream_t s);
// z = dsinv * (t - r)
void launch_schur_z(const double* dsinv, const double* t, const double* r, double* z, int64_t n,
                    hipStream_t s);
// dots[0] = <y,z>, dots[1] = <y, dsinv y>
void launch_schur_dots(const double* y, const double* z, const double* dsinv, double* partials,
                       double* dots, int64_t n, hipStream_t s);
// x_u += w - beta v ; x_p += beta z (beta = dots[0]/dots[1]); first: x = instead of +=
template <typename T>
void launch_smoother_update(const T* w, const T* vv, const double* z, const double* dots, T* x_u,
                            double* x_p, int64_t nu, int64_t np, bool first, hipStream_t s);

// s1, s2: FP64 fine-level scratch vectors (velocity length) for the intermediate passes
// BiCGStab(1) Schur step: b = t - r, p = D_S^{-1} b; s = b - alpha v (in place of b),
// q = D_S^{-1} s; x_u (+)= w - alpha t1 - omega t2, x_p (+)= alpha p + omega q with
// alpha = dots[0]/dots[1], omega = dots[2]/dots[3] (0 if dots[3] = 0)
void launch_bicg_start(const double* dsinv, const double* t, const double* r, double* b, double* p, int64_t n,
                       hipStream_t s);
void launch_bicg_mid(const double* dsinv, const double* dots, const double* v, double* b, double* q, int64_t n,
                     hipStream_t s);
template <typename T>
void launch_bicg_update(const T* w, const T* t1, const T* t2, const double* p, const double* q, const double* dots,
                        T* x_u, double* x_p, int64_t nu, int64_t np, bool first, hipStream_t s);
// rb_u, rb_p (may be null): restrict rf - rb instead of rf (the residual f - M x from f
// and M x, no separate subtraction)
template <typename T>
void launch_restrict(const Level& fine, const Level& coarse, const T* rf_u, const double* rf_p,
                     T* rc_u, double* rc_p, double* s1, double* s2, hipStream_t s, const T* rb_u = nullptr,
                     const double* rb_p = nullptr);
template <typename T>
void launch_prolongate_add(const Level& fine, const Level& coarse, const T* ec_u, const double* ec_p,
                           T* xf_u, double* xf_p, double* s1, double* s2, hipStream_t s);

// coarse level
void launch_coarse_assemble_impl(const Level& L, const double* K, const double* cv, const int* vrow,
                                 int64_t nfree_u, double* M, int64_t n, hipStream_t s, bool conv = false);
void launch_gj(double* M, int64_t n, int* piv, int* sigma, double* colk, double* tmp, int* flag, hipStream_t s);
template <typename T>
void launch_coarse_apply(const Coarse& C, const Level& L, const T* f_u, const double* f_p, T* x_u,
                         double* x_p, hipStream_t s);

// reductions and BLAS-1 (FP64 accumulation)
template <typename T>
void launch_dot(const T* x, const T* y, int64_t n, double* partials, double* out, hipStream_t s);
// out[j] = <V_j, w> for j < m (and out[m] = ||w||^2 with with_norm), V_j = V + j ldv
void launch_multi_dot(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* partials,
                      double* out, hipStream_t s, bool with_norm = false);
// w += sign sum_j coef_j V_j; *out_norm2 = ||w||^2 afterwards (partials: >= kReduceBlocks)
void launch_multi_axpy_norm(const double* V, int64_t ldv, int m, const double* coef_dev, double sign, double* w,
                            int64_t n, double* partials, double* out_norm2, hipStream_t s);
void launch_multi_axpy(const double* V, int64_t ldv, int m, const double* coef_dev, double sign,
                       double* w, int64_t n, hipStream_t s);
void launch_axpy_host(double a, const double* x, double* y, int64_t n, hipStream_t s);
void launch_xpby_host(const double* x, double b, double* y, int64_t n, hipStream_t s);   // y = x + b y
template <typename T>
void launch_add(T* x, const T* y, int64_t n, hipStream_t s);                              // x += y
void launch_clear_wall_bits(const uint4* in, uint4* out, int64_t n, hipStream_t s);
void launch_convection(const Level& L, const double* vconv, const double* r, double* cb64, double* cs64, float* cb32,
                       float* cs32, int* flag, hipStream_t s);
template <typename T>
void launch_coarse_apply_u(const Coarse& U, const Level& L, const T* f_u, T* x_u, hipStream_t s);
void launch_scale_host(double a, const double* x, double* y, int64_t n, hipStream_t s);
void launch_lanczos_start(const Level& L, double* v, hipStream_t s);
void launch_mul(const double* a, const double* b, double* c, int64_t n, hipStream_t s);
void launch_vsqrt(const double* a, double* c, int64_t n, hipStream_t s);
void launch_nonfinite(const double* x, int64_t n, int* flag, hipStream_t s);
void launch_sub_into(const double* g, const double* mx, double* r, int64_t n, hipStream_t s);
void launch_recip(const double* a, double* b, int64_t n, hipStream_t s);

constexpr int kReduceBlocks = 1024;

// ---------------------------------------------------------------- time step (kernels_gcsi.hip)
// u_out = gt w - a1 u1 - a2 u2 (velocity dofs; u2 may be null) and its values at the
// vertices, [dim][n_vert] (either output may be null)
void launch_gcsi_displacement(const Level& L, const double* w, const double* u1, const double* u2, double gt, double a1,
                              double a2, double* u_out, double* disp_out, hipStream_t s);
// c_m and eta per point from the solid indicator
void launch_gcsi_coefficients(const uint8_t* solid, double cm_f, double cm_s, double eta_f, double eta_s, double* cm,
                              double* eta, int64_t n, hipStream_t s);
// g = v on the fixed nodes, 0 elsewhere
void launch_fixed_values(const Level& L, const uint8_t* fixed, const double* v, double* g, hipStream_t s);
struct GcsiRhsArgs {
    int nx, ny, nz, vnx, vny, pnx, pny;
    int64_t nvn, nvert;
    double h[3];
    const double* disp;                   // [3][n_vert] vertex displacement of the explicit geometry
    const uint8_t* solid;                 // [n_cells][3^dim]
    const uint8_t* wall;                  // [n_vel_nodes] Dirichlet rows (left zero)
    const double *uh, *u1, *u2, *v1, *v2, *w1, *w2;
    double a1, a2, gt;                    // BDF alpha_1, alpha_2 and gamma tau
    double rho_f, rho_s, mu_s, inv_etaV;  // inv_etaV = 0: no volume correction
    double body[3];
    int predictor;
    double* g_u;                          // zeroed, accumulated with atomics
    double* g_p;
};
void launch_gcsi_rhs(const GcsiRhsArgs& a, int dim, int64_t nc, hipStream_t s);
// v° = v# - w# at the Gauss points of level L ([n_cells][27][3]) and the streamline
// parameter ([n_cells][27]); the fine-level fields are read at L's nodes (stride)
void launch_gcsi_convection(const Level& L, const Level& F, const double* vh, const double* wh, const double* eta,
                            int stride, double* vconv, double* r, hipStream_t s);

}  // namespace fsi
