// Auxiliary kernels of the hot path: geometry and coefficient setup (mapped
// spaces of Sec. 3.2, BDF mass coefficient of Sec. 3.1, viscosity splitting of
// Sec. 3.1.1), the diagonals diag(A) and diag(B diag(A)^{-1} B^T) used by the
// smoother of Sec. 4, the nested-space transfers of the level hierarchy
// (Sec. 4), the Chebyshev and MINRES vector updates, FP64 reductions and the
// dense coarsest-level solve.
#include "fsi_common.h"

namespace fsi {

constexpr int TPB = 256;
static inline unsigned nblocks(int64_t n, int tpb = TPB) {
    int64_t b = (n + tpb - 1) / tpb;
    if (b < 1) b = 1;
    return (unsigned)b;
}

__device__ __forceinline__ double dS(int q, int n) {
    return n == 1 ? (q == 1 ? 1.0 : 0.4) : (q == 1 ? 0.0 : ((q == 0) == (n == 0) ? 0.3 + kS15 : 0.3 - kS15));
}
__device__ __forceinline__ double dD(int q, int n) {
    if (q == 1) return n == 0 ? -1.0 : (n == 1 ? 0.0 : 1.0);
    const double sg = (q == 0) ? 1.0 : -1.0;   // D[2][n] = -D[0][2-n]
    const int m = (q == 0) ? n : 2 - n;
    const double v = m == 0 ? -1.0 - 4.0 * kS15 : (m == 1 ? 8.0 * kS15 : 1.0 - 4.0 * kS15);
    return sg * v;
}
__device__ __forceinline__ double dL(int q, int a) {
    if (q == 1) return 0.5;
    return ((q == 0) == (a == 0)) ? 0.5 + kS15 : 0.5 - kS15;
}
__device__ __forceinline__ double dLd(int a) { return a == 0 ? -1.0 : 1.0; }
__device__ __forceinline__ double dW(int q) { return q == 1 ? kW1 : kW0; }

// ---------------------------------------------------------------- geometry
struct GeoOut {
    int dim, NT, Q;
    int64_t nc, plane;
    GeoLayout geo;
    const int* lex2col;
    double* K;
    double* cw;
    float* K32;
    int* flag;
};

__device__ __forceinline__ void store_geometry(const GeoOut& g, int64_t cell, int q, const double* J) {
    const int dim = g.dim;
    const int qx = q % 3, t = q / 3;
    const int64_t col = g.lex2col[cell];
    const int64_t off = geo_off(g.geo, qx, col, t);
    double w = 1.0;
    int r = q;
    for (int d = 0; d < dim; ++d) {
        w *= dW(r % 3);
        r /= 3;
    }
    double inv[9];
    double det;
    if (dim == 2) {
        det = J[0] * J[3] - J[1] * J[2];
        const double id = 1.0 / det;
        inv[0] = J[3] * id; inv[1] = -J[1] * id; inv[2] = -J[2] * id; inv[3] = J[0] * id;
    } else {
        const double c00 = J[4] * J[8] - J[5] * J[7];
        const double c01 = J[5] * J[6] - J[3] * J[8];
        const double c02 = J[3] * J[7] - J[4] * J[6];
        det = J[0] * c00 + J[1] * c01 + J[2] * c02;
        const double id = 1.0 / det;
        inv[0] = c00 * id;
        inv[1] = (J[2] * J[7] - J[1] * J[8]) * id;
        inv[2] = (J[1] * J[5] - J[2] * J[4]) * id;
        inv[3] = c01 * id;
        inv[4] = (J[0] * J[8] - J[2] * J[6]) * id;
        inv[5] = (J[2] * J[3] - J[0] * J[5]) * id;
        inv[6] = c02 * id;
        inv[7] = (J[1] * J[6] - J[0] * J[7]) * id;
        inv[8] = (J[0] * J[4] - J[1] * J[3]) * id;
    }
    if (!(det > 0.0)) g.flag[0] = 1;
    const double cw = det * w;
    g.cw[off] = cw;
    // plane b*dim + a holds K_{ba} = cw (J^{-1})_{ba}
    for (int b = 0; b < dim; ++b)
        for (int a = 0; a < dim; ++a) {
            const double k = cw * inv[b * dim + a];
            g.K[(b * dim + a) * g.plane + off] = k;
            g.K32[(b * dim + a) * g.plane + off] = (float)k;
        }
}

__global__ void k_geometry(GeoOut g, const double* __restrict__ J) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.nc * g.Q) return;
    const int64_t cell = id / g.Q;
    const int q = (int)(id - cell * g.Q);
    const int dd = g.dim * g.dim;
    double Jl[9];
    for (int i = 0; i < dd; ++i) Jl[i] = J[id * dd + i];
    store_geometry(g, cell, q, Jl);
}

void launch_geometry(const Level& L, const double* J, double* K, double* cw, float* K32, int* flag,
                     hipStream_t s) {
    GeoOut g{L.dim, L.dim == 3 ? 9 : 3, L.Q, L.nc, L.plane(), L.geo, L.d_lex2col, K, cw, K32, flag};
    hipLaunchKernelGGL(k_geometry, dim3(nblocks(L.nc * L.Q)), dim3(TPB), 0, s, g, J);
}

struct DispIn {
    const double* disp;   // fine vertex displacement [dim][nvert_fine]
    int stride;           // level vertex -> fine vertex
    int fp[3];            // fine vertex counts per direction
    int64_t nvert_fine;
    int cells[3];
    double h[3];
};

__global__ void k_geometry_disp(GeoOut g, DispIn in) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.nc * g.Q) return;
    const int64_t cell = id / g.Q;
    const int q = (int)(id - cell * g.Q);
    const int dim = g.dim;
    int ci[3] = {0, 0, 0}, qi[3] = {0, 0, 0};
    int64_t r = cell;
    for (int d = 0; d < dim; ++d) {
        ci[d] = (int)(r % in.cells[d]);
        r /= in.cells[d];
    }
    int rq = q;
    for (int d = 0; d < dim; ++d) {
        qi[d] = rq % 3;
        rq /= 3;
    }
    // x = X + d: the box cell's own map X has Jacobian diag(h) exactly, so only the
    // displacement is differentiated (differences of positions X + d would lose
    // digits in proportion to |X| / h)
    double J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int nv = 1 << dim;
    for (int v = 0; v < nv; ++v) {
        int vi[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
        int64_t fidx = 0, st = 1;
        for (int d = 0; d < dim; ++d) {
            const int lv = ci[d] + vi[d];
            fidx += (int64_t)lv * in.stride * st;
            st *= in.fp[d];
        }
        for (int b = 0; b < dim; ++b) {
            double dl = 1.0;
            for (int d = 0; d < dim; ++d) dl *= (d == b) ? dLd(vi[d]) : dL(qi[d], vi[d]);
            for (int a = 0; a < dim; ++a) J[a * dim + b] += dl * in.disp[(int64_t)a * in.nvert_fine + fidx];
        }
    }
    for (int a = 0; a < dim; ++a) J[a * dim + a] += in.h[a];
    store_geometry(g, cell, q, J);
}

// h: the level's reference cell sizes (extent / cells)
void launch_geometry_from_disp(const Level& L, const double* disp_fine, int stride, const int* fine_pnodes,
                                 const double* h, double* K, double* cw, float* K32, int* flag, hipStream_t s) {
    GeoOut g{L.dim, L.dim == 3 ? 9 : 3, L.Q, L.nc, L.plane(), L.geo, L.d_lex2col, K, cw, K32, flag};
    DispIn in;
    in.disp = disp_fine;
    in.stride = stride;
    in.nvert_fine = 1;
    for (int d = 0; d < 3; ++d) {
        in.fp[d] = d < L.dim ? fine_pnodes[d] : 1;
        in.cells[d] = L.cells[d];
        in.h[d] = d < L.dim ? h[d] : 0.0;
    }
    for (int d = 0; d < L.dim; ++d) in.nvert_fine *= in.fp[d];
    hipLaunchKernelGGL(k_geometry_disp, dim3(nblocks(L.nc * L.Q)), dim3(TPB), 0, s, g, in);
}

// ---------------------------------------------------------------- coefficients
__global__ void k_coefficients(int dim, int64_t nc, int Q, GeoLayout geo, int64_t plane,
                               const int* __restrict__ lex2col, const double* __restrict__ cm,
                               const double* __restrict__ eta, const double* __restrict__ cw,
                               double* __restrict__ cv64, float* __restrict__ cv32, float* __restrict__ cq32,
                               double* __restrict__ cq64,
                               const double* __restrict__ K64, double* __restrict__ Ks64, float* __restrict__ Ks32,
                               int* flag) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nc * Q) return;
    const int64_t cell = id / Q;
    const int q = (int)(id - cell * Q);
    const int qx = q % 3, t = q / 3;
    const int64_t off = geo_off(geo, qx, lex2col[cell], t);
    const double m = cm[id], e = eta[id], w = cw[off];
    if (!isfinite(m) || !isfinite(e) || !(e >= 0.0)) flag[0] = 1;
    const double cvisc = 2.0 * e / w, cmass = m * w;
    cv64[off] = cvisc;
    cv64[plane + off] = cmass;
    cv32[off] = (float)cvisc;
    cv32[plane + off] = (float)cmass;
    if (cq32) {
        cq32[off] = (float)(2.0 * e);
        cq32[plane + off] = (float)m;
    }
    if (cq64) {
        cq64[off] = 2.0 * e;
        cq64[plane + off] = m;
    }
    const double sv = sqrt(cvisc);
    for (int pl = 0; pl < dim * dim; ++pl) {
        const double k = sv * K64[pl * plane + off];
        Ks64[pl * plane + off] = k;
        Ks32[pl * plane + off] = (float)k;
    }
}

// corrector-mode terms: per point (lexicographic cell, point) beta_b = sum_e K[b][e] v°_e
// and sigma = r / (det J w), written into the geometry layout in FP64 and FP32 (2D and 3D;
// vconv holds dim components per point)
__global__ void k_convection(int dim, int64_t nc, int Q, GeoLayout geo, int64_t plane, const int* __restrict__ lex2col,
                             const double* __restrict__ vconv, const double* __restrict__ r,
                             const double* __restrict__ K64, const double* __restrict__ cw,
                             double* __restrict__ cb64, double* __restrict__ cs64, float* __restrict__ cb32,
                             float* __restrict__ cs32, int* flag) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nc * Q) return;
    const int64_t cell = id / Q;
    const int q = (int)(id - cell * Q);
    const int64_t off = geo_off(geo, q % 3, lex2col[cell], q / 3);
    double v[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    for (int e = 0; e < dim; ++e) {
        v[e] = vconv[dim * id + e];
        bad |= !isfinite(v[e]);
    }
    const double rr = r[id];
    if (bad || !isfinite(rr) || !(rr >= 0.0)) flag[0] = 1;
    for (int b = 0; b < dim; ++b) {
        double be = 0.0;
        for (int e = 0; e < dim; ++e) be += K64[(dim * b + e) * plane + off] * v[e];
        cb64[b * plane + off] = be;
        cb32[b * plane + off] = (float)be;
    }
    const double sg = rr / cw[off];
    cs64[off] = sg;
    cs32[off] = (float)sg;
}
void launch_convection(const Level& L, const double* vconv, const double* r, double* cb64, double* cs64, float* cb32,
                       float* cs32, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_convection, dim3(nblocks(L.nc * L.Q)), dim3(TPB), 0, s, L.dim, L.nc, L.Q, L.geo, L.plane(),
                       L.d_lex2col, vconv, r, L.d_K64, L.d_cw64, cb64, cs64, cb32, cs32, flag);
}

void launch_coefficients(const Level& L, const double* cm, const double* eta, const double* cw, double* cv64,
                         float* cv32, float* cq32, double* cq64, const double* K64, double* Ks64, float* Ks32,
                         int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_coefficients, dim3(nblocks(L.nc * L.Q)), dim3(TPB), 0, s, L.dim, L.nc, L.Q, L.geo,
                       L.plane(), L.d_lex2col, cm, eta, cw, cv64, cv32, cq32, cq64, K64, Ks64, Ks32, flag);
}

// level vertex v (lexicographic) takes the fine displacement at fine vertex stride * v
__global__ void k_vertex_disp(int dim, int pn0, int pn1, int pn2, int stride, int fp0, int fp1, int64_t nvert_fine,
                              const double* __restrict__ disp, float4* __restrict__ out32,
                              double4* __restrict__ out64) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = (int64_t)pn0 * pn1 * pn2;
    if (v >= nv) return;
    const int i = (int)(v % pn0), j = (int)((v / pn0) % pn1), k = (int)(v / ((int64_t)pn0 * pn1));
    const int64_t f = (int64_t)i * stride + (int64_t)fp0 * ((int64_t)j * stride + (int64_t)fp1 * ((int64_t)k * stride));
    double c[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < dim; ++d) c[d] = disp[(int64_t)d * nvert_fine + f];
    out32[v] = make_float4((float)c[0], (float)c[1], (float)c[2], 0.f);
    out64[v] = make_double4(c[0], c[1], c[2], 0.0);
}
void launch_vertex_disp(const Level& L, const double* disp_fine, int stride, const int* fine_pnodes, float4* out32,
                        double4* out64, hipStream_t s) {
    int64_t nvf = 1;
    for (int d = 0; d < L.dim; ++d) nvf *= fine_pnodes[d];
    hipLaunchKernelGGL(k_vertex_disp, dim3(nblocks(L.np)), dim3(TPB), 0, s, L.dim, L.pnodes[0], L.pnodes[1],
                       L.pnodes[2], stride, fine_pnodes[0], L.dim > 1 ? fine_pnodes[1] : 1, nvf, disp_fine, out32,
                       out64);
}

// ---------------------------------------------------------------- diag(A)
// diag_(a,n) = sum_q cmass phi_n^2 + (cvisc/2)(|G_n|^2 + G_n[a]^2), G_n = K^T grad-hat phi_n
template <int DIM>
__global__ __launch_bounds__(TPB) void k_diagA(int64_t cbeg, int64_t cend, const int* __restrict__ col2lex, int nx, int xpar,
                        GeoLayout geo, int64_t nvn, int64_t plane,
                        const int* __restrict__ vmap, const uint4* __restrict__ info,
                        const double* __restrict__ K, const double* __restrict__ cv,
                        const double* __restrict__ cb, const double* __restrict__ cs, double rho,
                        double* __restrict__ diag) {
    // cb, cs (corrector mode, else null): beta = K v° planes and sigma = r / (det J w)
    constexpr int NLOC = DIM == 3 ? 27 : 9, NQZ = DIM == 3 ? 3 : 1;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = cbeg + id / NLOC;
    const int n = (int)(id % NLOC);
    if (cell >= cend) return;
    if ((col2lex[cell] % nx) % 2 != xpar) return;   // cells of a row share x-faces
    if ((info[cell].x >> n) & 1u) return;
    const int ni[3] = {n % 3, (n / 3) % 3, n / 9};
    double S1[1][3], D1[1][3];   // 1D value and derivative tables of the node along x
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        S1[0][q] = dS(q, ni[0]);
        D1[0][q] = dD(q, ni[0]);
    }
    double acc[3] = {0, 0, 0};
    // outer points in loops (tables re-evaluated there), the x points unrolled: a full
    // unroll hoists all 27 points' loads and runs out of registers
#pragma unroll 1
    for (int q2 = 0; q2 < NQZ; ++q2)
#pragma unroll 1
        for (int q1 = 0; q1 < 3; ++q1) {
            const double s2 = DIM == 3 ? dS(q2, ni[2]) : 1.0, d2 = DIM == 3 ? dD(q2, ni[2]) : 0.0;
            const double s1 = dS(q1, ni[1]), d1 = dD(q1, ni[1]);
#pragma unroll
            for (int q0 = 0; q0 < 3; ++q0) {
                const int64_t off = geo_off(geo, q0, cell, q1 + 3 * q2);
                const double phi = S1[0][q0] * s1 * s2;
                double gh[3];
                gh[0] = D1[0][q0] * s1 * s2;
                gh[1] = S1[0][q0] * d1 * s2;
                gh[2] = S1[0][q0] * s1 * d2;
                double G[3] = {0, 0, 0}, g2 = 0.0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
#pragma unroll
                    for (int b = 0; b < DIM; ++b) G[a] += K[(b * DIM + a) * plane + off] * gh[b];
                    g2 += G[a] * G[a];
                }
                const double cvisc = cv[off], cmass = cv[plane + off];
                double extra = 0.0;
                if (cb) {   // rho phi (v° . grad phi) + r (v° . grad phi)^2, times det(J) w
                    double cg = 0.0;
#pragma unroll
                    for (int b = 0; b < DIM; ++b) cg += gh[b] * cb[b * plane + off];
                    extra = rho * phi * cg + cs[off] * cg * cg;
                }
#pragma unroll
                for (int a = 0; a < DIM; ++a) acc[a] += cmass * phi * phi + 0.5 * cvisc * (g2 + G[a] * G[a]) + extra;
            }
        }
    const int node = vmap[cell * NLOC + n];
    for (int a = 0; a < DIM; ++a) diag[a * nvn + node] += acc[a];
}

void launch_diagA(const Level& L, const double* K, const double* cv, double* diag, hipStream_t s, bool conv) {
    const double* cb = conv ? L.d_cb64 : nullptr;
    const double* cs = conv ? L.d_cs64 : nullptr;
    const int nloc = L.dim == 3 ? 27 : 9;
    for (int ph = 0; ph < L.nphases(); ++ph)
        for (int xpar = 0; xpar < 2; ++xpar) {
            const int64_t n = (L.phase_off[ph + 1] - L.phase_off[ph]) * nloc;
            if (n == 0) continue;
            if (L.dim == 3)
                hipLaunchKernelGGL(k_diagA<3>, dim3(nblocks(n)), dim3(TPB), 0, s, L.phase_off[ph], L.phase_off[ph + 1],
                                   L.d_col2lex, L.cells[0], xpar, L.geo, L.nvn, L.plane(), L.d_vmap, L.d_info, K, cv,
                                   cb, cs, L.rho, diag);
            else
                hipLaunchKernelGGL(k_diagA<2>, dim3(nblocks(n)), dim3(TPB), 0, s, L.phase_off[ph], L.phase_off[ph + 1],
                                   L.d_col2lex, L.cells[0], xpar, L.geo, L.nvn, L.plane(), L.d_vmap, L.d_info, K, cv,
                                   cb, cs, L.rho, diag);
        }
}

__global__ void k_diag_finish(int64_t nv, double* __restrict__ diag, double* __restrict__ d64,
                              float* __restrict__ d32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const double d = diag[i];
    const double inv = d > 0.0 ? 1.0 / d : 1.0;   // wall dofs (zero accumulated) act as identity rows
    if (!(d > 0.0)) diag[i] = 1.0;
    d64[i] = inv;
    d32[i] = (float)inv;
}

void launch_diagA_finish(const Level& L, double* diag, double* dinv64, float* dinv32, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_finish, dim3(nblocks(L.nv)), dim3(TPB), 0, s, L.nv, diag, dinv64, dinv32);
}

// ---------------------------------------------------------------- diag(B diag(A)^{-1} B^T)
// s_k = sum_i (B_{k,i})^2 / A_ii over the velocity dofs i of the 5^dim node patch around
// vertex k.  One workgroup per pressure node: thread (c, n) evaluates, for cell c of the
// 2^dim cells around the vertex and its local node n, the three element-row entries
// B^K_{k,(a,n)} = sum_q psi_k(q) (K^T grad-hat phi_n)_a(q); thread p then sums the
// entries of patch node p over the cells containing it (fixed order, no atomics).
template <int DIM>
__global__ __launch_bounds__(256) void k_diagS(int c0, int c1, int c2, int vn0, int vn1, int vn2, GeoLayout geo, int64_t nvn,
                        int64_t plane, const int* __restrict__ lex2col, const uint8_t* __restrict__ wall,
                        const double* __restrict__ K, const double* __restrict__ dAinv,
                        double* __restrict__ dSinv) {
    constexpr int NLOC = DIM == 3 ? 27 : 9, NCELL = 1 << DIM, Q = NLOC, DD = DIM * DIM;
    constexpr int NQZ = DIM == 3 ? 3 : 1;
    __shared__ double be[NCELL][NLOC][DIM];   // [cell][local node][component]
    __shared__ double kg[NCELL][Q][DD];       // K of the cells around the vertex
    __shared__ double red[256];
    const int pn0 = c0 + 1, pn1 = c1 + 1;
    const int64_t k = blockIdx.x;
    const int kv[3] = {(int)(k % pn0), (int)((k / pn0) % pn1), DIM == 3 ? (int)(k / ((int64_t)pn0 * pn1)) : 0};
    const int tid = threadIdx.x;
    const int cells[3] = {c0, c1, c2};
    const int vn[3] = {vn0, vn1, vn2};
    // stage the geometry of the cells around the vertex once (each value is used by
    // every local node of its cell)
    for (int e = tid; e < NCELL * Q * DD; e += blockDim.x) {
        const int c = e / (Q * DD), r = e - c * (Q * DD), q = r / DD, pl = r - q * DD;
        int ce[3] = {0, 0, 0};
        bool in = true;
        for (int d = 0; d < DIM; ++d) {
            ce[d] = kv[d] - 1 + ((c >> d) & 1);
            if (ce[d] < 0 || ce[d] >= cells[d]) in = false;
        }
        double v = 0.0;
        if (in) {
            const int64_t lex = ce[0] + (int64_t)cells[0] * (ce[1] + (int64_t)cells[1] * ce[2]);
            v = K[pl * plane + geo_off(geo, q % 3, lex2col[lex], q / 3)];
        }
        kg[c][q][pl] = v;
    }
    __syncthreads();
    // element-row entries of the cells around the vertex: 1D tables of this thread's
    // node (values, derivatives) and of the vertex's Q1 function, then tensor products
    if (tid < NCELL * NLOC) {
        const int c = tid / NLOC, n = tid % NLOC;
        const int ni[3] = {n % 3, (n / 3) % 3, n / 9};
        bool in = true;
        int kl[3] = {0, 0, 0};
        for (int d = 0; d < DIM; ++d) {
            const int ce = kv[d] - 1 + ((c >> d) & 1);
            if (ce < 0 || ce >= cells[d]) in = false;
            kl[d] = kv[d] - ce;
        }
        double S1[3][3], D1[3][3], P1[3][3];   // [direction][point]
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                S1[d][q] = d < DIM ? dS(q, ni[d]) : 1.0;
                D1[d][q] = d < DIM ? dD(q, ni[d]) : 0.0;
                P1[d][q] = d < DIM ? dL(q, kl[d]) : 1.0;
            }
        double bs[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) bs[a] = 0.0;
        if (in) {
#pragma unroll
            for (int q2 = 0; q2 < NQZ; ++q2)
#pragma unroll
                for (int q1 = 0; q1 < 3; ++q1)
#pragma unroll
                    for (int q0 = 0; q0 < 3; ++q0) {
                        const int q = q0 + 3 * q1 + 9 * q2;
                        const double psi = P1[0][q0] * P1[1][q1] * P1[2][q2];
                        double gh[3];
                        gh[0] = D1[0][q0] * S1[1][q1] * S1[2][q2];
                        gh[1] = S1[0][q0] * D1[1][q1] * S1[2][q2];
                        gh[2] = S1[0][q0] * S1[1][q1] * D1[2][q2];
#pragma unroll
                        for (int a = 0; a < DIM; ++a) {
                            double G = 0.0;
#pragma unroll
                            for (int b = 0; b < DIM; ++b) G += kg[c][q][b * DIM + a] * gh[b];
                            bs[a] += psi * G;
                        }
                    }
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) be[c][n][a] = bs[a];
    }
    __syncthreads();
    // patch node p: sum its entries over the cells containing it
    double contrib = 0.0;
    const int npatch = DIM == 3 ? 125 : 25;
    if (tid < npatch) {
        const int pi[3] = {tid % 5, (tid / 5) % 5, DIM == 3 ? tid / 25 : 0};
        int g[3] = {0, 0, 0};
        bool ok = true;
        for (int d = 0; d < DIM; ++d) {
            g[d] = 2 * kv[d] - 2 + pi[d];
            if (g[d] < 0 || g[d] >= vn[d]) ok = false;
        }
        if (ok) {
            const int64_t node = g[0] + (int64_t)vn[0] * (g[1] + (int64_t)vn[1] * g[2]);
            if (!wall[node]) {
                double bsum[DIM];
                for (int a = 0; a < DIM; ++a) bsum[a] = 0.0;
                for (int c = 0; c < NCELL; ++c) {
                    int n = 0, st = 1;
                    bool inside = true;
                    for (int d = 0; d < DIM; ++d) {
                        const int l = pi[d] - 2 * ((c >> d) & 1);   // local index in cell c
                        if (l < 0 || l > 2) inside = false;
                        n += l * st;
                        st *= 3;
                    }
                    if (!inside) continue;                      // cells outside the mesh hold zeros
                    for (int a = 0; a < DIM; ++a) bsum[a] += be[c][n][a];
                }
                for (int a = 0; a < DIM; ++a) contrib += bsum[a] * bsum[a] * dAinv[a * nvn + node];
            }
        }
    }
    red[tid] = contrib;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) dSinv[k] = red[0] > 0.0 ? 1.0 / red[0] : 1.0;
}

void launch_diagS_impl(const Level& L, const uint8_t* d_wall, const double* K, const double* dAinv, double* dSinv,
                       hipStream_t s) {
    if (L.dim == 3)
        hipLaunchKernelGGL(k_diagS<3>, dim3((unsigned)L.np), dim3(256), 0, s, L.cells[0], L.cells[1], L.cells[2],
                           L.vnodes[0], L.vnodes[1], L.vnodes[2], L.geo, L.nvn, L.plane(), L.d_lex2col, d_wall, K,
                           dAinv, dSinv);
    else
        hipLaunchKernelGGL(k_diagS<2>, dim3((unsigned)L.np), dim3(256), 0, s, L.cells[0], L.cells[1], L.cells[2],
                           L.vnodes[0], L.vnodes[1], L.vnodes[2], L.geo, L.nvn, L.plane(), L.d_lex2col, d_wall, K,
                           dAinv, dSinv);
}

// ---------------------------------------------------------------- simple vector kernels
template <typename T>
__global__ void k_fill(T* x, T v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}
template <typename T>
void launch_fill(T* x, T val, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill<T>, dim3(nblocks(n)), dim3(TPB), 0, s, x, val, n);
}
template void launch_fill<double>(double*, double, int64_t, hipStream_t);
template void launch_fill<float>(float*, float, int64_t, hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);

template <typename T>
__global__ void k_dir_copy(const int* __restrict__ nodes, int64_t nd, int dim, int64_t nvn, const T* __restrict__ u,
                           T* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const int64_t n = nodes[i];
    for (int c = 0; c < dim; ++c) v[c * nvn + n] = u[c * nvn + n];
}
template <typename T>
void launch_dirichlet_copy(const Level& L, const T* u, T* v, hipStream_t s) {
    if (L.n_dir > 0)
        hipLaunchKernelGGL(k_dir_copy<T>, dim3(nblocks(L.n_dir)), dim3(TPB), 0, s, L.d_dir_nodes, L.n_dir, L.dim,
                           L.nvn, u, v);
}
template void launch_dirichlet_copy<double>(const Level&, const double*, double*, hipStream_t);
template void launch_dirichlet_copy<float>(const Level&, const float*, float*, hipStream_t);

// zero n elements: 16-byte stores over the body (x 16-byte aligned), element stores
// for the tail
template <typename T>
__global__ void k_zero16(T* __restrict__ x, int64_t n) {
    constexpr int E = 16 / sizeof(T);
    const int64_t nb = n / E;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) reinterpret_cast<uint4*>(x)[i] = make_uint4(0u, 0u, 0u, 0u);
    if (i < n - nb * E) x[nb * E + i] = T(0);
}
template <typename T>
static void launch_zero(T* x, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    if (reinterpret_cast<uintptr_t>(x) % 16 != 0) {
        launch_fill<T>(x, T(0), n, s);
        return;
    }
    constexpr int E = 16 / sizeof(T);
    const int64_t nb = n / E;
    hipLaunchKernelGGL(k_zero16<T>, dim3(nblocks(std::max<int64_t>(nb, n - nb * E))), dim3(TPB), 0, s, x, n);
}
// v = 0 and q = 0 in one launch (small levels, where launch latency dominates)
template <typename T>
__global__ void k_zero2(T* __restrict__ v, int64_t nv, double* __restrict__ q, int64_t np) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v && i < nv) v[i] = T(0);
    if (q && i < np) q[i] = 0.0;
}
// zero fill of a velocity vector (component-major, x fastest), node plane by node plane
// (kZeroPlaneParts blocks per plane), top planes first: the planes the atomic cell launch reaches first (low z; it walks the
// rows in natural order) are written last and are the likeliest to still sit in the
// memory-side cache when its adds arrive.  16-byte stores; a store unit that straddles
// two planes is written by both blocks (zeros either way); the array's last unit may run
// past the end and is written element by element.
constexpr int kZeroPlaneParts = 4;   // blocks per node plane and component
template <typename T>
__global__ void k_zero_planes_desc(T* __restrict__ x, int64_t nvn, int64_t plane, int nz, int ncomp, int64_t n) {
    constexpr int E = 16 / sizeof(T);
    const int part = (int)(blockIdx.x % kZeroPlaneParts), pc = (int)(blockIdx.x / kZeroPlaneParts);
    const int zz = pc / ncomp, c = pc % ncomp;
    const int64_t p0 = c * nvn + (int64_t)(nz - 1 - zz) * plane;
    const int64_t s0 = p0 + plane * part / kZeroPlaneParts, s1 = p0 + plane * (part + 1) / kZeroPlaneParts;
    const int64_t u0 = s0 / E, u1 = (s1 + E - 1) / E;
    for (int64_t u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
        if ((u + 1) * E <= n) {
            reinterpret_cast<uint4*>(x)[u] = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int64_t i = u * E; i < n; ++i) x[i] = T(0);
        }
    }
}

template <typename T>
void launch_atomic_init(const Level& L, T* v, double* q, hipStream_t s) {
    // large levels: streaming zero fills at full store width (3D velocity: plane by plane,
    // top planes first); small levels: one kernel
    if (L.nvn >= (int64_t(1) << 20)) {
        if (v && L.dim == 3 && reinterpret_cast<uintptr_t>(v) % 16 == 0) {
            const int64_t plane = (int64_t)L.vnodes[0] * L.vnodes[1];
            hipLaunchKernelGGL(k_zero_planes_desc<T>, dim3((unsigned)(L.vnodes[2] * L.dim * kZeroPlaneParts)), dim3(256), 0, s, v,
                               L.nvn, plane, L.vnodes[2], L.dim, L.nv);
        } else if (v) {
            launch_zero<T>(v, L.nv, s);
        }
        if (q) launch_zero<double>(q, L.np, s);
        return;
    }
    const int64_t n = std::max(v ? L.nv : 0, q ? L.np : 0);
    if (n > 0) hipLaunchKernelGGL(k_zero2<T>, dim3(nblocks(n)), dim3(TPB), 0, s, v, L.nv, q, L.np);
}
template void launch_atomic_init<double>(const Level&, double*, double*, hipStream_t);
template void launch_atomic_init<float>(const Level&, float*, double*, hipStream_t);

template <typename T>
__global__ void k_dir_zero(const int* __restrict__ nodes, int64_t nd, int dim, int64_t nvn, T* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const int64_t n = nodes[i];
    for (int c = 0; c < dim; ++c) v[c * nvn + n] = T(0);
}
template <typename T>
void launch_dirichlet_zero(const Level& L, T* v, hipStream_t s) {
    if (L.n_dir > 0)
        hipLaunchKernelGGL(k_dir_zero<T>, dim3(nblocks(L.n_dir)), dim3(TPB), 0, s, L.d_dir_nodes, L.n_dir, L.dim,
                           L.nvn, v);
}
template void launch_dirichlet_zero<double>(const Level&, double*, hipStream_t);
template void launch_dirichlet_zero<float>(const Level&, float*, hipStream_t);

template <typename T>
__global__ void k_dir_cheb(const int* __restrict__ nodes, int64_t nd, int dim, int64_t nvn, T* __restrict__ x,
                           T* __restrict__ d, const T* __restrict__ r, const T* __restrict__ dinv, T c1, T c2,
                           int first, int store_d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const int64_t n = nodes[i];
    for (int c = 0; c < dim; ++c) {
        const int64_t k = c * nvn + n;
        const T xk = x[k];
        const T dn = c1 * (first ? xk : d[k]) + c2 * dinv[k] * (r[k] - xk);   // wall row of A: identity
        if (store_d) d[k] = dn;
        x[k] = xk + dn;
    }
}
template <typename T>
void launch_dirichlet_cheb(const Level& L, T* x, T* d, const T* r, const T* dinv, double c1, double c2, bool first,
                           bool store_d, hipStream_t s) {
    if (L.n_dir > 0)
        hipLaunchKernelGGL(k_dir_cheb<T>, dim3(nblocks(L.n_dir)), dim3(TPB), 0, s, L.d_dir_nodes, L.n_dir, L.dim,
                           L.nvn, x, d, r, dinv, (T)c1, (T)c2, first ? 1 : 0, store_d ? 1 : 0);
}
template void launch_dirichlet_cheb<double>(const Level&, double*, double*, const double*, const double*, double,
                                            double, bool, bool, hipStream_t);
template void launch_dirichlet_cheb<float>(const Level&, float*, float*, const float*, const float*, double, double,
                                           bool, bool, hipStream_t);

template <typename T>
__global__ void k_dir_res(const int* __restrict__ nodes, int64_t nd, int dim, int64_t nvn, const T* __restrict__ f,
                          const T* __restrict__ u, T* __restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const int64_t n = nodes[i];
    for (int c = 0; c < dim; ++c) r[c * nvn + n] = f[c * nvn + n] - u[c * nvn + n];
}
template <typename T>
void launch_dirichlet_res(const Level& L, const T* f, const T* u, T* r, hipStream_t s) {
    if (L.n_dir > 0)
        hipLaunchKernelGGL(k_dir_res<T>, dim3(nblocks(L.n_dir)), dim3(TPB), 0, s, L.d_dir_nodes, L.n_dir, L.dim,
                           L.nvn, f, u, r);
}
template void launch_dirichlet_res<double>(const Level&, const double*, const double*, double*, hipStream_t);
template void launch_dirichlet_res<float>(const Level&, const float*, const float*, float*, hipStream_t);

template <typename TD, typename TS>
__global__ void k_cast(TD* __restrict__ d, const TS* __restrict__ s, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (TD)s[i];
}
template <typename TD, typename TS>
void launch_cast(TD* d, const TS* src, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL((k_cast<TD, TS>), dim3(nblocks(n)), dim3(TPB), 0, s, d, src, n);
}
template void launch_cast<float, double>(float*, const double*, int64_t, hipStream_t);
template void launch_cast<double, float>(double*, const float*, int64_t, hipStream_t);
template void launch_cast<double, double>(double*, const double*, int64_t, hipStream_t);
template void launch_cast<float, float>(float*, const float*, int64_t, hipStream_t);

// first Chebyshev iterate x = c0 D^{-1} r; the first direction equals it, so it is not stored
template <typename T>
__global__ void k_cheb_init(const T* __restrict__ dinv, const T* __restrict__ r, T* __restrict__ x, T c0,
                            int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] = dinv[i] * r[i] * c0;
}
template <typename T>
void launch_cheb_init(const T* dinv, const T* r, T* x, double c0, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_init<T>, dim3(nblocks(n)), dim3(TPB), 0, s, dinv, r, x, (T)c0, n);
}
template void launch_cheb_init<double>(const double*, const double*, double*, double, int64_t, hipStream_t);
template void launch_cheb_init<float>(const float*, const float*, float*, double, int64_t, hipStream_t);

// d' = c1 d + c2 D^{-1}(r - A x), x += d'; the first step takes d = x (nothing stored
// yet), the last one does not store d'
template <typename T>
__global__ void k_cheb_step(const T* __restrict__ dinv, const T* __restrict__ r, const T* __restrict__ ax,
                            T* __restrict__ x, T* __restrict__ d, T c1, T c2, int first, int store_d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T xi = x[i];
    const T dn = c1 * (first ? xi : d[i]) + c2 * dinv[i] * (r[i] - ax[i]);
    if (store_d) d[i] = dn;
    x[i] = xi + dn;
}
template <typename T>
void launch_cheb_step(const T* dinv, const T* r, const T* ax, T* x, T* d, double c1, double c2, bool first,
                      bool store_d, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cheb_step<T>, dim3(nblocks(n)), dim3(TPB), 0, s, dinv, r, ax, x, d, (T)c1, (T)c2,
                       first ? 1 : 0, store_d ? 1 : 0, n);
}
template void launch_cheb_step<double>(const double*, const double*, const double*, double*, double*, double, double,
                                       bool, bool, int64_t, hipStream_t);
template void launch_cheb_step<float>(const float*, const float*, const float*, float*, float*, double, double, bool,
                                      bool, int64_t, hipStream_t);

template <typename T>
__global__ void k_sub(const T* __restrict__ f, const T* __restrict__ a, T* __restrict__ r, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = f[i] - a[i];
}
template <typename T>
void launch_sub(const T* f, const T* a, T* r, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_sub<T>, dim3(nblocks(n)), dim3(TPB), 0, s, f, a, r, n);
}
template void launch_sub<double>(const double*, const double*, double*, int64_t, hipStream_t);
template void launch_sub<float>(const float*, const float*, float*, int64_t, hipStream_t);

__global__ void k_schur_z(const double* __restrict__ ds, const double* __restrict__ t, const double* __restrict__ r,
                          double* __restrict__ z, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = ds[i] * (t[i] - r[i]);
}
void launch_schur_z(const double* dsinv, const double* t, const double* r, double* z, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_schur_z, dim3(nblocks(n)), dim3(TPB), 0, s, dsinv, t, r, z, n);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (tid < st) sh[tid] += sh[tid + st];
        __syncthreads();
    }
    return sh[0];
}

template <typename T>
__global__ void k_dot_partial(const T* __restrict__ x, const T* __restrict__ y, int64_t n, double* __restrict__ part) {
    __shared__ double sh[TPB];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += (double)x[i] * (double)y[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_partials(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double sh[TPB];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = s;
}

static unsigned red_blocks(int64_t n) {
    int64_t b = (n + TPB - 1) / TPB;
    if (b > kReduceBlocks) b = kReduceBlocks;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <typename T>
void launch_dot(const T* x, const T* y, int64_t n, double* partials, double* out, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(nb), dim3(TPB), 0, s, x, y, n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(TPB), 0, s, partials, (int)nb, out);
}
template void launch_dot<double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template void launch_dot<float>(const float*, const float*, int64_t, double*, double*, hipStream_t);

__global__ void k_schur_dots_partial(const double* __restrict__ y, const double* __restrict__ z,
                                     const double* __restrict__ ds, int64_t n, double* __restrict__ part) {
    __shared__ double sh[TPB];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double yi = y[i];
        a += yi * z[i];
        b += yi * ds[i] * yi;
    }
    const double sa = block_sum(a, sh);
    __syncthreads();
    const double sb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = sb;
    }
}
__global__ void k_schur_dots_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double sh[TPB];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    const double sa = block_sum(a, sh);
    __syncthreads();
    const double sb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        out[0] = sa;
        out[1] = sb;
    }
}
void launch_schur_dots(const double* y, const double* z, const double* dsinv, double* partials, double* dots,
                       int64_t n, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_schur_dots_partial, dim3(nb), dim3(TPB), 0, s, y, z, dsinv, n, partials);
    hipLaunchKernelGGL(k_schur_dots_final, dim3(1), dim3(TPB), 0, s, partials, (int)nb, dots);
}

// x_u (+)= w - beta v ; x_p (+)= beta z with beta = dots[0]/dots[1] (one MINRES step)
template <typename T>
__global__ void k_smoother_update(const T* __restrict__ w, const T* __restrict__ vv, const double* __restrict__ z,
                                  const double* __restrict__ dots, T* __restrict__ xu, double* __restrict__ xp,
                                  int64_t nu, int64_t np, int first) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double den = dots[1];
    const double beta = den != 0.0 ? dots[0] / den : 0.0;
    if (i < nu) {
        const T inc = w[i] - (T)beta * vv[i];
        xu[i] = first ? inc : xu[i] + inc;
    } else if (i < nu + np) {
        const int64_t j = i - nu;
        const double inc = beta * z[j];
        xp[j] = first ? inc : xp[j] + inc;
    }
}
template <typename T>
void launch_smoother_update(const T* w, const T* vv, const double* z, const double* dots, T* x_u, double* x_p,
                            int64_t nu, int64_t np, bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_smoother_update<T>, dim3(nblocks(nu + np)), dim3(TPB), 0, s, w, vv, z, dots, x_u, x_p, nu, np,
                       first ? 1 : 0);
}
__global__ void k_bicg_start(const double* __restrict__ ds, const double* __restrict__ t,
                             const double* __restrict__ r, double* __restrict__ b, double* __restrict__ p,
                             int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double bi = t[i] - r[i];
        b[i] = bi;
        p[i] = ds[i] * bi;
    }
}
void launch_bicg_start(const double* dsinv, const double* t, const double* r, double* b, double* p, int64_t n,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_start, dim3(nblocks(n)), dim3(TPB), 0, s, dsinv, t, r, b, p, n);
}
__global__ void k_bicg_mid(const double* __restrict__ ds, const double* __restrict__ dots,
                           const double* __restrict__ v, double* __restrict__ b, double* __restrict__ q, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double alpha = dots[1] != 0.0 ? dots[0] / dots[1] : 0.0;
    if (i < n) {
        const double si = b[i] - alpha * v[i];
        b[i] = si;
        q[i] = ds[i] * si;
    }
}
void launch_bicg_mid(const double* dsinv, const double* dots, const double* v, double* b, double* q, int64_t n,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_mid, dim3(nblocks(n)), dim3(TPB), 0, s, dsinv, dots, v, b, q, n);
}
template <typename T>
__global__ void k_bicg_update(const T* __restrict__ w, const T* __restrict__ t1, const T* __restrict__ t2,
                              const double* __restrict__ p, const double* __restrict__ q,
                              const double* __restrict__ dots, T* __restrict__ xu, double* __restrict__ xp,
                              int64_t nu, int64_t np, int first) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double alpha = dots[1] != 0.0 ? dots[0] / dots[1] : 0.0;
    const double omega = dots[3] > 0.0 ? dots[2] / dots[3] : 0.0;
    if (i < nu) {
        const T inc = w[i] - (T)alpha * t1[i] - (T)omega * t2[i];
        xu[i] = first ? inc : xu[i] + inc;
    } else if (i < nu + np) {
        const int64_t j = i - nu;
        const double inc = alpha * p[j] + omega * q[j];
        xp[j] = first ? inc : xp[j] + inc;
    }
}
template <typename T>
void launch_bicg_update(const T* w, const T* t1, const T* t2, const double* p, const double* q, const double* dots,
                        T* x_u, double* x_p, int64_t nu, int64_t np, bool first, hipStream_t s) {
    hipLaunchKernelGGL(k_bicg_update<T>, dim3(nblocks(nu + np)), dim3(TPB), 0, s, w, t1, t2, p, q, dots, x_u, x_p,
                       nu, np, first ? 1 : 0);
}
template void launch_bicg_update<double>(const double*, const double*, const double*, const double*, const double*,
                                         const double*, double*, double*, int64_t, int64_t, bool, hipStream_t);
template void launch_bicg_update<float>(const float*, const float*, const float*, const double*, const double*,
                                        const double*, float*, double*, int64_t, int64_t, bool, hipStream_t);
template void launch_smoother_update<double>(const double*, const double*, const double*, const double*, double*,
                                             double*, int64_t, int64_t, bool, hipStream_t);
template void launch_smoother_update<float>(const float*, const float*, const double*, const double*, float*, double*,
                                            int64_t, int64_t, bool, hipStream_t);

// ---------------------------------------------------------------- transfers
// 1D prolongation weights of the nested Q2 space: fine node f, coarse cell e = f/4,
// r = f - 4e -> weights on coarse nodes 2e..2e+2.
__device__ __forceinline__ void q2_prol_1d(int f, int ncoarse_cells, int& base, double w[3]) {
    int e = f >> 2;
    if (e >= ncoarse_cells) e = ncoarse_cells - 1;
    const int r = f - 4 * e;
    base = 2 * e;
    switch (r) {
        case 0: w[0] = 1; w[1] = 0; w[2] = 0; break;
        case 1: w[0] = 0.375; w[1] = 0.75; w[2] = -0.125; break;
        case 2: w[0] = 0; w[1] = 1; w[2] = 0; break;
        case 3: w[0] = -0.125; w[1] = 0.75; w[2] = 0.375; break;
        default: w[0] = 0; w[1] = 0; w[2] = 1; break;
    }
}
__device__ __forceinline__ void q1_prol_1d(int f, int ncoarse_cells, int& base, double w[2]) {
    int e = f >> 1;
    if (e >= ncoarse_cells) e = ncoarse_cells - 1;
    const int r = f - 2 * e;
    base = e;
    if (r == 0) { w[0] = 1; w[1] = 0; }
    else if (r == 1) { w[0] = 0.5; w[1] = 0.5; }
    else { w[0] = 0; w[1] = 1; }
}
__device__ __forceinline__ int q1_rest_1d(int c, int nfine_nodes, int f[3], double w[3]) {
    int m = 0;
    const int fo[3] = {2 * c - 1, 2 * c, 2 * c + 1};
    const double wo[3] = {0.5, 1.0, 0.5};
    for (int i = 0; i < 3; ++i)
        if (fo[i] >= 0 && fo[i] < nfine_nodes) { f[m] = fo[i]; w[m] = wo[i]; ++m; }
    return m;
}

struct XferDims {
    int dim;
    int fv[3], cv[3];     // velocity node counts fine / coarse
    int fp[3], cp[3];     // pressure node counts
    int cc[3];            // coarse cells
    int64_t fnv, cnv, fnp, cnp;
};

// rb (may be null): restrict rf - rb (the residual f - M x from f and M x)
__global__ void k_restrict_p(XferDims x, const double* __restrict__ rf, const double* __restrict__ rb,
                             double* __restrict__ rc) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= x.cnp) return;
    int c[3] = {0, 0, 0};
    int64_t r = id;
    for (int d = 0; d < x.dim; ++d) { c[d] = (int)(r % x.cp[d]); r /= x.cp[d]; }
    int fi[3][3];
    double wi[3][3];
    int m[3] = {1, 1, 1};
    fi[1][0] = fi[2][0] = 0;
    wi[1][0] = wi[2][0] = 1.0;
    for (int d = 0; d < x.dim; ++d) m[d] = q1_rest_1d(c[d], x.fp[d], fi[d], wi[d]);
    double acc = 0.0;
    for (int k = 0; k < m[2]; ++k)
        for (int j = 0; j < m[1]; ++j)
            for (int i = 0; i < m[0]; ++i) {
                const int64_t fn = fi[0][i] + (int64_t)x.fp[0] * (fi[1][j] + (int64_t)x.fp[1] * fi[2][k]);
                acc += wi[0][i] * wi[1][j] * wi[2][k] * (rb ? rf[fn] - rb[fn] : rf[fn]);
            }
    rc[id] = acc;
}

// The velocity transfers are tensor products of the 1D Q2 stencils, so they run as
// one 1D pass per direction over a tensor viewed as [outer][n][inner] (inner = the
// faster directions, contiguous): each pass reads its input once, coalesced along
// the inner index.  Restriction contracts x, then y, then z (the last pass zeroes
// the coarse wall rows); prolongation expands z, then y, then x (the last pass adds
// into the fine vector, skipping its wall rows).  Sums are formed in FP64 and the
// intermediate tensors are FP64, so an FP32 transfer rounds once, at its output.
// SUB: the pass restricts in - inb (the first pass of the residual restriction, which
// then needs no separate subtraction kernel); the difference is formed in FP64
template <typename Tin, typename Tout, bool SUB>
__global__ void k_restrict_axis(const Tin* __restrict__ in, const Tin* __restrict__ inb, Tout* __restrict__ out,
                                int64_t outer, int nf, int nc, int64_t inner, const uint8_t* __restrict__ cwall,
                                int64_t cnv) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= outer * nc * inner) return;
    const int64_t b = id % inner, r = id / inner;
    const int c = (int)(r % nc);
    const int64_t a = r / nc;
    const Tin* src = in + a * nf * inner + b;
    const Tin* srb = SUB ? inb + a * nf * inner + b : nullptr;
    auto val = [&](int f) {
        return SUB ? double(src[(int64_t)f * inner]) - double(srb[(int64_t)f * inner]) : double(src[(int64_t)f * inner]);
    };
    const int e = c >> 1;
    double acc;
    if ((c & 1) == 0) {
        const int f0 = 4 * e;
        acc = val(f0);
        if (f0 - 1 >= 0) acc += 0.375 * val(f0 - 1);
        if (f0 + 1 < nf) acc += 0.375 * val(f0 + 1);
        if (f0 - 3 >= 0) acc -= 0.125 * val(f0 - 3);
        if (f0 + 3 < nf) acc -= 0.125 * val(f0 + 3);
    } else {
        const int f1 = 4 * e + 1;
        acc = 0.75 * (val(f1) + val(f1 + 2)) + val(f1 + 1);
    }
    if (cwall && cwall[id % cnv]) acc = 0.0;
    out[id] = Tout(acc);
}
template <typename Tin, typename Tout>
__global__ void k_prolong_axis(const Tin* __restrict__ in, Tout* __restrict__ out, int64_t outer, int ncells, int nf,
                               int64_t inner, const uint8_t* __restrict__ fwall, int64_t fnv) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= outer * nf * inner) return;
    if (fwall && fwall[id % fnv]) return;   // last pass: wall rows keep their value
    const int64_t b = id % inner, r = id / inner;
    const int f = (int)(r % nf);
    const int64_t a = r / nf;
    const int nc = 2 * ncells + 1;
    int base;
    double w[3];
    q2_prol_1d(f, ncells, base, w);
    const Tin* src = in + (a * nc + base) * inner + b;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (w[i] != 0.0) acc += w[i] * double(src[(int64_t)i * inner]);
    if (fwall) out[id] += Tout(acc);
    else out[id] = Tout(acc);
}
__global__ void k_prolong_p(XferDims x, const double* __restrict__ ec, double* __restrict__ xf) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= x.fnp) return;
    int f[3] = {0, 0, 0};
    int64_t r = id;
    for (int d = 0; d < x.dim; ++d) { f[d] = (int)(r % x.fp[d]); r /= x.fp[d]; }
    int base[3] = {0, 0, 0};
    double w[3][2] = {{1, 0}, {1, 0}, {1, 0}};
    int m[3] = {1, 1, 1};
    for (int d = 0; d < x.dim; ++d) { q1_prol_1d(f[d], x.cc[d], base[d], w[d]); m[d] = 2; }
    double acc = 0.0;
    for (int k = 0; k < m[2]; ++k)
        for (int j = 0; j < m[1]; ++j)
            for (int i = 0; i < m[0]; ++i) {
                const double ww = w[0][i] * w[1][j] * w[2][k];
                if (ww == 0.0) continue;
                const int64_t cn = (base[0] + i) + (int64_t)x.cp[0] * ((base[1] + j) + (int64_t)x.cp[1] * (base[2] + k));
                acc += ww * ec[cn];
            }
    xf[id] += acc;
}

static XferDims xdims(const Level& fine, const Level& coarse) {
    XferDims x;
    x.dim = fine.dim;
    for (int d = 0; d < 3; ++d) {
        x.fv[d] = fine.vnodes[d];
        x.cv[d] = coarse.vnodes[d];
        x.fp[d] = fine.pnodes[d];
        x.cp[d] = coarse.pnodes[d];
        x.cc[d] = coarse.cells[d];
    }
    x.fnv = fine.nvn;
    x.cnv = coarse.nvn;
    x.fnp = fine.np;
    x.cnp = coarse.np;
    return x;
}

// wall masks live on the device as uint8 per node (set up by the host)

namespace {
// one 1D pass of a transfer: tensor extents before the pass, the direction d, and
// the input / output types of the pass
struct AxisPass {
    int64_t outer, inner;
    int nin, nout;
};
AxisPass axis_pass(const int64_t ext[3], int d, int D, int nout) {
    AxisPass p;
    p.inner = 1;
    p.outer = D;
    for (int e = 0; e < d; ++e) p.inner *= ext[e];
    for (int e = d + 1; e < 3; ++e) p.outer *= ext[e];
    p.nin = (int)ext[d];
    p.nout = nout;
    return p;
}
template <typename Tin, typename Tout>
void restrict_pass(const Tin* in, Tout* out, const AxisPass& p, const uint8_t* cwall, int64_t cnv, hipStream_t s,
                   const Tin* inb = nullptr) {
    const int64_t n = p.outer * p.nout * p.inner;
    if (inb)
        hipLaunchKernelGGL((k_restrict_axis<Tin, Tout, true>), dim3(nblocks(n)), dim3(TPB), 0, s, in, inb, out,
                           p.outer, p.nin, p.nout, p.inner, cwall, cnv);
    else
        hipLaunchKernelGGL((k_restrict_axis<Tin, Tout, false>), dim3(nblocks(n)), dim3(TPB), 0, s, in, inb, out,
                           p.outer, p.nin, p.nout, p.inner, cwall, cnv);
}
template <typename Tin, typename Tout>
void prolong_pass(const Tin* in, Tout* out, const AxisPass& p, int ncells, const uint8_t* fwall, int64_t fnv,
                  hipStream_t s) {
    const int64_t n = p.outer * p.nout * p.inner;
    hipLaunchKernelGGL((k_prolong_axis<Tin, Tout>), dim3(nblocks(n)), dim3(TPB), 0, s, in, out, p.outer, ncells,
                       p.nout, p.inner, fwall, fnv);
}
}  // namespace

template <typename T>
void launch_restrict(const Level& fine, const Level& coarse, const T* rf_u, const double* rf_p, T* rc_u, double* rc_p,
                     double* s1, double* s2, hipStream_t s, const T* rb_u, const double* rb_p) {
    const XferDims x = xdims(fine, coarse);
    const int D = x.dim;
    // extents of the tensor [comp][z][y][x] as the passes shrink it
    int64_t ext[3] = {x.fv[0], x.fv[1], D == 3 ? x.fv[2] : 1};
    const uint8_t* cw = level_wall_mask(coarse);
    AxisPass p = axis_pass(ext, 0, D, x.cv[0]);
    restrict_pass<T, double>(rf_u, s1, p, nullptr, x.cnv, s, rb_u);
    ext[0] = x.cv[0];
    p = axis_pass(ext, 1, D, x.cv[1]);
    if (D == 2) {
        restrict_pass<double, T>(s1, rc_u, p, cw, x.cnv, s);
    } else {
        restrict_pass<double, double>(s1, s2, p, nullptr, x.cnv, s);
        ext[1] = x.cv[1];
        p = axis_pass(ext, 2, D, x.cv[2]);
        restrict_pass<double, T>(s2, rc_u, p, cw, x.cnv, s);
    }
    if (rf_p) hipLaunchKernelGGL(k_restrict_p, dim3(nblocks(x.cnp)), dim3(TPB), 0, s, x, rf_p, rb_p, rc_p);
}
template <typename T>
void launch_prolongate_add(const Level& fine, const Level& coarse, const T* ec_u, const double* ec_p, T* xf_u,
                           double* xf_p, double* s1, double* s2, hipStream_t s) {
    const XferDims x = xdims(fine, coarse);
    const int D = x.dim;
    int64_t ext[3] = {x.cv[0], x.cv[1], D == 3 ? x.cv[2] : 1};
    const uint8_t* fw = level_wall_mask(fine);
    const double* in = nullptr;
    if (D == 3) {
        AxisPass p = axis_pass(ext, 2, D, x.fv[2]);
        prolong_pass<T, double>(ec_u, s1, p, x.cc[2], nullptr, x.fnv, s);
        ext[2] = x.fv[2];
        p = axis_pass(ext, 1, D, x.fv[1]);
        prolong_pass<double, double>(s1, s2, p, x.cc[1], nullptr, x.fnv, s);
        in = s2;
    } else {
        AxisPass p = axis_pass(ext, 1, D, x.fv[1]);
        prolong_pass<T, double>(ec_u, s2, p, x.cc[1], nullptr, x.fnv, s);
        in = s2;
    }
    ext[1] = x.fv[1];
    AxisPass p = axis_pass(ext, 0, D, x.fv[0]);
    prolong_pass<double, T>(in, xf_u, p, x.cc[0], fw, x.fnv, s);
    if (ec_p) hipLaunchKernelGGL(k_prolong_p, dim3(nblocks(x.fnp)), dim3(TPB), 0, s, x, ec_p, xf_p);
}
template void launch_restrict<double>(const Level&, const Level&, const double*, const double*, double*, double*,
                                      double*, double*, hipStream_t, const double*, const double*);
template void launch_restrict<float>(const Level&, const Level&, const float*, const double*, float*, double*,
                                     double*, double*, hipStream_t, const float*, const double*);
template void launch_prolongate_add<double>(const Level&, const Level&, const double*, const double*, double*,
                                            double*, double*, double*, hipStream_t);
template void launch_prolongate_add<float>(const Level&, const Level&, const float*, const double*, float*, double*,
                                           double*, double*, hipStream_t);

// ---------------------------------------------------------------- coarse level
// One thread per (cell of one colour, test dof (a, n), column node m): the element
// matrix entries of A (mass + viscous) for the trial dofs (b, m), b = 0..dim-1, or
// (m >= NLOC) the B^T column / B row entries of pressure vertex m - NLOC, are added
// to the dense matrix restricted to free dofs (dof2row[dof] < 0 for wall dofs).
// Cells of one launch share no node, so every entry has one writer.
template <int DIM>
__global__ __launch_bounds__(64) void k_coarse_assemble(int64_t cbeg, int64_t cend, const int* __restrict__ col2lex, int nx, int xpar,
                                  GeoLayout geo, int64_t nvn, int64_t plane, const int* __restrict__ vmap,
                                  const int* __restrict__ pmap, const double* __restrict__ K,
                                  const double* __restrict__ cv, const double* __restrict__ cb,
                                  const double* __restrict__ cs, double rho, const int* __restrict__ vrow,
                                  int64_t nfree_u, double* __restrict__ M, int64_t n) {
    constexpr int NLOC = DIM == 3 ? 27 : 9, NPL = DIM == 3 ? 8 : 4, NQZ = DIM == 3 ? 3 : 1;
    constexpr int NCOL = NLOC + NPL, PER_CELL = DIM * NLOC * NCOL;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = cbeg + id / PER_CELL;
    if (cell >= cend) return;
    if ((col2lex[cell] % nx) % 2 != xpar) return;   // cells of a row share x-faces
    const int loc = (int)(id % PER_CELL);
    const int a = loc / (NLOC * NCOL), nrow = (loc / NCOL) % NLOC, m = loc % NCOL;
    const int row = vrow[a * nvn + vmap[cell * NLOC + nrow]];
    if (row < 0) return;
    const int ni[3] = {nrow % 3, (nrow / 3) % 3, nrow / 9};
    double Sn[3][3], Dn[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Sn[d][q] = d < DIM ? dS(q, ni[d]) : 1.0;
            Dn[d][q] = d < DIM ? dD(q, ni[d]) : 0.0;
        }
    if (m < NLOC) {
        const int mi[3] = {m % 3, (m / 3) % 3, m / 9};
        double Sm[3][3], Dm[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                Sm[d][q] = d < DIM ? dS(q, mi[d]) : 1.0;
                Dm[d][q] = d < DIM ? dD(q, mi[d]) : 0.0;
            }
        double acc[DIM];
#pragma unroll
        for (int b = 0; b < DIM; ++b) acc[b] = 0.0;
#pragma unroll 1
        for (int q2 = 0; q2 < NQZ; ++q2)
#pragma unroll 1
            for (int q1 = 0; q1 < 3; ++q1)
#pragma unroll
                for (int q0 = 0; q0 < 3; ++q0) {
                    const int64_t off = geo_off(geo, q0, cell, q1 + 3 * q2);
                    const double phin = Sn[0][q0] * Sn[1][q1] * Sn[2][q2];
                    const double phim = Sm[0][q0] * Sm[1][q1] * Sm[2][q2];
                    const double gn[3] = {Dn[0][q0] * Sn[1][q1] * Sn[2][q2], Sn[0][q0] * Dn[1][q1] * Sn[2][q2],
                                          Sn[0][q0] * Sn[1][q1] * Dn[2][q2]};
                    const double gm[3] = {Dm[0][q0] * Sm[1][q1] * Sm[2][q2], Sm[0][q0] * Dm[1][q1] * Sm[2][q2],
                                          Sm[0][q0] * Sm[1][q1] * Dm[2][q2]};
                    double Gn[3] = {0, 0, 0}, Gm[3] = {0, 0, 0};
#pragma unroll
                    for (int c = 0; c < DIM; ++c)
#pragma unroll
                        for (int e = 0; e < DIM; ++e) {
                            const double kk = K[(e * DIM + c) * plane + off];
                            Gn[c] += kk * gn[e];
                            Gm[c] += kk * gm[e];
                        }
                    const double cvisc = cv[off], cmass = cv[plane + off];
                    double dot = 0.0;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) dot += Gn[c] * Gm[c];
                    // corrector mode: rho phi_n (v° . grad phi_m) + r (v° . grad phi_n)(v° . grad phi_m)
                    double extra = 0.0;
                    if (cb) {
                        double cn = 0.0, cmv = 0.0;
#pragma unroll
                        for (int e = 0; e < DIM; ++e) {
                            const double be = cb[e * plane + off];
                            cn += gn[e] * be;
                            cmv += gm[e] * be;
                        }
                        extra = rho * phin * cmv + cs[off] * cn * cmv;
                    }
#pragma unroll
                    for (int b = 0; b < DIM; ++b) {
                        double v = 0.5 * cvisc * Gn[b] * Gm[a];
                        if (a == b) v += cmass * phin * phim + 0.5 * cvisc * dot + extra;
                        acc[b] += v;
                    }
                }
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const int col = vrow[b * nvn + vmap[cell * NLOC + m]];
            if (col >= 0) M[(int64_t)row * n + col] += acc[b];
        }
    } else {
        // B^T column / B row entries of pressure vertex kk of this cell
        const int kk = m - NLOC;
        const int ki[3] = {kk & 1, (kk >> 1) & 1, (kk >> 2) & 1};
        double P1[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 3; ++q) P1[d][q] = d < DIM ? dL(q, ki[d]) : 1.0;
        double acc = 0.0;
#pragma unroll 1
        for (int q2 = 0; q2 < NQZ; ++q2)
#pragma unroll 1
            for (int q1 = 0; q1 < 3; ++q1)
#pragma unroll
                for (int q0 = 0; q0 < 3; ++q0) {
                    const int64_t off = geo_off(geo, q0, cell, q1 + 3 * q2);
                    const double psi = P1[0][q0] * P1[1][q1] * P1[2][q2];
                    const double gn[3] = {Dn[0][q0] * Sn[1][q1] * Sn[2][q2], Sn[0][q0] * Dn[1][q1] * Sn[2][q2],
                                          Sn[0][q0] * Sn[1][q1] * Dn[2][q2]};
                    double G = 0.0;
#pragma unroll
                    for (int e = 0; e < DIM; ++e) G += K[(e * DIM + a) * plane + off] * gn[e];
                    acc += psi * G;
                }
        const int64_t prow = nfree_u + pmap[cell * NPL + kk];
        M[(int64_t)row * n + prow] += acc;
        M[prow * n + row] += acc;
    }
}

void launch_coarse_assemble_impl(const Level& L, const double* K, const double* cv, const int* vrow,
                                 int64_t nfree_u, double* M, int64_t n, hipStream_t s, bool conv) {
    const int nloc = L.dim == 3 ? 27 : 9, npl = L.dim == 3 ? 8 : 4;
    const double* cb = conv ? L.d_cb64 : nullptr;
    const double* cs = conv ? L.d_cs64 : nullptr;
    for (int ph = 0; ph < L.nphases(); ++ph)
        for (int xpar = 0; xpar < 2; ++xpar) {
            const int64_t cnt = (L.phase_off[ph + 1] - L.phase_off[ph]) * L.dim * nloc * (nloc + npl);
            if (cnt == 0) continue;
            if (L.dim == 3)
                hipLaunchKernelGGL(k_coarse_assemble<3>, dim3(nblocks(cnt, 64)), dim3(64), 0, s, L.phase_off[ph],
                                   L.phase_off[ph + 1], L.d_col2lex, L.cells[0], xpar, L.geo, L.nvn, L.plane(),
                                   L.d_vmap, L.d_pmap, K, cv, cb, cs, L.rho, vrow, nfree_u, M, n);
            else
                hipLaunchKernelGGL(k_coarse_assemble<2>, dim3(nblocks(cnt, 64)), dim3(64), 0, s, L.phase_off[ph],
                                   L.phase_off[ph + 1], L.d_col2lex, L.cells[0], xpar, L.geo, L.nvn, L.plane(),
                                   L.d_vmap, L.d_pmap, K, cv, cb, cs, L.rho, vrow, nfree_u, M, n);
        }
}

// Gauss-Jordan inversion with partial pivoting: per pivot step one single-workgroup
// launch (pivot search, row swap, copy of the pivot column, scaling of the pivot
// row) and one elimination launch over the whole matrix; the column swaps of the
// row pivoting are applied at the end as one permutation.
constexpr int kGjThreads = 1024;
__global__ __launch_bounds__(kGjThreads) void k_gj_prep(double* __restrict__ M, int64_t n, int64_t k,
                                                        int* __restrict__ piv, double* __restrict__ colk,
                                                        int* __restrict__ flag) {
    __shared__ double bv[kGjThreads];
    __shared__ int bi[kGjThreads];
    double best = -1.0;
    int bidx = (int)k;
    for (int64_t i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double v = fabs(M[i * n + k]);
        if (v > best) { best = v; bidx = (int)i; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double o = bv[threadIdx.x + st];
            const int oi = bi[threadIdx.x + st];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int64_t p = bi[0];
    if (threadIdx.x == 0) {
        piv[k] = (int)p;
        if (!(bv[0] > 0.0)) flag[0] = 1;
    }
    // swap rows k and p
    if (p != k)
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
            const double t = M[k * n + j];
            M[k * n + j] = M[p * n + j];
            M[p * n + j] = t;
        }
    __syncthreads();
    // pivot column (after the swap), then the scaled pivot row
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) colk[i] = M[i * n + k];
    __syncthreads();
    const double pv = M[k * n + k];
    __syncthreads();
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) M[k * n + j] = (j == k) ? 1.0 / pv : M[k * n + j] / pv;
}
__global__ void k_gj_eliminate(double* __restrict__ M, int64_t n, int64_t k, const double* __restrict__ colk) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * n) return;
    const int64_t i = id / n, j = id - (id / n) * n;
    if (i == k) return;
    const double f = colk[i];
    if (j == k) M[i * n + k] = -f * M[k * n + k];
    else M[i * n + j] -= f * M[k * n + j];
}
// the column swaps (k, piv[k]) for k = n-1 .. 0 compose to one permutation:
// column j of the result is column sigma[j] of the eliminated matrix
__global__ void k_gj_sigma(const int* __restrict__ piv, int64_t n, int* __restrict__ sigma) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int64_t j = 0; j < n; ++j) sigma[j] = (int)j;
    for (int64_t k = n - 1; k >= 0; --k) {
        const int64_t p = piv[k];
        const int t = sigma[k];
        sigma[k] = sigma[p];
        sigma[p] = t;
    }
}
__global__ void k_gj_permute(const double* __restrict__ M, int64_t n, const int* __restrict__ sigma,
                             double* __restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * n) return;
    const int64_t i = id / n, j = id - (id / n) * n;
    out[id] = M[i * n + sigma[j]];
}

// inverts M (n x n, row-major) in place; piv and sigma: n ints, colk: n doubles,
// tmp: n * n doubles of scratch
void launch_gj(double* M, int64_t n, int* piv, int* sigma, double* colk, double* tmp, int* flag, hipStream_t s) {
    if (n <= 0) return;
    for (int64_t k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_prep, dim3(1), dim3(kGjThreads), 0, s, M, n, k, piv, colk, flag);
        hipLaunchKernelGGL(k_gj_eliminate, dim3(nblocks(n * n)), dim3(TPB), 0, s, M, n, k, colk);
    }
    hipLaunchKernelGGL(k_gj_sigma, dim3(1), dim3(64), 0, s, piv, n, sigma);
    hipLaunchKernelGGL(k_gj_permute, dim3(nblocks(n * n)), dim3(TPB), 0, s, M, n, sigma, tmp);
    hipMemcpyAsync(M, tmp, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s);
}

// coarse apply: gather free dofs, dense GEMV with the inverse, scatter
template <typename T>
__global__ void k_coarse_gather(const int* __restrict__ uidx, int64_t nfu, int64_t np, const T* __restrict__ fu,
                                const double* __restrict__ fp, T* __restrict__ xin) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nfu) xin[i] = fu[uidx[i]];
    else if (i < nfu + np) xin[i] = (T)fp[i - nfu];
}
template <typename T>
__global__ void k_gemv(const T* __restrict__ A, const T* __restrict__ x, T* __restrict__ y, int64_t n) {
    // one 64-wide wavefront per row
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += 64) acc += (double)A[row * n + j] * (double)x[j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[row] = (T)acc;
}
template <typename T>
__global__ void k_coarse_scatter(const int* __restrict__ uidx, int64_t nfu, int64_t np, const T* __restrict__ xout,
                                 T* __restrict__ xu, double* __restrict__ xp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nfu) xu[uidx[i]] = xout[i];
    else if (i < nfu + np) xp[i - nfu] = (double)xout[i];
}

template <typename T>
void launch_coarse_apply_impl(const Coarse& C, const Level& L, const T* A, T* xin, T* xout, const T* f_u,
                              const double* f_p, T* x_u, double* x_p, hipStream_t s) {
    launch_fill<T>(x_u, T(0), L.nv, s);
    hipLaunchKernelGGL(k_coarse_gather<T>, dim3(nblocks(C.n)), dim3(TPB), 0, s, C.d_uidx, C.nfree_u, L.np, f_u, f_p,
                       xin);
    hipLaunchKernelGGL(k_gemv<T>, dim3((unsigned)((C.n + 3) / 4)), dim3(256), 0, s, A, xin, xout, C.n);
    hipLaunchKernelGGL(k_coarse_scatter<T>, dim3(nblocks(C.n)), dim3(TPB), 0, s, C.d_uidx, C.nfree_u, L.np, xout, x_u,
                       x_p);
}
template <typename T>
void launch_coarse_apply(const Coarse& C, const Level& L, const T* f_u, const double* f_p, T* x_u, double* x_p,
                         hipStream_t s) {
    if constexpr (sizeof(T) == 8)
        launch_coarse_apply_impl<T>(C, L, C.d_inv64, C.d_xin64, C.d_xout64, f_u, f_p, x_u, x_p, s);
    else
        launch_coarse_apply_impl<T>(C, L, C.d_inv32, C.d_xin32, C.d_xout32, f_u, f_p, x_u, x_p, s);
}
template void launch_coarse_apply<double>(const Coarse&, const Level&, const double*, const double*, double*, double*,
                                          hipStream_t);
// velocity-only coarse solve (the extension problem): U holds the inverse of the free
// velocity block of A_0
template <typename T>
void launch_coarse_apply_u(const Coarse& U, const Level& L, const T* f_u, T* x_u, hipStream_t s) {
    const T* A = nullptr;
    T *xin = nullptr, *xout = nullptr;
    if constexpr (sizeof(T) == 8) {
        A = U.d_inv64;
        xin = U.d_xin64;
        xout = U.d_xout64;
    } else {
        A = U.d_inv32;
        xin = U.d_xin32;
        xout = U.d_xout32;
    }
    launch_fill<T>(x_u, T(0), L.nv, s);
    hipLaunchKernelGGL(k_coarse_gather<T>, dim3(nblocks(U.n)), dim3(TPB), 0, s, U.d_uidx, U.nfree_u, (int64_t)0, f_u,
                       (const double*)nullptr, xin);
    hipLaunchKernelGGL(k_gemv<T>, dim3((unsigned)((U.n + 3) / 4)), dim3(256), 0, s, A, xin, xout, U.n);
    hipLaunchKernelGGL(k_coarse_scatter<T>, dim3(nblocks(U.n)), dim3(TPB), 0, s, U.d_uidx, U.nfree_u, (int64_t)0, xout,
                       x_u, (double*)nullptr);
}
template void launch_coarse_apply_u<double>(const Coarse&, const Level&, const double*, double*, hipStream_t);
template void launch_coarse_apply_u<float>(const Coarse&, const Level&, const float*, float*, hipStream_t);
template void launch_coarse_apply<float>(const Coarse&, const Level&, const float*, const double*, float*, double*,
                                         hipStream_t);

// ---------------------------------------------------------------- Krylov helpers (FP64)
// partial dots <V_j, w> for a group of kDotGroup basis vectors per block row, so that
// w is streamed once per group rather than once per vector
constexpr int kDotGroup = 8;
// Vector index mb (== number of basis vectors) stands for w itself when the total
// count m exceeds mb, which yields ||w||^2 in the same sweep.
__global__ void k_multi_dot_partial(const double* __restrict__ V, int64_t ldv, int mb, int m,
                                    const double* __restrict__ w, int64_t n, double* __restrict__ part) {
    __shared__ double sh[kDotGroup][TPB / 64];
    const int j0 = blockIdx.y * kDotGroup;
    const int ng = min(kDotGroup, m - j0);
    double acc[kDotGroup];
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) acc[g] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int g = 0; g < kDotGroup; ++g)
            if (g < ng) acc[g] += (j0 + g < mb ? V[(int64_t)(j0 + g) * ldv + i] : wi) * wi;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) {
        double v = acc[g];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (lane == 0) sh[g][wave] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < ng) {
        double sum = 0.0;
        for (int k = 0; k < TPB / 64; ++k) sum += sh[threadIdx.x][k];
        part[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] = sum;
    }
}
__global__ void k_multi_dot_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double sh[TPB];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[(int64_t)j * nb + i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[j] = s;
}
void launch_multi_dot(const double* V, int64_t ldv, int m, const double* w, int64_t n, double* partials, double* out,
                      hipStream_t s, bool with_norm) {
    const unsigned nb = 1024;
    const int mt = m + (with_norm ? 1 : 0);
    const unsigned groups = (unsigned)((mt + kDotGroup - 1) / kDotGroup);
    hipLaunchKernelGGL(k_multi_dot_partial, dim3(nb, groups), dim3(TPB), 0, s, V, ldv, m, mt, w, n, partials);
    hipLaunchKernelGGL(k_multi_dot_final, dim3(mt), dim3(TPB), 0, s, partials, (int)nb, out);
}
__global__ void k_multi_axpy(const double* __restrict__ V, int64_t ldv, int m, const double* __restrict__ coef,
                             double sign, double* __restrict__ w, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    int j = 0;
    for (; j + 8 <= m; j += 8) {
        double v[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) v[g] = V[(int64_t)(j + g) * ldv + i];
#pragma unroll
        for (int g = 0; g < 8; ++g) acc += coef[j + g] * v[g];
    }
    for (; j < m; ++j) acc += coef[j] * V[(int64_t)j * ldv + i];
    w[i] += sign * acc;
}
void launch_multi_axpy(const double* V, int64_t ldv, int m, const double* coef_dev, double sign, double* w, int64_t n,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(nblocks(n)), dim3(TPB), 0, s, V, ldv, m, coef_dev, sign, w, n);
}
constexpr int kAxpyBlocks = 4096;
// w += sign * sum_j coef[j] V_j, and ||w||^2 of the result in the same sweep; the
// basis loads are issued eight at a time so that each thread keeps several in flight
__global__ void k_multi_axpy_norm(const double* __restrict__ V, int64_t ldv, int m, const double* __restrict__ coef,
                                  double sign, double* __restrict__ w, int64_t n, double* __restrict__ part) {
    __shared__ double sh[TPB];
    double nrm = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        int j = 0;
        for (; j + 8 <= m; j += 8) {
            double v[8];
#pragma unroll
            for (int g = 0; g < 8; ++g) v[g] = V[(int64_t)(j + g) * ldv + i];
#pragma unroll
            for (int g = 0; g < 8; ++g) acc += coef[j + g] * v[g];
        }
        for (; j < m; ++j) acc += coef[j] * V[(int64_t)j * ldv + i];
        const double wn = w[i] + sign * acc;
        w[i] = wn;
        nrm += wn * wn;
    }
    const double t = block_sum(nrm, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}
void launch_multi_axpy_norm(const double* V, int64_t ldv, int m, const double* coef_dev, double sign, double* w,
                            int64_t n, double* partials, double* out_norm2, hipStream_t s) {
    hipLaunchKernelGGL(k_multi_axpy_norm, dim3(kAxpyBlocks), dim3(TPB), 0, s, V, ldv, m, coef_dev, sign, w, n,
                       partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(TPB), 0, s, partials, kAxpyBlocks, out_norm2);
}
__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}
__global__ void k_xpby(const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] + b * y[i];
}
void launch_xpby_host(const double* x, double b, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_xpby, dim3(nblocks(n)), dim3(TPB), 0, s, x, b, y, n);
}
template <typename T>
__global__ void k_add(T* __restrict__ x, const T* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += y[i];
}
template <typename T>
void launch_add(T* x, const T* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_add<T>, dim3(nblocks(n)), dim3(TPB), 0, s, x, y, n);
}
template void launch_add<double>(double*, const double*, int64_t, hipStream_t);
template void launch_add<float>(float*, const float*, int64_t, hipStream_t);
__global__ void k_clear_wall_bits(const uint4* __restrict__ in, uint4* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        uint4 v = in[i];
        v.x = 0u;
        out[i] = v;
    }
}
void launch_clear_wall_bits(const uint4* in, uint4* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_wall_bits, dim3(nblocks(n)), dim3(TPB), 0, s, in, out, n);
}
void launch_axpy_host(double a, const double* x, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(nblocks(n)), dim3(TPB), 0, s, a, x, y, n);
}
__global__ void k_scale(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}
void launch_scale_host(double a, const double* x, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3(nblocks(n)), dim3(TPB), 0, s, a, x, y, n);
}
__global__ void k_mul(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = a[i] * b[i];
}
void launch_mul(const double* a, const double* b, double* c, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_mul, dim3(nblocks(n)), dim3(TPB), 0, s, a, b, c, n);
}
__global__ void k_vsqrt(const double* __restrict__ a, double* __restrict__ c, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = sqrt(a[i]);
}
void launch_vsqrt(const double* a, double* c, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_vsqrt, dim3(nblocks(n)), dim3(TPB), 0, s, a, c, n);
}
// v_i = ((7919 i) mod 1021)/1021 - 1/2 on free dofs, 0 on wall dofs
__global__ void k_lanczos_start(int64_t nv, int64_t nvn, const uint8_t* __restrict__ wall, double* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const int64_t node = i % nvn;
    v[i] = wall[node] ? 0.0 : (double)((7919 * i) % 1021) / 1021.0 - 0.5;
}
void launch_lanczos_start(const Level& L, double* v, hipStream_t s) {
    hipLaunchKernelGGL(k_lanczos_start, dim3(nblocks(L.nv)), dim3(TPB), 0, s, L.nv, L.nvn, level_wall_mask(L), v);
}
__global__ void k_nonfinite(const double* __restrict__ x, int64_t n, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(x[i])) flag[0] = 1;
}
void launch_nonfinite(const double* x, int64_t n, int* flag, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_nonfinite, dim3(nblocks(n)), dim3(TPB), 0, s, x, n, flag);
}
__global__ void k_sub_into(const double* __restrict__ g, const double* __restrict__ mx, double* __restrict__ r,
                           int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = g[i] - mx[i];
}
void launch_sub_into(const double* g, const double* mx, double* r, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_into, dim3(nblocks(n)), dim3(TPB), 0, s, g, mx, r, n);
}
__global__ void k_recip(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = 1.0 / a[i];
}
void launch_recip(const double* a, double* b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_recip, dim3(nblocks(n)), dim3(TPB), 0, s, a, b, n);
}

}  // namespace fsi
