// Kernels of one GCSI_k(M_1, .., M_S) time step (Algorithm 1, Sec. 3.1.1) around the
// generalized-Stokes solve: the explicit displacement of the velocity splitting, the
// coefficients of the stress splitting, the right-hand sides g_vM (eq. form_g_j) and
// g_p (eq. form_g_p), the corrector's convective velocity with the streamline parameter
// of Sec. 3.2, and the boundary data of the extension Ext (Sec. 2).
//
// Readings of the paper (the library's documentation lists them with the entry points):
// the explicit solid stress is mu_s [-2 eps(sum_i alpha_i u^{n,i}) - (grad u#)^T grad u#]
// (the velocity splitting substituted into the solid stress of Sec. 2.3), moved to the
// right-hand side and tested with eps(v); the k = 2 predictor extrapolates the relative
// velocity, v° = 2 (v^{n,1} - w^{n,1}) - (v^{n,2} - w^{n,2}); the predictor's convective
// term is explicit as a whole; the volume correction differentiates the Q2 field u#
// on the reference cell.
#include <hip/hip_runtime.h>

#include "fsi_common.h"

namespace fsi {

namespace {

constexpr int TPB_G = 256;
inline unsigned nblk(int64_t n, int tpb = TPB_G) { return (unsigned)((n + tpb - 1) / tpb); }

// u_out = gt w - a1 u1 - a2 u2 on every velocity dof
__global__ void k_gcsi_disp(const double* __restrict__ w, const double* __restrict__ u1,
                            const double* __restrict__ u2, double gt, double a1, double a2, double* __restrict__ out,
                            int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = gt * w[i] - a1 * u1[i];
    if (u2) v -= a2 * u2[i];
    out[i] = v;
}

// the same combination at the mesh vertices (Q2 node (2i, 2j, 2k)): [dim][n_vert]
__global__ void k_gcsi_disp_vertices(const double* __restrict__ w, const double* __restrict__ u1,
                                     const double* __restrict__ u2, double gt, double a1, double a2,
                                     double* __restrict__ out, int pnx, int pny, int64_t nvert, int vnx, int vny,
                                     int64_t nvn, int dim) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)dim * nvert) return;
    const int c = (int)(i / nvert);
    const int64_t v = i - (int64_t)c * nvert;
    const int64_t vx = v % pnx, vy = (v / pnx) % pny, vz = v / ((int64_t)pnx * pny);
    const int64_t node = c * nvn + 2 * vx + (int64_t)vnx * (2 * vy + (int64_t)vny * 2 * vz);
    double r = gt * w[node] - a1 * u1[node];
    if (u2) r -= a2 * u2[node];
    out[i] = r;
}

// c_m = rho / (gamma tau), eta = eta_f or gamma tau mu_s, per point
__global__ void k_gcsi_coef(const uint8_t* __restrict__ solid, double cm_f, double cm_s, double eta_f, double eta_s,
                            double* __restrict__ cm, double* __restrict__ eta, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool s = solid[i] != 0;
    cm[i] = s ? cm_s : cm_f;
    eta[i] = s ? eta_s : eta_f;
}

// g = v on the fixed nodes, 0 elsewhere
__global__ void k_fixed_values(const uint8_t* __restrict__ fixed, const double* __restrict__ v, double* __restrict__ g,
                               int64_t nvn, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    g[i] = fixed[i % nvn] ? v[i] : 0.0;
}

// right-hand side: one 64-thread workgroup per cell.  Threads 0..NL-1 (NL = 3^dim local
// nodes and as many Gauss points) load the cell's nodal combinations and then own one Gauss
// point each (Jacobian of the multilinear map through the vertex displacement, physical
// gradients, the integrands scaled by det(J) w), then one test node each (sum over the
// points, atomic add into g_u, wall rows left zero); threads NL..NL+2^dim-1 own the cell's
// vertices (g_p).
template <int DIM>
__global__ __launch_bounds__(64) void k_gcsi_rhs(GcsiRhsArgs a) {
    constexpr int NL = DIM == 3 ? 27 : 9, NV = DIM == 3 ? 8 : 4;
    const int64_t c = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t cx = c % a.nx, cy = (c / a.nx) % a.ny, cz = DIM == 3 ? c / ((int64_t)a.nx * a.ny) : 0;
    __shared__ double s_uh[3][27], s_us[3][27], s_vs[3][27], s_vt[3][27], s_vc[3][27];
    __shared__ double s_d[3][8];
    __shared__ double s_F[27][3], s_T[27][9], s_Ji[27][9], s_gp[27];
    auto loc = [](int i, int& ix, int& iy, int& iz) {
        ix = i % 3;
        iy = (i / 3) % 3;
        iz = DIM == 3 ? i / 9 : 0;
    };
    auto node_of = [&](int i) -> int64_t {
        int ix, iy, iz;
        loc(i, ix, iy, iz);
        return (2 * cx + ix) + (int64_t)a.vnx * ((2 * cy + iy) + (int64_t)a.vny * (2 * cz + iz));
    };
    auto vertex_of = [&](int v) -> int64_t {
        const int vx = v & 1, vy = (v >> 1) & 1, vz = DIM == 3 ? v >> 2 : 0;
        return (cx + vx) + (int64_t)a.pnx * ((cy + vy) + (int64_t)a.pny * (cz + vz));
    };
    if (t < NL) {
        const int64_t node = node_of(t);
        for (int k = 0; k < DIM; ++k) {
            const int64_t n = k * a.nvn + node;
            s_uh[k][t] = a.uh[n];
            s_us[k][t] = a.a1 * a.u1[n] + (a.u2 ? a.a2 * a.u2[n] : 0.0);
            const double v1 = a.v1[n], v2 = a.v2 ? a.v2[n] : 0.0;
            s_vs[k][t] = a.a1 * v1 + a.a2 * v2;
            if (a.predictor) {
                const double w1 = a.w1[n];
                if (a.v2) {
                    s_vt[k][t] = 2.0 * v1 - v2;
                    s_vc[k][t] = 2.0 * (v1 - w1) - (v2 - a.w2[n]);
                } else {
                    s_vt[k][t] = v1;
                    s_vc[k][t] = v1 - w1;
                }
            }
        }
    } else if (t < NL + NV) {
        const int v = t - NL;
        const int64_t vtx = vertex_of(v);
        for (int k = 0; k < DIM; ++k) s_d[k][v] = a.disp[k * a.nvert + vtx];
    }
    __syncthreads();
    if (t < NL) {
        const int q = t;
        int qx, qy, qz;
        loc(q, qx, qy, qz);
        // J[r][b] = h_r d_rb + sum_v d_v[r] d psi_v / d xi_b
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int r = 0; r < DIM; ++r) J[r][r] = a.h[r];
        for (int v = 0; v < NV; ++v) {
            const int vx = v & 1, vy = (v >> 1) & 1, vz = DIM == 3 ? v >> 2 : 0;
            const double Lx = Tab::L[qx][vx], Ly = Tab::L[qy][vy], Lz = DIM == 3 ? Tab::L[qz][vz] : 1.0;
            const double dp[3] = {(vx ? 1.0 : -1.0) * Ly * Lz, Lx * (vy ? 1.0 : -1.0) * Lz, Lx * Ly * (vz ? 1.0 : -1.0)};
            for (int r = 0; r < DIM; ++r)
                for (int b = 0; b < DIM; ++b) J[r][b] += s_d[r][v] * dp[b];
        }
        double Ji[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // Ji[b][x] = d xi_b / d x_x
        double det;
        if constexpr (DIM == 3) {
            double adj[3][3];
            adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
            adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
            adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
            adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
            const double idet = 1.0 / det;
            for (int b = 0; b < 3; ++b)
                for (int x = 0; x < 3; ++x) Ji[b][x] = adj[b][x] * idet;
        } else {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double idet = 1.0 / det;
            Ji[0][0] = J[1][1] * idet;
            Ji[0][1] = -J[0][1] * idet;
            Ji[1][0] = -J[1][0] * idet;
            Ji[1][1] = J[0][0] * idet;
        }
        const double wq = Tab::W[qx] * Tab::W[qy] * (DIM == 3 ? Tab::W[qz] : 1.0);
        const double wd = wq * det;
        // reference gradients (d / d xi_b) and point values
        double guh[3][3] = {}, gus[3][3] = {}, gvt[3][3] = {}, vs[3] = {}, vc[3] = {};
        for (int i = 0; i < NL; ++i) {
            int ix, iy, iz;
            loc(i, ix, iy, iz);
            const double sx = Tab::S[qx][ix], sy = Tab::S[qy][iy], sz = DIM == 3 ? Tab::S[qz][iz] : 1.0;
            const double dphi[3] = {Tab::D[qx][ix] * sy * sz, sx * Tab::D[qy][iy] * sz,
                                    DIM == 3 ? sx * sy * Tab::D[qz][iz] : 0.0};
            const double phi = sx * sy * sz;
            for (int k = 0; k < DIM; ++k) {
                vs[k] += phi * s_vs[k][i];
                for (int b = 0; b < DIM; ++b) {
                    guh[k][b] += s_uh[k][i] * dphi[b];
                    gus[k][b] += s_us[k][i] * dphi[b];
                }
                if (a.predictor) {
                    vc[k] += phi * s_vc[k][i];
                    for (int b = 0; b < DIM; ++b) gvt[k][b] += s_vt[k][i] * dphi[b];
                }
            }
        }
        // physical gradients: P[k][x] = sum_b R[k][b] Ji[b][x]
        double gh[3][3] = {}, gs[3][3] = {};
        for (int k = 0; k < DIM; ++k)
            for (int x = 0; x < DIM; ++x)
                for (int b = 0; b < DIM; ++b) {
                    gh[k][x] += guh[k][b] * Ji[b][x];
                    gs[k][x] += gus[k][b] * Ji[b][x];
                }
        const bool solid = a.solid[c * NL + q] != 0;
        const double rho = solid ? a.rho_s : a.rho_f;
        for (int k = 0; k < DIM; ++k) {
            double f = rho * (a.body[k] - vs[k] / a.gt);
            if (a.predictor) {
                double cv = 0.0;
                for (int x = 0; x < DIM; ++x) {
                    double gv = 0.0;
                    for (int b = 0; b < DIM; ++b) gv += gvt[k][b] * Ji[b][x];
                    cv += gv * vc[x];
                }
                f -= rho * cv;
            }
            s_F[q][k] = wd * f;
        }
        for (int k = 0; k < DIM; ++k)
            for (int x = 0; x < DIM; ++x) {
                double T = 0.0;
                if (solid) {
                    double tq = 0.0;
                    for (int b = 0; b < DIM; ++b) tq += gh[b][k] * gh[b][x];
                    T = a.mu_s * (gs[k][x] + gs[x][k] + tq);
                }
                s_T[q][k * 3 + x] = wd * T;
                s_Ji[q][k * 3 + x] = Ji[k][x];
            }
        // volume correction: J# = det(I + grad-hat u#), grad-hat = d/d xi / h
        double gp = 0.0;
        if (solid && a.inv_etaV > 0.0) {
            double F[3][3];
            for (int k = 0; k < DIM; ++k)
                for (int b = 0; b < DIM; ++b) F[k][b] = (k == b ? 1.0 : 0.0) + guh[k][b] / a.h[b];
            double Jh, hv;
            if constexpr (DIM == 3) {
                Jh = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                     F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
                hv = a.h[0] * a.h[1] * a.h[2];
            } else {
                Jh = F[0][0] * F[1][1] - F[0][1] * F[1][0];
                hv = a.h[0] * a.h[1];
            }
            gp = -a.inv_etaV * (Jh - 1.0) * wq * hv;
        }
        s_gp[q] = gp;
    }
    __syncthreads();
    if (t < NL) {
        const int i = t;
        int ix, iy, iz;
        loc(i, ix, iy, iz);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < NL; ++q) {
            int qx, qy, qz;
            loc(q, qx, qy, qz);
            const double sx = Tab::S[qx][ix], sy = Tab::S[qy][iy], sz = DIM == 3 ? Tab::S[qz][iz] : 1.0;
            const double dphi[3] = {Tab::D[qx][ix] * sy * sz, sx * Tab::D[qy][iy] * sz,
                                    DIM == 3 ? sx * sy * Tab::D[qz][iz] : 0.0};
            const double phi = sx * sy * sz;
            double gx[3] = {0.0, 0.0, 0.0};
            for (int x = 0; x < DIM; ++x)
                for (int b = 0; b < DIM; ++b) gx[x] += dphi[b] * s_Ji[q][b * 3 + x];
            for (int k = 0; k < DIM; ++k) {
                double sacc = s_F[q][k] * phi;
                for (int x = 0; x < DIM; ++x) sacc += s_T[q][k * 3 + x] * gx[x];
                acc[k] += sacc;
            }
        }
        const int64_t node = node_of(i);
        if (!a.wall[node])
            for (int k = 0; k < DIM; ++k) atomicAdd(&a.g_u[k * a.nvn + node], acc[k]);
    } else if (t < NL + NV && a.inv_etaV > 0.0) {
        const int v = t - NL, vx = v & 1, vy = (v >> 1) & 1, vz = DIM == 3 ? v >> 2 : 0;
        double acc = 0.0;
        for (int q = 0; q < NL; ++q) {
            int qx, qy, qz;
            loc(q, qx, qy, qz);
            acc += s_gp[q] * Tab::L[qx][vx] * Tab::L[qy][vy] * (DIM == 3 ? Tab::L[qz][vz] : 1.0);
        }
        atomicAdd(&a.g_p[vertex_of(v)], acc);
    }
}

// corrector convection inputs of one level: v° = v# - w# (fine nodal fields read at the
// level's nodes, stride s) at the Gauss points, and the Peclet-law streamline parameter
// per cell (Sec. 3.2, p1 = 2): Pe = |v°|_max h_K / (2 eta_mean p1),
// r = h_K / (2 |v°|_max p1) (coth Pe - 1/Pe) for Pe >= 1, else 0.  Two cells per
// 64-thread workgroup, one Gauss point per thread; vconv is [n_cells][3^dim][dim].
template <int DIM>
__global__ __launch_bounds__(64) void k_gcsi_conv(const double* __restrict__ vh, const double* __restrict__ wh,
                                                  const double* __restrict__ eta, int nx, int ny, int64_t nc,
                                                  int stride, int vnx_f, int vny_f, int64_t nvn_f, double hK,
                                                  double* __restrict__ vconv, double* __restrict__ r) {
    constexpr int NL = DIM == 3 ? 27 : 9;
    const int half = threadIdx.x >> 5, t = threadIdx.x & 31;
    const int64_t c = (int64_t)blockIdx.x * 2 + half;
    __shared__ double s_v[2][3][27];
    __shared__ double s_m[2][27], s_e[2][27];
    const bool on = c < nc;
    const int64_t cx = on ? c % nx : 0, cy = on ? (c / nx) % ny : 0, cz = (on && DIM == 3) ? c / ((int64_t)nx * ny) : 0;
    if (on && t < NL) {
        const int lx = t % 3, ly = (t / 3) % 3, lz = DIM == 3 ? t / 9 : 0;
        const int64_t node = (int64_t)stride * (2 * cx + lx) +
                             (int64_t)vnx_f * ((int64_t)stride * (2 * cy + ly) + (int64_t)vny_f * stride * (2 * cz + lz));
        for (int k = 0; k < DIM; ++k) s_v[half][k][t] = vh[k * nvn_f + node] - wh[k * nvn_f + node];
    }
    __syncthreads();
    if (on && t < NL) {
        const int q = t, qx = q % 3, qy = (q / 3) % 3, qz = DIM == 3 ? q / 9 : 0;
        double v[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < NL; ++i) {
            const double phi = Tab::S[qx][i % 3] * Tab::S[qy][(i / 3) % 3] * (DIM == 3 ? Tab::S[qz][i / 9] : 1.0);
            for (int k = 0; k < DIM; ++k) v[k] += phi * s_v[half][k][i];
        }
        double m2 = 0.0;
        for (int k = 0; k < DIM; ++k) {
            vconv[(c * NL + q) * DIM + k] = v[k];
            m2 += v[k] * v[k];
        }
        s_m[half][q] = sqrt(m2);
        s_e[half][q] = eta[c * NL + q];
    }
    __syncthreads();
    if (on && t < NL) {
        double vmax = 0.0, es = 0.0;
        for (int q = 0; q < NL; ++q) {
            vmax = fmax(vmax, s_m[half][q]);
            es += s_e[half][q];
        }
        const double mu = es / NL, p1 = 2.0;
        const double pe = vmax * hK / (2.0 * mu * p1);
        double rr = 0.0;
        if (pe >= 1.0) rr = hK / (2.0 * vmax * p1) * (1.0 / tanh(pe) - 1.0 / pe);
        r[c * NL + t] = rr;
    }
}

}  // namespace

void launch_gcsi_displacement(const Level& L, const double* w, const double* u1, const double* u2, double gt, double a1,
                              double a2, double* u_out, double* disp_out, hipStream_t s) {
    if (u_out) hipLaunchKernelGGL(k_gcsi_disp, dim3(nblk(L.nv)), dim3(TPB_G), 0, s, w, u1, u2, gt, a1, a2, u_out, L.nv);
    if (disp_out)
        hipLaunchKernelGGL(k_gcsi_disp_vertices, dim3(nblk((int64_t)L.dim * L.nvert)), dim3(TPB_G), 0, s, w, u1, u2, gt,
                           a1, a2, disp_out, L.pnodes[0], L.pnodes[1], L.nvert, L.vnodes[0], L.vnodes[1], L.nvn, L.dim);
}

void launch_gcsi_coefficients(const uint8_t* solid, double cm_f, double cm_s, double eta_f, double eta_s, double* cm,
                              double* eta, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_gcsi_coef, dim3(nblk(n)), dim3(TPB_G), 0, s, solid, cm_f, cm_s, eta_f, eta_s, cm, eta, n);
}

void launch_fixed_values(const Level& L, const uint8_t* fixed, const double* v, double* g, hipStream_t s) {
    hipLaunchKernelGGL(k_fixed_values, dim3(nblk(L.nv)), dim3(TPB_G), 0, s, fixed, v, g, L.nvn, L.nv);
}

void launch_gcsi_rhs(const GcsiRhsArgs& a, int dim, int64_t nc, hipStream_t s) {
    if (dim == 3) hipLaunchKernelGGL(k_gcsi_rhs<3>, dim3((unsigned)nc), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_gcsi_rhs<2>, dim3((unsigned)nc), dim3(64), 0, s, a);
}

void launch_gcsi_convection(const Level& L, const Level& F, const double* vh, const double* wh, const double* eta,
                            int stride, double* vconv, double* r, hipStream_t s) {
    double h2 = 0.0;
    for (int d = 0; d < L.dim; ++d) h2 += L.h[d] * L.h[d];
    const double hK = sqrt(h2);
    if (L.dim == 3)
        hipLaunchKernelGGL(k_gcsi_conv<3>, dim3((unsigned)((L.nc + 1) / 2)), dim3(64), 0, s, vh, wh, eta, L.cells[0],
                           L.cells[1], L.nc, stride, F.vnodes[0], F.vnodes[1], F.nvn, hK, vconv, r);
    else
        hipLaunchKernelGGL(k_gcsi_conv<2>, dim3((unsigned)((L.nc + 1) / 2)), dim3(64), 0, s, vh, wh, eta, L.cells[0],
                           L.cells[1], L.nc, stride, F.vnodes[0], F.vnodes[1], F.nvn, hK, vconv, r);
}

}  // namespace fsi
