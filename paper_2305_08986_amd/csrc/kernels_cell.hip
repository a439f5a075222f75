// Matrix-free cell operator of the Q2-Q1 generalized-Stokes system (Sec. 4
// block system; forms a and b of Sec. 3.1.1 in predictor mode):
//
//   A: v_K = int c_m u.phi + 2 eta eps(u):eps(phi)      (mass + variable viscosity)
//   B: q_K = int psi div u                               (discrete divergence)
//   B^T: v_K += int p div phi
//
// evaluated by sum factorisation on the ALE-mapped cell (Sec. 3.2).  Per
// quadrature point the kernel reads K = det(J) w_q J^{-1} and the scalars
// cvisc = 2 eta / (det J w_q), cmass = c_m det J w_q; with H = (grad-hat u) K
// (= det J w_q grad u) the viscous flux is F = cvisc sym(H) K^T and the
// divergence is tr(H), so A, B and B^T share the same 9(+2) stored values.
//
// Thread layout (64-wide wavefronts): one thread per line of 3 points of a
// cell, NT = 3^(dim-1) threads per cell, CPW cells per wavefront.  The three
// 1D contraction sweeps run in registers; between sweep directions the lines
// are transposed through LDS (wavefront-private).  Cells of one colour share
// no node, so the scatter is a plain read-modify-write (no atomics); the host
// launches the 2^dim colours one after another.
#include "fsi_common.h"

namespace fsi {

template <typename T> __device__ __forceinline__ T cS(int q, int n) { return T(Tab::S[q][n]); }
template <typename T> __device__ __forceinline__ T cD(int q, int n) { return T(Tab::D[q][n]); }
template <typename T> __device__ __forceinline__ T cL(int q, int a) { return T(Tab::L[q][a]); }
// Q1 basis at a runtime Gauss index
template <typename T> __device__ __forceinline__ T rL(int q, int a) {
    const T lo = T(0.5 - kS15), hi = T(0.5 + kS15);
    if (q == 1) return T(0.5);
    return ((q == 0) == (a == 0)) ? hi : lo;
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t x = b & 7, qd = nb >> 3, r = nb & 7;
    const int64_t base = (x < r) ? x * (qd + 1) : r * (qd + 1) + (x - r) * qd;
    return base + (b >> 3);
}

template <typename T>
struct CellArgs {
    int64_t cbeg, cend, nc, nvn, plane;
    const int* __restrict__ vmap;
    const uint32_t* __restrict__ dmask;
    const int* __restrict__ pmap;
    const T* __restrict__ K;
    const T* __restrict__ cv;
    const T* __restrict__ u;
    const double* __restrict__ p;
    T* __restrict__ v;
    double* __restrict__ q;
};

// ============================================================== 3D
template <typename T, int MODE, int WPB, bool REMAP>
__global__ __launch_bounds__(64 * WPB) void cell3d(CellArgs<T> a) {
    constexpr int NT = 9, CPW = 7, NLOC = 27, BUF = 243;
    constexpr bool FWD = (MODE & (OP_A | OP_B)) != 0;
    constexpr bool BWD = (MODE & (OP_A | OP_BT)) != 0;
    __shared__ T sbuf[WPB][CPW][BUF];
    __shared__ double pbuf[(MODE & OP_B) ? WPB : 1][CPW][NT][8];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / NT, t = lane - slot * NT;
    const bool inwave = slot < CPW;
    const int64_t lb = REMAP ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t cell = a.cbeg + (lb * WPB + wave) * CPW + slot;
    const bool act = inwave && cell < a.cend;
    T* B = sbuf[wave][inwave ? slot : 0];
    const int64_t P = a.plane;

    // ---------------- forward: values and reference gradients at the 27 points
    T val[3][3], g0[3][3], g1[3][3], g2[3][3];   // [comp][qx] at this thread's (qy,qz)
    if constexpr (FWD) {
        T uu[3][3];
        if (act) {
            const uint32_t dm = a.dmask[cell];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ln = t + 9 * k;
                const int node = a.vmap[cell * NLOC + ln];
                const bool wall = (dm >> ln) & 1u;
#pragma unroll
                for (int c = 0; c < 3; ++c) uu[c][k] = wall ? T(0) : a.u[c * a.nvn + node];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) uu[c][k] = T(0);
        }
        // stage A (t = i + 3j): z-sweep
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int qz = 0; qz < 3; ++qz) {
                    T s = T(0), d = T(0);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        s += cS<T>(qz, k) * uu[c][k];
                        d += cD<T>(qz, k) * uu[c][k];
                    }
                    B[((c * 2 + 0) * 3 + qz) * 9 + t] = s;
                    B[((c * 2 + 1) * 3 + qz) * 9 + t] = d;
                }
        }
        __syncthreads();
        // stage B (t = i + 3 qz): y-sweep
        const int ib = t % 3, qzb = t / 3;
        T ya[3][3], yb[3][3], yc[3][3];
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T zs[3], zd[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    zs[j] = B[((c * 2 + 0) * 3 + qzb) * 9 + ib + 3 * j];
                    zd[j] = B[((c * 2 + 1) * 3 + qzb) * 9 + ib + 3 * j];
                }
#pragma unroll
                for (int qy = 0; qy < 3; ++qy) {
                    T s = T(0), d = T(0), e = T(0);
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        s += cS<T>(qy, j) * zs[j];
                        d += cD<T>(qy, j) * zs[j];
                        e += cS<T>(qy, j) * zd[j];
                    }
                    ya[c][qy] = s;
                    yb[c][qy] = d;
                    yc[c][qy] = e;
                }
            }
        }
        __syncthreads();
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int qy = 0; qy < 3; ++qy) {
                    B[((c * 3 + 0) * 9 + qy + 3 * qzb) * 3 + ib] = ya[c][qy];
                    B[((c * 3 + 1) * 9 + qy + 3 * qzb) * 3 + ib] = yb[c][qy];
                    B[((c * 3 + 2) * 9 + qy + 3 * qzb) * 3 + ib] = yc[c][qy];
                }
        }
        __syncthreads();
        // stage C (t = qy + 3 qz): x-sweep
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T ga[3], gb[3], gc[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ga[i] = inwave ? B[((c * 3 + 0) * 9 + t) * 3 + i] : T(0);
                gb[i] = inwave ? B[((c * 3 + 1) * 9 + t) * 3 + i] : T(0);
                gc[i] = inwave ? B[((c * 3 + 2) * 9 + t) * 3 + i] : T(0);
            }
#pragma unroll
            for (int qx = 0; qx < 3; ++qx) {
                T s = T(0), d = T(0), e = T(0), f = T(0);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    s += cS<T>(qx, i) * ga[i];
                    d += cD<T>(qx, i) * ga[i];
                    e += cS<T>(qx, i) * gb[i];
                    f += cS<T>(qx, i) * gc[i];
                }
                val[c][qx] = s;
                g0[c][qx] = d;
                g1[c][qx] = e;
                g2[c][qx] = f;
            }
        }
    }

    const int qy = t % 3, qz = t / 3;
    // ---------------- pressure at the quadrature points (B^T)
    T pq[3] = {T(0), T(0), T(0)};
    if constexpr ((MODE & OP_BT) != 0) {
        if (act) {
            double pv[8];
#pragma unroll
            for (int n = 0; n < 8; ++n) pv[n] = a.p[a.pmap[cell * 8 + n]];
            const T ly0 = rL<T>(qy, 0), ly1 = rL<T>(qy, 1), lz0 = rL<T>(qz, 0), lz1 = rL<T>(qz, 1);
            T tx[2];
#pragma unroll
            for (int ax = 0; ax < 2; ++ax)
                tx[ax] = ly0 * lz0 * T(pv[ax]) + ly1 * lz0 * T(pv[ax + 2]) + ly0 * lz1 * T(pv[ax + 4]) +
                         ly1 * lz1 * T(pv[ax + 6]);
#pragma unroll
            for (int qx = 0; qx < 3; ++qx) pq[qx] = cL<T>(qx, 0) * tx[0] + cL<T>(qx, 1) * tx[1];
        }
    }

    // ---------------- quadrature-point operation
    T F0[3][3], F1[3][3], F2[3][3], Fv[3][3];   // [comp][qx]
    T divq[3];
#pragma unroll
    for (int qx = 0; qx < 3; ++qx) {
        T Km[3][3];
        const int64_t off = ((int64_t)qx * a.nc + cell) * NT + t;
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) Km[b][aa] = act ? a.K[(b * 3 + aa) * P + off] : T(0);
        T Tm[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) Tm[c][aa] = T(0);
        divq[qx] = T(0);
        if constexpr (FWD) {
            T H[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int aa = 0; aa < 3; ++aa)
                    H[c][aa] = g0[c][qx] * Km[0][aa] + g1[c][qx] * Km[1][aa] + g2[c][qx] * Km[2][aa];
            if constexpr ((MODE & OP_B) != 0) divq[qx] = H[0][0] + H[1][1] + H[2][2];
            if constexpr ((MODE & OP_A) != 0) {
                const T cvisc = act ? a.cv[off] : T(0);
                const T cmass = act ? a.cv[P + off] : T(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Tm[c][c] = cvisc * H[c][c];
                    Fv[c][qx] = cmass * val[c][qx];
                }
                const T e01 = T(0.5) * cvisc * (H[0][1] + H[1][0]);
                const T e02 = T(0.5) * cvisc * (H[0][2] + H[2][0]);
                const T e12 = T(0.5) * cvisc * (H[1][2] + H[2][1]);
                Tm[0][1] = e01; Tm[1][0] = e01;
                Tm[0][2] = e02; Tm[2][0] = e02;
                Tm[1][2] = e12; Tm[2][1] = e12;
            }
        }
        if constexpr ((MODE & OP_A) == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Fv[c][qx] = T(0);
        }
        if constexpr ((MODE & OP_BT) != 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Tm[c][c] += pq[qx];
        }
        if constexpr (BWD) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                F0[c][qx] = Tm[c][0] * Km[0][0] + Tm[c][1] * Km[0][1] + Tm[c][2] * Km[0][2];
                F1[c][qx] = Tm[c][0] * Km[1][0] + Tm[c][1] * Km[1][1] + Tm[c][2] * Km[1][2];
                F2[c][qx] = Tm[c][0] * Km[2][0] + Tm[c][1] * Km[2][1] + Tm[c][2] * Km[2][2];
            }
        }
    }

    // ---------------- divergence tested with the Q1 basis (B)
    if constexpr ((MODE & OP_B) != 0) {
        T r[2];
#pragma unroll
        for (int ax = 0; ax < 2; ++ax)
            r[ax] = cL<T>(0, ax) * divq[0] + cL<T>(1, ax) * divq[1] + cL<T>(2, ax) * divq[2];
        if (inwave) {
            const T ly[2] = {rL<T>(qy, 0), rL<T>(qy, 1)};
            const T lz[2] = {rL<T>(qz, 0), rL<T>(qz, 1)};
#pragma unroll
            for (int cz = 0; cz < 2; ++cz)
#pragma unroll
                for (int by = 0; by < 2; ++by)
#pragma unroll
                    for (int ax = 0; ax < 2; ++ax)
                        pbuf[wave][slot][t][ax + 2 * by + 4 * cz] = double(ly[by] * lz[cz] * r[ax]);
        }
        __syncthreads();
        if (act && t < 8) {
            double s = 0.0;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) s += pbuf[wave][slot][tt][t];
            const int node = a.pmap[cell * 8 + t];
            a.q[node] += s;
        }
    }

    // ---------------- backward: test with the gradients / values of the Q2 basis
    if constexpr (BWD) {
        T wa[3][3], wb[3][3], wc[3][3];   // [comp][i]
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T s = T(0), d = T(0), e = T(0);
#pragma unroll
                for (int qx = 0; qx < 3; ++qx) {
                    s += cS<T>(qx, i) * Fv[c][qx] + cD<T>(qx, i) * F0[c][qx];
                    d += cS<T>(qx, i) * F1[c][qx];
                    e += cS<T>(qx, i) * F2[c][qx];
                }
                wa[c][i] = s;
                wb[c][i] = d;
                wc[c][i] = e;
            }
        __syncthreads();
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    B[((c * 3 + 0) * 9 + t) * 3 + i] = wa[c][i];
                    B[((c * 3 + 1) * 9 + t) * 3 + i] = wb[c][i];
                    B[((c * 3 + 2) * 9 + t) * 3 + i] = wc[c][i];
                }
        }
        __syncthreads();
        const int ib = t % 3, qzb = t / 3;
        T vs[3][3], vd[3][3];   // [comp][j]
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T WA[3], WB[3], WC[3];
#pragma unroll
            for (int q2 = 0; q2 < 3; ++q2) {
                WA[q2] = inwave ? B[((c * 3 + 0) * 9 + q2 + 3 * qzb) * 3 + ib] : T(0);
                WB[q2] = inwave ? B[((c * 3 + 1) * 9 + q2 + 3 * qzb) * 3 + ib] : T(0);
                WC[q2] = inwave ? B[((c * 3 + 2) * 9 + q2 + 3 * qzb) * 3 + ib] : T(0);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T s = T(0), d = T(0);
#pragma unroll
                for (int q2 = 0; q2 < 3; ++q2) {
                    s += cS<T>(q2, j) * WA[q2] + cD<T>(q2, j) * WB[q2];
                    d += cS<T>(q2, j) * WC[q2];
                }
                vs[c][j] = s;
                vd[c][j] = d;
            }
        }
        __syncthreads();
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    B[((c * 2 + 0) * 3 + qzb) * 9 + ib + 3 * j] = vs[c][j];
                    B[((c * 2 + 1) * 3 + qzb) * 9 + ib + 3 * j] = vd[c][j];
                }
        }
        __syncthreads();
        if (act) {
            const uint32_t dm = a.dmask[cell];
            T out[3][3];   // [comp][k]
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T VS[3], VD[3];
#pragma unroll
                for (int q3 = 0; q3 < 3; ++q3) {
                    VS[q3] = B[((c * 2 + 0) * 3 + q3) * 9 + t];
                    VD[q3] = B[((c * 2 + 1) * 3 + q3) * 9 + t];
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T s = T(0);
#pragma unroll
                    for (int q3 = 0; q3 < 3; ++q3) s += cS<T>(q3, k) * VS[q3] + cD<T>(q3, k) * VD[q3];
                    out[c][k] = s;
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int ln = t + 9 * k;
                if ((dm >> ln) & 1u) continue;
                const int node = a.vmap[cell * NLOC + ln];
#pragma unroll
                for (int c = 0; c < 3; ++c) a.v[c * a.nvn + node] += out[c][k];
            }
        }
    }
}

// ============================================================== 2D
template <typename T, int MODE, int WPB, bool REMAP>
__global__ __launch_bounds__(64 * WPB) void cell2d(CellArgs<T> a) {
    constexpr int NT = 3, CPW = 21, NLOC = 9, BUF = 36;
    constexpr bool FWD = (MODE & (OP_A | OP_B)) != 0;
    constexpr bool BWD = (MODE & (OP_A | OP_BT)) != 0;
    __shared__ T sbuf[WPB][CPW][BUF];
    __shared__ double pbuf[(MODE & OP_B) ? WPB : 1][CPW][NT][4];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / NT, t = lane - slot * NT;
    const bool inwave = slot < CPW;
    const int64_t lb = REMAP ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t cell = a.cbeg + (lb * WPB + wave) * CPW + slot;
    const bool act = inwave && cell < a.cend;
    T* B = sbuf[wave][inwave ? slot : 0];
    const int64_t P = a.plane;

    T val[2][3], g0[2][3], g1[2][3];
    if constexpr (FWD) {
        T uu[2][3];
        if (act) {
            const uint32_t dm = a.dmask[cell];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int ln = t + 3 * j;
                const int node = a.vmap[cell * NLOC + ln];
                const bool wall = (dm >> ln) & 1u;
#pragma unroll
                for (int c = 0; c < 2; ++c) uu[c][j] = wall ? T(0) : a.u[c * a.nvn + node];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j) uu[c][j] = T(0);
        }
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int qy = 0; qy < 3; ++qy) {
                    T s = T(0), d = T(0);
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        s += cS<T>(qy, j) * uu[c][j];
                        d += cD<T>(qy, j) * uu[c][j];
                    }
                    B[((c * 2 + 0) * 3 + qy) * 3 + t] = s;
                    B[((c * 2 + 1) * 3 + qy) * 3 + t] = d;
                }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            T sa[3], da[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                sa[i] = inwave ? B[((c * 2 + 0) * 3 + t) * 3 + i] : T(0);
                da[i] = inwave ? B[((c * 2 + 1) * 3 + t) * 3 + i] : T(0);
            }
#pragma unroll
            for (int qx = 0; qx < 3; ++qx) {
                T s = T(0), d = T(0), e = T(0);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    s += cS<T>(qx, i) * sa[i];
                    d += cD<T>(qx, i) * sa[i];
                    e += cS<T>(qx, i) * da[i];
                }
                val[c][qx] = s;
                g0[c][qx] = d;
                g1[c][qx] = e;
            }
        }
    }

    const int qy = t;
    T pq[3] = {T(0), T(0), T(0)};
    if constexpr ((MODE & OP_BT) != 0) {
        if (act) {
            double pv[4];
#pragma unroll
            for (int n = 0; n < 4; ++n) pv[n] = a.p[a.pmap[cell * 4 + n]];
            const T ly0 = rL<T>(qy, 0), ly1 = rL<T>(qy, 1);
            const T tx0 = ly0 * T(pv[0]) + ly1 * T(pv[2]);
            const T tx1 = ly0 * T(pv[1]) + ly1 * T(pv[3]);
#pragma unroll
            for (int qx = 0; qx < 3; ++qx) pq[qx] = cL<T>(qx, 0) * tx0 + cL<T>(qx, 1) * tx1;
        }
    }

    T F0[2][3], F1[2][3], Fv[2][3];
    T divq[3];
#pragma unroll
    for (int qx = 0; qx < 3; ++qx) {
        T Km[2][2];
        const int64_t off = ((int64_t)qx * a.nc + cell) * NT + t;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) Km[b][aa] = act ? a.K[(b * 2 + aa) * P + off] : T(0);
        T Tm[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
        divq[qx] = T(0);
        if constexpr (FWD) {
            T H[2][2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int aa = 0; aa < 2; ++aa) H[c][aa] = g0[c][qx] * Km[0][aa] + g1[c][qx] * Km[1][aa];
            if constexpr ((MODE & OP_B) != 0) divq[qx] = H[0][0] + H[1][1];
            if constexpr ((MODE & OP_A) != 0) {
                const T cvisc = act ? a.cv[off] : T(0);
                const T cmass = act ? a.cv[P + off] : T(0);
                Tm[0][0] = cvisc * H[0][0];
                Tm[1][1] = cvisc * H[1][1];
                const T e01 = T(0.5) * cvisc * (H[0][1] + H[1][0]);
                Tm[0][1] = e01;
                Tm[1][0] = e01;
#pragma unroll
                for (int c = 0; c < 2; ++c) Fv[c][qx] = cmass * val[c][qx];
            }
        }
        if constexpr ((MODE & OP_A) == 0) {
#pragma unroll
            for (int c = 0; c < 2; ++c) Fv[c][qx] = T(0);
        }
        if constexpr ((MODE & OP_BT) != 0) {
            Tm[0][0] += pq[qx];
            Tm[1][1] += pq[qx];
        }
        if constexpr (BWD) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                F0[c][qx] = Tm[c][0] * Km[0][0] + Tm[c][1] * Km[0][1];
                F1[c][qx] = Tm[c][0] * Km[1][0] + Tm[c][1] * Km[1][1];
            }
        }
    }

    if constexpr ((MODE & OP_B) != 0) {
        T r[2];
#pragma unroll
        for (int ax = 0; ax < 2; ++ax)
            r[ax] = cL<T>(0, ax) * divq[0] + cL<T>(1, ax) * divq[1] + cL<T>(2, ax) * divq[2];
        if (inwave) {
            const T ly[2] = {rL<T>(qy, 0), rL<T>(qy, 1)};
#pragma unroll
            for (int by = 0; by < 2; ++by)
#pragma unroll
                for (int ax = 0; ax < 2; ++ax) pbuf[wave][slot][t][ax + 2 * by] = double(ly[by] * r[ax]);
        }
        __syncthreads();
        if (act) {
            // 3 threads per cell, 4 vertices: thread t sums vertex t (and t = 0 also vertex 3)
#pragma unroll
            for (int rep = 0; rep < 2; ++rep) {
                const int vtx = rep == 0 ? t : 3;
                if (rep == 1 && t != 0) break;
                double s = pbuf[wave][slot][0][vtx] + pbuf[wave][slot][1][vtx] + pbuf[wave][slot][2][vtx];
                a.q[a.pmap[cell * 4 + vtx]] += s;
            }
        }
    }

    if constexpr (BWD) {
        T ws[2][3], wd[2][3];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T s = T(0), d = T(0);
#pragma unroll
                for (int qx = 0; qx < 3; ++qx) {
                    s += cS<T>(qx, i) * Fv[c][qx] + cD<T>(qx, i) * F0[c][qx];
                    d += cS<T>(qx, i) * F1[c][qx];
                }
                ws[c][i] = s;
                wd[c][i] = d;
            }
        __syncthreads();
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    B[((c * 2 + 0) * 3 + t) * 3 + i] = ws[c][i];
                    B[((c * 2 + 1) * 3 + t) * 3 + i] = wd[c][i];
                }
        }
        __syncthreads();
        if (act) {
            const uint32_t dm = a.dmask[cell];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                T WS[3], WD[3];
#pragma unroll
                for (int q2 = 0; q2 < 3; ++q2) {
                    WS[q2] = B[((c * 2 + 0) * 3 + q2) * 3 + t];
                    WD[q2] = B[((c * 2 + 1) * 3 + q2) * 3 + t];
                }
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    T s = T(0);
#pragma unroll
                    for (int q2 = 0; q2 < 3; ++q2) s += cS<T>(q2, j) * WS[q2] + cD<T>(q2, j) * WD[q2];
                    const int ln = t + 3 * j;
                    if ((dm >> ln) & 1u) continue;
                    const int node = a.vmap[cell * NLOC + ln];
                    a.v[c * a.nvn + node] += s;
                }
            }
        }
    }
}

// ============================================================== launchers
// variant: bits 0-1 waves per block (0:1, 1:2, 2:4), bit 2: disable XCD remap
constexpr int kNumVariants = 6;

template <typename T, int MODE, int WPB, bool REMAP>
static void launch_one(const Level& L, const CellArgs<T>& args, int64_t ncell, hipStream_t s) {
    const int cpw = L.dim == 3 ? Shape<3>::CPW : Shape<2>::CPW;
    const int64_t per_block = (int64_t)cpw * WPB;
    const int64_t grid = (ncell + per_block - 1) / per_block;
    if (grid <= 0) return;
    if (L.dim == 3)
        hipLaunchKernelGGL((cell3d<T, MODE, WPB, REMAP>), dim3((unsigned)grid), dim3(64 * WPB), 0, s, args);
    else
        hipLaunchKernelGGL((cell2d<T, MODE, WPB, REMAP>), dim3((unsigned)grid), dim3(64 * WPB), 0, s, args);
}

template <typename T, int MODE>
static void launch_mode(const Level& L, int variant, const CellArgs<T>& args, int64_t ncell, hipStream_t s) {
    switch (variant) {
        case 0: launch_one<T, MODE, 1, true>(L, args, ncell, s); break;
        case 1: launch_one<T, MODE, 2, true>(L, args, ncell, s); break;
        case 2: launch_one<T, MODE, 4, true>(L, args, ncell, s); break;
        case 3: launch_one<T, MODE, 1, false>(L, args, ncell, s); break;
        case 4: launch_one<T, MODE, 2, false>(L, args, ncell, s); break;
        default: launch_one<T, MODE, 4, false>(L, args, ncell, s); break;
    }
}

template <typename T>
void launch_cell(const Level& L, int mode, int variant, int color, const T* K, const T* cv, const T* u,
                 const double* p, T* v, double* q, hipStream_t s) {
    CellArgs<T> args;
    args.cbeg = L.color_off[color];
    args.cend = L.color_off[color + 1];
    args.nc = L.nc;
    args.nvn = L.nvn;
    args.plane = L.plane();
    args.vmap = L.d_vmap;
    args.dmask = L.d_dmask;
    args.pmap = L.d_pmap;
    args.K = K;
    args.cv = cv;
    args.u = u;
    args.p = p;
    args.v = v;
    args.q = q;
    const int64_t ncell = args.cend - args.cbeg;
    switch (mode) {
        case OP_A: launch_mode<T, OP_A>(L, variant, args, ncell, s); break;
        case OP_B: launch_mode<T, OP_B>(L, variant, args, ncell, s); break;
        case OP_BT: launch_mode<T, OP_BT>(L, variant, args, ncell, s); break;
        case OP_A | OP_BT: launch_mode<T, OP_A | OP_BT>(L, variant, args, ncell, s); break;
        default: launch_mode<T, OP_A | OP_BT | OP_B>(L, variant, args, ncell, s); break;
    }
}

template <typename T>
void launch_cell_all(const Level& L, int mode, int variant, const T* K, const T* cv, const T* u,
                     const double* p, T* v, double* q, hipStream_t s) {
    for (int c = 0; c < L.ncolors; ++c) launch_cell<T>(L, mode, variant, c, K, cv, u, p, v, q, s);
}

template void launch_cell<double>(const Level&, int, int, int, const double*, const double*, const double*,
                                  const double*, double*, double*, hipStream_t);
template void launch_cell<float>(const Level&, int, int, int, const float*, const float*, const float*,
                                 const double*, float*, double*, hipStream_t);
template void launch_cell_all<double>(const Level&, int, int, const double*, const double*, const double*,
                                      const double*, double*, double*, hipStream_t);
template void launch_cell_all<float>(const Level&, int, int, const float*, const float*, const float*,
                                     const double*, float*, double*, hipStream_t);

}  // namespace fsi
