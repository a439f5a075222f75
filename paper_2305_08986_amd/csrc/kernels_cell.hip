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
// In FP32 on 3D levels whose geometry comes from vertex displacements (the
// multilinear ALE map), the kernel can instead form det(J) w_q J^{-1} = w_q adj(J)
// at each point from the cell's 8 vertex displacements and read only
// (2 eta, c_m) per point.
//
// Thread layout (64-wide wavefronts): one thread per line of 3 points of a
// cell, NT = 3^(dim-1) threads per cell, CPW cells per wavefront.  The three
// 1D contraction sweeps run in registers; between sweep directions the lines
// are transposed through LDS (wavefront-private).  Cells of one colour share
// no node, so the scatter is a plain store (first touch of a node in phase
// order) or read-modify-write (later touches), with no atomics; the host
// launches the processing phases one after another.
#include <type_traits>

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

// 1D Gauss weight at a runtime index
template <typename T> __device__ __forceinline__ T rW(int q) { return q == 1 ? T(kW1) : T(kW0); }

// geometry is read exactly once per application: optionally stream it past the caches
template <bool NT, typename T>
__device__ __forceinline__ T gload(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// ordering of LDS traffic among the lanes of one wavefront: a wavefront's LDS
// instructions execute in issue order, so only compiler code motion has to be
// stopped (no s_barrier, no wait for outstanding memory operations)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t x = b & 7, qd = nb >> 3, r = nb & 7;
    const int64_t base = (x < r) ? x * (qd + 1) : r * (qd + 1) + (x - r) * qd;
    return base + (b >> 3);
}

template <typename T>
struct CellArgs {
    int64_t cbeg, cend, nc, nvn, plane;
    int64_t nrows;      // rows of cells (along x) in this phase
    int nx, nchunks;    // cells per row, chunks of CPW cells per row
    int wlast;          // cells in the last (ragged) chunk of a row
    int64_t chunk0;     // geometry chunk index of the phase's first chunk
    int64_t nchk;       // geometry chunks on the level (stride of the qx blocks)
    const int* __restrict__ vmap;
    const uint4* __restrict__ info;
    const int* __restrict__ rowmap;   // OP_ATOM: phase-major row of each dispatch slot
    // OP_FIXW (the 3D atomic A on a level with fixed cells): the per-node wall mask, which
    // replaces the wall bits derived from the box faces
    const uint8_t* __restrict__ wallmask;
    const int* __restrict__ pmap;
    const T* __restrict__ K;
    const T* __restrict__ cv;
    const T* __restrict__ u;
    const double* __restrict__ p;
    T* __restrict__ v;
    double* __restrict__ q;
    // fused epilogues (OP_CHEB: iterate x, direction d, right-hand side r, 1/diag A;
    // OP_RES: right-hand sides r (velocity) and fp (pressure))
    T* __restrict__ x;
    T* __restrict__ d;
    const T* __restrict__ r;
    const T* __restrict__ dinv;
    const double* __restrict__ fp;
    T c1, c2;
    int first;          // OP_CHEB: first step, the direction is the iterate itself
    int store_d;
    // geometry from vertices (FP32, 3D): per-vertex displacement of the level's
    // multilinear ALE map, reference cell sizes, and per point (2 eta, c_m) in the
    // geometry layout (2 planes)
    const float4* __restrict__ vd;
    const double4* __restrict__ vd64;
    const T* __restrict__ cq;
    T hx, hy, hz;
    // corrector-mode terms (OP_CONV): beta = K v° (3 planes) and sigma = r / (det J w)
    // in the geometry layout, and the density
    const T* __restrict__ cb;
    const T* __restrict__ cs;
    T rho;
    // OP_ATOM: cell->node and cell->vertex indices and wall bits follow from the cell's
    // coordinates on the structured box (no map or cell-info reads): cells per direction
    // (y, z), Q2 node counts, Q1 vertex counts (x, y), Dirichlet face bits
    int cny, cnz;
    int vnx, vny, vnz;
    int pnx, pny;
    unsigned dfaces;
    // OP_ATOM, one wavefront per row (no row sharing): each row is cut into nseg segments
    // of segch chunks, one dispatch slot per segment (shorter work units, a shorter tail
    // at the end of the launch); the x-face node two segments share takes atomics from
    // both.  nseg = 1: whole rows
    int nseg, segch;
};

// ============================================================== 3D
// A row of cells along x is walked in chunks of CPW = 7 cells (9 threads per cell:
// one per line of 3 points), one chunk per wavefront.  RS = false: each wavefront
// of the workgroup owns its own row.  RS = true: the WPB wavefronts share one row
// and take WPB consecutive chunks per step, so a step covers 14 WPB nodes of every
// node line (fewer cache lines shared with the next step) and the row has WPB
// times more wavefronts in flight; the x-face hand-over then crosses wavefronts.
// Only the two hand-overs (x-face values and pressure partial sums) synchronise the
// workgroup; the LDS transposes between sweep directions are wavefront-private.
// ZG > 1 (the atomic form): a workgroup takes ZG consecutive rows along z at the same y
// and walks them chunk by chunk, z innermost; the node plane two neighbouring rows of the
// group share is summed in registers and stored once, so only the group's outer z-planes
// and the y-faces take atomics.
template <typename T, int MODE, int WPB, bool RS, bool NTL, int WPE, bool VG, int ZG>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(WPE))) void cell3d(CellArgs<T> a) {
    constexpr int NT = 9, CPW = 7, NLOC = 27, BUF = 243;
    constexpr bool FWD = (MODE & (OP_A | OP_B)) != 0;
    constexpr bool BWD = (MODE & (OP_A | OP_BT)) != 0;
    constexpr bool HAS_B = (MODE & OP_B) != 0;
    constexpr bool HAS_BT = (MODE & OP_BT) != 0;
    constexpr bool HAS_A = (MODE & OP_A) != 0;
    constexpr bool CHEB = (MODE & OP_CHEB) != 0;
    constexpr bool RES = (MODE & OP_RES) != 0;
    constexpr bool CONV = (MODE & OP_CONV) != 0;
    // every phase in one launch: each touch adds atomically (outputs zeroed beforehand)
    constexpr bool ATOM = (MODE & OP_ATOM) != 0;
    constexpr bool FIXW = (MODE & OP_FIXW) != 0;
    static_assert(!FIXW || MODE == (OP_A | OP_ATOM | OP_FIXW), "the fixed-node wall mask goes with the atomic A");
    static_assert(!ATOM || !(CHEB || RES), "the atomic form has no epilogue");
    static_assert(!CHEB || MODE == (OP_A | OP_CHEB), "the Chebyshev epilogue goes with A alone");
    static_assert(!CONV || ((MODE & ~OP_ATOM) == (OP_A | OP_CONV) || (MODE & ~OP_ATOM) == (OP_A | OP_BT | OP_B | OP_CONV)),
                  "the corrector terms go with A or the Stokes apply");
    static_assert(!CONV || !VG, "the corrector terms use the stored geometry");
    static_assert(!RES || MODE == (OP_A | OP_BT | OP_B | OP_RES), "the residual epilogue goes with the Stokes apply");

    static_assert(ZG == 1 || ATOM, "row groups along z belong to the atomic form");
    // A alone reads K' = sqrt(cvisc) K (no cvisc plane): sym(grad-hat u K') K'^T = cvisc sym(H) K^T
    constexpr bool SCALED = !VG && ((MODE & ~(OP_ATOM | OP_FIXW)) == OP_A || MODE == (OP_A | OP_CHEB));
    __shared__ T sbuf[WPB][CPW][BUF];
    __shared__ double pbuf[HAS_B ? WPB : 1][CPW][NT][8];
    // x-face hand-over between neighbouring cells of the row: [slot][j][comp][k],
    // carry from the last slot of a chunk to the first slot of the next one
    // (double-buffered by step parity, so that a wavefront may start the next step
    // while its right neighbour still reads the previous step's values)
    __shared__ T xb[2][WPB][CPW][27];
    __shared__ T xcarry[WPB][ZG][2][27];
    __shared__ double pxb[2][HAS_B ? WPB : 1][CPW][4];
    __shared__ double pcarry[HAS_B ? WPB : 1][ZG][2][4];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / NT, t = lane - slot * NT;
    const bool inwave = slot < CPW;
    const int64_t slot_row = RS ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * WPB + wave;
    const bool slotact = slot_row < a.nrows;
    // the atomic form has no order to keep: dispatch slot g takes segment g mod nseg of
    // the natural rows (iy, iz) = (r mod ny, ZG (r div ny) + z), r = g div nseg, whose
    // geometry sits at the phase-major row that the row map gives
    int siy = 0, siz0 = 0;
    int chb = 0, che = a.nchunks;   // the slot's chunks [chb, che) of its rows
    if constexpr (ATOM) {
        const int64_t rslot = slot_row / a.nseg;
        siy = (int)(rslot % a.cny);
        siz0 = (int)(rslot / a.cny) * ZG;
        if constexpr (!RS) {
            chb = (int)(slot_row - rslot * a.nseg) * a.segch;
            che = min(a.nchunks, chb + a.segch);
        }
    }
    // cells [xbeg, xend) of the row; the x-face columns at a segment seam are shared with
    // the neighbouring segment
    const int xbeg = chb * CPW, xend = min(a.nx, che * CPW);
    // row z of the slot's group active; its geometry row (loaded once, before the walk,
    // so that no step's geometry loads wait for a row-map load)
    auto zact = [&](int z) { return ATOM ? (slotact && siz0 + z < a.cnz) : slotact; };
    int zr[4] = {0, 0, 0, 0};
    if constexpr (ATOM) {
#pragma unroll
        for (int z = 0; z < ZG; ++z)
            zr[z] = zact(z) ? __builtin_amdgcn_readfirstlane(a.rowmap[siy + (int64_t)a.cny * (siz0 + z)]) : 0;
    }
    auto zrow = [&](int z) -> int64_t {
        if constexpr (ATOM) return z == 0 ? zr[0] : (z == 1 ? zr[1] : (z == 2 ? zr[2] : zr[3]));
        else return slot_row;
    };
    const int nsteps = RS ? (a.nchunks + WPB - 1) / WPB : max(0, che - chb);
    const int cw = RS ? 0 : wave;                  // owner of the chunk-to-chunk carry
    const bool carry_out = !RS || wave == WPB - 1; // this wavefront's last cell feeds the next step
    T* B = sbuf[wave][inwave ? slot : 0];
    const int64_t P = a.plane;
    // thread roles: stage A / scatter column (ic, jc) = (t % 3, t / 3); stage B line (ib, qzb)
    // = (t % 3, t / 3); stage C line (qy, qz) = (t % 3, t / 3)
    const int ic = t % 3, jc = t / 3;
    const int qy = t % 3, qz = t / 3;
    const int pax = t & 1, pyz = t >> 1;

    // cell info and node indices of a step: the Stokes modes (one or two wavefronts per
    // SIMD) fetch the next step's while their own gathers are in flight, which takes one
    // dependent round trip out of the step; the other modes fetch them in the step
    // itself (measured faster there: 7 more live registers cost them more than the
    // round trip)
    constexpr bool PREF = HAS_A && HAS_BT && !ATOM;
    uint4 inf_nx = make_uint4(0u, 0u, 0u, 0u);
    int node_nx[3] = {0, 0, 0};
    auto fetch_idx = [&](int stp) {
        const int chp = RS ? stp * WPB + wave : stp;
        const int ixp = chp * CPW + slot;
        const bool actp = slotact && inwave && stp < nsteps && ixp < a.nx;
        const int64_t cellp = a.cbeg + slot_row * a.nx + ixp;
        inf_nx = actp ? a.info[cellp] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int k = 0; k < 3; ++k) node_nx[k] = actp ? a.vmap[cellp * NLOC + t + 9 * k] : 0;
    };
    if constexpr (PREF) fetch_idx(0);
    // the node plane a row of a z-group shares with the next row: this thread's sums
    // there (the writer threads' complete x-face values), added at the next z
    T zc[3] = {T(0), T(0), T(0)};
    for (int st = 0; st < nsteps; ++st)
#pragma unroll 1
    for (int z = 0; z < ZG; ++z) {
        const int ls = st * ZG + z;                        // linear step: hand-over buffer parity
        const bool rowact = zact(z);
        const int64_t row = __builtin_amdgcn_readfirstlane((int)zrow(z));
        if constexpr (!PREF && !ATOM) fetch_idx(st);
        const int ch = RS ? st * WPB + wave : chb + st;
        const int ix = ch * CPW + slot;
        const bool act = rowact && inwave && ix < xend;
        const int64_t cell = a.cbeg + row * a.nx + ix;   // phase cells are stored row by row
        // the chunk is wavefront-uniform: keep it scalar so that every geometry load is
        // a scalar base plus the lane's fixed offset (no per-plane vector addresses)
        const int64_t chunk = __builtin_amdgcn_readfirstlane((int)(a.chunk0 + row * a.nchunks + ch));
        const uint4 inf = inf_nx;
        // does this thread write its column (x-face columns go to the right neighbour)?
        const bool vwriter = act && (ic != 2 || ix == xend - 1);
        const bool pwriter = act && t < 8 && (pax == 0 || ix == xend - 1);
        // a column on a seam between two segments of the row: its sums are partial
        const bool xseam = ATOM && ((ic == 0 && ix == xbeg && ix > 0) || (ic == 2 && xend < a.nx));
        // the atomic form: node indices, wall bits of this thread's column and the cell's
        // vertices from the cell coordinates (ix, iy, iz)
        const int iz = siz0 + z;
        int node[3] = {node_nx[0], node_nx[1], node_nx[2]};
        unsigned wbits = 0;   // bit k: node (ic, jc, k) lies on a Dirichlet face
        if constexpr (ATOM) {
            const int gx = 2 * ix + ic, gy = 2 * siy + jc;
            const bool wxy = ((a.dfaces & 1u) && gx == 0) || ((a.dfaces & 2u) && gx == a.vnx - 1) ||
                             ((a.dfaces & 4u) && gy == 0) || ((a.dfaces & 8u) && gy == a.vny - 1);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int gz = 2 * iz + k;
                node[k] = gx + a.vnx * (gy + a.vny * gz);
                const bool w = wxy || ((a.dfaces & 16u) && gz == 0) || ((a.dfaces & 32u) && gz == a.vnz - 1);
                wbits |= (w ? 1u : 0u) << k;
            }
            if constexpr (FIXW) {   // fixed nodes inside the box
                wbits = 0;
#pragma unroll
                for (int k = 0; k < 3; ++k) wbits |= ((act && a.wallmask[node[k]]) ? 1u : 0u) << k;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) wbits |= ((inf.x >> (t + 9 * k)) & 1u) << k;
        }
        // Q1 vertex n = (n & 1, (n >> 1) & 1, n >> 2) of the cell
        auto vert = [&](int n) -> int {
            if constexpr (ATOM)
                return (ix + (n & 1)) + a.pnx * ((siy + ((n >> 1) & 1)) + a.pny * (iz + (n >> 2)));
            else
                return a.pmap[cell * 8 + n];
        };

        // ---------------- loads
        T uu[3][3];     // [comp][k] velocity of the column nodes
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const bool wall = (wbits >> k) & 1u;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                uu[c][k] = (FWD && act && !wall) ? (CHEB ? a.x : a.u)[c * a.nvn + node[k]] : T(0);
        }
        if constexpr (PREF) fetch_idx(st + 1);
        // the first point's geometry (per-point path): issued before the forward sweeps,
        // whose work hides its latency
        constexpr bool PERQX0 = !VG && (sizeof(T) == 8 || (HAS_A && HAS_BT) || CONV);
        // FP64 geometry from the vertices: the backward x-sweep accumulates in the
        // transpose buffer (the registers go to the Jacobian data)
        constexpr bool LACC = VG && sizeof(T) == 8 && BWD;
        T g0[11];
        if constexpr (PERQX0) {
            const int64_t off0 = chunk * kGeoSlots + (slot * NT + t);
#pragma unroll
            for (int e = 0; e < 9; ++e) g0[e] = act ? gload<NTL>(a.K + e * P + off0) : T(0);
            g0[9] = (SCALED || !HAS_A || !act) ? T(1) : gload<NTL>(a.cv + off0);
            g0[10] = (HAS_A && act) ? gload<NTL>(a.cv + P + off0) : T(0);
            __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the sweeps
        }
        int pnode = 0;
        if constexpr (HAS_B) {
            if (pwriter) pnode = vert(t);
        }
        T pv[8];
        if constexpr (HAS_BT) {
            // threads t < 8 of a cell fetch one vertex value each; the cell's other
            // threads read them across lanes (one memory round trip instead of
            // eight index + eight value loads per thread)
            const T mine = (act && t < 8) ? T(a.p[vert(t)]) : T(0);
            const int base = lane - t;   // lane of the cell's first thread
#pragma unroll
            for (int n = 0; n < 8; ++n) pv[n] = __shfl(mine, base + n, 64);
        }
        // geometry from vertices: at this thread's (qy, qz) the Jacobian columns of the
        // multilinear map x = X + sum_v N_v d_v are dx/dxi_0 = g0 (constant in qx) and
        // dx/dxi_1 = L0(qx) b0 + L1(qx) b1, dx/dxi_2 = L0(qx) f0 + L1(qx) f1, where the
        // reference cell sizes are folded in (L0 + L1 = 1); vertex v = i + 2j + 4k
        T vg0[3], vb0[3], vb1[3], vf0[3], vf1[3];
        if constexpr (VG) {
            using V4 = std::conditional_t<sizeof(T) == 8, double4, float4>;
            const V4* vdp;
            if constexpr (sizeof(T) == 8) vdp = a.vd64;
            else vdp = a.vd;
            V4 dv[8];
#pragma unroll
            for (int n = 0; n < 8; ++n) dv[n] = act ? vdp[vert(n)] : V4{};
            const T ly0 = rL<T>(qy, 0), ly1 = rL<T>(qy, 1), lz0 = rL<T>(qz, 0), lz1 = rL<T>(qz, 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T d[8];
#pragma unroll
                for (int n = 0; n < 8; ++n) d[n] = c == 0 ? dv[n].x : (c == 1 ? dv[n].y : dv[n].z);
                vg0[c] = (c == 0 ? a.hx : T(0)) + ly0 * lz0 * (d[1] - d[0]) + ly1 * lz0 * (d[3] - d[2]) +
                         ly0 * lz1 * (d[5] - d[4]) + ly1 * lz1 * (d[7] - d[6]);
                vb0[c] = (c == 1 ? a.hy : T(0)) + lz0 * (d[2] - d[0]) + lz1 * (d[6] - d[4]);
                vb1[c] = (c == 1 ? a.hy : T(0)) + lz0 * (d[3] - d[1]) + lz1 * (d[7] - d[5]);
                vf0[c] = (c == 2 ? a.hz : T(0)) + ly0 * (d[4] - d[0]) + ly1 * (d[6] - d[2]);
                vf1[c] = (c == 2 ? a.hz : T(0)) + ly0 * (d[5] - d[1]) + ly1 * (d[7] - d[3]);
            }
        }

        // ---------------- forward sweeps z (A), y (B); x happens per point in stage C
        T ga[3][3], gb[3][3], gc[3][3];   // [comp][i] at this thread's (qy, qz)
        if constexpr (FWD) {
            if (inwave) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q3 = 0; q3 < 3; ++q3) {
                        T sv = T(0), dv = T(0);
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            sv += cS<T>(q3, k) * uu[c][k];
                            dv += cD<T>(q3, k) * uu[c][k];
                        }
                        B[((c * 2 + 0) * 3 + q3) * 9 + t] = sv;
                        B[((c * 2 + 1) * 3 + q3) * 9 + t] = dv;
                    }
            }
            wave_sync();
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
                    for (int q2 = 0; q2 < 3; ++q2) {
                        T sv = T(0), dv = T(0), ev = T(0);
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            sv += cS<T>(q2, j) * zs[j];
                            dv += cD<T>(q2, j) * zs[j];
                            ev += cS<T>(q2, j) * zd[j];
                        }
                        ya[c][q2] = sv;
                        yb[c][q2] = dv;
                        yc[c][q2] = ev;
                    }
                }
            }
            wave_sync();
            if (inwave) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int q2 = 0; q2 < 3; ++q2) {
                        B[((c * 3 + 0) * 9 + q2 + 3 * qzb) * 3 + ib] = ya[c][q2];
                        B[((c * 3 + 1) * 9 + q2 + 3 * qzb) * 3 + ib] = yb[c][q2];
                        B[((c * 3 + 2) * 9 + q2 + 3 * qzb) * 3 + ib] = yc[c][q2];
                    }
            }
            wave_sync();
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ga[c][i] = inwave ? B[((c * 3 + 0) * 9 + t) * 3 + i] : T(0);
                    gb[c][i] = inwave ? B[((c * 3 + 1) * 9 + t) * 3 + i] : T(0);
                    gc[c][i] = inwave ? B[((c * 3 + 2) * 9 + t) * 3 + i] : T(0);
                }
        }

        // ---------------- stage C: per quadrature point (qx, qy, qz); the backward
        // x-sweep is accumulated on the fly into wa/wb/wc
        T wa[3][3], wb[3][3], wc[3][3];   // [comp][i]
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i) wa[c][i] = wb[c][i] = wc[c][i] = T(0);
        T r0 = T(0), r1 = T(0);           // divergence tested with the two Q1 x-factors
        T tx0 = T(0), tx1 = T(0);         // pressure contracted in y and z
        if constexpr (HAS_BT) {
            const T ly0 = rL<T>(qy, 0), ly1 = rL<T>(qy, 1), lz0 = rL<T>(qz, 0), lz1 = rL<T>(qz, 1);
            tx0 = ly0 * lz0 * pv[0] + ly1 * lz0 * pv[2] + ly0 * lz1 * pv[4] + ly1 * lz1 * pv[6];
            tx1 = ly0 * lz0 * pv[1] + ly1 * lz0 * pv[3] + ly0 * lz1 * pv[5] + ly1 * lz1 * pv[7];
        }
        // point-by-point accumulation of the backward x-sweep needs fewer live registers;
        // FP64 always uses it, FP32 for the Stokes modes (A + B^T [+ B]), whose extra
        // pressure state would otherwise halve the wavefronts per SIMD
        constexpr bool PERQX = sizeof(T) == 8 || (HAS_A && HAS_BT && !VG) || CONV;
        if constexpr (PERQX) {
        // accumulate the backward x-sweep point by point (fewer live registers)
#pragma unroll
        for (int qx = 0; qx < 3; ++qx) {
            // keep one point's geometry in flight at a time (register budget)
            __builtin_amdgcn_sched_barrier(0);
            // geometry of the point: K = det(J) w J^{-1} (row-major 3x3), cvisc, cmass
            T Kq[9];
            const int64_t off = ((int64_t)qx * a.nchk + chunk) * kGeoSlots + (slot * NT + t);
            T cvq, cmq;
            if constexpr (VG) {
                // det(J) w J^{-1} = w adj(J) from the multilinear map (no division for K);
                // J[r][a] = dx_r/dxi_a
                const T lx0 = rL<T>(qx, 0), lx1 = rL<T>(qx, 1);
                T Jm[9];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    Jm[r * 3 + 0] = vg0[r];
                    Jm[r * 3 + 1] = lx0 * vb0[r] + lx1 * vb1[r];
                    Jm[r * 3 + 2] = lx0 * vf0[r] + lx1 * vf1[r];
                }
                const T wq = rW<T>(qx) * rW<T>(qy) * rW<T>(qz);
                const T c00 = Jm[4] * Jm[8] - Jm[5] * Jm[7];
                const T c01 = Jm[5] * Jm[6] - Jm[3] * Jm[8];
                const T c02 = Jm[3] * Jm[7] - Jm[4] * Jm[6];
                const T det = Jm[0] * c00 + Jm[1] * c01 + Jm[2] * c02;
                Kq[0] = wq * c00;
                Kq[1] = wq * (Jm[2] * Jm[7] - Jm[1] * Jm[8]);
                Kq[2] = wq * (Jm[1] * Jm[5] - Jm[2] * Jm[4]);
                Kq[3] = wq * c01;
                Kq[4] = wq * (Jm[0] * Jm[8] - Jm[2] * Jm[6]);
                Kq[5] = wq * (Jm[2] * Jm[3] - Jm[0] * Jm[5]);
                Kq[6] = wq * c02;
                Kq[7] = wq * (Jm[1] * Jm[6] - Jm[0] * Jm[7]);
                Kq[8] = wq * (Jm[0] * Jm[4] - Jm[1] * Jm[3]);
                const T cw = det * wq;
                cvq = (HAS_A && act) ? gload<NTL>(a.cq + off) / cw : T(0);       // 2 eta / (det J w)
                cmq = (HAS_A && act) ? gload<NTL>(a.cq + a.plane + off) * cw : T(0);   // c_m det J w
            } else if (qx == 0) {
#pragma unroll
                for (int e = 0; e < 9; ++e) Kq[e] = g0[e];
                cvq = SCALED ? T(1) : ((HAS_A && act) ? g0[9] : T(0));
                cmq = g0[10];
            } else {
#pragma unroll
                for (int e = 0; e < 9; ++e) Kq[e] = act ? gload<NTL>(a.K + e * P + off) : T(0);
                cvq = SCALED ? T(1) : ((HAS_A && act) ? gload<NTL>(a.cv + off) : T(0));
                cmq = (HAS_A && act) ? gload<NTL>(a.cv + P + off) : T(0);
            }
            // corrector terms: with beta = K v°, (grad-hat u_c) . beta = det(J) w (v° . grad u_c)
            T be[3] = {T(0), T(0), T(0)}, sg = T(0), cvc[3] = {T(0), T(0), T(0)};
            if constexpr (CONV) {
#pragma unroll
                for (int b = 0; b < 3; ++b) be[b] = act ? gload<NTL>(a.cb + b * P + off) : T(0);
                sg = act ? gload<NTL>(a.cs + off) : T(0);
            }
            T Tm[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int e = 0; e < 3; ++e) Tm[c][e] = T(0);
            T Fv[3] = {T(0), T(0), T(0)};
            if constexpr (FWD) {
                T H[3][3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T vv = T(0), d0 = T(0), d1 = T(0), d2 = T(0);
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        vv += cS<T>(qx, i) * ga[c][i];
                        d0 += cD<T>(qx, i) * ga[c][i];
                        d1 += cS<T>(qx, i) * gb[c][i];
                        d2 += cS<T>(qx, i) * gc[c][i];
                    }
#pragma unroll
                    for (int e = 0; e < 3; ++e) H[c][e] = d0 * Kq[e] + d1 * Kq[3 + e] + d2 * Kq[6 + e];
                    if constexpr (HAS_A) Fv[c] = cmq * vv;
                    if constexpr (CONV) {
                        cvc[c] = d0 * be[0] + d1 * be[1] + d2 * be[2];
                        Fv[c] += a.rho * cvc[c];      // rho (v° . grad u_c) det(J) w, tested with phi
                    }
                }
                if constexpr (HAS_B) {
                    const T dv = H[0][0] + H[1][1] + H[2][2];
                    r0 += cL<T>(qx, 0) * dv;
                    r1 += cL<T>(qx, 1) * dv;
                }
                if constexpr (HAS_A) {
                    const T cv = cvq;
                    Tm[0][0] = cv * H[0][0];
                    Tm[1][1] = cv * H[1][1];
                    Tm[2][2] = cv * H[2][2];
                    const T e01 = T(0.5) * cv * (H[0][1] + H[1][0]);
                    const T e02 = T(0.5) * cv * (H[0][2] + H[2][0]);
                    const T e12 = T(0.5) * cv * (H[1][2] + H[2][1]);
                    Tm[0][1] = e01; Tm[1][0] = e01;
                    Tm[0][2] = e02; Tm[2][0] = e02;
                    Tm[1][2] = e12; Tm[2][1] = e12;
                }
            }
            if constexpr (HAS_BT) {
                const T pq = cL<T>(qx, 0) * tx0 + cL<T>(qx, 1) * tx1;
                Tm[0][0] += pq;
                Tm[1][1] += pq;
                Tm[2][2] += pq;
            }
            if constexpr (BWD) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    // F[c][b] = sum_e Tm[c][e] K[b][e]
                    T F0 = Tm[c][0] * Kq[0] + Tm[c][1] * Kq[1] + Tm[c][2] * Kq[2];
                    T F1 = Tm[c][0] * Kq[3] + Tm[c][1] * Kq[4] + Tm[c][2] * Kq[5];
                    T F2 = Tm[c][0] * Kq[6] + Tm[c][1] * Kq[7] + Tm[c][2] * Kq[8];
                    if constexpr (CONV) {
                        // streamline term, tested with (grad-hat w_c) . beta / (det J w)
                        const T st = sg * cvc[c];
                        F0 += st * be[0];
                        F1 += st * be[1];
                        F2 += st * be[2];
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const T da = cS<T>(qx, i) * Fv[c] + cD<T>(qx, i) * F0;
                        const T db = cS<T>(qx, i) * F1;
                        const T dc = cS<T>(qx, i) * F2;
                        if constexpr (LACC) {
                            // the thread's own slots of the transpose buffer, which hold
                            // the backward sweep's input in this layout afterwards (its
                            // forward values were already read into registers)
                            if (inwave) {
                                T* pa = &B[((c * 3 + 0) * 9 + t) * 3 + i];
                                T* pb = &B[((c * 3 + 1) * 9 + t) * 3 + i];
                                T* pc = &B[((c * 3 + 2) * 9 + t) * 3 + i];
                                *pa = (qx == 0 ? T(0) : *pa) + da;
                                *pb = (qx == 0 ? T(0) : *pb) + db;
                                *pc = (qx == 0 ? T(0) : *pc) + dc;
                            }
                        } else {
                            wa[c][i] += da;
                            wb[c][i] += db;
                            wc[c][i] += dc;
                        }
                    }
                }
            }
        }

        } else {
        // FP32: registers are plentiful; all points first, then the backward x-sweep
        T Fva[3][3], F0a[3][3], F1a[3][3], F2a[3][3];   // [comp][qx]
#pragma unroll
        for (int qx = 0; qx < 3; ++qx) {
            // geometry of the point: K = det(J) w J^{-1} (row-major 3x3), cvisc, cmass
            T Kq[9], cvq = T(0), cmq = T(0);
            const int64_t off = ((int64_t)qx * a.nchk + chunk) * kGeoSlots + (slot * NT + t);
            if constexpr (VG) {
                // det(J) w J^{-1} = w adj(J): no division; J[r][a] = dx_r/dxi_a
                const T lx0 = rL<T>(qx, 0), lx1 = rL<T>(qx, 1);
                T Jm[9];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    Jm[r * 3 + 0] = vg0[r];
                    Jm[r * 3 + 1] = lx0 * vb0[r] + lx1 * vb1[r];
                    Jm[r * 3 + 2] = lx0 * vf0[r] + lx1 * vf1[r];
                }
                const T wq = rW<T>(qx) * rW<T>(qy) * rW<T>(qz);
                const T c00 = Jm[4] * Jm[8] - Jm[5] * Jm[7];
                const T c01 = Jm[5] * Jm[6] - Jm[3] * Jm[8];
                const T c02 = Jm[3] * Jm[7] - Jm[4] * Jm[6];
                const T det = Jm[0] * c00 + Jm[1] * c01 + Jm[2] * c02;
                Kq[0] = wq * c00;
                Kq[1] = wq * (Jm[2] * Jm[7] - Jm[1] * Jm[8]);
                Kq[2] = wq * (Jm[1] * Jm[5] - Jm[2] * Jm[4]);
                Kq[3] = wq * c01;
                Kq[4] = wq * (Jm[0] * Jm[8] - Jm[2] * Jm[6]);
                Kq[5] = wq * (Jm[2] * Jm[3] - Jm[0] * Jm[5]);
                Kq[6] = wq * c02;
                Kq[7] = wq * (Jm[1] * Jm[6] - Jm[0] * Jm[7]);
                Kq[8] = wq * (Jm[0] * Jm[4] - Jm[1] * Jm[3]);
                if constexpr (HAS_A) {
                    if (act) {
                        const T cw = det * wq;
                        // hardware reciprocal (about 1 ulp): this is the FP32 preconditioner path
                        cvq = gload<NTL>(a.cq + off) * __builtin_amdgcn_rcpf(cw);   // 2 eta / (det J w)
                        cmq = gload<NTL>(a.cq + P + off) * cw;                       // c_m det J w
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < 9; ++e) Kq[e] = act ? gload<NTL>(a.K + e * P + off) : T(0);
                cvq = SCALED ? T(1) : ((HAS_A && act) ? gload<NTL>(a.cv + off) : T(0));
                cmq = (HAS_A && act) ? gload<NTL>(a.cv + P + off) : T(0);
            }
            T Tm[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int e = 0; e < 3; ++e) Tm[c][e] = T(0);
            T Fv[3] = {T(0), T(0), T(0)};
            if constexpr (FWD) {
                T H[3][3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T vv = T(0), d0 = T(0), d1 = T(0), d2 = T(0);
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        vv += cS<T>(qx, i) * ga[c][i];
                        d0 += cD<T>(qx, i) * ga[c][i];
                        d1 += cS<T>(qx, i) * gb[c][i];
                        d2 += cS<T>(qx, i) * gc[c][i];
                    }
#pragma unroll
                    for (int e = 0; e < 3; ++e) H[c][e] = d0 * Kq[e] + d1 * Kq[3 + e] + d2 * Kq[6 + e];
                    if constexpr (HAS_A) Fv[c] = cmq * vv;
                }
                if constexpr (HAS_B) {
                    const T dv = H[0][0] + H[1][1] + H[2][2];
                    r0 += cL<T>(qx, 0) * dv;
                    r1 += cL<T>(qx, 1) * dv;
                }
                if constexpr (HAS_A) {
                    const T cv = cvq;
                    Tm[0][0] = cv * H[0][0];
                    Tm[1][1] = cv * H[1][1];
                    Tm[2][2] = cv * H[2][2];
                    const T e01 = T(0.5) * cv * (H[0][1] + H[1][0]);
                    const T e02 = T(0.5) * cv * (H[0][2] + H[2][0]);
                    const T e12 = T(0.5) * cv * (H[1][2] + H[2][1]);
                    Tm[0][1] = e01; Tm[1][0] = e01;
                    Tm[0][2] = e02; Tm[2][0] = e02;
                    Tm[1][2] = e12; Tm[2][1] = e12;
                }
            }
            if constexpr (HAS_BT) {
                const T pq = cL<T>(qx, 0) * tx0 + cL<T>(qx, 1) * tx1;
                Tm[0][0] += pq;
                Tm[1][1] += pq;
                Tm[2][2] += pq;
            }
            if constexpr (BWD) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    // F[c][b] = sum_e Tm[c][e] K[b][e]
                    const T F0 = Tm[c][0] * Kq[0] + Tm[c][1] * Kq[1] + Tm[c][2] * Kq[2];
                    const T F1 = Tm[c][0] * Kq[3] + Tm[c][1] * Kq[4] + Tm[c][2] * Kq[5];
                    const T F2 = Tm[c][0] * Kq[6] + Tm[c][1] * Kq[7] + Tm[c][2] * Kq[8];
                    Fva[c][qx] = Fv[c];
                    F0a[c][qx] = F0;
                    F1a[c][qx] = F1;
                    F2a[c][qx] = F2;
                }
            }
        }

        if constexpr (BWD) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    T sv = T(0), dv = T(0), ev = T(0);
#pragma unroll
                    for (int qx = 0; qx < 3; ++qx) {
                        sv += cS<T>(qx, i) * Fva[c][qx] + cD<T>(qx, i) * F0a[c][qx];
                        dv += cS<T>(qx, i) * F1a[c][qx];
                        ev += cS<T>(qx, i) * F2a[c][qx];
                    }
                    wa[c][i] = sv;
                    wb[c][i] = dv;
                    wc[c][i] = ev;
                }
        }
        }
        // ---------------- divergence tested with the Q1 basis (B); x-shared vertices
        // are summed along the row before the write
        if constexpr (HAS_B) {
            // partial sum of earlier phases (RES at the last touch: f_p - partial), fetched
            // here so that it is not live through stage C; the reduction below hides it
            double qold = 0.0;
            bool plast = false;
            if (pwriter) {
                if (!ATOM && !((inf.z >> t) & 1u)) qold = a.q[pnode];
                if constexpr (RES) {
                    plast = (inf.z >> (16 + t)) & 1u;
                    if (plast) qold = a.fp[pnode] - qold;
                }
            }
            if (inwave) {
                const T ly[2] = {rL<T>(qy, 0), rL<T>(qy, 1)};
                const T lz[2] = {rL<T>(qz, 0), rL<T>(qz, 1)};
#pragma unroll
                for (int cz = 0; cz < 2; ++cz)
#pragma unroll
                    for (int by = 0; by < 2; ++by) {
                        pbuf[wave][slot][t][0 + 2 * by + 4 * cz] = double(ly[by] * lz[cz] * r0);
                        pbuf[wave][slot][t][1 + 2 * by + 4 * cz] = double(ly[by] * lz[cz] * r1);
                    }
            }
            wave_sync();
            double sq = 0.0;
            if (inwave && t < 8) {
#pragma unroll
                for (int tt = 0; tt < NT; ++tt) sq += pbuf[wave][slot][tt][t];
                if (pax == 1) pxb[ls & 1][wave][slot][pyz] = sq;
            }
            __syncthreads();   // pxb crosses wavefronts (row sharing)
            if (act && t < 8) {
                if (pax == 0 && ix > xbeg)
                    sq += slot > 0 ? pxb[ls & 1][wave][slot - 1][pyz]
                                   : ((RS && wave > 0) ? pxb[ls & 1][wave - 1][CPW - 1][pyz]
                                                       : pcarry[cw][z][(st + 1) & 1][pyz]);
                if (pwriter) {
                    if constexpr (ATOM) unsafeAtomicAdd(&a.q[pnode], sq);
                    else a.q[pnode] = plast ? qold - sq : qold + sq;
                } else if (slot == CPW - 1 && carry_out) {
                    pcarry[cw][z][st & 1][pyz] = sq;
                }
            }
        }

        // ---------------- backward sweeps y (B) and z (A), x-face hand-over, stores
        // fused epilogue operands [comp][k]: partial sum of earlier phases, right-hand
        // side, and for the Chebyshev step the iterate, direction and 1/diag A
        T ep[3][3], er[3][3], ex[3][3], ed[3][3], eg[3][3];
        if constexpr (BWD) {
            wave_sync();
            if (inwave && !LACC) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        B[((c * 3 + 0) * 9 + t) * 3 + i] = wa[c][i];
                        B[((c * 3 + 1) * 9 + t) * 3 + i] = wb[c][i];
                        B[((c * 3 + 2) * 9 + t) * 3 + i] = wc[c][i];
                    }
            }
            wave_sync();
            // ---------------- fused epilogue operands, fetched behind the barrier that
            // ends stage C (so they do not add to its register peak) and combined only
            // at the store, after the backward sweeps whose work hides their latency
            if constexpr (CHEB || RES) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int ln = t + 9 * k;
                    const bool last = vwriter && !((wbits >> k) & 1u) && ((inf.w >> ln) & 1u);
                    // every node this step adds to: earlier phases' partial sum
                    const bool part = vwriter && !((wbits >> k) & 1u) && !((inf.y >> ln) & 1u);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int64_t i = c * a.nvn + node[k];
                        ep[c][k] = part ? a.v[i] : T(0);
                        er[c][k] = last ? a.r[i] : T(0);
                        if constexpr (CHEB) {
                            ex[c][k] = last ? a.x[i] : T(0);
                            ed[c][k] = (last && !a.first) ? a.d[i] : T(0);
                            eg[c][k] = last ? a.dinv[i] : T(0);
                        }
                    }
                }
            } else {
                // the earlier phases' partial sums of the nodes this step adds to (plain
                // modes), fetched here so that their latency hides behind the backward sweeps
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int ln = t + 9 * k;
                    const bool part = !ATOM && vwriter && !((wbits >> k) & 1u) && !((inf.y >> ln) & 1u);
#pragma unroll
                    for (int c = 0; c < 3; ++c) ep[c][k] = part ? a.v[c * a.nvn + node[k]] : T(0);
                }
            }
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
                    T sv = T(0), dv = T(0);
#pragma unroll
                    for (int q2 = 0; q2 < 3; ++q2) {
                        sv += cS<T>(q2, j) * WA[q2] + cD<T>(q2, j) * WB[q2];
                        dv += cS<T>(q2, j) * WC[q2];
                    }
                    vs[c][j] = sv;
                    vd[c][j] = dv;
                }
            }
            wave_sync();
            if (inwave) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        B[((c * 2 + 0) * 3 + qzb) * 9 + ib + 3 * j] = vs[c][j];
                        B[((c * 2 + 1) * 3 + qzb) * 9 + ib + 3 * j] = vd[c][j];
                    }
            }
            wave_sync();
            T out[3][3];   // [comp][k] for the nodes (ic, jc, k) of this thread's column
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T VS[3], VD[3];
#pragma unroll
                for (int q3 = 0; q3 < 3; ++q3) {
                    VS[q3] = inwave ? B[((c * 2 + 0) * 3 + q3) * 9 + t] : T(0);
                    VD[q3] = inwave ? B[((c * 2 + 1) * 3 + q3) * 9 + t] : T(0);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T sv = T(0);
#pragma unroll
                    for (int q3 = 0; q3 < 3; ++q3) sv += cS<T>(q3, k) * VS[q3] + cD<T>(q3, k) * VD[q3];
                    out[c][k] = sv;
                }
            }
            if (inwave && ic == 2) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int k = 0; k < 3; ++k) xb[ls & 1][wave][slot][jc * 9 + c * 3 + k] = out[c][k];
            }
            __syncthreads();   // xb crosses wavefronts (row sharing)
            if (act) {
                if (ic == 0 && ix > xbeg) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            out[c][k] += slot > 0 ? xb[ls & 1][wave][slot - 1][jc * 9 + c * 3 + k]
                                                  : ((RS && wave > 0) ? xb[ls & 1][wave - 1][CPW - 1][jc * 9 + c * 3 + k]
                                                                      : xcarry[cw][z][(st + 1) & 1][jc * 9 + c * 3 + k]);
                }
                if (ATOM && vwriter) {
                    // z-group: the plane shared with the previous row of the group is complete
                    // once that row's sums are added; the plane shared with the next row is
                    // carried; the group's outer planes and the y-faces (jc 0 and 2, shared
                    // with the neighbouring y rows) take atomics.  Wall rows: v = u (A and
                    // the Stokes apply; B^T leaves the zeroed output), written by one owner
                    // per node: the x writer, at jc > 0 or iy = 0, at k > 0 or iz = 0.
                    const bool carry_next = ZG > 1 && z + 1 < ZG && zact(z + 1);
                    if (ZG > 1 && z > 0) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) out[c][0] += zc[c];
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const int64_t nd = node[k];
                        if ((wbits >> k) & 1u) {
                            if (HAS_A && (jc > 0 || siy == 0) && (k > 0 || iz == 0)) {
#pragma unroll
                                for (int c = 0; c < 3; ++c) a.v[c * a.nvn + nd] = a.u[c * a.nvn + nd];
                            }
                            continue;
                        }
                        if (k == 0 && ZG > 1 && z > 0 && jc != 1) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) unsafeAtomicAdd(&a.v[c * a.nvn + nd], out[c][0]);
                            continue;
                        }
                        if (k == 2 && carry_next) continue;   // added at the next z
                        const bool plain = !xseam && jc == 1 && (k == 1 || (k == 0 && ZG > 1 && z > 0));
                        if (plain) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) a.v[c * a.nvn + nd] = out[c][k];
                        } else {
#pragma unroll
                            for (int c = 0; c < 3; ++c) unsafeAtomicAdd(&a.v[c * a.nvn + nd], out[c][k]);
                        }
                    }
                    if (ZG > 1) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) zc[c] = out[c][2];
                    }
                } else if (vwriter) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const int ln = t + 9 * k;
                        if ((wbits >> k) & 1u) continue;
                        const bool first = (inf.y >> ln) & 1u;   // first touch of the node in phase order
                        if ((CHEB || RES) && ((inf.w >> ln) & 1u)) {
                            // last touch: the row of A x (M u) is complete here
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                const int64_t i = c * a.nvn + node[k];
                                const T tot = ep[c][k] + out[c][k];
                                if constexpr (CHEB) {
                                    const T dprev = a.first ? ex[c][k] : ed[c][k];
                                    const T dn = a.c1 * dprev + a.c2 * eg[c][k] * (er[c][k] - tot);
                                    if (a.store_d) a.d[i] = dn;
                                    a.x[i] = ex[c][k] + dn;
                                } else {
                                    a.v[i] = er[c][k] - tot;
                                }
                            }
                        } else if (first) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) a.v[c * a.nvn + node[k]] = out[c][k];
                        } else {
#pragma unroll
                            for (int c = 0; c < 3; ++c) a.v[c * a.nvn + node[k]] = ep[c][k] + out[c][k];
                        }
                    }
                }
                if (!vwriter && slot == CPW - 1 && carry_out) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int k = 0; k < 3; ++k) xcarry[cw][z][st & 1][jc * 9 + c * 3 + k] = out[c][k];
                }
            }
        }
        wave_sync();
    }   // chunk and z loops
}

// ============================================================== 2D
template <typename T, int MODE, int WPB, bool REMAP, bool NTL>
__global__ __launch_bounds__(64 * WPB) void cell2d(CellArgs<T> a) {
    constexpr int NT = 3, CPW = 21, NLOC = 9, BUF = 36;
    constexpr bool FWD = (MODE & (OP_A | OP_B)) != 0;
    constexpr bool BWD = (MODE & (OP_A | OP_BT)) != 0;
    constexpr bool CHEB = (MODE & OP_CHEB) != 0;
    constexpr bool RES = (MODE & OP_RES) != 0;
    constexpr bool CONV = (MODE & OP_CONV) != 0;
    // OP_ATOM: every row of every phase in one launch; shared nodes take hardware atomic
    // adds into the zeroed output, and wall rows take v = u (plain stores of one value)
    constexpr bool ATOM = (MODE & OP_ATOM) != 0;
    constexpr int MB = MODE & ~OP_ATOM;
    static_assert(!ATOM || !(CHEB || RES), "the atomic form has no epilogue");
    static_assert(!CHEB || MODE == (OP_A | OP_CHEB), "the Chebyshev epilogue goes with A alone");
    static_assert(!RES || MODE == (OP_A | OP_BT | OP_B | OP_RES), "the residual epilogue goes with the Stokes apply");
    static_assert(!CONV || MB == (OP_A | OP_CONV) || MB == (OP_A | OP_BT | OP_B | OP_CONV),
                  "the corrector terms go with A or the Stokes apply");
    constexpr bool SCALED = MB == OP_A || MODE == (OP_A | OP_CHEB);   // K' = sqrt(cvisc) K, no cvisc plane
    __shared__ T sbuf[WPB][CPW][BUF];
    __shared__ double pbuf[(MODE & OP_B) ? WPB : 1][CPW][NT][4];

    __shared__ T xb[WPB][CPW][6];
    __shared__ T xcarry[WPB][2][6];
    __shared__ double pxb[(MODE & OP_B) ? WPB : 1][CPW][2];
    __shared__ double pcarry[(MODE & OP_B) ? WPB : 1][2][2];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / NT, t = lane - slot * NT;
    const bool inwave = slot < CPW;
    const int64_t lb = REMAP ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t row = lb * WPB + wave;
    const bool rowact = row < a.nrows;
    T* B = sbuf[wave][inwave ? slot : 0];
    const int64_t P = a.plane;

    for (int ch = 0; ch < a.nchunks; ++ch) {
    const int ix = ch * CPW + slot;
    const bool act = rowact && inwave && ix < a.nx;
    const int64_t cell = a.cbeg + row * a.nx + ix;   // phase cells are stored row by row
    const int64_t chunk = __builtin_amdgcn_readfirstlane((int)(a.chunk0 + row * a.nchunks + ch));

    T val[2][3], g0[2][3], g1[2][3];
    if constexpr (FWD) {
        T uu[2][3];
        if (act) {
            const uint32_t dm = a.info[cell].x;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int ln = t + 3 * j;
                const int node = a.vmap[cell * NLOC + ln];
                const bool wall = (dm >> ln) & 1u;
#pragma unroll
                for (int c = 0; c < 2; ++c) uu[c][j] = wall ? T(0) : (CHEB ? a.x : a.u)[c * a.nvn + node];
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
        wave_sync();
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
        const int64_t off = ((int64_t)qx * a.nchk + chunk) * kGeoSlots + (slot * NT + t);
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) Km[b][aa] = act ? gload<NTL>(a.K + (b * 2 + aa) * P + off) : T(0);
        T Tm[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
        divq[qx] = T(0);
        // corrector terms: with beta = K v°, (grad-hat u_c) . beta = det(J) w (v° . grad u_c)
        T be[2] = {T(0), T(0)}, sg = T(0), cvc[2] = {T(0), T(0)};
        if constexpr (CONV) {
#pragma unroll
            for (int b = 0; b < 2; ++b) be[b] = act ? gload<NTL>(a.cb + b * P + off) : T(0);
            sg = act ? gload<NTL>(a.cs + off) : T(0);
        }
        if constexpr (FWD) {
            T H[2][2];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int aa = 0; aa < 2; ++aa) H[c][aa] = g0[c][qx] * Km[0][aa] + g1[c][qx] * Km[1][aa];
            if constexpr ((MODE & OP_B) != 0) divq[qx] = H[0][0] + H[1][1];
            if constexpr ((MODE & OP_A) != 0) {
                const T cvisc = SCALED ? T(1) : (act ? gload<NTL>(a.cv + off) : T(0));
                const T cmass = act ? gload<NTL>(a.cv + P + off) : T(0);
                Tm[0][0] = cvisc * H[0][0];
                Tm[1][1] = cvisc * H[1][1];
                const T e01 = T(0.5) * cvisc * (H[0][1] + H[1][0]);
                Tm[0][1] = e01;
                Tm[1][0] = e01;
#pragma unroll
                for (int c = 0; c < 2; ++c) Fv[c][qx] = cmass * val[c][qx];
                if constexpr (CONV) {
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        cvc[c] = g0[c][qx] * be[0] + g1[c][qx] * be[1];
                        Fv[c][qx] += a.rho * cvc[c];   // rho (v° . grad u_c) det(J) w, tested with phi
                    }
                }
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
                if constexpr (CONV) {   // streamline term, tested with (grad-hat w_c) . beta / (det J w)
                    F0[c][qx] += sg * cvc[c] * be[0];
                    F1[c][qx] += sg * cvc[c] * be[1];
                }
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
        wave_sync();
        // thread t < 2 sums the vertices (0, t) and (1, t); the x-shared vertex (1, t)
        // is added into the right neighbour's (0, t) along the row
        double s0 = 0.0, s1 = 0.0;
        if (inwave && t < 2) {
            s0 = pbuf[wave][slot][0][2 * t] + pbuf[wave][slot][1][2 * t] + pbuf[wave][slot][2][2 * t];
            s1 = pbuf[wave][slot][0][2 * t + 1] + pbuf[wave][slot][1][2 * t + 1] + pbuf[wave][slot][2][2 * t + 1];
            pxb[wave][slot][t] = s1;
        }
        wave_sync();
        if (act && t < 2) {
            if (ix > 0) s0 += slot > 0 ? pxb[wave][slot - 1][t] : pcarry[wave][(ch + 1) & 1][t];
            const uint32_t pf = a.info[cell].z;
            const int n0 = a.pmap[cell * 4 + 2 * t], n1 = a.pmap[cell * 4 + 2 * t + 1];
            if constexpr (ATOM) {
                unsafeAtomicAdd(&a.q[n0], s0);
                if (ix == a.nx - 1) unsafeAtomicAdd(&a.q[n1], s1);
                else if (slot == CPW - 1) pcarry[wave][ch & 1][t] = s1;
            } else {
                {
                    const double tot = ((pf >> (2 * t)) & 1u) ? s0 : a.q[n0] + s0;
                    a.q[n0] = (RES && ((pf >> (16 + 2 * t)) & 1u)) ? a.fp[n0] - tot : tot;
                }
                if (ix == a.nx - 1) {
                    const double tot = ((pf >> (2 * t + 1)) & 1u) ? s1 : a.q[n1] + s1;
                    a.q[n1] = (RES && ((pf >> (16 + 2 * t + 1)) & 1u)) ? a.fp[n1] - tot : tot;
                } else if (slot == CPW - 1) {
                    pcarry[wave][ch & 1][t] = s1;
                }
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
        wave_sync();
        if (inwave) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    B[((c * 2 + 0) * 3 + t) * 3 + i] = ws[c][i];
                    B[((c * 2 + 1) * 3 + t) * 3 + i] = wd[c][i];
                }
        }
        wave_sync();
        T out[2][3];   // [comp][j] for the nodes (i, j) of this thread's column
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            T WS[3], WD[3];
#pragma unroll
            for (int q2 = 0; q2 < 3; ++q2) {
                WS[q2] = inwave ? B[((c * 2 + 0) * 3 + q2) * 3 + t] : T(0);
                WD[q2] = inwave ? B[((c * 2 + 1) * 3 + q2) * 3 + t] : T(0);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T s = T(0);
#pragma unroll
                for (int q2 = 0; q2 < 3; ++q2) s += cS<T>(q2, j) * WS[q2] + cD<T>(q2, j) * WD[q2];
                out[c][j] = s;
            }
        }
        if (inwave && t == 2) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j) xb[wave][slot][c * 3 + j] = out[c][j];
        }
        wave_sync();
        if (act) {
            if (t == 0 && ix > 0) {
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        out[c][j] += slot > 0 ? xb[wave][slot - 1][c * 3 + j] : xcarry[wave][(ch + 1) & 1][c * 3 + j];
            }
            if (t != 2 || ix == a.nx - 1) {
                const uint4 inf = a.info[cell];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int ln = t + 3 * j;
                    if constexpr (ATOM) {
                        const int node = a.vmap[cell * NLOC + ln];
                        if ((inf.x >> ln) & 1u) {
                            if constexpr ((MODE & OP_A) != 0) {
#pragma unroll
                                for (int c = 0; c < 2; ++c) a.v[c * a.nvn + node] = a.u[c * a.nvn + node];
                            }
                            continue;
                        }
#pragma unroll
                        for (int c = 0; c < 2; ++c) unsafeAtomicAdd(&a.v[c * a.nvn + node], out[c][j]);
                        continue;
                    }
                    if ((inf.x >> ln) & 1u) continue;
                    const int node = a.vmap[cell * NLOC + ln];
                    const bool first = (inf.y >> ln) & 1u;
                    if ((CHEB || RES) && ((inf.w >> ln) & 1u)) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const int64_t i = c * a.nvn + node;
                            const T tot = first ? out[c][j] : a.v[i] + out[c][j];
                            if constexpr (CHEB) {
                                const T xi = a.x[i];
                                const T dn = a.c1 * (a.first ? xi : a.d[i]) + a.c2 * a.dinv[i] * (a.r[i] - tot);
                                if (a.store_d) a.d[i] = dn;
                                a.x[i] = xi + dn;
                            } else {
                                a.v[i] = a.r[i] - tot;
                            }
                        }
                    } else if (first) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) a.v[c * a.nvn + node] = out[c][j];
                    } else {
#pragma unroll
                        for (int c = 0; c < 2; ++c) a.v[c * a.nvn + node] += out[c][j];
                    }
                }
            } else if (slot == CPW - 1) {
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j) xcarry[wave][ch & 1][c * 3 + j] = out[c][j];
            }
        }
    }
    wave_sync();
    }   // chunk loop
}

// ============================================================== launchers
// Phase p holds whole rows of cells (cells[0] each); one wavefront walks a row.
// WPB > 1: in 3D the wavefronts of a workgroup share a row (one row per workgroup);
// in 2D each wavefront keeps its own row (two per workgroup)
template <typename T, int MODE, int WPB, bool NTL, int WPE, int ZG = 1>
static void launch_one(const Level& L, const CellArgs<T>& args, hipStream_t s) {
    if (args.nrows <= 0) return;
    if (L.dim == 3) {
        constexpr bool RS = WPB > 1;
        const int64_t grid = args.nrows;   // one workgroup per row (per z-group of rows)
        // the corrector terms use the stored geometry, also where the FP32 applies form it
        // from the vertices
        if constexpr ((MODE & OP_CONV) == 0) {
            if (args.vd || args.vd64) {
                // forming the geometry takes more registers: at most three wavefronts per SIMD
                constexpr int WV = WPE > 3 ? 3 : WPE;
                hipLaunchKernelGGL((cell3d<T, MODE, WPB, RS, NTL, WV, true, ZG>), dim3((unsigned)grid), dim3(64 * WPB),
                                   0, s, args);
                return;
            }
        }
        hipLaunchKernelGGL((cell3d<T, MODE, WPB, RS, NTL, WPE, false, ZG>), dim3((unsigned)grid), dim3(64 * WPB), 0, s,
                           args);
    } else {
        constexpr int W2 = WPB > 1 ? 2 : 1;   // 2D: one row per wavefront, at most two
        const int64_t grid = (args.nrows + W2 - 1) / W2;   // one wavefront per row of cells
        hipLaunchKernelGGL((cell2d<T, MODE, W2, false, NTL>), dim3((unsigned)grid), dim3(64 * W2), 0, s, args);
    }
}

// launch variant v (0 .. 15): for v < 12, v % 3 selects 1, 2 or 4 wavefronts per
// workgroup (in 3D the wavefronts share one row; in 2D they own a row each, at most
// two); (v / 3) % 2 selects cached instead of streaming geometry loads; v / 6 caps the
// registers for one wavefront per SIMD more than the class reaches unconstrained
// (spills allowed).  v = 12 .. 15: three wavefronts share a row, (v - 12) % 2 cached
// loads, (v - 12) / 2 the register cap.  Three wavefronts fit five workgroups where
// four fit four (FP32 A, B classes), which fills the chip better when the rows of a
// phase are not a multiple of the four-wavefront slots (96^3: 2304 rows per phase).
// Unconstrained occupancy (3D): FP64 2 (A, B classes) or 1 (Stokes classes); FP32
// 3-4 (A, B classes) or 2 (Stokes classes).
template <typename T, int MODE, int WPB, bool NTL>
static void launch_capped(const Level& L, int cap, const CellArgs<T>& args, hipStream_t s) {
    constexpr bool STOKES = (MODE & OP_A) && (MODE & OP_BT);
    constexpr int W1 = sizeof(T) == 8 ? (STOKES ? 2 : 3) : (STOKES ? 3 : 4);
    // uncapped: FP64 A and B classes fit two wavefronts per SIMD (the row-shared
    // launches would otherwise take a few registers more and drop to one)
    constexpr int W0 = (sizeof(T) == 8 && !STOKES) ? 2 : 1;
    if (cap == 0) launch_one<T, MODE, WPB, NTL, W0>(L, args, s);
    else launch_one<T, MODE, WPB, NTL, W1>(L, args, s);
}

template <typename T, int MODE>
static void launch_mode(const Level& L, int variant, const CellArgs<T>& args, hipStream_t s) {
    if (variant >= 12) {
        const int w = variant - 12;
        const int cap = (w >> 1) & 1;
        if (w & 1) launch_capped<T, MODE, 3, false>(L, cap, args, s);
        else launch_capped<T, MODE, 3, true>(L, cap, args, s);
        return;
    }
    const int cap = (variant / 6) & 1;
    const bool plain = ((variant / 3) & 1) != 0;
    switch (variant % 3) {
        case 0: plain ? launch_capped<T, MODE, 1, false>(L, cap, args, s) : launch_capped<T, MODE, 1, true>(L, cap, args, s); break;
        case 1: plain ? launch_capped<T, MODE, 2, false>(L, cap, args, s) : launch_capped<T, MODE, 2, true>(L, cap, args, s); break;
        default: plain ? launch_capped<T, MODE, 4, false>(L, cap, args, s) : launch_capped<T, MODE, 4, true>(L, cap, args, s); break;
    }
}

template <typename T>
static CellArgs<T> phase_args(const Level& L, int phase, const T* K, const T* cv) {
    CellArgs<T> args{};
    args.cbeg = L.phase_off[phase];
    args.cend = L.phase_off[phase + 1];
    args.nx = L.geo.nx;   // cells per row: a whole x-line in 3D, a segment of one in 2D
    args.nrows = (args.cend - args.cbeg) / L.geo.nx;
    args.nchunks = L.geo.nchunks;
    args.wlast = L.geo.nx - (args.nchunks - 1) * L.geo.cpw;
    args.chunk0 = (args.cbeg / L.geo.nx) * args.nchunks;
    args.nchk = L.geo.nchk;
    args.nc = L.nc;
    args.nvn = L.nvn;
    args.plane = L.plane();
    args.vmap = L.d_vmap;
    args.info = L.d_info;
    args.pmap = L.d_pmap;
    args.K = K;
    args.cv = cv;
    if constexpr (sizeof(T) == 8) {
        args.cb = L.d_cb64;
        args.cs = L.d_cs64;
    } else {
        args.cb = L.d_cb32;
        args.cs = L.d_cs32;
    }
    args.rho = (T)L.rho;
    if constexpr (sizeof(T) == 4) {
        if (L.vgeo && L.dim == 3) {
            args.vd = L.d_vd32;
            args.cq = L.d_cq32;
            args.hx = (T)L.h[0];
            args.hy = (T)L.h[1];
            args.hz = (T)L.h[2];
        }
    } else {
        if (L.vgeo64 && L.dim == 3) {
            args.vd64 = L.d_vd64;
            args.cq = L.d_cq64;
            args.hx = L.h[0];
            args.hy = L.h[1];
            args.hz = L.h[2];
        }
    }
    return args;
}

template <typename T>
void launch_cell(const Level& L, int mode, int variant, int phase, const T* K, const T* cv, const T* u,
                 const double* p, T* v, double* q, hipStream_t s) {
    CellArgs<T> args = phase_args<T>(L, phase, K, cv);
    args.u = u;
    args.p = p;
    args.v = v;
    args.q = q;
    switch (mode) {
        case OP_A: launch_mode<T, OP_A>(L, variant, args, s); break;
        case OP_B: launch_mode<T, OP_B>(L, variant, args, s); break;
        case OP_BT: launch_mode<T, OP_BT>(L, variant, args, s); break;
        case OP_A | OP_BT: launch_mode<T, OP_A | OP_BT>(L, variant, args, s); break;
        case OP_A | OP_CONV: launch_mode<T, OP_A | OP_CONV>(L, variant, args, s); break;
        case OP_A | OP_BT | OP_B | OP_CONV: launch_mode<T, OP_A | OP_BT | OP_B | OP_CONV>(L, variant, args, s); break;
        default: launch_mode<T, OP_A | OP_BT | OP_B>(L, variant, args, s); break;
    }
}

template <typename T>
void launch_cell_all(const Level& L, int mode, int variant, const T* K, const T* cv, const T* u,
                     const double* p, T* v, double* q, hipStream_t s) {
    for (int ph = 0; ph < L.nphases(); ++ph) launch_cell<T>(L, mode, variant, ph, K, cv, u, p, v, q, s);
}

// every phase in one launch (modes A, B, B^T, A + B^T + B, and A or the Stokes apply
// with the corrector terms): one kernel zeroes the
// outputs, then each cell adds its contributions atomically and the cell kernel writes
// the wall rows itself (v = u when A is applied; B^T alone leaves them zero).  Shapes
// in 3D (kAtomShapes): 0 one wavefront per row; 1 four wavefronts share a row; 2, 3 one
// wavefront takes two or four rows along z (the plane they share summed in registers);
// 4 four wavefronts share a pair of rows along z; 5, 6 one wavefront per half or quarter
// row; the wall bits follow from the box faces,
// or on a level with fixed cells from the per-node wall mask.  In 2D (kAtomShapes2D): one
// wavefront per row segment, one (0) or two (1) wavefronts per workgroup; the cell info
// and the node map supply the wall bits, so fixed cells are honoured.
template <int ZG>
static int64_t atom_slots(const Level& L) {
    return (int64_t)L.cells[1] * ((L.cells[2] + ZG - 1) / ZG);
}

template <typename T>
void launch_cell_atomic(const Level& L, int mode, int shape, const T* K, const T* cv, const T* u, const double* p,
                        T* v, double* q, hipStream_t s) {
    CellArgs<T> args = phase_args<T>(L, 0, K, cv);
    args.cend = L.phase_off[L.nphases()];
    args.rowmap = L.d_atom_rows;
    args.wallmask = L.d_wall;
    args.cny = L.cells[1];
    args.cnz = L.cells[2];
    args.vnx = L.vnodes[0];
    args.vny = L.vnodes[1];
    args.vnz = L.vnodes[2];
    args.pnx = L.pnodes[0];
    args.pny = L.pnodes[1];
    args.dfaces = L.dfaces;
    args.u = u;
    args.p = p;
    args.v = v;
    args.q = q;
    launch_atomic_init<T>(L, (mode & (OP_A | OP_BT)) ? v : nullptr, (mode & OP_B) ? q : nullptr, s);
    auto go = [&](auto mc) {
        constexpr int M = decltype(mc)::value | OP_ATOM;
        if constexpr ((M & OP_FIXW) == 0) {
            if (L.dim == 2) {
                // every row segment of every phase; shape 0 one wavefront per workgroup, else two
                args.nrows = (args.cend - args.cbeg) / L.geo.nx;
                if (shape == 0) launch_one<T, M, 1, true, 1, 1>(L, args, s);
                else launch_one<T, M, 2, true, 1, 1>(L, args, s);
                return;
            }
        }
        // waves per SIMD the unfused classes reach: FP64 two (A, B, B^T), FP32 four; the
        // Stokes classes are left unconstrained
        constexpr bool STOKES = (M & OP_A) && (M & OP_BT);
        constexpr int W0 = (STOKES || (M & OP_CONV)) ? 1 : (sizeof(T) == 8 ? 2 : 4);
        // shapes 5 and 6: shape 0 with every row cut into two or four segments
        args.nseg = shape == 5 ? 2 : (shape == 6 ? 4 : 1);
        args.segch = (args.nchunks + args.nseg - 1) / args.nseg;
        switch (shape) {
            case 0: args.nrows = atom_slots<1>(L); launch_one<T, M, 1, true, W0, 1>(L, args, s); break;
            case 1: args.nrows = atom_slots<1>(L); launch_one<T, M, 4, true, W0, 1>(L, args, s); break;
            case 2: args.nrows = atom_slots<2>(L); launch_one<T, M, 1, true, W0, 2>(L, args, s); break;
            case 3: args.nrows = atom_slots<4>(L); launch_one<T, M, 1, true, W0, 4>(L, args, s); break;
            case 5:
            case 6: args.nrows = atom_slots<1>(L) * args.nseg; launch_one<T, M, 1, true, W0, 1>(L, args, s); break;
            default: args.nrows = atom_slots<2>(L); launch_one<T, M, 4, true, W0, 2>(L, args, s); break;
        }
    };
    switch (mode) {
        case OP_A:
            if (L.fixed_nodes && L.dim == 3) go(std::integral_constant<int, OP_A | OP_FIXW>{});
            else go(std::integral_constant<int, OP_A>{});
            break;
        case OP_B: go(std::integral_constant<int, OP_B>{}); break;
        case OP_BT: go(std::integral_constant<int, OP_BT>{}); break;
        case OP_A | OP_BT: go(std::integral_constant<int, OP_A | OP_BT>{}); break;
        case OP_A | OP_CONV: go(std::integral_constant<int, OP_A | OP_CONV>{}); break;
        case OP_A | OP_BT | OP_B | OP_CONV: go(std::integral_constant<int, OP_A | OP_BT | OP_B | OP_CONV>{}); break;
        default: go(std::integral_constant<int, OP_A | OP_BT | OP_B>{}); break;
    }
}

template <typename T>
void launch_cell_cheb(const Level& L, int variant, int phase, const T* K, const T* cv, T* x, T* d, const T* r,
                      const T* dinv, T* v, double c1, double c2, bool first, bool store_d, hipStream_t s) {
    CellArgs<T> args = phase_args<T>(L, phase, K, cv);
    args.v = v;
    args.x = x;
    args.d = d;
    args.r = r;
    args.dinv = dinv;
    args.c1 = (T)c1;
    args.c2 = (T)c2;
    args.first = first ? 1 : 0;
    args.store_d = store_d ? 1 : 0;
    launch_mode<T, OP_A | OP_CHEB>(L, variant, args, s);
}

template <typename T>
void launch_cell_cheb_all(const Level& L, int variant, const T* K, const T* cv, T* x, T* d, const T* r,
                          const T* dinv, T* v, double c1, double c2, bool first, bool store_d, hipStream_t s) {
    for (int ph = 0; ph < L.nphases(); ++ph)
        launch_cell_cheb<T>(L, variant, ph, K, cv, x, d, r, dinv, v, c1, c2, first, store_d, s);
}

template <typename T>
void launch_cell_res(const Level& L, int variant, int phase, const T* K, const T* cv, const T* u, const double* p,
                     const T* f_u, const double* f_p, T* r_u, double* r_p, hipStream_t s) {
    CellArgs<T> args = phase_args<T>(L, phase, K, cv);
    args.u = u;
    args.p = p;
    args.v = r_u;
    args.q = r_p;
    args.r = f_u;
    args.fp = f_p;
    launch_mode<T, OP_A | OP_BT | OP_B | OP_RES>(L, variant, args, s);
}

template <typename T>
void launch_cell_res_all(const Level& L, int variant, const T* K, const T* cv, const T* u, const double* p,
                         const T* f_u, const double* f_p, T* r_u, double* r_p, hipStream_t s) {
    for (int ph = 0; ph < L.nphases(); ++ph) launch_cell_res<T>(L, variant, ph, K, cv, u, p, f_u, f_p, r_u, r_p, s);
}

template void launch_cell_atomic<double>(const Level&, int, int, const double*, const double*, const double*,
                                         const double*, double*, double*, hipStream_t);
template void launch_cell_atomic<float>(const Level&, int, int, const float*, const float*, const float*,
                                        const double*, float*, double*, hipStream_t);
template void launch_cell<double>(const Level&, int, int, int, const double*, const double*, const double*,
                                  const double*, double*, double*, hipStream_t);
template void launch_cell<float>(const Level&, int, int, int, const float*, const float*, const float*,
                                 const double*, float*, double*, hipStream_t);
template void launch_cell_all<double>(const Level&, int, int, const double*, const double*, const double*,
                                      const double*, double*, double*, hipStream_t);
template void launch_cell_all<float>(const Level&, int, int, const float*, const float*, const float*,
                                     const double*, float*, double*, hipStream_t);
template void launch_cell_cheb_all<double>(const Level&, int, const double*, const double*, double*, double*,
                                           const double*, const double*, double*, double, double, bool, bool,
                                           hipStream_t);
template void launch_cell_cheb_all<float>(const Level&, int, const float*, const float*, float*, float*,
                                          const float*, const float*, float*, double, double, bool, bool, hipStream_t);
template void launch_cell_cheb<double>(const Level&, int, int, const double*, const double*, double*, double*,
                                       const double*, const double*, double*, double, double, bool, bool, hipStream_t);
template void launch_cell_cheb<float>(const Level&, int, int, const float*, const float*, float*, float*,
                                      const float*, const float*, float*, double, double, bool, bool, hipStream_t);
template void launch_cell_res<double>(const Level&, int, int, const double*, const double*, const double*,
                                      const double*, const double*, const double*, double*, double*, hipStream_t);
template void launch_cell_res<float>(const Level&, int, int, const float*, const float*, const float*,
                                     const double*, const float*, const double*, float*, double*, hipStream_t);
template void launch_cell_res_all<double>(const Level&, int, const double*, const double*, const double*,
                                          const double*, const double*, const double*, double*, double*,
                                          hipStream_t);
template void launch_cell_res_all<float>(const Level&, int, const float*, const float*, const float*,
                                         const double*, const float*, const double*, float*, double*, hipStream_t);

}  // namespace fsi
