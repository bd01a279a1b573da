// IFEM volume kernel for gfx950 (the comparison path, Sec. 2.3 and Tab.
// flops "IFEM"): the exact stencil of every interior node assembled on the
// fly from the stiffness rows of its 24 fine tetrahedra, fused into y = L x,
// r = f - L x and the multicolour Gauss-Seidel update.
//
// Same work decomposition as the surrogate kernel (a workgroup owns one
// macro, a slab of R planes and whole rows of the slab's bottom plane; each
// lane owns a column and marches up in k).  The blended coordinates of the
// level's nodes are computed once and kept in HBM (24 bytes per node); for
// every plane the workgroup stages x and the coordinates of rows j0-1 .. j1
// in LDS, loading the next plane while the current one is assembled, and a
// node reads its 15 neighbours of planes k-1, k, k+1 from the three staged
// planes.  Four plane buffers: the buffer of plane p is rewritten four planes
// later, after the barriers of the planes in between.  One translation unit
// per staging width KPT (the macro TS_KPT).
#include "ts_surrogate.h"

#ifndef TS_KPT
#error "TS_KPT must be defined"
#endif
// instruction kinds the scheduler may move across the per-tetrahedron
// barriers (0x100: LDS reads, so the next points load early)
#ifndef TS_IFEM_SCHED_MASK
#define TS_IFEM_SCHED_MASK 0x100
#endif

namespace ts {

// three plane buffers (48 KiB of LDS at staging width 2) and a 3-wave
// register budget: three workgroups per CU (with four buffers, 64 KiB, two)
#ifndef TS_IFEM_WAVES
#define TS_IFEM_WAVES 3
#endif
#ifndef TS_IFEM_NB
#define TS_IFEM_NB 3
#endif

// The macro's vertices in ascending global-id order, held in registers for
// the whole kernel; point() repeats node_xyz operation for operation, so
// every kernel computes bitwise the same blended coordinates.
struct OrderedGeom {
    double v[4][3], r[4];
    int ord[4];
    int affine;
    __device__ __forceinline__ void load(const MacroGeom& g) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int a = g.ord[q];
            ord[q] = a;
            v[q][0] = g.v[a][0];
            v[q][1] = g.v[a][1];
            v[q][2] = g.v[a][2];
            r[q] = g.r[a];
        }
        affine = g.affine;
    }
    __device__ __forceinline__ void point(int N, int i, int j, int k, double x[3]) const {
        const int m0 = N - i - j - k;
        double y0 = 0, y1 = 0, y2 = 0, rho = 0;
        const double invN = 1.0 / (double)N;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int a = ord[q];
            const int mu = a == 0 ? m0 : a == 1 ? i : a == 2 ? j : k;
            const double w = (double)mu * invN;
            y0 += w * v[q][0];
            y1 += w * v[q][1];
            y2 += w * v[q][2];
            rho += w * r[q];
        }
        if (affine) {
            x[0] = y0; x[1] = y1; x[2] = y2;
            return;
        }
        const double sc = rho / sqrt(y0 * y0 + y1 * y1 + y2 * y2);
        x[0] = sc * y0; x[1] = sc * y1; x[2] = sc * y2;
    }
};

// stiffness_row0 with the reciprocal of 6 |T| from the hardware estimate
// and two Newton steps (each doubles the correct bits: full FP64 precision)
// instead of a correctly rounded division, which costs about twice the
// instructions; the rows differ from stiffness_row0's by a few ulps
__device__ __forceinline__ void stiffness_row0_fast(const double* P0, const double* P1,
                                                    const double* P2, const double* P3,
                                                    double K[4]) {
    const double a0 = P1[0] - P0[0], a1 = P1[1] - P0[1], a2 = P1[2] - P0[2];
    const double b0 = P2[0] - P0[0], b1 = P2[1] - P0[1], b2 = P2[2] - P0[2];
    const double c0 = P3[0] - P0[0], c1 = P3[1] - P0[1], c2 = P3[2] - P0[2];
    const double g10 = b1 * c2 - b2 * c1, g11 = b2 * c0 - b0 * c2, g12 = b0 * c1 - b1 * c0;
    const double g20 = c1 * a2 - c2 * a1, g21 = c2 * a0 - c0 * a2, g22 = c0 * a1 - c1 * a0;
    const double g30 = a1 * b2 - a2 * b1, g31 = a2 * b0 - a0 * b2, g32 = a0 * b1 - a1 * b0;
    const double g00 = -(g10 + g20 + g30), g01 = -(g11 + g21 + g31), g02 = -(g12 + g22 + g32);
    const double det = a0 * g10 + a1 * g11 + a2 * g12;
    const double d6 = 6.0 * fabs(det);
    double sc = __builtin_amdgcn_rcp(d6);
    sc = fma(fma(-d6, sc, 1.0), sc, sc);
    sc = fma(fma(-d6, sc, 1.0), sc, sc);
    K[0] = (g00 * g00 + g01 * g01 + g02 * g02) * sc;
    K[1] = (g00 * g10 + g01 * g11 + g02 * g12) * sc;
    K[2] = (g00 * g20 + g01 * g21 + g02 * g22) * sc;
    K[3] = (g00 * g30 + g01 * g31 + g02 * g32) * sc;
}

#ifndef TS_IFEM_FAST_RCP
#define TS_IFEM_FAST_RCP 1
#endif

template <typename T, int MODE, int R, int KPT>
__global__ __launch_bounds__(VOL_THREADS) __attribute__((amdgpu_waves_per_eu(TS_IFEM_WAVES)))
void k_ifem_lds(
    const T* x, T* y, const T* __restrict__ f, const double* __restrict__ xyz,
    const int4* __restrict__ tiles, int n_tiles, int nt, const int* __restrict__ mlist,
    const unsigned* __restrict__ lanes, int N, int64_t B, int colour) {
    int macro, tile;
    if (!decode_block(n_tiles, nt, macro, tile, mlist)) return;
    const int4 td = tiles[tile];
    const int k0 = td.x, j0 = td.y, j1 = td.z;
    const int tid = (int)threadIdx.x;
    int i = 1, j = j0;
    const unsigned e0 = lanes[(size_t)tile * VOL_THREADS + tid];
    const bool act = e0 != 0xFFFFFFFFu;
    if (act) {
        i = (int)(e0 & 0xFFFFu);
        j = (int)(e0 >> 16);
    }
    const int nlive = act ? min(N - 1 - i - j, k0 + R - 1) - k0 + 1 : 0;
    const size_t base = (size_t)macro * B;
    const int64_t bbytes = B * (int64_t)sizeof(T);
    const __amdgpu_buffer_rsrc_t rx = block_rsrc(x + base, bbytes);
    const __amdgpu_buffer_rsrc_t ry = block_rsrc(y + base, bbytes);
    const __amdgpu_buffer_rsrc_t rf = block_rsrc(f ? f + base : x + base, bbytes);
    const __amdgpu_buffer_rsrc_t rc = block_rsrc(xyz + 3 * base, 3 * B * (int64_t)sizeof(double));

    // plane buffers: with four, the buffer of plane p is rewritten four
    // planes later, after the barriers in between; with three (less LDS, a
    // third workgroup per CU) a second barrier per plane keeps the next
    // write behind this plane's reads
    constexpr int NB = TS_IFEM_NB;
    __shared__ T bx[NB][KPT * VOL_THREADS];
    __shared__ double bp[NB][3][KPT * VOL_THREADS];

    const int jb = j0 - 1, jtri = jb * (jb - 1) / 2;
    const int nb = j - jb;
    const int srow = (jb + j - 1) * nb / 2;
    int po = (int)plane_off(N, k0 - 1);       // first point of the plane being staged
    int c = nb * (N + 2 - k0) - srow + i;     // lane's LDS index in plane k0 - 1
    int qa = N + 2 - k0 - j;
    int idx = (int)plane_off(N, k0) + j * (N + 1 - k0) - j * (j - 1) / 2 + i;
    int col = (i + 2 * j + 3 * k0) & 3;

    // staged registers: x and (x, y, z) of the lane's KPT entries of the
    // next plane (entries past the plane's range are never read)
    T sx[KPT];
    double sp[KPT][3];
    auto load_plane = [&](int p) {
        const int A = N + 1 - p;
        const int g0 = p <= N ? po + jb * A - jtri : 0;
#pragma unroll
        for (int s2 = 0; s2 < KPT; s2++) {
            const int e = g0 + tid + s2 * VOL_THREADS;
            sx[s2] = bload<T>(rx, e * (int)sizeof(T));
            sp[s2][0] = bload<double>(rc, (3 * e) * 8);
            sp[s2][1] = bload<double>(rc, (3 * e + 1) * 8);
            sp[s2][2] = bload<double>(rc, (3 * e + 2) * 8);
        }
        po += A * (A + 1) / 2;
    };
    load_plane(k0 - 1);
#pragma unroll
    for (int st = 0; st < R + 2; st++) {
        const int p = k0 - 1 + st;
        {
            const int b = st % NB;
#pragma unroll
            for (int s2 = 0; s2 < KPT; s2++) {
                const int e = tid + s2 * VOL_THREADS;
                bx[b][e] = sx[s2];
                bp[b][0][e] = sp[s2][0];
                bp[b][1][e] = sp[s2][1];
                bp[b][2][e] = sp[s2][2];
            }
        }
        __syncthreads();
        if (st + 1 < R + 2) load_plane(p + 1);
        if (st >= 2) {
            const int r = st - 2;  // node (i, j, k0 + r)
            const bool live = r < nlive;
            const bool upd = MODE == 2 ? (live && col == colour) : live;
            if (upd) {
                // the 15 neighbours: plane k from buffer (st-1), k-1 from
                // (st-2), k+1 from st; LDS index and row offset per plane
                const int bm = (st + NB - 2) % NB, b0 = (st + NB - 1) % NB, bq = st % NB;
                const int cq = c, qq = qa;               // plane k + 1
                const int c0 = c + nb, q0 = qa + 1;      // plane k
                const int cm = c + 2 * nb, qm = qa + 2;  // plane k - 1
                int li[NW], lb[NW];
                li[0] = c0;            lb[0] = b0;
                li[1] = c0 - 1;        lb[1] = b0;
                li[2] = c0 + 1;        lb[2] = b0;
                li[3] = c0 - q0 - 1;   lb[3] = b0;
                li[4] = c0 + q0;       lb[4] = b0;
                li[5] = c0 - q0;       lb[5] = b0;
                li[6] = c0 + q0 - 1;   lb[6] = b0;
                li[7] = cm;            lb[7] = bm;
                li[8] = cm + 1;        lb[8] = bm;
                li[9] = cm + qm;       lb[9] = bm;
                li[10] = cm + qm - 1;  lb[10] = bm;
                li[11] = cq;           lb[11] = bq;
                li[12] = cq - 1;       lb[12] = bq;
                li[13] = cq - qq - 1;  lb[13] = bq;
                li[14] = cq - qq;      lb[14] = bq;
                // the node's point, then per tetrahedron its three other
                // points read from LDS just before use (scheduling barriers
                // between tetrahedra keep the live register set small)
                const double P0[3] = {bp[b0][0][c0], bp[b0][1][c0], bp[b0][2][c0]};
                double s[NW];
#pragma unroll
                for (int w = 0; w < NW; w++) s[w] = 0.0;
#pragma unroll
                for (int t = 0; t < 24; t++) {
                    const int w1 = kTets24.t[t][1], w2 = kTets24.t[t][2], w3 = kTets24.t[t][3];
                    const double P1[3] = {bp[lb[w1]][0][li[w1]], bp[lb[w1]][1][li[w1]],
                                          bp[lb[w1]][2][li[w1]]};
                    const double P2[3] = {bp[lb[w2]][0][li[w2]], bp[lb[w2]][1][li[w2]],
                                          bp[lb[w2]][2][li[w2]]};
                    const double P3[3] = {bp[lb[w3]][0][li[w3]], bp[lb[w3]][1][li[w3]],
                                          bp[lb[w3]][2][li[w3]]};
                    double K[4];
                    if constexpr (TS_IFEM_FAST_RCP)
                        stiffness_row0_fast(P0, P1, P2, P3, K);
                    else
                        stiffness_row0(P0, P1, P2, P3, K);
                    s[0] += K[0];
                    s[w1] += K[1];
                    s[w2] += K[2];
                    s[w3] += K[3];
                    __builtin_amdgcn_sched_barrier(TS_IFEM_SCHED_MASK);
                }
                T off = (T)0;
#pragma unroll
                for (int w = 1; w < NW; w++) off += (T)s[w] * bx[lb[w]][li[w]];
                const int o = idx * (int)sizeof(T);
                if (MODE == 2) {
                    bstore<T>(ry, o, (bload<T>(rf, o) - off) / (T)s[0]);
                } else {
                    const T v = (T)s[0] * bx[b0][c0] + off;
                    bstore<T>(ry, o, MODE == 0 ? v : bload<T>(rf, o) - v);
                }
            }
            const int Ak = N + 1 - (k0 + r);
            idx += Ak * (Ak + 1) / 2 - j;
            col = (col + 3) & 3;
        }
        c -= nb;
        qa -= 1;
        if constexpr (NB == 3) __syncthreads();
    }
}

#define TS_CAT2(a, b, c, d) a##b##c##d
#define TS_CAT(a, b, c, d) TS_CAT2(a, b, c, d)

void TS_CAT(launch_ifem, _k, TS_KPT, )(const Level& L, const double* xyz, int nt,
                                        const int* mlist, int dtype, int mode, const void* x,
                                        void* y, const void* f, int colour, hipStream_t s) {
    const dim3 grid((unsigned)(((nt + 7) / 8) * 8 * L.n_lds_tiles)), blk(VOL_THREADS);
    const unsigned* lanes = mode == 2 ? L.gs_lanes.p : L.ap_lanes.p;
#define TS_GO(T_, M_)                                                                       \
    k_ifem_lds<T_, M_, VOL_R, TS_KPT><<<grid, blk, 0, s>>>(                                  \
        (const T_*)x, (T_*)y, (const T_*)f, xyz, L.lds_tiles.p, L.n_lds_tiles, nt, mlist,     \
        lanes, L.N, L.B, colour)
    if (dtype == TS_F64) {
        if (mode == 0) TS_GO(double, 0); else if (mode == 1) TS_GO(double, 1); else TS_GO(double, 2);
    } else {
        if (mode == 0) TS_GO(float, 0); else if (mode == 1) TS_GO(float, 1); else TS_GO(float, 2);
    }
#undef TS_GO
}

}  // namespace ts
