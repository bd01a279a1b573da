// Stencil kernels for gfx950 besides the surrogate volume kernel: IFEM
// volume rows (Sec. 2.3, element-wise assembly from the 24 fine tetrahedra
// at a node; the comparison path), lower-primitive rows (faces, edges,
// vertices: element-wise assembly over all adjacent macros, with the
// per-copy partial stencils stored once per level), and the dispatch of the
// surrogate volume kernel.  Each kernel serves y = L x, r = f - L x and the
// Gauss-Seidel update u_I = (f_I - sum_{w != mc} s_w u_{I_w}) / s_mc
// (eq. iteration-scheme).
#include "ts_surrogate.h"

namespace ts {

// The 7 points (i,j), (i-1,j), (i+1,j), (i,j-1), (i,j+1), (i+1,j-1), (i-1,j+1)
// of plane p.  c is the block index of (i, j, p) and A = N + 1 - p the side
// of plane p (row j holds A - j points), so row j-1 starts A - j + 1 points
// before row j and row j+1 starts A - j points after it.  The two points with
// index sum i + j + 1 exist only if i + j + 2 <= A.
template <typename T>
__device__ __forceinline__ void load7(const T* xm, int c, int A, int i, int j, T o[7]) {
    const bool hi = i + j + 2 <= A;
    const int rs = c - (A - j + 1);
    const int rn = c + (A - j);
    o[0] = xm[c];
    o[1] = xm[c - 1];
    o[2] = hi ? xm[c + 1] : (T)0;
    o[3] = xm[rs];
    o[4] = hi ? xm[rn] : (T)0;
    o[5] = xm[rs + 1];
    o[6] = xm[rn - 1];
}

// IFEM: the exact stencil from the 24 fine tetrahedra at the node.
struct IfemW {
    MacroGeom g;
    int N, i, j;
    __device__ __forceinline__ void weights(int k, double s[NW]) const {
        ifem_partial_stencil(g, N, i, j, k, s);
    }
};

// Volume kernel body ----------------------------------------------------------
// MODE 0: y = L x; 1: y = f - L x; 2: Gauss-Seidel update of colour `colour`
// in place (x == y).  Block indices advance incrementally: from plane p to
// p + 1 the index of (i, j) grows by T(A) - j with T(A) = A (A + 1) / 2 the
// size of plane p and A = N + 1 - p.
template <typename T, typename W, int MODE, int R, class WP>
__device__ __forceinline__ void volume_body(const T* xm, T* ym, const T* fm, WP& wp, int N,
                                            int i, int j, int k0, int kend, int colour) {
    T pm[7], p0[7], pp[7];
    int A = N + 2 - k0;  // side of plane k0 - 1
    int c = (int)bidx(N, i, j, k0 - 1);
    load7(xm, c, A, i, j, pm);
    c += A * (A + 1) / 2 - j;
    A -= 1;
    load7(xm, c, A, i, j, p0);
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int k = k0 + r;
        if (k > kend) break;
        const int cn = c + A * (A + 1) / 2 - j;
        load7(xm, cn, A - 1, i, j, pp);
        if (MODE == 2) {
            if (((i + 2 * j + 3 * k) & 3) == colour) {
                W s[NW];
                wp.weights(k, s);
                const T off = off_sum<T, W>(s, pm, p0, pp);
                ym[c] = (fm[c] - off) / (T)s[0];
            }
        } else {
            W s[NW];
            wp.weights(k, s);
            const T v = (T)s[0] * p0[0] + off_sum<T, W>(s, pm, p0, pp);
            if (MODE == 0)
                ym[c] = v;
            else
                ym[c] = fm[c] - v;
        }
#pragma unroll
        for (int q = 0; q < 7; q++) {
            pm[q] = p0[q];
            p0[q] = pp[q];
        }
        c = cn;
        A -= 1;
    }
}

template <typename T, int MODE, int R>
__global__ __launch_bounds__(VOL_THREADS) void k_ifem_volume(
    const T* x, T* y, const T* __restrict__ f, const MacroGeom* __restrict__ geom,
    const int2* __restrict__ tiles, int n_tiles, int nt, const int* __restrict__ mlist, int N,
    int64_t B, int colour) {
    int macro, tile;
    if (!decode_block(n_tiles, nt, macro, tile, mlist)) return;
    const int2 td = tiles[tile];
    const int k0 = td.x, Mr = N - 1 - k0;
    const int pos = td.y + (int)threadIdx.x;
    if (pos >= (Mr - 1) * Mr / 2) return;
    int i, j;
    pos_to_ij(pos, Mr, i, j);
    const int kend = min(N - 1 - i - j, k0 + R - 1);
    IfemW wp;
    wp.g = geom[macro];
    wp.N = N;
    wp.i = i;
    wp.j = j;
    const size_t base = (size_t)macro * B;
    volume_body<T, double, MODE, R>(x + base, y + base, f ? f + base : nullptr, wp, N, i, j, k0,
                                 kend, colour);
}

// Lower primitives -------------------------------------------------------------
// Block-index offsets of the 15 stencil neighbours of the node at block index
// base = (i, j, k), from its row j and the side A = N + 1 - k of its plane:
// rows j-1 / j+1 start A - j + 1 points before / A - j points after row j;
// plane k+1 starts T(A) - j points after (i, j, k) (T(A) = A (A + 1) / 2) and
// plane k-1 ends T(A + 1) - j points before it.
__device__ __forceinline__ void nbr_index(int base, int A, int j, int o[NW]) {
    const int rs = base - (A - j + 1), rn = base + (A - j);
    const int bm = base - (A + 1) * (A + 2) / 2 + j;
    const int tp = base + A * (A + 1) / 2 - j;
    o[0] = base;
    o[1] = base - 1;
    o[2] = base + 1;
    o[3] = rs;
    o[4] = rn;
    o[5] = rs + 1;
    o[6] = rn - 1;
    o[7] = bm;
    o[8] = bm + 1;
    o[9] = bm + (A + 1 - j);
    o[10] = bm + (A - j);
    o[11] = tp;
    o[12] = tp - 1;
    o[13] = tp - (A - j);
    o[14] = tp - (A - j) + 1;
}

// General path: one thread per listed face/edge/vertex node, summing over the
// node's copies the element-wise partial stencil of each adjacent macro,
// assembled on the fly.  MODE 0: y = L x; 1: y = f - L x, written to every
// copy; 2: Gauss-Seidel value (f - off) / diag into tmp[t].
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_iface(
    const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ f,
    const int* __restrict__ off, const int4* __restrict__ cp,
    const unsigned char* __restrict__ flag, const int* __restrict__ list, int n,
    const MacroGeom* __restrict__ geom, int N, int64_t B, double* __restrict__ tmp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int node = list ? list[t] : t;
    const int c0 = off[node], c1 = off[node + 1];
    const int4 q0 = cp[c0];
    const size_t s0 = (size_t)q0.x * B + bidx(N, q0.y, q0.z, q0.w);
    if (flag[node] & 1) {
        if (MODE != 2)
            for (int c = c0; c < c1; c++) {
                const int4 q = cp[c];
                y[(size_t)q.x * B + bidx(N, q.y, q.z, q.w)] = (T)0;
            }
        return;
    }
    double dg = 0.0, of = 0.0;
    for (int c = c0; c < c1; c++) {
        const int4 q = cp[c];
        double s[NW];
        ifem_partial_stencil(geom[q.x], N, q.y, q.z, q.w, s);
        const T* xm = x + (size_t)q.x * B;
        int o[NW];
        nbr_index((int)bidx(N, q.y, q.z, q.w), N + 1 - q.w, q.z, o);
        dg += s[0];
#pragma unroll
        for (int w = 1; w < NW; w++)
            if (inside(N, q.y + dir_i(w), q.z + dir_j(w), q.w + dir_k(w))) of += s[w] * (double)xm[o[w]];
    }
    if (MODE == 2) {
        tmp[t] = ((double)f[s0] - of) / dg;
        return;
    }
    double v = dg * (double)x[s0] + of;
    if (MODE == 1) v = (double)f[s0] - v;
    for (int c = c0; c < c1; c++) {
        const int4 q = cp[c];
        y[(size_t)q.x * B + bidx(N, q.y, q.z, q.w)] = (T)v;
    }
}

// Face path: free nodes of interior faces, each with exactly two copies.  The
// element-wise partial stencils of both copies are stored once per level as
// struct of arrays [copy][w][node], so consecutive lanes load consecutive
// weights.  Same modes as k_iface; list (optional) selects positions.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_face2(
    const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ f,
    const int4* __restrict__ cp, const double* __restrict__ sten, int n2,
    const int* __restrict__ list, int n, int N, int64_t B, double* __restrict__ tmp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int q = list ? list[t] : t;
    double dg = 0.0, of = 0.0;
    size_t slot[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const int4 c = cp[(size_t)r * n2 + q];
        const double* sw = sten + (size_t)r * NW * n2 + q;
        const T* xm = x + (size_t)c.x * B;
        int o[NW];
        const int base = (int)bidx(N, c.y, c.z, c.w);
        nbr_index(base, N + 1 - c.w, c.z, o);
        slot[r] = (size_t)c.x * B + base;
        dg += sw[0];
#pragma unroll
        for (int w = 1; w < NW; w++)
            if (inside(N, c.y + dir_i(w), c.z + dir_j(w), c.w + dir_k(w)))
                of += sw[(size_t)w * n2] * (double)xm[o[w]];
    }
    if (MODE == 2) {
        tmp[t] = ((double)f[slot[0]] - of) / dg;
        return;
    }
    double v = dg * (double)x[slot[0]] + of;
    if (MODE == 1) v = (double)f[slot[0]] - v;
    y[slot[0]] = (T)v;
    y[slot[1]] = (T)v;
}

__global__ __launch_bounds__(128) void k_face2_stencils(const int4* __restrict__ cp, int n2,
                                                        const MacroGeom* __restrict__ geom, int N,
                                                        double* __restrict__ sten) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * n2) return;
    const int r = t / n2, q = t - r * n2;
    const int4 c = cp[t];
    double s[NW];
    ifem_partial_stencil(geom[c.x], N, c.y, c.z, c.w, s);
#pragma unroll
    for (int w = 0; w < NW; w++) sten[((size_t)r * NW + w) * n2 + q] = s[w];
}

const double* face_stencils(Mesh& M, int lam, hipStream_t s) {
    Level& L = M.level(lam);
    if (!L.f2_sten.p && L.n_f2) {
        L.f2_sten.alloc((size_t)2 * NW * L.n_f2);
        k_face2_stencils<<<(2 * L.n_f2 + 127) / 128, 128, 0, s>>>(L.f2_cp.p, L.n_f2, M.d_geom.p, L.N, L.f2_sten.p);
        TS_HIP(hipGetLastError());
    }
    return L.f2_sten.p;
}

template <typename T>
__global__ __launch_bounds__(256) void k_iface_scatter(
    T* __restrict__ u, const double* __restrict__ tmp, const int* __restrict__ off,
    const int4* __restrict__ cp, const int* __restrict__ list, int n, int N, int64_t B) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int node = list[t];
    const T v = (T)tmp[t];
    for (int c = off[node]; c < off[node + 1]; c++) {
        const int4 q = cp[c];
        u[(size_t)q.x * B + bidx(N, q.y, q.z, q.w)] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_face2_scatter(T* __restrict__ u, const double* __restrict__ tmp,
                                                       const int4* __restrict__ cp, int n2,
                                                       const int* __restrict__ list, int n, int N,
                                                       int64_t B) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int q = list[t];
    const T v = (T)tmp[t];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const int4 c = cp[(size_t)r * n2 + q];
        u[(size_t)c.x * B + bidx(N, c.y, c.z, c.w)] = v;
    }
}

// Launchers --------------------------------------------------------------------

static int grid_volume(const Level& L, int64_t nt) {
    return (int)(((nt + 7) / 8) * 8 * L.n_tiles);
}

#define TS_DECL(Q, K)                                                                     \
    void launch_surr_q##Q##_k##K(const Level& L, int nt, const LevelOp& lo, int dtype,    \
                                 int center, int mode, const void* x, void* y,            \
                                 const void* f, int colour, hipStream_t s);
TS_DECL(1, 2) TS_DECL(1, 4) TS_DECL(1, 8)
TS_DECL(2, 2) TS_DECL(2, 4) TS_DECL(2, 8)
TS_DECL(3, 2) TS_DECL(3, 4) TS_DECL(3, 8)
TS_DECL(4, 2) TS_DECL(4, 4) TS_DECL(4, 8)
#undef TS_DECL

void launch_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                   const void* f, int colour, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const LevelOp& lo = *op->lv.at(lam);
    const int nt = (int)M.nt, q = op->p.q, c = op->p.center;
    if (lo.n_ifem)  // selective surrogate: these macros keep IFEM rows
        launch_ifem_volume(op, lam, dtype == TS_F16W ? TS_F32 : dtype, mode, x, y, f, colour, s,
                           lo.ifem_list.p, lo.n_ifem);
    if (lo.n_sur == 0) return;
    const int kpt = L.lds_kpt <= 2 ? 2 : L.lds_kpt <= 4 ? 4 : 8;
    TS_REQUIRE(L.lds_kpt <= 8, TS_EINVAL, "level too large for the surrogate volume kernel");
#define TS_GO(Q, K) launch_surr_q##Q##_k##K(L, nt, lo, dtype, c, mode, x, y, f, colour, s)
    switch (q * 16 + kpt) {
        case 18: TS_GO(1, 2); break;
        case 20: TS_GO(1, 4); break;
        case 24: TS_GO(1, 8); break;
        case 34: TS_GO(2, 2); break;
        case 36: TS_GO(2, 4); break;
        case 40: TS_GO(2, 8); break;
        case 50: TS_GO(3, 2); break;
        case 52: TS_GO(3, 4); break;
        case 56: TS_GO(3, 8); break;
        case 66: TS_GO(4, 2); break;
        case 68: TS_GO(4, 4); break;
        case 72: TS_GO(4, 8); break;
        default: throw Error{TS_EINVAL, "unsupported surrogate degree"};
    }
#undef TS_GO
    TS_HIP(hipGetLastError());
}

template <typename T>
static void run_ifem_volume(const Mesh& M, const Level& L, int mode, const void* x, void* y,
                            const void* f, int colour, hipStream_t s, const int* ml, int nt) {
    const dim3 grid(grid_volume(L, nt)), blk(VOL_THREADS);
    if (grid.x == 0) return;
    const T* xp = (const T*)x;
    T* yp = (T*)y;
    const T* fp = (const T*)f;
    if (mode == 0)
        k_ifem_volume<T, 0, VOL_R><<<grid, blk, 0, s>>>(xp, yp, fp, M.d_geom.p, L.tiles.p, L.n_tiles, nt, ml, L.N, L.B, colour);
    else if (mode == 1)
        k_ifem_volume<T, 1, VOL_R><<<grid, blk, 0, s>>>(xp, yp, fp, M.d_geom.p, L.tiles.p, L.n_tiles, nt, ml, L.N, L.B, colour);
    else
        k_ifem_volume<T, 2, VOL_R><<<grid, blk, 0, s>>>(yp, yp, fp, M.d_geom.p, L.tiles.p, L.n_tiles, nt, ml, L.N, L.B, colour);
}

void launch_ifem_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                        const void* f, int colour, hipStream_t s, const int* mlist, int n_list) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const int nt = n_list >= 0 ? n_list : (int)M.nt;
    if (nt == 0) return;
    if (dtype == TS_F64)
        run_ifem_volume<double>(M, L, mode, x, y, f, colour, s, mlist, nt);
    else
        run_ifem_volume<float>(M, L, mode, x, y, f, colour, s, mlist, nt);
    TS_HIP(hipGetLastError());
}

// Lower-primitive rows: phase < 0 handles every node (apply / residual);
// phase >= 0 computes the Gauss-Seidel values of that phase into tmp (face
// fast path first, then the general nodes after it in tmp).
void launch_iface(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                  const void* f, int phase, double* tmp, hipStream_t s) {
    Mesh& M = op->mesh->m;
    const Level& L = M.level(lam);
    const double* sten = face_stencils(M, lam, s);
    const int* l2 = phase >= 0 ? L.f2_phase[phase].p : nullptr;
    const int n2 = phase >= 0 ? L.n_f2_phase[phase] : L.n_f2;
    const int* lr = phase >= 0 ? L.rest_phase[phase].p : L.rest.p;
    const int nr = phase >= 0 ? L.n_rest_phase[phase] : L.n_rest;
    double* tmp_r = tmp ? tmp + n2 : nullptr;
#define TS_F2(T_, M_)                                                                         \
    k_face2<T_, M_><<<(n2 + 255) / 256, 256, 0, s>>>((const T_*)x, (T_*)y, (const T_*)f,       \
                                                     L.f2_cp.p, sten, L.n_f2, l2, n2, L.N,    \
                                                     L.B, tmp)
#define TS_IF(T_, M_)                                                                         \
    k_iface<T_, M_><<<(nr + 255) / 256, 256, 0, s>>>((const T_*)x, (T_*)y, (const T_*)f,       \
                                                     L.if_off.p, L.if_copy.p, L.if_flag.p, lr, \
                                                     nr, M.d_geom.p, L.N, L.B, tmp_r)
    if (n2) {
        if (dtype == TS_F64) {
            if (mode == 0) TS_F2(double, 0); else if (mode == 1) TS_F2(double, 1); else TS_F2(double, 2);
        } else {
            if (mode == 0) TS_F2(float, 0); else if (mode == 1) TS_F2(float, 1); else TS_F2(float, 2);
        }
    }
    if (nr) {
        if (dtype == TS_F64) {
            if (mode == 0) TS_IF(double, 0); else if (mode == 1) TS_IF(double, 1); else TS_IF(double, 2);
        } else {
            if (mode == 0) TS_IF(float, 0); else if (mode == 1) TS_IF(float, 1); else TS_IF(float, 2);
        }
    }
#undef TS_F2
#undef TS_IF
    TS_HIP(hipGetLastError());
}

void launch_iface_scatter(const ts_op* op, int lam, int dtype, int phase, const double* tmp,
                          void* u, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const int n2 = L.n_f2_phase[phase], nr = L.n_rest_phase[phase];
    if (n2) {
        if (dtype == TS_F64)
            k_face2_scatter<double><<<(n2 + 255) / 256, 256, 0, s>>>((double*)u, tmp, L.f2_cp.p, L.n_f2, L.f2_phase[phase].p, n2, L.N, L.B);
        else
            k_face2_scatter<float><<<(n2 + 255) / 256, 256, 0, s>>>((float*)u, tmp, L.f2_cp.p, L.n_f2, L.f2_phase[phase].p, n2, L.N, L.B);
    }
    if (nr) {
        if (dtype == TS_F64)
            k_iface_scatter<double><<<(nr + 255) / 256, 256, 0, s>>>((double*)u, tmp + n2, L.if_off.p, L.if_copy.p, L.rest_phase[phase].p, nr, L.N, L.B);
        else
            k_iface_scatter<float><<<(nr + 255) / 256, 256, 0, s>>>((float*)u, tmp + n2, L.if_off.p, L.if_copy.p, L.rest_phase[phase].p, nr, L.N, L.B);
    }
    TS_HIP(hipGetLastError());
}

}  // namespace ts
