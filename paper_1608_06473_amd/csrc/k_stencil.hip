// Stencil kernels for gfx950: surrogate volume rows (Sec. 3.4 eq. ts with
// the line-wise 1D reduction of the surrogate polynomials), IFEM volume rows
// (Sec. 2.3, element-wise assembly from the 24 fine tetrahedra at a node),
// and lower-primitive rows (faces, edges, vertices: element-wise assembly
// over all adjacent macros).  Each kernel serves y = L x, r = f - L x and the
// Gauss-Seidel update u_I = (f_I - sum_{w != mc} s_w u_{I_w}) / s_mc
// (eq. iteration-scheme).
//
// Volume work decomposition: a workgroup takes one macro, a slab of
// VOL_R planes k0 .. k0+VOL_R-1 and 256 consecutive (i, j) positions of
// plane k0's interior triangle; each lane owns a column (i, j) and marches up
// in k.  Neighbour values of planes k-1, k, k+1 stay in registers (a rolling
// 3-plane window of 7 points each), so every step loads only the 7 points of
// plane k+1; consecutive lanes are consecutive i in a row, so the loads and
// stores are coalesced.  The 15 surrogate polynomials are reduced once per
// lane to 1D polynomials in zeta (the line-wise reduction of Sec. 3.4) and
// evaluated with q FMAs per weight and step.
#include "ts_internal.h"

namespace ts {

template <int Q>
struct Basis {
    static constexpr int MQ = (Q + 1) * (Q + 2) * (Q + 3) / 6;
    int l[MQ], m[MQ], n[MQ];
    constexpr Basis() : l(), m(), n() {
        int c = 0;
        for (int d = 0; d <= Q; d++)
            for (int a = d; a >= 0; a--)
                for (int b = d - a; b >= 0; b--) {
                    l[c] = a;
                    m[c] = b;
                    n[c] = d - a - b;
                    c++;
                }
    }
};

// position in the interior triangle of plane k0 -> (i, j); rows j = 1..Mr-1
// hold Mr - j positions each (Mr = N - 1 - k0)
__device__ __forceinline__ void pos_to_ij(int pos, int Mr, int& i, int& j) {
    const double a = 2.0 * Mr - 1.0;
    int J = (int)((a - sqrt(a * a - 8.0 * pos)) * 0.5);
    if (J < 0) J = 0;
    while (J > 0 && J * (2 * Mr - J - 1) / 2 > pos) J--;
    while ((J + 1) * (2 * Mr - J - 2) / 2 <= pos) J++;
    j = J + 1;
    i = pos - J * (2 * Mr - J - 1) / 2 + 1;
}

// the 7 points (i,j), (i-1,j), (i+1,j), (i,j-1), (i,j+1), (i+1,j-1), (i-1,j+1)
// of plane p; the two points with i+j+1 are guarded (they exist only if
// i + j + 1 + p <= N)
template <typename T>
__device__ __forceinline__ void load7(const T* xm, int N, int i, int j, int p, T o[7]) {
    const int po = (int)plane_off(N, p);
    const int rj = po + (int)row_off(N, j, p);
    const int rs = po + (int)row_off(N, j - 1, p);
    const int rn = po + (int)row_off(N, j + 1, p);
    const bool hi = i + j + 1 + p <= N;
    o[0] = xm[rj + i];
    o[1] = xm[rj + i - 1];
    o[2] = hi ? xm[rj + i + 1] : (T)0;
    o[3] = xm[rs + i];
    o[4] = hi ? xm[rn + i] : (T)0;
    o[5] = xm[rs + i + 1];
    o[6] = xm[rn + i - 1];
}

// weights x neighbours: mc mw me ms mn mse mnw from plane k, bc be bn bnw
// from k-1, tc tw ts tse from k+1
template <typename T, typename W>
__device__ __forceinline__ T off_sum(const W s[NW], const T pm[7], const T p0[7], const T pp[7]) {
    T a = (T)s[1] * p0[1];
    a += (T)s[2] * p0[2];
    a += (T)s[3] * p0[3];
    a += (T)s[4] * p0[4];
    a += (T)s[5] * p0[5];
    a += (T)s[6] * p0[6];
    a += (T)s[7] * pm[0];
    a += (T)s[8] * pm[2];
    a += (T)s[9] * pm[4];
    a += (T)s[10] * pm[6];
    a += (T)s[11] * pp[0];
    a += (T)s[12] * pp[1];
    a += (T)s[13] * pp[3];
    a += (T)s[14] * pp[5];
    return a;
}

// XCD-aware block decode: workgroup b runs on XCD b % 8; all tiles of a macro
// go to the same XCD so that the planes shared by neighbouring tiles stay in
// that XCD's L2.
__device__ __forceinline__ bool decode_block(int n_tiles, int nt, int& macro, int& tile) {
    const int b = blockIdx.x;
    const int xcd = b & 7, loc = b >> 3;
    const int grp = loc / n_tiles;
    macro = grp * 8 + xcd;
    tile = loc - grp * n_tiles;
    return macro < nt;
}

// Weight providers ------------------------------------------------------------

// Surrogate: per lane, the 1D polynomials d_w(zeta) = sum_n d[w][n] zeta^n of
// the column (i, j), from the 3D coefficients a_w (monomials of the centred,
// scaled coordinates).  W is the arithmetic type of the weights.
template <int Q, typename W, int CENTER>
struct SurrogateW {
    W d[NW][Q + 1];
    W invN;
    __device__ __forceinline__ void init(const W* __restrict__ a, int N, int i, int j) {
        constexpr Basis<Q> BS{};
        constexpr int MQ = Basis<Q>::MQ;
        invN = (W)1 / (W)N;
        const W xi = (W)i * invN - (W)0.25, eta = (W)j * invN - (W)0.25;
        W xp[Q + 1], ep[Q + 1];
        xp[0] = ep[0] = (W)1;
#pragma unroll
        for (int q = 1; q <= Q; q++) {
            xp[q] = xp[q - 1] * xi;
            ep[q] = ep[q - 1] * eta;
        }
#pragma unroll
        for (int w = 0; w < NW; w++) {
#pragma unroll
            for (int n = 0; n <= Q; n++) d[w][n] = (W)0;
#pragma unroll
            for (int c = 0; c < MQ; c++) d[w][BS.n[c]] += a[w * MQ + c] * (xp[BS.l[c]] * ep[BS.m[c]]);
        }
    }
    __device__ __forceinline__ void weights(int k, W s[NW]) const {
        const W z = (W)k * invN - (W)0.25;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            W v = d[w][Q];
#pragma unroll
            for (int n = Q - 1; n >= 0; n--) v = v * z + d[w][n];
            s[w] = v;
        }
        if (CENTER == TS_CENTER_ROWSUM) {
            W c = (W)0;
#pragma unroll
            for (int w = 1; w < NW; w++) c -= s[w];
            s[0] = c;
        }
    }
};

// FP16 weight evaluation: the 1D column polynomials are evaluated in half
// precision on coefficients pre-scaled by N (weights of order one), the
// products and sums stay in FP32.
template <int Q>
struct SurrogateHalfW {
    _Float16 d[NW][Q + 1];
    float invN;
    __device__ __forceinline__ void init(const float* __restrict__ a, int N, int i, int j) {
        constexpr Basis<Q> BS{};
        constexpr int MQ = Basis<Q>::MQ;
        invN = 1.0f / (float)N;
        const float xi = (float)i * invN - 0.25f, eta = (float)j * invN - 0.25f;
        float xp[Q + 1], ep[Q + 1];
        xp[0] = ep[0] = 1.0f;
#pragma unroll
        for (int q = 1; q <= Q; q++) {
            xp[q] = xp[q - 1] * xi;
            ep[q] = ep[q - 1] * eta;
        }
#pragma unroll
        for (int w = 0; w < NW; w++) {
            float t[Q + 1];
#pragma unroll
            for (int n = 0; n <= Q; n++) t[n] = 0.0f;
#pragma unroll
            for (int c = 0; c < MQ; c++) t[BS.n[c]] += a[w * MQ + c] * (xp[BS.l[c]] * ep[BS.m[c]]);
#pragma unroll
            for (int n = 0; n <= Q; n++) d[w][n] = (_Float16)t[n];
        }
    }
    __device__ __forceinline__ void weights(int k, float s[NW]) const {
        const _Float16 z = (_Float16)((float)k * invN - 0.25f);
        const float scale = invN;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            _Float16 v = d[w][Q];
#pragma unroll
            for (int n = Q - 1; n >= 0; n--) v = v * z + d[w][n];
            s[w] = (float)v * scale;
        }
    }
};

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
// in place (x == y).
template <typename T, typename W, int MODE, class WP>
__device__ __forceinline__ void volume_body(const T* xm, T* ym, const T* fm, WP& wp, int N,
                                            int i, int j, int k0, int kend, int colour) {
    T pm[7], p0[7], pp[7];
    load7(xm, N, i, j, k0 - 1, pm);
    load7(xm, N, i, j, k0, p0);
#pragma unroll
    for (int r = 0; r < VOL_R; r++) {
        const int k = k0 + r;
        if (k > kend) break;
        load7(xm, N, i, j, k + 1, pp);
        const int idx = (int)bidx(N, i, j, k);
        if (MODE == 2) {
            if (((i + 2 * j + 3 * k) & 3) == colour) {
                W s[NW];
                wp.weights(k, s);
                const T off = off_sum<T, W>(s, pm, p0, pp);
                ym[idx] = (fm[idx] - off) / (T)s[0];
            }
        } else {
            W s[NW];
            wp.weights(k, s);
            const T v = (T)s[0] * p0[0] + off_sum<T, W>(s, pm, p0, pp);
            if (MODE == 0)
                ym[idx] = v;
            else
                ym[idx] = fm[idx] - v;
        }
#pragma unroll
        for (int q = 0; q < 7; q++) {
            pm[q] = p0[q];
            p0[q] = pp[q];
        }
    }
}

template <int Q, typename T, typename W, int MODE, int CENTER>
__global__ __launch_bounds__(VOL_THREADS) void k_surrogate(
    const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ f,
    const W* __restrict__ coef, const int2* __restrict__ tiles, int n_tiles, int nt, int N,
    int64_t B, int colour) {
    int macro, tile;
    if (!decode_block(n_tiles, nt, macro, tile)) return;
    const int2 td = tiles[tile];
    const int k0 = td.x, Mr = N - 1 - k0;
    const int pos = td.y + (int)threadIdx.x;
    if (pos >= (Mr - 1) * Mr / 2) return;
    int i, j;
    pos_to_ij(pos, Mr, i, j);
    const int kend = min(N - 1 - i - j, k0 + VOL_R - 1);
    constexpr int MQ = Basis<Q>::MQ;
    SurrogateW<Q, W, CENTER> wp;
    wp.init(coef + (size_t)macro * NW * MQ, N, i, j);
    const size_t base = (size_t)macro * B;
    volume_body<T, W, MODE>(x + base, y + base, f ? f + base : nullptr, wp, N, i, j, k0, kend,
                            colour);
}

// Gauss-Seidel variant: x and y alias (in-place update)
template <int Q, typename T, typename W, int CENTER>
__global__ __launch_bounds__(VOL_THREADS) void k_surrogate_gs(
    T* u, const T* __restrict__ f, const W* __restrict__ coef, const int2* __restrict__ tiles,
    int n_tiles, int nt, int N, int64_t B, int colour) {
    int macro, tile;
    if (!decode_block(n_tiles, nt, macro, tile)) return;
    const int2 td = tiles[tile];
    const int k0 = td.x, Mr = N - 1 - k0;
    const int pos = td.y + (int)threadIdx.x;
    if (pos >= (Mr - 1) * Mr / 2) return;
    int i, j;
    pos_to_ij(pos, Mr, i, j);
    const int kend = min(N - 1 - i - j, k0 + VOL_R - 1);
    constexpr int MQ = Basis<Q>::MQ;
    SurrogateW<Q, W, CENTER> wp;
    wp.init(coef + (size_t)macro * NW * MQ, N, i, j);
    const size_t base = (size_t)macro * B;
    volume_body<T, W, 2>(u + base, u + base, f + base, wp, N, i, j, k0, kend, colour);
}

template <int Q, int MODE>
__global__ __launch_bounds__(VOL_THREADS) void k_surrogate_half(
    const float* x, float* y, const float* __restrict__ f, const float* __restrict__ coef,
    const int2* __restrict__ tiles, int n_tiles, int nt, int N, int64_t B, int colour) {
    int macro, tile;
    if (!decode_block(n_tiles, nt, macro, tile)) return;
    const int2 td = tiles[tile];
    const int k0 = td.x, Mr = N - 1 - k0;
    const int pos = td.y + (int)threadIdx.x;
    if (pos >= (Mr - 1) * Mr / 2) return;
    int i, j;
    pos_to_ij(pos, Mr, i, j);
    const int kend = min(N - 1 - i - j, k0 + VOL_R - 1);
    constexpr int MQ = Basis<Q>::MQ;
    SurrogateHalfW<Q> wp;
    wp.init(coef + (size_t)macro * NW * MQ, N, i, j);
    const size_t base = (size_t)macro * B;
    volume_body<float, float, MODE>(x + base, y + base, f ? f + base : nullptr, wp, N, i, j,
                                    k0, kend, colour);
}

template <typename T, int MODE>
__global__ __launch_bounds__(VOL_THREADS) void k_ifem_volume(
    const T* x, T* y, const T* __restrict__ f, const MacroGeom* __restrict__ geom,
    const int2* __restrict__ tiles, int n_tiles, int nt, int N, int64_t B, int colour) {
    int macro, tile;
    if (!decode_block(n_tiles, nt, macro, tile)) return;
    const int2 td = tiles[tile];
    const int k0 = td.x, Mr = N - 1 - k0;
    const int pos = td.y + (int)threadIdx.x;
    if (pos >= (Mr - 1) * Mr / 2) return;
    int i, j;
    pos_to_ij(pos, Mr, i, j);
    const int kend = min(N - 1 - i - j, k0 + VOL_R - 1);
    IfemW wp;
    wp.g = geom[macro];
    wp.N = N;
    wp.i = i;
    wp.j = j;
    const size_t base = (size_t)macro * B;
    volume_body<T, double, MODE>(x + base, y + base, f ? f + base : nullptr, wp, N, i, j, k0,
                                 kend, colour);
}

// Lower primitives -------------------------------------------------------------
// One thread per unique face/edge/vertex node.  The row is the sum over the
// node's copies (one per adjacent macro) of that macro's element-wise
// partial stencil.  MODE 0: y = L x; 1: y = f - L x, written to every copy;
// 2: Gauss-Seidel value (f - off) / diag into tmp[t].
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
        dg += s[0];
#pragma unroll
        for (int w = 1; w < NW; w++) {
            const int a = q.y + dir_i(w), b = q.z + dir_j(w), cc = q.w + dir_k(w);
            if (inside(N, a, b, cc)) of += s[w] * (double)xm[bidx(N, a, b, cc)];
        }
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

// Launchers --------------------------------------------------------------------

static int grid_volume(const Level& L, int64_t nt) {
    return (int)(((nt + 7) / 8) * 8 * L.n_tiles);
}

template <int Q, typename T, typename W>
static void run_surrogate(const Level& L, int nt, const W* coef, int center, int mode,
                          const void* x, void* y, const void* f, int colour, hipStream_t s) {
    const dim3 grid(grid_volume(L, nt)), blk(VOL_THREADS);
    if (grid.x == 0) return;
    const T* xp = (const T*)x;
    T* yp = (T*)y;
    const T* fp = (const T*)f;
    if (mode == 2) {
        if (center == TS_CENTER_POLY)
            k_surrogate_gs<Q, T, W, TS_CENTER_POLY><<<grid, blk, 0, s>>>(yp, fp, coef, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
        else
            k_surrogate_gs<Q, T, W, TS_CENTER_ROWSUM><<<grid, blk, 0, s>>>(yp, fp, coef, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
        return;
    }
#define TS_LAUNCH(MODE_, C_)                                                                 \
    k_surrogate<Q, T, W, MODE_, C_><<<grid, blk, 0, s>>>(xp, yp, fp, coef, L.tiles.p, L.n_tiles, \
                                                          nt, L.N, L.B, colour)
    if (center == TS_CENTER_POLY) {
        if (mode == 0) TS_LAUNCH(0, TS_CENTER_POLY); else TS_LAUNCH(1, TS_CENTER_POLY);
    } else {
        if (mode == 0) TS_LAUNCH(0, TS_CENTER_ROWSUM); else TS_LAUNCH(1, TS_CENTER_ROWSUM);
    }
#undef TS_LAUNCH
}

template <int Q>
static void run_half(const Level& L, int nt, const float* coef, int mode, const void* x,
                     void* y, const void* f, int colour, hipStream_t s) {
    const dim3 grid(grid_volume(L, nt)), blk(VOL_THREADS);
    if (grid.x == 0) return;
    const float* xp = (const float*)x;
    float* yp = (float*)y;
    const float* fp = (const float*)f;
    if (mode == 0)
        k_surrogate_half<Q, 0><<<grid, blk, 0, s>>>(xp, yp, fp, coef, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
    else if (mode == 1)
        k_surrogate_half<Q, 1><<<grid, blk, 0, s>>>(xp, yp, fp, coef, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
    else
        k_surrogate_half<Q, 2><<<grid, blk, 0, s>>>(yp, yp, fp, coef, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
}

void launch_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                   const void* f, int colour, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const LevelOp& lo = *op->lv.at(lam);
    const int nt = (int)M.nt, q = op->p.q, c = op->p.center;
    if (dtype == TS_F64) {
        const double* cf = lo.coef64.p;
        switch (q) {
            case 1: run_surrogate<1, double, double>(L, nt, cf, c, mode, x, y, f, colour, s); break;
            case 2: run_surrogate<2, double, double>(L, nt, cf, c, mode, x, y, f, colour, s); break;
            case 3: run_surrogate<3, double, double>(L, nt, cf, c, mode, x, y, f, colour, s); break;
            case 4: run_surrogate<4, double, double>(L, nt, cf, c, mode, x, y, f, colour, s); break;
        }
    } else if (dtype == TS_F32) {
        const float* cf = lo.coef32.p;
        switch (q) {
            case 1: run_surrogate<1, float, float>(L, nt, cf, c, mode, x, y, f, colour, s); break;
            case 2: run_surrogate<2, float, float>(L, nt, cf, c, mode, x, y, f, colour, s); break;
            case 3: run_surrogate<3, float, float>(L, nt, cf, c, mode, x, y, f, colour, s); break;
            case 4: run_surrogate<4, float, float>(L, nt, cf, c, mode, x, y, f, colour, s); break;
        }
    } else {
        const float* cf = lo.coef16s.p;
        switch (q) {
            case 1: run_half<1>(L, nt, cf, mode, x, y, f, colour, s); break;
            case 2: run_half<2>(L, nt, cf, mode, x, y, f, colour, s); break;
            case 3: run_half<3>(L, nt, cf, mode, x, y, f, colour, s); break;
            case 4: run_half<4>(L, nt, cf, mode, x, y, f, colour, s); break;
        }
    }
    TS_HIP(hipGetLastError());
}

template <typename T>
static void run_ifem_volume(const Mesh& M, const Level& L, int mode, const void* x, void* y,
                            const void* f, int colour, hipStream_t s) {
    const int nt = (int)M.nt;
    const dim3 grid(grid_volume(L, nt)), blk(VOL_THREADS);
    if (grid.x == 0) return;
    const T* xp = (const T*)x;
    T* yp = (T*)y;
    const T* fp = (const T*)f;
    if (mode == 0)
        k_ifem_volume<T, 0><<<grid, blk, 0, s>>>(xp, yp, fp, M.d_geom.p, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
    else if (mode == 1)
        k_ifem_volume<T, 1><<<grid, blk, 0, s>>>(xp, yp, fp, M.d_geom.p, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
    else
        k_ifem_volume<T, 2><<<grid, blk, 0, s>>>(yp, yp, fp, M.d_geom.p, L.tiles.p, L.n_tiles, nt, L.N, L.B, colour);
}

void launch_ifem_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                        const void* f, int colour, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    if (dtype == TS_F64)
        run_ifem_volume<double>(M, L, mode, x, y, f, colour, s);
    else
        run_ifem_volume<float>(M, L, mode, x, y, f, colour, s);
    TS_HIP(hipGetLastError());
}

void launch_iface(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                  const void* f, int phase, double* tmp, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const int* list = phase >= 0 ? L.phase_list[phase].p : nullptr;
    const int n = phase >= 0 ? L.n_phase[phase] : (int)L.n_if;
    if (n == 0) return;
    const dim3 grid((n + 255) / 256), blk(256);
#define TS_IF(T_, M_)                                                                         \
    k_iface<T_, M_><<<grid, blk, 0, s>>>((const T_*)x, (T_*)y, (const T_*)f, L.if_off.p,      \
                                         L.if_copy.p, L.if_flag.p, list, n, M.d_geom.p,       \
                                         L.N, L.B, tmp)
    if (dtype == TS_F64) {
        if (mode == 0) TS_IF(double, 0); else if (mode == 1) TS_IF(double, 1); else TS_IF(double, 2);
    } else {
        if (mode == 0) TS_IF(float, 0); else if (mode == 1) TS_IF(float, 1); else TS_IF(float, 2);
    }
#undef TS_IF
    TS_HIP(hipGetLastError());
}

void launch_iface_scatter(const ts_op* op, int lam, int dtype, int phase, const double* tmp,
                          void* u, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const int n = L.n_phase[phase];
    if (n == 0) return;
    const dim3 grid((n + 255) / 256), blk(256);
    if (dtype == TS_F64)
        k_iface_scatter<double><<<grid, blk, 0, s>>>((double*)u, tmp, L.if_off.p, L.if_copy.p, L.phase_list[phase].p, n, L.N, L.B);
    else
        k_iface_scatter<float><<<grid, blk, 0, s>>>((float*)u, tmp, L.if_off.p, L.if_copy.p, L.phase_list[phase].p, n, L.N, L.B);
    TS_HIP(hipGetLastError());
}

}  // namespace ts
