// Surrogate volume kernel for gfx950 (shared by the per-degree instantiation
// units): y = L~ x, r = f - L~ x and the multicolour Gauss-Seidel update on
// the volume primitives (Sec. 3.4 eq. ts; eq. iteration-scheme).
//
// Work decomposition: a workgroup owns one macro, a slab of R planes
// k0 .. k0+R-1 and whole rows j0 .. j1-1 of plane k0's interior; each lane
// owns a column (i, j) and marches up in k.  The surrogate polynomials are
// reduced once per lane to 1D polynomials in zeta (the line-wise reduction of
// Sec. 3.4) and evaluated with q FMAs per weight and step.  For every plane
// p = k0-1 .. k0+R the rows j0-1 .. j1 form one contiguous range of the block
// layout: the workgroup copies it into LDS with coalesced loads issued PF
// planes ahead into registers, and every lane reads the 7 points of its
// column from LDS into a rolling 3-plane register window.  All index
// arithmetic advances incrementally from plane to plane.
#pragma once

#include "ts_face.h"
#include "ts_internal.h"

#ifndef TS_GS_G
#define TS_GS_G 3
#endif

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

// position of the basis monomial xi^l eta^m zeta^n (degree d = l + m + n):
// all terms of lower degree come first, then l descending, then m descending
constexpr int basis_index(int l, int m, int n) {
    const int d = l + m + n;
    return d * (d + 1) * (d + 2) / 6 + (d - l) * (d - l + 1) / 2 + (d - l - m);
}

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
// mlist (optional) maps the nt list positions to macro ids.
__device__ __forceinline__ bool decode_block(int n_tiles, int nt, int& macro, int& tile,
                                             const int* __restrict__ mlist = nullptr,
                                             int b = -1) {
    if (b < 0) b = blockIdx.x;
    const int xcd = b & 7, loc = b >> 3;
    const int grp = loc / n_tiles;
    macro = grp * 8 + xcd;
    tile = loc - grp * n_tiles;
    if (macro >= nt) return false;
    if (mlist) macro = mlist[macro];
    return true;
}

// Surrogate: per lane, the 1D polynomials d_w(zeta) = sum_n d[w][n] zeta^n of
// the column (i, j), from the 3D coefficients a_w (monomials of the centred,
// scaled coordinates).  W is the arithmetic type of the weights.
template <int Q, typename W, int CENTER>
struct SurrogateW {
    static constexpr int kQ = Q;
    W d[NW][Q + 1];
    W invN;
    __device__ __forceinline__ void init_from(const float* __restrict__ cf,
                                              const double* __restrict__ cd, int macro, int N,
                                              int i, int j) {
        constexpr int MQ = Basis<Q>::MQ;
        if constexpr (sizeof(W) == 8)
            init((const W*)cd + (size_t)macro * NW * MQ, N, i, j);
        else
            init((const W*)cf + (size_t)macro * NW * MQ, N, i, j);
    }
    __device__ __forceinline__ void init(const W* a, int N, int i, int j) {
        constexpr Basis<Q> BS{};
        constexpr int MQ = Basis<Q>::MQ;
        invN = (W)1 / (W)N;
        const W xi = (W)i * invN - (W)0.25, eta = (W)j * invN - (W)0.25;
        // d_n = sum_l xi^l (sum_m a[l, m, n] eta^m): nested Horner, one FMA per
        // basis term beyond the first of each n.  Weights are processed in
        // groups of 3 so that only their coefficients are live in SGPRs.
#pragma unroll
        for (int g = 0; g < NW; g += 3) {
#pragma unroll
            for (int w = g; w < g + 3; w++) {
#pragma unroll
                for (int n = 0; n <= Q; n++) {
                    W acc = (W)0;
                    bool first = true;
#pragma unroll
                    for (int l = Q - n; l >= 0; l--) {
                        W inner = (W)0;
                        bool ifirst = true;
#pragma unroll
                        for (int m = Q - n - l; m >= 0; m--) {
                            const W av = a[w * MQ + basis_index(l, m, n)];
                            inner = ifirst ? av : inner * eta + av;
                            ifirst = false;
                        }
                        acc = first ? inner : acc * xi + inner;
                        first = false;
                    }
                    d[w][n] = acc;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        pin();
    }
    // Keep the column coefficients in VGPRs: some of them are wave-uniform
    // (the top-degree ones), and held in SGPRs they overflow the scalar file.
    __device__ __forceinline__ void pin() {
#pragma unroll
        for (int w = 0; w < NW; w++)
#pragma unroll
            for (int n = 0; n <= Q; n++) asm volatile("" : "+v"(d[w][n]));
    }
    __device__ __forceinline__ void weights_z(W z, W s[NW]) const {
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
// products and sums stay in FP32.  Two weights share one half2 register, so
// each Horner step is one packed FP16 FMA for both (the same per-component
// rounding as two scalar FP16 FMAs); weight 15 of the last pair is unused.
template <int Q>
struct SurrogateHalfW {
    static constexpr int kQ = Q;
    static constexpr int NP = (NW + 1) / 2;
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 d[NP][Q + 1];
    float invN;
    __device__ __forceinline__ void init_from(const float* __restrict__ cf,
                                              const double* __restrict__ cd, int macro, int N,
                                              int i, int j) {
        constexpr Basis<Q> BS{};
        constexpr int MQ = Basis<Q>::MQ;
        (void)cd;
        const float* a = cf + (size_t)macro * NW * MQ;
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
        for (int g = 0; g < NW; g += 3) {
#pragma unroll
            for (int w = g; w < g + 3; w++) {
                float t[Q + 1];
#pragma unroll
                for (int n = 0; n <= Q; n++) t[n] = 0.0f;
#pragma unroll
                for (int c = 0; c < MQ; c++) t[BS.n[c]] += a[w * MQ + c] * (xp[BS.l[c]] * ep[BS.m[c]]);
#pragma unroll
                for (int n = 0; n <= Q; n++) d[w / 2][n][w % 2] = (_Float16)t[n];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int n = 0; n <= Q; n++) d[NP - 1][n][1] = (_Float16)0.0f;
#pragma unroll
        for (int p = 0; p < NP; p++)
#pragma unroll
            for (int n = 0; n <= Q; n++) asm volatile("" : "+v"(d[p][n]));
    }
    // weights of order one (coefficients pre-scaled by N) evaluated in half
    // precision, returned in float after scaling back by 1/N
    __device__ __forceinline__ void weights_z(float zf, float s[NW]) const {
        const _Float16 zh = (_Float16)zf;
        const h2 z = {zh, zh};
#pragma unroll
        for (int p = 0; p < NP; p++) {
            h2 v = d[p][Q];
#pragma unroll
            for (int n = Q - 1; n >= 0; n--) v = v * z + d[p][n];
            s[2 * p] = (float)v[0] * invN;
            if (2 * p + 1 < NW) s[2 * p + 1] = (float)v[1] * invN;
        }
    }
};

// Raw buffer accesses over one macro block: a resource with the block's base
// and size, and a 32-bit byte offset per lane.  The hardware checks every
// offset against the size: reads at or past it return 0 and writes there are
// dropped, so no lane can touch memory outside its macro block.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int off, T v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}

// Staging loads of one plane range: KPT consecutive entries per lane from
// element g on; entries past the range are never used by a live step (and
// read 0 past the block's end).
template <typename T, int KPT>
__device__ __forceinline__ void stage_load(__amdgpu_buffer_rsrc_t rx, int g, T r[KPT]) {
#pragma unroll
    for (int s = 0; s < KPT; s++)
        r[s] = bload<T>(rx, (g + (int)threadIdx.x + s * VOL_THREADS) * (int)sizeof(T));
}

// WP: weight provider (SurrogateW or SurrogateHalfW), T: vector type, W:
// weight arithmetic type (float for the FP16 provider's products).
// Minimum wavefronts per SIMD the compiler is held to (register budget):
// the apply and residual at q <= 2 with narrow staging; no bound otherwise.
// FF: the fused face rows take the face fits (degree kQ) instead of the
// stored exact rows
template <class WP, typename T, typename W, int MODE, int R, int KPT, bool FF = false>
__global__ __launch_bounds__(VOL_THREADS)
__attribute__((amdgpu_waves_per_eu(MODE != 2 && WP::kQ <= 2 && KPT <= 2 ? TS_VOL_WAVES_EU : 1)))
void k_surr_lds(const T* x, T* y, const T* __restrict__ f, const float* __restrict__ coef_f,
                const double* __restrict__ coef_d, const int4* __restrict__ tiles, int n_tiles,
                int nt, const int* __restrict__ mlist, const unsigned* __restrict__ lanes,
                const int* __restrict__ stage, int N, int64_t B, int colour,
                const int4* __restrict__ f2cp = nullptr,
                const T* __restrict__ f2sten = nullptr,
                const double* __restrict__ f2coef = nullptr, int n2 = 0) {
    // the residual's f ring needs registers: shorter staging prefetch there
    // when the kernel is compiled for three waves
    constexpr int PF = MODE == 1 && WP::kQ <= 2 && KPT <= 2 ? 2 : TS_VOL_PF;
    int bx = (int)blockIdx.x;
    if (MODE != 2 && n2 > 0) {
        // fused launch: per XCD, positions blockIdx / 8 in groups of three,
        // two volume workgroups then one workgroup of 256 face rows (the
        // face rows' gathers overlap the volume march on the same CUs)
        const int xcd = bx & 7, loc = bx >> 3, grp = loc / 3, r3 = loc - 3 * grp;
        if (r3 == 2) {
            const int t = (grp * 8 + xcd) * VOL_THREADS + (int)threadIdx.x;
            if (t < n2)
                face2_node<T, MODE, FF ? WP::kQ : 0>(x, y, f, f2cp, f2sten, f2coef, n2, nullptr,
                                                     t, N, B, nullptr);
            return;
        }
        bx = ((grp * 2 + r3) << 3) | xcd;
    }
    int macro, tile;
    if (!decode_block(n_tiles, nt, macro, tile, mlist, bx)) return;
    const int4 td = tiles[tile];
    const int k0 = td.x, j0 = td.y, j1 = td.z;
    const int tid = (int)threadIdx.x;
    // lanes without a column park at (1, j0): every index they form below
    // stays inside the staged range, so reads need no guard
    int i = 1, j = j0;
    bool act;
    {
        // column order of the tile (Gauss-Seidel: by colour class first)
        const unsigned e = lanes[(size_t)tile * VOL_THREADS + tid];
        act = e != 0xFFFFFFFFu;
        if (act) {
            i = (int)(e & 0xFFFFu);
            j = (int)(e >> 16);
        }
    }
    // number of live steps of this lane's column in the slab
    const int nlive = act ? min(N - 1 - i - j, k0 + R - 1) - k0 + 1 : 0;
    WP wp;
    wp.init_from(coef_f, coef_d, macro, N, i, j);

    // G planes are staged per barrier into one half of 2G plane buffers; a
    // buffer is rewritten two groups later, after the next group's barrier.
    // The smoother, which computes on a quarter of the planes, takes larger
    // groups (fewer barriers); the apply and residual are faster with 2.
    constexpr int G = MODE == 2 ? TS_GS_G : TS_VOL_G;
    __shared__ T buf[2 * G][KPT * VOL_THREADS];
    const size_t base = (size_t)macro * B;
    const int64_t bbytes = B * (int64_t)sizeof(T);
    const __amdgpu_buffer_rsrc_t rx = block_rsrc(x + base, bbytes);
    const __amdgpu_buffer_rsrc_t ry = block_rsrc(y + base, bbytes);
    const __amdgpu_buffer_rsrc_t rf = block_rsrc(f ? f + base : x + base, bbytes);

    // Staged range of plane p = k0 - 1 + st: rows jb = j0 - 1 .. min(j1, N - p)
    // from element plane_off(p) + row_off(jb, p) of the block.  FP32
    // kernels read it from the per-level table stage[tile][st]; the FP64
    // kernels, at their register limit, advance it incrementally instead
    // (plane p has side A = N + 1 - p, and plane_off grows by A (A + 1) / 2).
    const int* __restrict__ sgt = stage + (size_t)tile * (R + 2);
    const int jb = j0 - 1, jtri = jb * (jb - 1) / 2;
    int po_pf = (int)plane_off(N, k0 - 1);
    auto sg = [&](int st) {
        if constexpr (sizeof(T) == 4) {
            return sgt[st];
        } else {
            const int p = k0 - 1 + st;
            const int A = N + 1 - p;
            const int jl = min(j1, N - p);
            const int g = (p <= N && jl >= jb) ? po_pf + jb * A - jtri : 0;
            po_pf += A * (A + 1) / 2;
            return g;
        }
    };
    // lane: LDS index c of (i, j) = sum_{jb <= r < j} (A - r) + i; it drops by
    // nb = j - jb from one plane to the next; qa = A - j drops by 1
    const int nb = j - jb;
    const int srow = (jb + j - 1) * nb / 2;
    T pf[PF][KPT];
#pragma unroll
    for (int d = 0; d < PF; d++) stage_load<T, KPT>(rx, sg(d), pf[d]);
    int A0 = N + 2 - k0;                 // side of plane k0 - 1
    int c = nb * A0 - srow + i;          // LDS index in plane k0 - 1
    int qa = A0 - j;
    // global index of (i, j, k0)
    int idx = (int)plane_off(N, k0) + j * (N + 1 - k0) - j * (j - 1) / 2 + i;
    const W invN = (W)1 / (W)N;
    W z = (W)k0 * invN - (W)0.25;
    int col = (i + 2 * j + 3 * k0) & 3;
    // Right-hand side, loaded ahead of use: a Gauss-Seidel lane needs f only
    // on the steps of the colour being updated (every fourth), all issued
    // here; the residual streams f through a ring PF steps ahead.
    constexpr int NG = (R + 3) / 4;
    T fg[MODE == 2 ? NG : 1];
    T fr[MODE == 1 ? PF : 1];
    int idf = idx;
    if constexpr (MODE == 2) {
        const int r0 = (3 * (colour - col)) & 3;  // col + 3 r = colour (mod 4)
#pragma unroll
        for (int r = 0; r < R; r++) {
            if ((r & 3) == r0) fg[r >> 2] = r < nlive ? bload<T>(rf, idf * (int)sizeof(T)) : (T)0;
            const int Af = N + 1 - (k0 + r);
            idf += Af * (Af + 1) / 2 - j;
        }
    }
    if constexpr (MODE == 1) {
#pragma unroll
        for (int d = 0; d < PF; d++) {
            fr[d] = d < nlive ? bload<T>(rf, idf * (int)sizeof(T)) : (T)0;
            const int Af = N + 1 - (k0 + d);
            idf += Af * (Af + 1) / 2 - j;
        }
    }
    T pm[7], p0[7], pp[7];
#pragma unroll
    for (int g0 = 0; g0 < R + 2; g0 += G) {
#pragma unroll
    for (int st = g0; st < g0 + G && st < R + 2; st++) {
        T* bb = buf[st % (2 * G)];
#pragma unroll
        for (int s2 = 0; s2 < KPT; s2++) bb[tid + s2 * VOL_THREADS] = pf[st % PF][s2];
        if (st + PF <= R + 1) stage_load<T, KPT>(rx, sg(st + PF), pf[st % PF]);
    }
    __syncthreads();
#pragma unroll
    for (int st = g0; st < g0 + G && st < R + 2; st++) {
        const T* bb = buf[st % (2 * G)];
        // the 7 points of plane p: (i,j) c, (i-1,j), (i+1,j), (i,j-1) c-qa-1,
        // (i+1,j-1), (i,j+1) c+qa, (i-1,j+1)
        {
            const int rs = c - qa - 1, rn = c + qa;
            pp[0] = bb[c];
            pp[1] = bb[c - 1];
            pp[2] = bb[c + 1];
            pp[3] = bb[rs];
            pp[4] = bb[rn];
            pp[5] = bb[rs + 1];
            pp[6] = bb[rn - 1];
        }
        if (st >= 2) {
            const int r = st - 2;  // step k = k0 + r
            const bool live = r < nlive;
            if (MODE == 2) {
                // only the lanes of the colour being updated evaluate weights;
                // with the colour-class lane order whole wavefronts skip
                if (live && col == colour) {
                    W sw[NW];
                    wp.weights_z(z, sw);
                    const T off = off_sum<T, W>(sw, pm, p0, pp);
                    bstore<T>(ry, idx * (int)sizeof(T), (fg[r >> 2] - off) / (T)sw[0]);
                }
                col = (col + 3) & 3;
            } else {
                W sw[NW];
                wp.weights_z(z, sw);
                const T off = off_sum<T, W>(sw, pm, p0, pp);
                const T v = (T)sw[0] * p0[0] + off;
                if (MODE == 0) {
                    if (live) bstore<T>(ry, idx * (int)sizeof(T), v);
                } else {
                    if (live) bstore<T>(ry, idx * (int)sizeof(T), fr[r % PF] - v);
                    if (r + PF < R) {
                        fr[r % PF] = r + PF < nlive ? bload<T>(rf, idf * (int)sizeof(T)) : (T)0;
                        const int Af = N + 1 - (k0 + r + PF);
                        idf += Af * (Af + 1) / 2 - j;
                    }
                }
            }
            const int Ak = N + 1 - (k0 + r);  // side of plane k
            idx += Ak * (Ak + 1) / 2 - j;
            z += invN;
        }
        c -= nb;
        qa -= 1;
#pragma unroll
        for (int q = 0; q < 7; q++) {
            pm[q] = p0[q];
            p0[q] = pp[q];
        }
    }
    }
}

}  // namespace ts
