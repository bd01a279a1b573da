// Rows of the two-copy interior-face nodes (the face fast path), shared by
// the stand-alone face kernel and the fused surrogate volume launch.
#pragma once

#include "ts_internal.h"

namespace ts {

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

// Face path: free nodes of interior faces, each with exactly two copies A
// and B.  A face node of macro A lies on one of its faces: i = 0, j = 0,
// k = 0 or i + j + k = N (face type 0..3).  Of the 15 directions, 7 stay in
// the face, 4 point into the macro and 4 out of it.  The node's row is stored
// once per level as 15 combined weights (struct of arrays [15][n2]): slots
// 0..10 the non-outward directions of A in increasing order (in-face weights
// summed over both sides), slots 11..14 the inward directions of B.
struct FaceDirs {
    int a[4][11];  // non-outward directions of a copy on face type f
    int b[4][4];   // inward directions
};
constexpr int kDI[NW] = {0, -1, 1, 0, 0, 1, -1, 0, 1, 0, -1, 0, -1, 0, 1};
constexpr int kDJ[NW] = {0, 0, 0, -1, 1, -1, 1, 0, 0, 1, 1, 0, 0, -1, -1};
constexpr int kDK[NW] = {0, 0, 0, 0, 0, 0, 0, -1, -1, -1, -1, 1, 1, 1, 1};
// signed distance of direction w from face type f (< 0 outward, > 0 inward)
constexpr int face_side(int f, int w) {
    return f == 0 ? kDI[w] : f == 1 ? kDJ[w] : f == 2 ? kDK[w] : -(kDI[w] + kDJ[w] + kDK[w]);
}
constexpr FaceDirs make_face_dirs() {
    FaceDirs d{};
    for (int f = 0; f < 4; f++) {
        int na = 0, nb = 0;
        for (int w = 0; w < NW; w++) {
            if (face_side(f, w) >= 0) d.a[f][na++] = w;
            if (face_side(f, w) > 0) d.b[f][nb++] = w;
        }
    }
    return d;
}
inline constexpr FaceDirs kFaceDirs = make_face_dirs();

__device__ __forceinline__ int face_type(int N, int i, int j, int k) {
    return i == 0 ? 0 : j == 0 ? 1 : k == 0 ? 2 : 3;
}

// element index, within its macro, of row entry e of a face node: entries
// 0..10 through the first copy's directions (offsets oa), 11..14 through the
// second copy's inward directions (offsets ob)
template <int F>
__device__ __forceinline__ void face_ix_a(const int oa[NW], int ix[NW]) {
#pragma unroll
    for (int e = 0; e < 11; e++) ix[e] = oa[kFaceDirs.a[F][e]];
}
template <int F>
__device__ __forceinline__ void face_ix_b(const int ob[NW], int ix[NW]) {
#pragma unroll
    for (int e = 0; e < 4; e++) ix[11 + e] = ob[kFaceDirs.b[F][e]];
}

template <int FQ>
struct FaceBasis {
    static constexpr int M2 = (FQ + 1) * (FQ + 2) / 2;
};

// monomial c of the face basis at (u, v): exponents (d - l, l) for the c-th
// pair in the order (d, l) = (0,0), (1,0), (1,1), (2,0), ...
template <int C>
struct FaceExp {
    static constexpr int d() {
        int dd = 0, c = C;
        while (c > dd) {
            c -= dd + 1;
            dd++;
        }
        return dd;
    }
    static constexpr int l() {
        int dd = 0, c = C;
        while (c > dd) {
            c -= dd + 1;
            dd++;
        }
        return c;
    }
};

__device__ __forceinline__ double ipow_c(double x, int n) {
    double r = 1.0;
    for (int a = 0; a < n; a++) r *= x;
    return r;
}

template <int FQ, int C = 0>
__device__ __forceinline__ void face_phi(double u, double v, double* phi) {
    if constexpr (C < FaceBasis<FQ>::M2) {
        constexpr int d = FaceExp<C>::d(), l = FaceExp<C>::l();
        phi[C] = ipow_c(u, d - l) * ipow_c(v, l);
        face_phi<FQ, C + 1>(u, v, phi);
    }
}

// the face basis at the first copy (i, j, k) on face type fa
template <int FQ>
__device__ __forceinline__ void face_basis(int N, int fa, int i, int j, int k,
                                           double phi[FaceBasis<FQ>::M2]) {
    const double invN = 1.0 / (double)N;
    const double u = (double)(fa == 0 ? j : i) * invN - 1.0 / 3.0;
    const double v = (double)(fa <= 1 ? k : j) * invN - 1.0 / 3.0;
    face_phi<FQ>(u, v, phi);
}

// One face fast-path node t (position q = list ? list[t] : t); same modes as
// k_iface.  FQ = 0: the stored exact row (its weights in the vector type T:
// rounded to FP32 for FP32 vectors; sums in FP64); FQ > 0: the face fit of
// degree FQ.
// Gauss-Seidel (MODE 2): nodes t < n_direct write the new value to both
// copies, the others to tmp[t - n_direct].
template <typename T, int MODE, int FQ = 0>
__device__ __forceinline__ void face2_node(const T* __restrict__ x, T* __restrict__ y,
                                           const T* __restrict__ f,
                                           const int4* __restrict__ cp,
                                           const T* __restrict__ sten,
                                           const double* __restrict__ fcoef, int n2,
                                           const int* __restrict__ list, int t, int N, int64_t B,
                                           double* __restrict__ tmp, int n_direct = 0) {
    const int q = list ? list[t] : t;
    const int4 ca = cp[q], cb = cp[(size_t)n2 + q];
    const int ba = (int)bidx(N, ca.y, ca.z, ca.w), bb = (int)bidx(N, cb.y, cb.z, cb.w);
    const T* xa = x + (size_t)ca.x * B;
    const T* xb = x + (size_t)cb.x * B;
    const int fa = face_type(N, ca.y, ca.z, ca.w);
    int ix[NW];
    {
        int o[NW];
        nbr_index(ba, N + 1 - ca.w, ca.z, o);
        switch (fa) {
            case 0: face_ix_a<0>(o, ix); break;
            case 1: face_ix_a<1>(o, ix); break;
            case 2: face_ix_a<2>(o, ix); break;
            default: face_ix_a<3>(o, ix); break;
        }
        nbr_index(bb, N + 1 - cb.w, cb.z, o);
        switch (face_type(N, cb.y, cb.z, cb.w)) {
            case 0: face_ix_b<0>(o, ix); break;
            case 1: face_ix_b<1>(o, ix); break;
            case 2: face_ix_b<2>(o, ix); break;
            default: face_ix_b<3>(o, ix); break;
        }
    }
    // entry e: its weight (stored row, or the face fit at this node) times x
    // at its neighbour; the fitted weights are formed one at a time
    double of = 0.0, dg;
    if constexpr (FQ == 0) {
        const T* sw = sten + q;
        dg = (double)sw[0];
#pragma unroll
        for (int e = 1; e < NW; e++)
            of += (double)sw[(size_t)e * n2] * (double)(e < 11 ? xa : xb)[ix[e]];
    } else {
        constexpr int M2 = FaceBasis<FQ>::M2;
        double phi[M2];
        face_basis<FQ>(N, fa, ca.y, ca.z, ca.w, phi);
        const int blk = ca.x * 4 + fa;
        // Almost every wavefront lies on one face: then the coefficient block
        // is wave-uniform and is read through the scalar cache; wavefronts
        // across two faces read it per lane.
        const int b0 = __builtin_amdgcn_readfirstlane(blk);
        if (__builtin_amdgcn_ballot_w64(blk != b0) == 0) {
            const double* cf = fcoef + (size_t)b0 * (NW * M2);
            dg = 0.0;
#pragma unroll
            for (int c = 0; c < M2; c++) dg += cf[c] * phi[c];
#pragma unroll
            for (int e = 1; e < NW; e++) {
                double we = 0.0;
#pragma unroll
                for (int c = 0; c < M2; c++) we += cf[e * M2 + c] * phi[c];
                of += we * (double)(e < 11 ? xa : xb)[ix[e]];
                if (e % 2 == 0) asm volatile("" : "+s"(cf) : "v"(of));
            }
        } else {
            const double* cf = fcoef + (size_t)blk * (NW * M2);
            dg = 0.0;
#pragma unroll
            for (int c = 0; c < M2; c++) dg += cf[c] * phi[c];
#pragma unroll
            for (int e = 1; e < NW; e++) {
                double we = 0.0;
#pragma unroll
                for (int c = 0; c < M2; c++) we += cf[e * M2 + c] * phi[c];
                of += we * (double)(e < 11 ? xa : xb)[ix[e]];
                // One entry's coefficients in flight: the face rows share the
                // register budget of the fused volume kernel.  The empty asm
                // takes this entry's weight and hands back the coefficient
                // pointer, so the next entry's loads cannot be issued before
                // the weight is formed (the gathers of x stay free to run
                // ahead).
                asm volatile("" : "+v"(cf) : "v"(of));
            }
        }
    }
    const size_t sa = (size_t)ca.x * B + ba, sb = (size_t)cb.x * B + bb;
    if (MODE == 2) {
        const double g = ((double)f[sa] - of) / dg;
        if (t < n_direct) {
            y[sa] = (T)g;
            y[sb] = (T)g;
        } else {
            tmp[t - n_direct] = g;
        }
        return;
    }
    double v = dg * (double)xa[ba] + of;
    if (MODE == 1) v = (double)f[sa] - v;
    y[sa] = (T)v;
    y[sb] = (T)v;
}


}  // namespace ts
