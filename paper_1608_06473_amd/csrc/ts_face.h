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

template <int F, typename T>
__device__ __forceinline__ void face_acc_a(const double* __restrict__ sw, int n2, const T* xm,
                                           const int o[NW], double& of) {
#pragma unroll
    for (int e = 1; e < 11; e++) of += sw[(size_t)e * n2] * (double)xm[o[kFaceDirs.a[F][e]]];
}
template <int F, typename T>
__device__ __forceinline__ void face_acc_b(const double* __restrict__ sw, int n2, const T* xm,
                                           const int o[NW], double& of) {
#pragma unroll
    for (int e = 0; e < 4; e++) of += sw[(size_t)(11 + e) * n2] * (double)xm[o[kFaceDirs.b[F][e]]];
}

// One face fast-path node t (position q = list ? list[t] : t); same modes as
// k_iface.
template <typename T, int MODE>
__device__ __forceinline__ void face2_node(const T* __restrict__ x, T* __restrict__ y,
                                           const T* __restrict__ f,
                                           const int4* __restrict__ cp,
                                           const double* __restrict__ sten, int n2,
                                           const int* __restrict__ list, int t, int N, int64_t B,
                                           double* __restrict__ tmp) {
    const int q = list ? list[t] : t;
    const int4 ca = cp[q], cb = cp[(size_t)n2 + q];
    const int ba = (int)bidx(N, ca.y, ca.z, ca.w), bb = (int)bidx(N, cb.y, cb.z, cb.w);
    const T* xa = x + (size_t)ca.x * B;
    const T* xb = x + (size_t)cb.x * B;
    const double* sw = sten + q;
    int o[NW];
    double of = 0.0;
    nbr_index(ba, N + 1 - ca.w, ca.z, o);
    switch (face_type(N, ca.y, ca.z, ca.w)) {
        case 0: face_acc_a<0>(sw, n2, xa, o, of); break;
        case 1: face_acc_a<1>(sw, n2, xa, o, of); break;
        case 2: face_acc_a<2>(sw, n2, xa, o, of); break;
        default: face_acc_a<3>(sw, n2, xa, o, of); break;
    }
    nbr_index(bb, N + 1 - cb.w, cb.z, o);
    switch (face_type(N, cb.y, cb.z, cb.w)) {
        case 0: face_acc_b<0>(sw, n2, xb, o, of); break;
        case 1: face_acc_b<1>(sw, n2, xb, o, of); break;
        case 2: face_acc_b<2>(sw, n2, xb, o, of); break;
        default: face_acc_b<3>(sw, n2, xb, o, of); break;
    }
    const double dg = sw[0];
    const size_t sa = (size_t)ca.x * B + ba, sb = (size_t)cb.x * B + bb;
    if (MODE == 2) {
        tmp[t] = ((double)f[sa] - of) / dg;
        return;
    }
    double v = dg * (double)xa[ba] + of;
    if (MODE == 1) v = (double)f[sa] - v;
    y[sa] = (T)v;
    y[sb] = (T)v;
}


}  // namespace ts
