// Geometry of the refined macro tetrahedra: lattice, blending map, P1
// stiffness of a fine tetrahedron.  Host and device (gfx950) inline code.
//
// Paper: Sec. 2.2 (affine map Psi_T of the reference tetrahedron, blending
// map Phi_T onto the spherical shell, eq. (algebraic)), Sec. 2.3 (regular
// refinement, 15-point stencil with directions W).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define TS_HD __host__ __device__ __forceinline__

namespace ts {

constexpr int NW = 15;

// Stencil directions (di, dj, dk) in the library's order:
//  0 mc  1 mw  2 me  3 ms  4 mn  5 mse  6 mnw  7 bc  8 be  9 bn 10 bnw
// 11 tc 12 tw 13 ts 14 tse  (m/b/t = plane k, k-1, k+1; e/w = +-i; n/s = +-j)
TS_HD int dir_i(int w) {
    constexpr int d[NW] = {0, -1, 1, 0, 0, 1, -1, 0, 1, 0, -1, 0, -1, 0, 1};
    return d[w];
}
TS_HD int dir_j(int w) {
    constexpr int d[NW] = {0, 0, 0, -1, 1, -1, 1, 0, 0, 1, 1, 0, 0, -1, -1};
    return d[w];
}
TS_HD int dir_k(int w) {
    constexpr int d[NW] = {0, 0, 0, 0, 0, 0, 0, -1, -1, -1, -1, 1, 1, 1, 1};
    return d[w];
}
// direction index of an offset with components in {-1, 0, 1}; -1 if none
TS_HD int dir_index(int di, int dj, int dk) {
    for (int w = 0; w < NW; w++)
        if (dir_i(w) == di && dir_j(w) == dj && dir_k(w) == dk) return w;
    return -1;
}

// Index helpers for the packed tetrahedral block of one macro: nodes
// (i, j, k) >= 0 with i + j + k <= N, k outer, j, i inner.
TS_HD int64_t tri_n(int64_t n) { return n * (n + 1) / 2; }
TS_HD int64_t tet_n(int64_t n) { return n * (n + 1) * (n + 2) / 6; }
TS_HD int64_t block_size(int N) { return tet_n(N + 1); }
// first index of plane k
TS_HD int64_t plane_off(int N, int k) { return tet_n(N + 1) - tet_n(N + 1 - k); }
// first index of row j inside plane k
TS_HD int64_t row_off(int N, int j, int k) {
    return (int64_t)j * (N + 1 - k) - (int64_t)j * (j - 1) / 2;
}
TS_HD int64_t bidx(int N, int i, int j, int k) {
    return plane_off(N, k) + row_off(N, j, k) + i;
}
TS_HD bool inside(int N, int i, int j, int k) {
    return i >= 0 && j >= 0 && k >= 0 && i + j + k <= N;
}

// Per-macro geometry record (FP64).  v: vertices in frame order (v0..v3),
// r: their radii, ord: frame positions sorted by ascending global vertex id
// (sums over the vertices run in that order so that all macros sharing a
// node compute bitwise the same point), affine: 1 for Phi = Id.
struct MacroGeom {
    double v[4][3];
    double r[4];
    int ord[4];
    int affine;
    int pad;
};

// Fine node (i, j, k) of the macro: barycentric weights
// mu = (N-i-j-k, i, j, k)/N, affine point y = sum mu_v v, radius
// rho = sum mu_v |v|; blended point x = rho y / |y| (spherical layers).
TS_HD void node_xyz(const MacroGeom& g, int N, int i, int j, int k, double x[3]) {
    const int mu[4] = {N - i - j - k, i, j, k};
    double y0 = 0, y1 = 0, y2 = 0, rho = 0;
    const double invN = 1.0 / (double)N;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int a = g.ord[q];
        const double w = (double)mu[a] * invN;
        y0 += w * g.v[a][0];
        y1 += w * g.v[a][1];
        y2 += w * g.v[a][2];
        rho += w * g.r[a];
    }
    if (g.affine) {
        x[0] = y0; x[1] = y1; x[2] = y2;
        return;
    }
    const double s = rho / sqrt(y0 * y0 + y1 * y1 + y2 * y2);
    x[0] = s * y0; x[1] = s * y1; x[2] = s * y2;
}

// Row of vertex 0 of the P1 stiffness matrix of the straight tetrahedron
// P0..P3: K[q] = |T| grad(l_0) . grad(l_q).  With e_a = P_a - P0 the
// gradients are the rows of the inverse edge matrix: grad(l_a) = c_a / det
// with c_1 = e2 x e3, c_2 = e3 x e1, c_3 = e1 x e2, grad(l_0) = -sum.
// Returns |T|.
TS_HD double stiffness_row0(const double* P0, const double* P1, const double* P2,
                            const double* P3, double K[4]) {
    const double a0 = P1[0] - P0[0], a1 = P1[1] - P0[1], a2 = P1[2] - P0[2];
    const double b0 = P2[0] - P0[0], b1 = P2[1] - P0[1], b2 = P2[2] - P0[2];
    const double c0 = P3[0] - P0[0], c1 = P3[1] - P0[1], c2 = P3[2] - P0[2];
    const double g10 = b1 * c2 - b2 * c1, g11 = b2 * c0 - b0 * c2, g12 = b0 * c1 - b1 * c0;
    const double g20 = c1 * a2 - c2 * a1, g21 = c2 * a0 - c0 * a2, g22 = c0 * a1 - c1 * a0;
    const double g30 = a1 * b2 - a2 * b1, g31 = a2 * b0 - a0 * b2, g32 = a0 * b1 - a1 * b0;
    const double g00 = -(g10 + g20 + g30), g01 = -(g11 + g21 + g31), g02 = -(g12 + g22 + g32);
    const double det = a0 * g10 + a1 * g11 + a2 * g12;
    const double ad = fabs(det);
    const double sc = 1.0 / (6.0 * ad);
    K[0] = (g00 * g00 + g01 * g01 + g02 * g02) * sc;
    K[1] = (g00 * g10 + g01 * g11 + g02 * g12) * sc;
    K[2] = (g00 * g20 + g01 * g21 + g02 * g22) * sc;
    K[3] = (g00 * g30 + g01 * g31 + g02 * g32) * sc;
    return ad / 6.0;
}

// The 24 fine tetrahedra around a node, each as 4 direction indices with
// the node itself (mc = 0) first.  Built from the six tetrahedra of a
// lattice cell (Bey's refinement): up {0, e1, e2, e3}; the octahedron
// {e1, e2, e3, e1+e2, e1+e3, e2+e3} cut around its e2 -- e1+e3 diagonal;
// down {e1+e2, e1+e3, e2+e3, e1+e2+e3}.
struct Tets24 {
    signed char t[24][4];
};

constexpr int cdir_index(int di, int dj, int dk) {
    constexpr int I[NW] = {0, -1, 1, 0, 0, 1, -1, 0, 1, 0, -1, 0, -1, 0, 1};
    constexpr int J[NW] = {0, 0, 0, -1, 1, -1, 1, 0, 0, 1, 1, 0, 0, -1, -1};
    constexpr int K[NW] = {0, 0, 0, 0, 0, 0, 0, -1, -1, -1, -1, 1, 1, 1, 1};
    for (int w = 0; w < NW; w++)
        if (I[w] == di && J[w] == dj && K[w] == dk) return w;
    return -1;
}

constexpr Tets24 make_tets24() {
    constexpr int cell[6][4][3] = {
        {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
        {{0, 1, 0}, {1, 0, 1}, {1, 0, 0}, {0, 0, 1}},
        {{0, 1, 0}, {1, 0, 1}, {0, 0, 1}, {0, 1, 1}},
        {{0, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 0}},
        {{0, 1, 0}, {1, 0, 1}, {1, 1, 0}, {1, 0, 0}},
        {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}}};
    Tets24 T{};
    int n = 0;
    for (int ty = 0; ty < 6; ty++)
        for (int role = 0; role < 4; role++) {
            T.t[n][0] = 0;
            int q = 1;
            for (int w = 0; w < 4; w++) {
                if (w == role) continue;
                T.t[n][q++] = (signed char)cdir_index(cell[ty][w][0] - cell[ty][role][0],
                                                      cell[ty][w][1] - cell[ty][role][1],
                                                      cell[ty][w][2] - cell[ty][role][2]);
            }
            n++;
        }
    return T;
}

// compile-time table: fully unrolled loops index the coordinate registers
// statically
inline constexpr Tets24 kTets24 = make_tets24();

// IFEM stencil at local node (i, j, k) of a macro (Sec. 2.3 / Tab. flops
// "IFEM"): the stiffness rows of every fine tetrahedron of this macro that
// contains the node, summed per direction.  Tetrahedra reaching outside the
// closed macro are skipped, so for nodes on the macro boundary this is the
// macro's partial row.  vol (optional) gets sum |T| over those tetrahedra.
TS_HD void ifem_partial_stencil(const MacroGeom& g, int N, int i, int j, int k, double s[NW],
                                double* vol = nullptr) {
    double xs[NW][3];
    unsigned valid = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const int a = i + dir_i(w), b = j + dir_j(w), c = k + dir_k(w);
        s[w] = 0.0;
        if (inside(N, a, b, c)) {
            valid |= 1u << w;
            node_xyz(g, N, a, b, c, xs[w]);
        }
    }
    double vs = 0;
#pragma unroll
    for (int t = 0; t < 24; t++) {
        const int w0 = kTets24.t[t][0], w1 = kTets24.t[t][1], w2 = kTets24.t[t][2],
                  w3 = kTets24.t[t][3];
        const unsigned need = (1u << w0) | (1u << w1) | (1u << w2) | (1u << w3);
        if ((valid & need) != need) continue;
        double K[4];
        vs += stiffness_row0(xs[w0], xs[w1], xs[w2], xs[w3], K);
        s[w0] += K[0];
        s[w1] += K[1];
        s[w2] += K[2];
        s[w3] += K[3];
    }
    if (vol) *vol = vs;
}

}  // namespace ts
