/*
 * ts_oracle.c -- plain FP64 CPU oracle of the two-scale surrogate-stencil
 * method (Bauer, Mohr, Ruede, Weismueller, Wittmann, Wohlmuth: "A two-scale
 * approach for efficient on-the-fly operator assembly in massively parallel
 * high performance multigrid codes", arXiv 1608.06473).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library: every definition below is written out again here from
 * the paper, slowly and directly, so that a reader can check it by eye.
 *
 * Conventions (the paper's level l has 2^(l+2) intervals per macro edge; this
 * code takes N, the number of intervals, directly):
 *  - A macro tetrahedron T = (v0, v1, v2, v3) in the given vertex order.  Its
 *    fine nodes are the index triples (i, j, k) >= 0 with i + j + k <= N; the
 *    node's barycentric weights are mu = (N-i-j-k, i, j, k) / N (Sec. 2.2,
 *    the affine map Psi_T of the reference tetrahedron).
 *  - Geometry (Sec. 2.2, blending map Phi_T): y = sum_v mu_v v (affine point),
 *    rho = sum_v mu_v |v|; the fine node sits at x = rho * y / |y| for the
 *    spherical-shell blending, or at x = y for the affine geometry (Phi = Id).
 *    On a shared face rho and y depend only on the face vertices, so Phi is
 *    continuous; vertices are fixed; interior macros form spherical layers.
 *  - Fine tetrahedra (Sec. 2.3, Bey's regular refinement): for each lattice
 *    cell base c, the "up" tetrahedron {c, c+e1, c+e2, c+e3}, the octahedron
 *    {c+e1, c+e2, c+e3, c+e1+e2, c+e1+e3, c+e2+e3} cut into 4 tetrahedra
 *    around its diagonal c+e2 -- c+e1+e3, and the "down" tetrahedron
 *    {c+e1+e2, c+e1+e3, c+e2+e3, c+e1+e2+e3}; exactly those whose vertices
 *    lie in the closed macro.  24 of them meet at an interior node.
 *  - The 15 stencil directions W (Sec. 2.3) in this order:
 *      0 mc (0,0,0)   1 mw (-1,0,0)   2 me (1,0,0)    3 ms (0,-1,0)
 *      4 mn (0,1,0)   5 mse (1,-1,0)  6 mnw (-1,1,0)  7 bc (0,0,-1)
 *      8 be (1,0,-1)  9 bn (0,1,-1)  10 bnw (-1,1,-1) 11 tc (0,0,1)
 *     12 tw (-1,0,1) 13 ts (0,-1,1)  14 tse (1,-1,1)
 *  - P1 stiffness on straight fine tetrahedra between mapped vertices
 *    (Sec. 2.2, eq. (algebraic)): K_T[a][b] = |T| grad(lambda_a).grad(lambda_b).
 *  - Dirichlet nodes: every node on a mesh-boundary face (face of one macro).
 *
 * Canonical order of the unique nodes (the vector format of this oracle):
 *   vertices by global id; then edges (g0 < g1) in lexicographic order with
 *   their interior points a = 1..N-1 (weight of g1 = a/N); then faces
 *   (g0 < g1 < g2) in lexicographic order with interior points (a, b),
 *   b = 1..N-2 outer, a = 1..N-1-b inner (weights of g1, g2 = a/N, b/N); then
 *   for each macro in input order its interior points (i, j, k) >= 1,
 *   i + j + k <= N-1, k outer, j, i inner.
 * Block order (the HIP library's vector format): macro-major; inside a macro
 *   all (N+1)(N+2)(N+3)/6 nodes, k outer, j, i inner; interface nodes are
 *   repeated in every macro that contains them.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define NW 15

static const int DIR[NW][3] = {
    {0, 0, 0},  {-1, 0, 0}, {1, 0, 0},  {0, -1, 0}, {0, 1, 0},
    {1, -1, 0}, {-1, 1, 0}, {0, 0, -1}, {1, 0, -1}, {0, 1, -1},
    {-1, 1, -1}, {0, 0, 1}, {-1, 0, 1}, {0, -1, 1}, {1, -1, 1}};

/* ------------------------------------------------------------------------ */
/* mesh and topology                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t nv, nt, ne, nf;
    int affine;          /* 1: Phi = Id, 0: spherical blending */
    double *vtx;         /* nv x 3 */
    double *vrad;        /* |v| */
    int64_t *tet;        /* nt x 4 */
    int64_t *edges;      /* ne x 2, g0 < g1, lexicographic */
    int64_t *faces;      /* nf x 3, g0 < g1 < g2, lexicographic */
    int *face_count;     /* macros per face */
    unsigned char *vdir, *edir, *fdir; /* Dirichlet flags per primitive */
    /* incidence (CSR): primitive -> macros containing it */
    int64_t *v_off, *v_tet, *e_off, *e_tet, *f_off, *f_tet;
} or_mesh;

static int cmp2(const void *a, const void *b) {
    const int64_t *x = a, *y = b;
    for (int i = 0; i < 2; i++) {
        if (x[i] < y[i]) return -1;
        if (x[i] > y[i]) return 1;
    }
    return 0;
}
static int cmp3(const void *a, const void *b) {
    const int64_t *x = a, *y = b;
    for (int i = 0; i < 3; i++) {
        if (x[i] < y[i]) return -1;
        if (x[i] > y[i]) return 1;
    }
    return 0;
}
static void sort_small(int64_t *v, int n) {
    for (int a = 0; a < n; a++)
        for (int b = a + 1; b < n; b++)
            if (v[b] < v[a]) { int64_t t = v[a]; v[a] = v[b]; v[b] = t; }
}

static int64_t find_edge(const or_mesh *M, int64_t a, int64_t b) {
    int64_t key[2] = {a < b ? a : b, a < b ? b : a};
    int64_t lo = 0, hi = M->ne - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int c = cmp2(key, M->edges + 2 * mid);
        if (c == 0) return mid;
        if (c < 0) hi = mid - 1; else lo = mid + 1;
    }
    return -1;
}
static int64_t find_face(const or_mesh *M, int64_t a, int64_t b, int64_t c) {
    int64_t key[3] = {a, b, c};
    sort_small(key, 3);
    int64_t lo = 0, hi = M->nf - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int r = cmp3(key, M->faces + 3 * mid);
        if (r == 0) return mid;
        if (r < 0) hi = mid - 1; else lo = mid + 1;
    }
    return -1;
}

static void build_csr(int64_t n, int64_t nt, const int64_t *tet_items, int per,
                      int64_t **off_out, int64_t **tet_out) {
    int64_t *off = calloc(n + 1, sizeof(int64_t));
    for (int64_t t = 0; t < nt; t++)
        for (int p = 0; p < per; p++) off[tet_items[t * per + p] + 1]++;
    for (int64_t i = 0; i < n; i++) off[i + 1] += off[i];
    int64_t *fill = calloc(n, sizeof(int64_t));
    int64_t *lst = malloc(sizeof(int64_t) * (off[n] > 0 ? off[n] : 1));
    for (int64_t t = 0; t < nt; t++)
        for (int p = 0; p < per; p++) {
            int64_t id = tet_items[t * per + p];
            lst[off[id] + fill[id]++] = t;
        }
    free(fill);
    *off_out = off;
    *tet_out = lst;
}

or_mesh *or_mesh_new(const double *vtx, int64_t nv, const int64_t *tet,
                     int64_t nt, int affine) {
    or_mesh *M = calloc(1, sizeof(or_mesh));
    M->nv = nv;
    M->nt = nt;
    M->affine = affine;
    M->vtx = malloc(sizeof(double) * 3 * nv);
    memcpy(M->vtx, vtx, sizeof(double) * 3 * nv);
    M->vrad = malloc(sizeof(double) * nv);
    for (int64_t v = 0; v < nv; v++)
        M->vrad[v] = sqrt(vtx[3 * v] * vtx[3 * v] + vtx[3 * v + 1] * vtx[3 * v + 1] +
                          vtx[3 * v + 2] * vtx[3 * v + 2]);
    M->tet = malloc(sizeof(int64_t) * 4 * nt);
    memcpy(M->tet, tet, sizeof(int64_t) * 4 * nt);

    /* edges */
    int64_t *e = malloc(sizeof(int64_t) * 12 * nt);
    int64_t n = 0;
    for (int64_t t = 0; t < nt; t++)
        for (int a = 0; a < 4; a++)
            for (int b = a + 1; b < 4; b++) {
                int64_t x = tet[4 * t + a], y = tet[4 * t + b];
                e[2 * n] = x < y ? x : y;
                e[2 * n + 1] = x < y ? y : x;
                n++;
            }
    qsort(e, n, 2 * sizeof(int64_t), cmp2);
    int64_t ne = 0;
    for (int64_t i = 0; i < n; i++)
        if (ne == 0 || cmp2(e + 2 * i, e + 2 * (ne - 1)) != 0) {
            e[2 * ne] = e[2 * i];
            e[2 * ne + 1] = e[2 * i + 1];
            ne++;
        }
    M->ne = ne;
    M->edges = e;

    /* faces */
    int64_t *f = malloc(sizeof(int64_t) * 12 * nt);
    n = 0;
    for (int64_t t = 0; t < nt; t++)
        for (int o = 0; o < 4; o++) {
            int64_t key[3];
            int c = 0;
            for (int a = 0; a < 4; a++)
                if (a != o) key[c++] = tet[4 * t + a];
            sort_small(key, 3);
            memcpy(f + 3 * n, key, sizeof key);
            n++;
        }
    qsort(f, n, 3 * sizeof(int64_t), cmp3);
    int64_t nf = 0;
    for (int64_t i = 0; i < n; i++)
        if (nf == 0 || cmp3(f + 3 * i, f + 3 * (nf - 1)) != 0) {
            memcpy(f + 3 * nf, f + 3 * i, 3 * sizeof(int64_t));
            nf++;
        }
    M->nf = nf;
    M->faces = f;

    /* incidence lists */
    int64_t *te = malloc(sizeof(int64_t) * 6 * nt);
    int64_t *tf = malloc(sizeof(int64_t) * 4 * nt);
    for (int64_t t = 0; t < nt; t++) {
        int c = 0;
        for (int a = 0; a < 4; a++)
            for (int b = a + 1; b < 4; b++)
                te[6 * t + c++] = find_edge(M, tet[4 * t + a], tet[4 * t + b]);
        for (int o = 0; o < 4; o++) {
            int64_t key[3];
            int q = 0;
            for (int a = 0; a < 4; a++)
                if (a != o) key[q++] = tet[4 * t + a];
            tf[4 * t + o] = find_face(M, key[0], key[1], key[2]);
        }
    }
    build_csr(nv, nt, tet, 4, &M->v_off, &M->v_tet);
    build_csr(ne, nt, te, 6, &M->e_off, &M->e_tet);
    build_csr(nf, nt, tf, 4, &M->f_off, &M->f_tet);
    free(te);
    free(tf);

    /* Dirichlet: all primitives of faces that belong to one macro only */
    M->face_count = calloc(nf, sizeof(int));
    for (int64_t i = 0; i < nf; i++) M->face_count[i] = (int)(M->f_off[i + 1] - M->f_off[i]);
    M->vdir = calloc(nv, 1);
    M->edir = calloc(ne, 1);
    M->fdir = calloc(nf, 1);
    for (int64_t i = 0; i < nf; i++) {
        if (M->face_count[i] != 1) continue;
        const int64_t *g = M->faces + 3 * i;
        M->fdir[i] = 1;
        for (int a = 0; a < 3; a++) M->vdir[g[a]] = 1;
        M->edir[find_edge(M, g[0], g[1])] = 1;
        M->edir[find_edge(M, g[0], g[2])] = 1;
        M->edir[find_edge(M, g[1], g[2])] = 1;
    }
    return M;
}

void or_mesh_free(or_mesh *M) {
    if (!M) return;
    free(M->vtx); free(M->vrad); free(M->tet); free(M->edges); free(M->faces);
    free(M->face_count); free(M->vdir); free(M->edir); free(M->fdir);
    free(M->v_off); free(M->v_tet); free(M->e_off); free(M->e_tet);
    free(M->f_off); free(M->f_tet);
    free(M);
}

int64_t or_mesh_counts(const or_mesh *M, int64_t *out4) {
    out4[0] = M->nv; out4[1] = M->ne; out4[2] = M->nf; out4[3] = M->nt;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* canonical numbering                                                       */
/* ------------------------------------------------------------------------ */

static int64_t n_face_int(int N) { return (int64_t)(N - 1) * (N - 2) / 2; }
static int64_t n_vol_int(int N) { return (int64_t)(N - 1) * (N - 2) * (N - 3) / 6; }

int64_t or_num_unique(const or_mesh *M, int N) {
    return M->nv + M->ne * (N - 1) + M->nf * n_face_int(N) + M->nt * n_vol_int(N);
}

/* offset of face-interior point (a, b) among the interior points of a face */
static int64_t face_off(int N, int a, int b) {
    int64_t o = 0;
    for (int bb = 1; bb < b; bb++) o += N - 1 - bb;
    return o + (a - 1);
}
/* offset of interior point (i, j, k) among the interior points of a macro:
   planes kk < k hold T(N-2-kk) interior points each (T(m) = m(m+1)/2), rows
   jj < j of plane k hold N-1-k-jj points each */
static int64_t tetn(int64_t m) { return m * (m + 1) * (m + 2) / 6; }
static int64_t vol_off(int N, int i, int j, int k) {
    int64_t planes = tetn(N - 3) - tetn(N - 2 - k);
    int64_t rows = (int64_t)(j - 1) * (N - 1 - k) - (int64_t)(j - 1) * j / 2;
    return planes + rows + (i - 1);
}

/* canonical id of the local node (i, j, k) of macro t; *dir (optional) gets
   its Dirichlet flag */
static int64_t canon_d(const or_mesh *M, int N, int64_t t, int i, int j, int k, int *dir) {
    int mu[4] = {N - i - j - k, i, j, k};
    const int64_t *g = M->tet + 4 * t;
    int loc[4], nz = 0;
    for (int a = 0; a < 4; a++)
        if (mu[a] != 0) loc[nz++] = a;
    if (nz == 1) {
        if (dir) *dir = M->vdir[g[loc[0]]];
        return g[loc[0]];
    }
    if (nz == 2) {
        int a = loc[0], b = loc[1];
        if (g[a] > g[b]) { int s = a; a = b; b = s; }
        int64_t e = find_edge(M, g[a], g[b]);
        if (dir) *dir = M->edir[e];
        return M->nv + e * (N - 1) + (mu[b] - 1);
    }
    if (nz == 3) {
        /* sort the three local vertices by global id */
        for (int x = 0; x < 3; x++)
            for (int y = x + 1; y < 3; y++)
                if (g[loc[y]] < g[loc[x]]) { int s = loc[x]; loc[x] = loc[y]; loc[y] = s; }
        int64_t f = find_face(M, g[loc[0]], g[loc[1]], g[loc[2]]);
        int a = mu[loc[1]], b = mu[loc[2]];
        if (dir) *dir = M->fdir[f];
        return M->nv + M->ne * (N - 1) + f * n_face_int(N) + face_off(N, a, b);
    }
    if (dir) *dir = 0;
    return M->nv + M->ne * (N - 1) + M->nf * n_face_int(N) + t * n_vol_int(N) +
           vol_off(N, i, j, k);
}

int64_t or_canon(const or_mesh *M, int N, int64_t t, int i, int j, int k) {
    return canon_d(M, N, t, i, j, k, NULL);
}

/* kind: 0 vertex, 1 edge, 2 face, 3 volume */
typedef struct {
    int kind;
    int64_t prim;   /* vertex / edge / face / macro id */
    int a, b;       /* edge: a; face: (a, b) */
    int i, j, k;    /* volume */
} or_node;

static or_node decode(const or_mesh *M, int N, int64_t u) {
    or_node n;
    memset(&n, 0, sizeof n);
    if (u < M->nv) { n.kind = 0; n.prim = u; return n; }
    u -= M->nv;
    if (u < M->ne * (N - 1)) {
        n.kind = 1; n.prim = u / (N - 1); n.a = (int)(u % (N - 1)) + 1; return n;
    }
    u -= M->ne * (N - 1);
    if (u < M->nf * n_face_int(N)) {
        n.kind = 2; n.prim = u / n_face_int(N);
        int64_t r = u % n_face_int(N);
        for (int b = 1; b <= N - 2; b++) {
            int64_t len = N - 1 - b;
            if (r < len) { n.b = b; n.a = (int)r + 1; break; }
            r -= len;
        }
        return n;
    }
    u -= M->nf * n_face_int(N);
    n.kind = 3; n.prim = u / n_vol_int(N);
    int64_t r = u % n_vol_int(N);
    int k = 1;
    while (k < N - 3 && vol_off(N, 1, 1, k + 1) <= r) k++;
    r -= vol_off(N, 1, 1, k);
    int j = 1;
    while (j < N - 2 - k && r >= (int64_t)(N - 1 - k - j)) { r -= N - 1 - k - j; j++; }
    n.i = (int)r + 1; n.j = j; n.k = k;
    return n;
}

int or_is_dirichlet(const or_mesh *M, int N, int64_t u) {
    if (u >= M->nv + M->ne * (N - 1) + M->nf * n_face_int(N)) return 0;
    or_node n = decode(M, N, u);
    if (n.kind == 0) return M->vdir[n.prim];
    if (n.kind == 1) return M->edir[n.prim];
    if (n.kind == 2) return M->fdir[n.prim];
    return 0;
}

/* copies of a unique node: the macros containing it and its local indices */
static int copies(const or_mesh *M, int N, int64_t u, int64_t *ct, int (*cijk)[3],
                  int maxc) {
    or_node n = decode(M, N, u);
    if (n.kind == 3) {
        ct[0] = n.prim; cijk[0][0] = n.i; cijk[0][1] = n.j; cijk[0][2] = n.k;
        return 1;
    }
    const int64_t *off, *lst;
    int64_t id = n.prim;
    if (n.kind == 0) { off = M->v_off; lst = M->v_tet; }
    else if (n.kind == 1) { off = M->e_off; lst = M->e_tet; }
    else { off = M->f_off; lst = M->f_tet; }
    int c = 0;
    for (int64_t p = off[id]; p < off[id + 1] && c < maxc; p++, c++) {
        int64_t t = lst[p];
        const int64_t *g = M->tet + 4 * t;
        int mu[4] = {0, 0, 0, 0};
        for (int a = 0; a < 4; a++) {
            if (n.kind == 0) {
                if (g[a] == id) mu[a] = N;
            } else if (n.kind == 1) {
                const int64_t *e = M->edges + 2 * id;
                if (g[a] == e[0]) mu[a] = N - n.a;
                if (g[a] == e[1]) mu[a] = n.a;
            } else {
                const int64_t *f = M->faces + 3 * id;
                if (g[a] == f[0]) mu[a] = N - n.a - n.b;
                if (g[a] == f[1]) mu[a] = n.a;
                if (g[a] == f[2]) mu[a] = n.b;
            }
        }
        ct[c] = t;
        cijk[c][0] = mu[1]; cijk[c][1] = mu[2]; cijk[c][2] = mu[3];
    }
    return c;
}

int or_copies(const or_mesh *M, int N, int64_t u, int64_t *ct, int *cijk, int maxc) {
    return copies(M, N, u, ct, (int (*)[3])cijk, maxc);
}

/* ------------------------------------------------------------------------ */
/* geometry: Psi_T then Phi_T                                                */
/* ------------------------------------------------------------------------ */

static void node_xyz_g(const or_mesh *M, int N, int64_t t, int i, int j, int k,
                       double x[3], int affine);
static void node_xyz(const or_mesh *M, int N, int64_t t, int i, int j, int k,
                     double x[3]) {
    node_xyz_g(M, N, t, i, j, k, x, M->affine);
}

/* The fine node (i, j, k) of macro t: the affine point y = Psi_T((i,j,k)/N)
   (affine != 0: Phi = Id, the unmapped macro) or its blended image
   x = rho(y) y / |y| (Sec. 2.2). */
static void node_xyz_g(const or_mesh *M, int N, int64_t t, int i, int j, int k,
                       double x[3], int affine) {
    const int64_t *g = M->tet + 4 * t;
    int mu[4] = {N - i - j - k, i, j, k};
    /* sum over the macro vertices in ascending global-id order, so that every
       macro sharing the node produces bitwise the same point */
    int ord[4] = {0, 1, 2, 3};
    for (int a = 0; a < 4; a++)
        for (int b = a + 1; b < 4; b++)
            if (g[ord[b]] < g[ord[a]]) { int s = ord[a]; ord[a] = ord[b]; ord[b] = s; }
    double y[3] = {0, 0, 0}, rho = 0;
    for (int q = 0; q < 4; q++) {
        int a = ord[q];
        double w = (double)mu[a] / (double)N;
        for (int d = 0; d < 3; d++) y[d] += w * M->vtx[3 * g[a] + d];
        rho += w * M->vrad[g[a]];
    }
    if (affine) {
        for (int d = 0; d < 3; d++) x[d] = y[d];
        return;
    }
    double ny = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    for (int d = 0; d < 3; d++) x[d] = rho * y[d] / ny;
}

void or_node_xyz(const or_mesh *M, int N, int64_t t, int i, int j, int k, double *x) {
    node_xyz(M, N, t, i, j, k, x);
}

void or_coords(const or_mesh *M, int N, double *xyz) {
    int64_t nu = or_num_unique(M, N);
    for (int64_t u = 0; u < nu; u++) {
        /* the first copy is enough: every copy gives the same point */
        int64_t ct[256];
        int cijk[256][3];
        copies(M, N, u, ct, cijk, 256);
        node_xyz(M, N, ct[0], cijk[0][0], cijk[0][1], cijk[0][2], xyz + 3 * u);
    }
}

/* ------------------------------------------------------------------------ */
/* fine tetrahedra around a node                                             */
/* ------------------------------------------------------------------------ */

/* The fine tetrahedra of cell base c, as offsets from c. */
static const int CELL_TETS[6][4][3] = {
    /* up */
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    /* octahedron, diagonal (0,1,0)-(1,0,1), equator cycle
       (1,0,0) -> (0,0,1) -> (0,1,1) -> (1,1,0) -> (1,0,0) */
    {{0, 1, 0}, {1, 0, 1}, {1, 0, 0}, {0, 0, 1}},
    {{0, 1, 0}, {1, 0, 1}, {0, 0, 1}, {0, 1, 1}},
    {{0, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 0}},
    {{0, 1, 0}, {1, 0, 1}, {1, 1, 0}, {1, 0, 0}},
    /* down */
    {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}}};

static int inside(int N, int i, int j, int k) {
    return i >= 0 && j >= 0 && k >= 0 && i + j + k <= N;
}

/* All fine tetrahedra of macro t that contain local node p; each returned as
   4 local index triples with p first.  Returns the count (24 at an interior
   node). */
static int tets_at(int N, const int p[3], int out[][4][3]) {
    int cnt = 0;
    for (int type = 0; type < 6; type++)
        for (int v = 0; v < 4; v++) {
            int c[3];
            for (int d = 0; d < 3; d++) c[d] = p[d] - CELL_TETS[type][v][d];
            int ok = 1;
            int vv[4][3];
            for (int w = 0; w < 4; w++) {
                for (int d = 0; d < 3; d++) vv[w][d] = c[d] + CELL_TETS[type][w][d];
                if (!inside(N, vv[w][0], vv[w][1], vv[w][2])) ok = 0;
            }
            if (!ok) continue;
            /* p first, then the others in their listed order */
            int q = 1;
            for (int d = 0; d < 3; d++) out[cnt][0][d] = p[d];
            for (int w = 0; w < 4; w++) {
                if (w == v) continue;
                for (int d = 0; d < 3; d++) out[cnt][q][d] = vv[w][d];
                q++;
            }
            cnt++;
        }
    return cnt;
}

/* Row of vertex 0 of the P1 stiffness matrix of the tetrahedron x[0..3]. */
static void stiff_row0(double x[4][3], double K[4], double *vol) {
    double a[3], b[3], c[3];
    for (int d = 0; d < 3; d++) {
        a[d] = x[1][d] - x[0][d];
        b[d] = x[2][d] - x[0][d];
        c[d] = x[3][d] - x[0][d];
    }
    double g[4][3];
    g[1][0] = b[1] * c[2] - b[2] * c[1];
    g[1][1] = b[2] * c[0] - b[0] * c[2];
    g[1][2] = b[0] * c[1] - b[1] * c[0];
    g[2][0] = c[1] * a[2] - c[2] * a[1];
    g[2][1] = c[2] * a[0] - c[0] * a[2];
    g[2][2] = c[0] * a[1] - c[1] * a[0];
    g[3][0] = a[1] * b[2] - a[2] * b[1];
    g[3][1] = a[2] * b[0] - a[0] * b[2];
    g[3][2] = a[0] * b[1] - a[1] * b[0];
    for (int d = 0; d < 3; d++) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    double det = a[0] * g[1][0] + a[1] * g[1][1] + a[2] * g[1][2];
    double adet = fabs(det);
    /* grad(lambda_q) = g[q] / det; |T| = |det| / 6 */
    for (int q = 0; q < 4; q++)
        K[q] = (g[0][0] * g[q][0] + g[0][1] * g[q][1] + g[0][2] * g[q][2]) / (6.0 * adet);
    if (vol) *vol = adet / 6.0;
}

/* IFEM stencil of the interior node (i, j, k) of macro t (Sec. 2.3): the sum
   over its 24 fine tetrahedra of the stiffness entries coupling it to each of
   its 14 neighbours, and to itself for mc. */
void or_ifem_stencil(const or_mesh *M, int N, int64_t t, int i, int j, int k,
                     double *s) {
    int p[3] = {i, j, k};
    int tl[32][4][3];
    int n = tets_at(N, p, tl);
    for (int w = 0; w < NW; w++) s[w] = 0.0;
    for (int q = 0; q < n; q++) {
        double x[4][3], K[4];
        for (int v = 0; v < 4; v++) node_xyz(M, N, t, tl[q][v][0], tl[q][v][1], tl[q][v][2], x[v]);
        stiff_row0(x, K, NULL);
        s[0] += K[0];
        for (int v = 1; v < 4; v++) {
            int d[3] = {tl[q][v][0] - i, tl[q][v][1] - j, tl[q][v][2] - k};
            for (int w = 1; w < NW; w++)
                if (DIR[w][0] == d[0] && DIR[w][1] == d[1] && DIR[w][2] == d[2]) s[w] += K[v];
        }
    }
}

/* Number of fine tetrahedra at local node (i,j,k) of a macro at N. */
int or_tets_at_count(int N, int i, int j, int k) {
    int p[3] = {i, j, k};
    int tl[32][4][3];
    return tets_at(N, p, tl);
}

/* Sum of the volumes of the fine tetrahedra of macro t (tiling check). */
double or_macro_fine_volume(const or_mesh *M, int N, int64_t t) {
    double vol = 0;
    for (int k = 0; k <= N; k++)
        for (int j = 0; j + k <= N; j++)
            for (int i = 0; i + j + k <= N; i++)
                for (int type = 0; type < 6; type++) {
                    int ok = 1, vv[4][3];
                    for (int w = 0; w < 4; w++) {
                        vv[w][0] = i + CELL_TETS[type][w][0];
                        vv[w][1] = j + CELL_TETS[type][w][1];
                        vv[w][2] = k + CELL_TETS[type][w][2];
                        if (!inside(N, vv[w][0], vv[w][1], vv[w][2])) ok = 0;
                    }
                    if (!ok) continue;
                    double x[4][3], K[4], v;
                    for (int w = 0; w < 4; w++) node_xyz(M, N, t, vv[w][0], vv[w][1], vv[w][2], x[w]);
                    stiff_row0(x, K, &v);
                    vol += v;
                }
    return vol;
}

/* ------------------------------------------------------------------------ */
/* surrogate polynomials (Sec. 3.1-3.3)                                      */
/* ------------------------------------------------------------------------ */

/* Basis: monomials xi^l eta^m zeta^n with xi = i/N - 1/4 (same for j, k),
   l + m + n <= q, ordered by total degree d = 0..q, then l descending, then m
   descending. */
int or_num_coeffs(int q) { return (q + 1) * (q + 2) * (q + 3) / 6; }

static int basis_exps(int q, int (*e)[3]) {
    int c = 0;
    for (int d = 0; d <= q; d++)
        for (int l = d; l >= 0; l--)
            for (int m = d - l; m >= 0; m--) {
                e[c][0] = l; e[c][1] = m; e[c][2] = d - l - m;
                c++;
            }
    return c;
}

static double ipow(double x, int n) {
    double r = 1.0;
    for (int a = 0; a < n; a++) r *= x;
    return r;
}

static void basis_row(int q, int N, int i, int j, int k, double *row) {
    int e[64][3];
    int mq = basis_exps(q, e);
    double xi = (double)i / N - 0.25, eta = (double)j / N - 0.25, zeta = (double)k / N - 0.25;
    for (int c = 0; c < mq; c++)
        row[c] = ipow(xi, e[c][0]) * ipow(eta, e[c][1]) * ipow(zeta, e[c][2]);
}

double or_poly_eval(int q, int N, const double *a, int i, int j, int k) {
    double row[64];
    basis_row(q, N, i, j, k, row);
    int mq = or_num_coeffs(q);
    double s = 0;
    for (int c = 0; c < mq; c++) s += a[c] * row[c];
    return s;
}

/* Sampling points of a level with N intervals.
   method 1 (LSQP): S = M_m embedded at stride N / 2^(m+2), with the paper's
     level l = log2(N) - 2 and m = min(l, max(1, jsamp))  (eq.
     samplingSetFunctions);
   method 2 (IPOLY, q = 2): the ten points of Sec. 3.1 with a = N - 3,
     b = N/2 - 1.
   Returns the count; pts may be NULL to query it. */
int64_t or_sample_points(int N, int method, int jsamp, int *pts) {
    if (method == 2) {
        int a = N - 3, b = N / 2 - 1;
        int P[10][3] = {{1, 1, 1}, {1, 1, a}, {1, a, 1}, {a, 1, 1}, {1, 1, b},
                        {1, b, 1}, {b, 1, 1}, {1, b, b}, {b, 1, b}, {b, b, 1}};
        if (pts) memcpy(pts, P, sizeof P);
        return 10;
    }
    int l = 0;
    while ((4 << l) < N) l++;
    int m = jsamp < 1 ? 1 : jsamp;
    if (m > l) m = l;
    int Ns = 4 << m;
    int stride = N / Ns;
    int64_t c = 0;
    for (int k = 1; k <= Ns - 3; k++)
        for (int j = 1; j <= Ns - 2 - k; j++)
            for (int i = 1; i <= Ns - 1 - j - k; i++) {
                if (pts) {
                    pts[3 * c] = i * stride;
                    pts[3 * c + 1] = j * stride;
                    pts[3 * c + 2] = k * stride;
                }
                c++;
            }
    return c;
}

/* Least-squares solve min ||A z - B||_2 for nrhs right-hand sides by
   Householder QR (A is m x n, m >= n, row-major; B is m x nrhs, row-major;
   the solution overwrites X (n x nrhs)).  Returns 0 on success. */
static int householder_lsq(int m, int n, double *A, double *B, int nrhs, double *X) {
    double *v = malloc(sizeof(double) * m);
    for (int c = 0; c < n; c++) {
        double nrm = 0;
        for (int r = c; r < m; r++) nrm += A[r * n + c] * A[r * n + c];
        nrm = sqrt(nrm);
        if (nrm == 0) { free(v); return 1; }
        double alpha = A[c * n + c] > 0 ? -nrm : nrm;
        for (int r = 0; r < m; r++) v[r] = 0;
        for (int r = c; r < m; r++) v[r] = A[r * n + c];
        v[c] -= alpha;
        double vv = 0;
        for (int r = c; r < m; r++) vv += v[r] * v[r];
        if (vv == 0) continue;
        /* apply H = I - 2 v v^T / (v^T v) to A[:, c:] and B */
        for (int cc = c; cc < n; cc++) {
            double d = 0;
            for (int r = c; r < m; r++) d += v[r] * A[r * n + cc];
            d = 2 * d / vv;
            for (int r = c; r < m; r++) A[r * n + cc] -= d * v[r];
        }
        for (int cc = 0; cc < nrhs; cc++) {
            double d = 0;
            for (int r = c; r < m; r++) d += v[r] * B[r * nrhs + cc];
            d = 2 * d / vv;
            for (int r = c; r < m; r++) B[r * nrhs + cc] -= d * v[r];
        }
    }
    /* back substitution R X = (Q^T B)[0:n] */
    for (int cc = 0; cc < nrhs; cc++)
        for (int r = n - 1; r >= 0; r--) {
            double s = B[r * nrhs + cc];
            for (int q = r + 1; q < n; q++) s -= A[r * n + q] * X[q * nrhs + cc];
            X[r * nrhs + cc] = s / A[r * n + r];
        }
    free(v);
    return 0;
}

/* Fit the surrogate coefficients of every macro at N intervals.
   method 1 = LSQP (sampling jsamp), 2 = IPOLY (q must be 2).
   coeffs: nt x 15 x m_q (row-major).  Returns 0 on success. */
int or_fit(const or_mesh *M, int N, int method, int q, int jsamp, double *coeffs) {
    if (method == 2 && q != 2) return 1;
    int mq = or_num_coeffs(q);
    int64_t ns = or_sample_points(N, method, jsamp, NULL);
    int *pts = malloc(sizeof(int) * 3 * ns);
    or_sample_points(N, method, jsamp, pts);
    double *A = malloc(sizeof(double) * ns * mq);
    double *B = malloc(sizeof(double) * ns * NW);
    double *X = malloc(sizeof(double) * mq * NW);
    int err = 0;
    for (int64_t t = 0; t < M->nt && !err; t++) {
        for (int64_t s = 0; s < ns; s++) {
            basis_row(q, N, pts[3 * s], pts[3 * s + 1], pts[3 * s + 2], A + s * mq);
            or_ifem_stencil(M, N, t, pts[3 * s], pts[3 * s + 1], pts[3 * s + 2], B + s * NW);
        }
        err = householder_lsq((int)ns, mq, A, B, NW, X);
        for (int w = 0; w < NW; w++)
            for (int c = 0; c < mq; c++) coeffs[(t * NW + w) * mq + c] = X[c * NW + w];
    }
    free(pts); free(A); free(B); free(X);
    return err;
}

/* ------------------------------------------------------------------------ */
/* symmetric surrogate (remark at the end of Sec. 3.4): one polynomial per   */
/* edge direction, evaluated at the midpoint of the edge                     */
/* ------------------------------------------------------------------------ */

/* the direction opposite to w */
static int dir_opposite(int w) {
    for (int v = 0; v < NW; v++)
        if (DIR[v][0] == -DIR[w][0] && DIR[v][1] == -DIR[w][1] && DIR[v][2] == -DIR[w][2])
            return v;
    return -1;
}

/* the seven edge directions: pair p joins directions w < w' = opposite(w) */
static int sym_pairs(int pw[7][2]) {
    int n = 0;
    for (int w = 1; w < NW; w++) {
        int o = dir_opposite(w);
        if (o > w) { pw[n][0] = w; pw[n][1] = o; n++; }
    }
    return n;
}

/* pair index of direction w (1..14) */
static int sym_pair_of(int w) {
    int pw[7][2];
    sym_pairs(pw);
    for (int p = 0; p < 7; p++)
        if (pw[p][0] == w || pw[p][1] == w) return p;
    return -1;
}

/* The basis at the midpoint of the edge from (i, j, k) in direction w: the
   point (i + w/2, ...) has index coordinates that are integers on the level
   with 2N intervals, so the monomials are those of that level at
   (2i + w_i, 2j + w_j, 2k + w_k). */
static void basis_row_mid(int q, int N, int i, int j, int k, int w, double *row) {
    basis_row(q, 2 * N, 2 * i + DIR[w][0], 2 * j + DIR[w][1], 2 * k + DIR[w][2], row);
}

/* Least-squares fit of the pair polynomials from values at the sampling
   points: vals[s][w] is the exact weight of direction w at sample s, i.e. the
   weight of the edge whose midpoint is sample + w/2; pair p is fitted to the
   weights of its two directions at all samples (2 x ns points).  out:
   7 x mq.  Returns 0 on success. */
static int fit_sym_from(int N, int q, int64_t ns, const int *pts, const double *vals,
                        double *out) {
    int mq = or_num_coeffs(q);
    int pw[7][2];
    sym_pairs(pw);
    double *A = malloc(sizeof(double) * 2 * ns * mq);
    double *B = malloc(sizeof(double) * 2 * ns);
    double X[64];
    int err = 0;
    for (int p = 0; p < 7 && !err; p++) {
        for (int h = 0; h < 2; h++) {
            int w = pw[p][h];
            for (int64_t t = 0; t < ns; t++) {
                basis_row_mid(q, N, pts[3 * t], pts[3 * t + 1], pts[3 * t + 2], w,
                              A + (h * ns + t) * mq);
                B[h * ns + t] = vals[t * NW + w];
            }
        }
        err = householder_lsq((int)(2 * ns), mq, A, B, 1, X);
        for (int c = 0; c < mq; c++) out[p * mq + c] = X[c];
    }
    free(A); free(B);
    return err;
}

/* Fit the pair polynomials of every macro at N intervals (LSQP sampling with
   jsamp); coeffs: nt x 7 x m_q.  Returns 0 on success. */
int or_fit_sym(const or_mesh *M, int N, int q, int jsamp, double *coeffs) {
    int mq = or_num_coeffs(q);
    int64_t ns = or_sample_points(N, 1, jsamp, NULL);
    int *pts = malloc(sizeof(int) * 3 * ns);
    or_sample_points(N, 1, jsamp, pts);
    double *V = malloc(sizeof(double) * ns * NW);
    int err = 0;
    for (int64_t t = 0; t < M->nt && !err; t++) {
        for (int64_t s2 = 0; s2 < ns; s2++)
            or_ifem_stencil(M, N, t, pts[3 * s2], pts[3 * s2 + 1], pts[3 * s2 + 2], V + s2 * NW);
        err = fit_sym_from(N, q, ns, pts, V, coeffs + t * 7 * mq);
    }
    free(pts); free(V);
    return err;
}

/* the same fit for given values (ns x 15) at the LSQP sampling points */
int or_fit_sym_values(int N, int q, int jsamp, const double *vals, double *out) {
    int64_t ns = or_sample_points(N, 1, jsamp, NULL);
    int *pts = malloc(sizeof(int) * 3 * ns);
    or_sample_points(N, 1, jsamp, pts);
    int err = fit_sym_from(N, q, ns, pts, vals, out);
    free(pts);
    return err;
}

/* value of a polynomial (m_q coefficients) at the midpoint of the edge from
   (i, j, k) in direction w */
double or_poly_eval_mid(int q, int N, const double *a, int i, int j, int k, int w) {
    double row[64];
    basis_row_mid(q, N, i, j, k, w, row);
    double s = 0;
    for (int c = 0; c < or_num_coeffs(q); c++) s += a[c] * row[c];
    return s;
}

/* ------------------------------------------------------------------------ */
/* surrogate rows on interior faces (the remark after eq.                    */
/* numInteriorPoints: the same fitting applies to face nodes)                */
/* ------------------------------------------------------------------------ */

/* Which face of the macro a face copy (i, j, k) lies on: 0 i = 0, 1 j = 0,
   2 k = 0, 3 i + j + k = N (exactly one barycentric weight is 0). */
static int face_type_of(int N, const int c[3]) {
    if (c[0] == 0) return 0;
    if (c[1] == 0) return 1;
    if (c[2] == 0) return 2;
    (void)N;
    return 3;
}

/* signed distance of direction w from face type f: < 0 leaves the macro,
   0 stays in the face, > 0 points into the macro */
static int dir_side(int f, int w) {
    if (f == 0) return DIR[w][0];
    if (f == 1) return DIR[w][1];
    if (f == 2) return DIR[w][2];
    return -(DIR[w][0] + DIR[w][1] + DIR[w][2]);
}

static int dir_index(int di, int dj, int dk) {
    for (int w = 0; w < NW; w++)
        if (DIR[w][0] == di && DIR[w][1] == dj && DIR[w][2] == dk) return w;
    return -1;
}

/* The 15 entries of the row of a free node of an interior face, whose two
   copies are A (the first macro listed for the face) and B: entry 0 the node,
   entries 1..10 the other directions of A that do not leave A (the six
   in-face neighbours and four points inside A) in increasing order, entries
   11..14 the directions of B that point into B, in increasing order.  nbr
   gets each entry's unique id and dir its Dirichlet flag. */
typedef struct {
    int64_t t[2];
    int c[2][3];
    int fa, fb;
    int wa[11], wb[4];
    int64_t nbr[NW];
    int dir[NW];
} face_row;

static void face_row_setup(const or_mesh *M, int N, int64_t u, face_row *F) {
    int cijk[2][3];
    copies(M, N, u, F->t, cijk, 2);
    for (int c = 0; c < 2; c++)
        for (int d = 0; d < 3; d++) F->c[c][d] = cijk[c][d];
    F->fa = face_type_of(N, F->c[0]);
    F->fb = face_type_of(N, F->c[1]);
    int na = 0, nb = 0;
    for (int w = 0; w < NW; w++) {
        if (dir_side(F->fa, w) >= 0) F->wa[na++] = w;
        if (dir_side(F->fb, w) > 0) F->wb[nb++] = w;
    }
    for (int e = 0; e < 11; e++) {
        int w = F->wa[e];
        F->nbr[e] = canon_d(M, N, F->t[0], F->c[0][0] + DIR[w][0], F->c[0][1] + DIR[w][1],
                            F->c[0][2] + DIR[w][2], &F->dir[e]);
    }
    for (int e = 0; e < 4; e++) {
        int w = F->wb[e];
        F->nbr[11 + e] = canon_d(M, N, F->t[1], F->c[1][0] + DIR[w][0], F->c[1][1] + DIR[w][1],
                                 F->c[1][2] + DIR[w][2], &F->dir[11 + e]);
    }
}

/* exact (element-wise, Sec. 2.3) weights of the 15 entries: the stiffness
   rows of the fine tetrahedra at both copies, each coupling added to the
   entry of the node it reaches */
static void face_row_exact(const or_mesh *M, int N, const face_row *F, double s[NW]) {
    for (int e = 0; e < NW; e++) s[e] = 0;
    for (int c = 0; c < 2; c++) {
        int tl[32][4][3];
        int nt = tets_at(N, F->c[c], tl);
        for (int q = 0; q < nt; q++) {
            double xx[4][3], K[4];
            for (int v = 0; v < 4; v++)
                node_xyz(M, N, F->t[c], tl[q][v][0], tl[q][v][1], tl[q][v][2], xx[v]);
            stiff_row0(xx, K, NULL);
            s[0] += K[0];
            for (int v = 1; v < 4; v++) {
                int w = dir_index(tl[q][v][0] - F->c[c][0], tl[q][v][1] - F->c[c][1],
                                  tl[q][v][2] - F->c[c][2]);
                int e = -1;
                if (c == 0) {
                    for (int r = 0; r < 11; r++)
                        if (F->wa[r] == w) e = r;
                } else if (dir_side(F->fb, w) > 0) {
                    for (int r = 0; r < 4; r++)
                        if (F->wb[r] == w) e = 11 + r;
                } else {
                    int64_t g = canon_d(M, N, F->t[1], tl[q][v][0], tl[q][v][1], tl[q][v][2],
                                        NULL);
                    for (int r = 1; r < 11; r++)
                        if (F->nbr[r] == g) e = r;
                }
                s[e] += K[v];
            }
        }
    }
}

/* 2D monomials of total degree <= q in the face frame, alpha = a/N - 1/3,
   beta = b/N - 1/3 (centred on the face), by degree, then by falling power
   of alpha */
int or_num_coeffs2(int q) { return (q + 1) * (q + 2) / 2; }

static void basis_row2(int q, int N, int a, int b, double *row) {
    double al = (double)a / N - 1.0 / 3.0, be = (double)b / N - 1.0 / 3.0;
    int c = 0;
    for (int d = 0; d <= q; d++)
        for (int l = 0; l <= d; l++) row[c++] = ipow(al, d - l) * ipow(be, l);
}

/* Face sampling points (a, b): the interior points of the face lattice of
   level m at stride N / 2^(m+2), with m chosen as for the volume fit. */
int64_t or_face_sample_points(int N, int jsamp, int *pts) {
    int l = 0;
    while ((4 << l) < N) l++;
    int m = jsamp < 1 ? 1 : jsamp;
    if (m > l) m = l;
    int Ns = 4 << m, st = N / Ns;
    int64_t c = 0;
    for (int b = 1; b <= Ns - 2; b++)
        for (int a = 1; a <= Ns - 1 - b; a++) {
            if (pts) {
                pts[2 * c] = a * st;
                pts[2 * c + 1] = b * st;
            }
            c++;
        }
    return c;
}

/* Fit the 15 entries of every free interior face (two macros, not on the
   boundary) by least squares over the face sampling points (Householder
   QR).  fcoef: nf x 15 x m2 (faces not fitted stay 0).  Returns 0 on
   success. */
int or_face_fit(const or_mesh *M, int N, int q, int jsamp, double *fcoef) {
    int m2 = or_num_coeffs2(q);
    int64_t ns = or_face_sample_points(N, jsamp, NULL);
    if (ns < m2) return 1;
    int *pts = malloc(sizeof(int) * 2 * ns);
    or_face_sample_points(N, jsamp, pts);
    memset(fcoef, 0, sizeof(double) * M->nf * NW * m2);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t f = 0; f < M->nf; f++) {
        if (M->face_count[f] != 2 || M->fdir[f]) continue;
        double *A = malloc(sizeof(double) * ns * m2);
        double *B = malloc(sizeof(double) * ns * NW);
        double *X = malloc(sizeof(double) * m2 * NW);
        for (int64_t s = 0; s < ns; s++) {
            int a = pts[2 * s], b = pts[2 * s + 1];
            int64_t u = M->nv + M->ne * (N - 1) + f * n_face_int(N) + face_off(N, a, b);
            face_row F;
            face_row_setup(M, N, u, &F);
            face_row_exact(M, N, &F, B + s * NW);
            basis_row2(q, N, a, b, A + s * m2);
        }
        err |= householder_lsq((int)ns, m2, A, B, NW, X);
        for (int e = 0; e < NW; e++)
            for (int c = 0; c < m2; c++) fcoef[(f * NW + e) * m2 + c] = X[c * NW + e];
        free(A); free(B); free(X);
    }
    free(pts);
    return err;
}

/* value at face node (a, b) of the 2D polynomial with coefficients c (m2) */
double or_face_poly_eval(int q, int N, const double *c, int a, int b) {
    double row[64];
    basis_row2(q, N, a, b, row);
    double s = 0;
    for (int k = 0; k < or_num_coeffs2(q); k++) s += c[k] * row[k];
    return s;
}

/* The same least-squares fit for given values at the face sampling points
   (ns x 15, row-major); out: 15 x m2.  Returns 0 on success. */
int or_face_fit_values(int N, int q, int jsamp, const double *vals, double *out) {
    int m2 = or_num_coeffs2(q);
    int64_t ns = or_face_sample_points(N, jsamp, NULL);
    if (ns < m2) return 1;
    int *pts = malloc(sizeof(int) * 2 * ns);
    or_face_sample_points(N, jsamp, pts);
    double *A = malloc(sizeof(double) * ns * m2);
    double *B = malloc(sizeof(double) * ns * NW);
    double *X = malloc(sizeof(double) * m2 * NW);
    for (int64_t s = 0; s < ns; s++) basis_row2(q, N, pts[2 * s], pts[2 * s + 1], A + s * m2);
    memcpy(B, vals, sizeof(double) * ns * NW);
    int err = householder_lsq((int)ns, m2, A, B, NW, X);
    for (int e = 0; e < NW; e++)
        for (int c = 0; c < m2; c++) out[e * m2 + c] = X[c * NW + e];
    free(pts); free(A); free(B); free(X);
    return err;
}

/* the exact 15 entries of a face node (unique id u), for checks */
int or_face_row_exact(const or_mesh *M, int N, int64_t u, double *s, int64_t *nbr) {
    face_row F;
    face_row_setup(M, N, u, &F);
    face_row_exact(M, N, &F, s);
    if (nbr)
        for (int e = 0; e < NW; e++) nbr[e] = F.nbr[e];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the operator                                                              */
/* ------------------------------------------------------------------------ */

/* Operator on one level: kind 0 = IFEM everywhere; kind 1 = surrogate rows on
   the volume primitives (coefficients nt x 15 x m_q) with IFEM rows on the
   lower primitives (Sec. 3.4); kind 2 = the symmetric surrogate (coefficients
   nt x 7 x m_q, one per edge direction, centre from the row sum); kind 3 =
   the constant stencil of the unmapped geometry on the volume primitives
   (the paper's lower bound in Sec. 4.2.1 and Sec. 5: the volume rows of the
   fine tetrahedra of the affine macro, Phi = Id, with IFEM rows of the mesh
   geometry on the lower primitives).  center 0: own polynomial for mc; 1: mc
   from the row sum (Alg. 1). */
typedef struct {
    int kind, q, center;
    const double *coeffs;
    const unsigned char *ifem; /* per macro: 1 = IFEM rows on the volume (NULL: none) */
    const double *fcoef;       /* kind 1: per-face fits (nf x 15 x m2) for the rows
                                  of interior faces; NULL: IFEM rows there */
} or_op;

static int64_t vol_base(const or_mesh *M, int N) {
    return M->nv + M->ne * (N - 1) + M->nf * n_face_int(N);
}

/* Gauss-Seidel phase of a free unique node:
   0 vertices; 1-2 edges by a mod 2; 3-5 faces by (a + 2b) mod 3 in the face
   frame; 6-9 volume by (i + 2j + 3k) mod 4. */
int or_gs_phase(const or_mesh *M, int N, int64_t u) {
    or_node n = decode(M, N, u);
    if (n.kind == 0) return 0;
    if (n.kind == 1) return 1 + n.a % 2;
    if (n.kind == 2) return 3 + (n.a + 2 * n.b) % 3;
    return 6 + (n.i + 2 * n.j + 3 * n.k) % 4;
}

/* IFEM row (Sec. 2.3): sum over every copy of the node and every fine
   tetrahedron at that copy of the stiffness row; diag = a_II and
   off = sum_{J != I} a_IJ x_J with x = 0 at Dirichlet nodes. */
static void row_ifem_g(const or_mesh *M, int N, const int64_t *ct, int (*cijk)[3], int nc,
                       const double *x, double *diag, double *off, int affine);
static void row_ifem(const or_mesh *M, int N, const int64_t *ct, int (*cijk)[3], int nc,
                     const double *x, double *diag, double *off) {
    row_ifem_g(M, N, ct, cijk, nc, x, diag, off, M->affine);
}
/* affine != 0: the fine tetrahedra of the unmapped macros (Phi = Id) */
static void row_ifem_g(const or_mesh *M, int N, const int64_t *ct, int (*cijk)[3], int nc,
                       const double *x, double *diag, double *off, int affine) {
    double dg = 0, of = 0;
    for (int c = 0; c < nc; c++) {
        int tl[32][4][3];
        int nt = tets_at(N, cijk[c], tl);
        for (int q = 0; q < nt; q++) {
            double xx[4][3], K[4];
            for (int v = 0; v < 4; v++)
                node_xyz_g(M, N, ct[c], tl[q][v][0], tl[q][v][1], tl[q][v][2], xx[v], affine);
            stiff_row0(xx, K, NULL);
            dg += K[0];
            for (int v = 1; v < 4; v++) {
                int dir;
                int64_t w = canon_d(M, N, ct[c], tl[q][v][0], tl[q][v][1], tl[q][v][2], &dir);
                of += K[v] * (dir ? 0.0 : x[w]);
            }
        }
    }
    *diag = dg;
    *off = of;
}

/* Surrogate row of the interior node (i, j, k) of macro t (Sec. 3.4): each
   weight is its polynomial evaluated at the node's own index triple; mc from
   its own polynomial or from the row sum. */
static void row_surrogate(const or_mesh *M, int N, const or_op *op, int64_t t, int i,
                          int j, int k, const double *x, double *diag, double *off) {
    int mq = or_num_coeffs(op->q);
    const double *a = op->coeffs + t * NW * mq;
    double s[NW];
    for (int w = 0; w < NW; w++) s[w] = or_poly_eval(op->q, N, a + w * mq, i, j, k);
    if (op->center == 1) {
        s[0] = 0;
        for (int w = 1; w < NW; w++) s[0] -= s[w];
    }
    double of = 0;
    for (int w = 1; w < NW; w++) {
        int dir;
        int64_t v = canon_d(M, N, t, i + DIR[w][0], j + DIR[w][1], k + DIR[w][2], &dir);
        of += s[w] * (dir ? 0.0 : x[v]);
    }
    *diag = s[0];
    *off = of;
}

/* Surrogate row of a free node (a, b) of the interior face f: every entry
   from its fitted 2D polynomial, the centre from its own polynomial. */
static void row_face_surrogate(const or_mesh *M, int N, const or_op *op, int64_t u, int64_t f,
                               int a, int b, const double *x, double *diag, double *off) {
    int m2 = or_num_coeffs2(op->q);
    double row[64];
    basis_row2(op->q, N, a, b, row);
    face_row F;
    face_row_setup(M, N, u, &F);
    const double *fc = op->fcoef + f * NW * m2;
    double of = 0;
    for (int e = 1; e < NW; e++) {
        double se = 0;
        for (int c = 0; c < m2; c++) se += fc[e * m2 + c] * row[c];
        of += se * (F.dir[e] ? 0.0 : x[F.nbr[e]]);
    }
    double s0 = 0;
    for (int c = 0; c < m2; c++) s0 += fc[c] * row[c];
    *diag = s0;
    *off = of;
}

/* Symmetric surrogate row of the interior node (i, j, k) of macro t: the
   weight of direction w is its pair polynomial at the midpoint of the edge,
   the centre weight minus the sum of the others (coefficients nt x 7 x m_q). */
static void row_surrogate_sym(const or_mesh *M, int N, const or_op *op, int64_t t, int i,
                              int j, int k, const double *x, double *diag, double *off) {
    int mq = or_num_coeffs(op->q);
    const double *a = op->coeffs + t * 7 * mq;
    double of = 0, sum = 0;
    for (int w = 1; w < NW; w++) {
        double sw = or_poly_eval_mid(op->q, N, a + sym_pair_of(w) * mq, i, j, k, w);
        sum += sw;
        int dir;
        int64_t v = canon_d(M, N, t, i + DIR[w][0], j + DIR[w][1], k + DIR[w][2], &dir);
        of += sw * (dir ? 0.0 : x[v]);
    }
    *diag = -sum;
    *off = of;
}

/* row of the interior node (i, j, k) of macro t under op */
static void row_volume(const or_mesh *M, int N, const or_op *op, int64_t t, int i, int j,
                       int k, const double *x, double *diag, double *off) {
    if (op->kind == 2 && !(op->ifem && op->ifem[t])) {
        row_surrogate_sym(M, N, op, t, i, j, k, x, diag, off);
    } else if (op->kind == 1 && !(op->ifem && op->ifem[t])) {
        row_surrogate(M, N, op, t, i, j, k, x, diag, off);
    } else if (op->kind == 3) {
        int64_t ct[1] = {t};
        int cijk[1][3] = {{i, j, k}};
        row_ifem_g(M, N, ct, cijk, 1, x, diag, off, 1);
    } else {
        int64_t ct[1] = {t};
        int cijk[1][3] = {{i, j, k}};
        row_ifem(M, N, ct, cijk, 1, x, diag, off);
    }
}

/* row of any free unique node u */
static void row_eval(const or_mesh *M, int N, const or_op *op, int64_t u,
                     const double *x, double *diag, double *off) {
    or_node n = decode(M, N, u);
    if (n.kind == 3) {
        row_volume(M, N, op, n.prim, n.i, n.j, n.k, x, diag, off);
        return;
    }
    if (n.kind == 2 && op->kind == 1 && op->fcoef && M->face_count[n.prim] == 2) {
        row_face_surrogate(M, N, op, u, n.prim, n.a, n.b, x, diag, off);
        return;
    }
    int64_t ct[256];
    int cijk[256][3];
    int nc = copies(M, N, u, ct, cijk, 256);
    row_ifem(M, N, ct, cijk, nc, x, diag, off);
}

/* Visit every free row of GS phase `phase` (all rows if phase < 0): first the
   lower-primitive rows (unique ids below the volume block), then the interior
   points of every macro in canonical order.  The callback gets the unique
   id and the row's diag and off terms. */
typedef void (*row_fn)(void *ctx, int64_t u, double diag, double off);

static void for_rows(const or_mesh *M, int N, const or_op *op, const double *x,
                     int phase, row_fn fn, void *ctx) {
    int64_t vb = vol_base(M, N);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < vb; u++) {
        if (or_is_dirichlet(M, N, u)) continue;
        if (phase >= 0 && or_gs_phase(M, N, u) != phase) continue;
        double dg, of;
        row_eval(M, N, op, u, x, &dg, &of);
        fn(ctx, u, dg, of);
    }
    if (phase >= 0 && phase < 6) return;
    int64_t V = n_vol_int(N);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < M->nt; t++) {
        int64_t u = vb + t * V;
        for (int k = 1; k <= N - 3; k++)
            for (int j = 1; j <= N - 2 - k; j++)
                for (int i = 1; i <= N - 1 - j - k; i++, u++) {
                    if (phase >= 0 && 6 + (i + 2 * j + 3 * k) % 4 != phase) continue;
                    double dg, of;
                    row_volume(M, N, op, t, i, j, k, x, &dg, &of);
                    fn(ctx, u, dg, of);
                }
    }
}

typedef struct { const double *x, *f; double *y; } rows_ctx;

static void cb_apply(void *c, int64_t u, double dg, double of) {
    rows_ctx *r = c;
    r->y[u] = dg * r->x[u] + of;
}
static void cb_residual(void *c, int64_t u, double dg, double of) {
    rows_ctx *r = c;
    r->y[u] = r->f[u] - (dg * r->x[u] + of);
}
static void cb_gs(void *c, int64_t u, double dg, double of) {
    rows_ctx *r = c;
    r->y[u] = (r->f[u] - of) / dg;
}

static void zero_dirichlet(const or_mesh *M, int N, double *y) {
    int64_t vb = vol_base(M, N);
    for (int64_t u = 0; u < vb; u++)
        if (or_is_dirichlet(M, N, u)) y[u] = 0;
}

/* Per-macro IFEM fallback flags used by the operator entry points below
   (set with or_set_ifem_flags; NULL: surrogate rows on every macro). */
static const unsigned char *g_flags = NULL;
void or_set_ifem_flags(const unsigned char *flags) { g_flags = flags; }

/* Per-face fits used by the surrogate operator entry points below (set with
   or_set_face_coeffs; NULL: element-wise rows on every face). */
static const double *g_fcoef = NULL;
void or_set_face_coeffs(const double *fcoef) { g_fcoef = fcoef; }

/* y = L x over the free rows; Dirichlet rows of y are set to 0. */
void or_apply(const or_mesh *M, int N, int kind, int q, int center,
              const double *coeffs, const double *x, double *y) {
    or_op op = {kind, q, center, coeffs, g_flags, g_fcoef};
    rows_ctx c = {x, NULL, y};
    zero_dirichlet(M, N, y);
    for_rows(M, N, &op, x, -1, cb_apply, &c);
}

/* y_r = (L x)_{rows[r]} for selected rows only. */
void or_apply_rows(const or_mesh *M, int N, int kind, int q, int center,
                   const double *coeffs, const double *x, const int64_t *rows,
                   int64_t nrows, double *y) {
    or_op op = {kind, q, center, coeffs, g_flags, g_fcoef};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t u = rows[r];
        if (or_is_dirichlet(M, N, u)) { y[r] = 0; continue; }
        double dg, of;
        row_eval(M, N, &op, u, x, &dg, &of);
        y[r] = dg * x[u] + of;
    }
}

/* The Gauss-Seidel update of eq. iteration-scheme at the listed rows,
   out[r] = (f_u - sum_{J != u} a_uJ x_J) / a_uu with the row of unique node
   u = rows[r] (as in or_gs_sweep); 0 on Dirichlet rows.  With x the values
   at the start of a node's phase this is the value the sweep gives it. */
void or_gs_rows(const or_mesh *M, int N, int kind, int q, int center, const double *coeffs,
                const double *f, const double *x, const int64_t *rows, int64_t nrows,
                double *out) {
    or_op op = {kind, q, center, coeffs, g_flags, g_fcoef};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t u = rows[r];
        if (or_is_dirichlet(M, N, u)) { out[r] = 0; continue; }
        double dg, of;
        row_eval(M, N, &op, u, x, &dg, &of);
        out[r] = (f[u] - of) / dg;
    }
}

/* Unique ids of the free nodes that share a fine edge with node u: the
   neighbours in the 14 stencil directions of every copy of u that stay in
   that copy's macro, each once.  Returns their number (at most maxn). */
int or_row_neighbours(const or_mesh *M, int N, int64_t u, int64_t *out, int maxn) {
    int64_t ct[256];
    int cijk[256][3];
    int nc = copies(M, N, u, ct, cijk, 256), n = 0;
    for (int c = 0; c < nc; c++)
        for (int w = 1; w < NW; w++) {
            int i = cijk[c][0] + DIR[w][0], j = cijk[c][1] + DIR[w][1], k = cijk[c][2] + DIR[w][2];
            if (i < 0 || j < 0 || k < 0 || i + j + k > N) continue;
            int dir;
            int64_t v = canon_d(M, N, ct[c], i, j, k, &dir);
            if (dir) continue;
            int seen = 0;
            for (int e = 0; e < n; e++) seen |= out[e] == v;
            if (!seen && n < maxn) out[n++] = v;
        }
    return n;
}

/* r = f - L u on the free rows, 0 on Dirichlet rows. */
void or_residual(const or_mesh *M, int N, int kind, int q, int center,
                 const double *coeffs, const double *f, const double *u, double *r) {
    or_op op = {kind, q, center, coeffs, g_flags, g_fcoef};
    rows_ctx c = {u, f, r};
    zero_dirichlet(M, N, r);
    for_rows(M, N, &op, u, -1, cb_residual, &c);
}

/* One multicolour Gauss-Seidel sweep (eq. iteration-scheme): phases 0..9 in
   order; inside a phase every node is updated from the values at the start
   of that phase. */
/* Ordering of the sweep (an experiment on the smoother, not the operator):
   0 the multicolour phases below (default); 1 the same volume colours, but
   every free face, edge and vertex node updated one after the other in
   canonical order, each from the newest values (true Gauss-Seidel on the
   interface); 2 every free node one after the other in canonical order
   (interface, then each macro's interior with i fastest: the lexicographic
   Gauss-Seidel of eq. iteration-scheme). */
static int g_gs_order = 0;
void or_set_gs_order(int mode) { g_gs_order = mode; }

static void gs_node_seq(const or_mesh *M, int N, const or_op *op, const double *f, double *u,
                        int64_t v) {
    if (or_is_dirichlet(M, N, v)) return;
    double dg, of;
    row_eval(M, N, op, v, u, &dg, &of);
    u[v] = (f[v] - of) / dg;
}

void or_gs_sweep(const or_mesh *M, int N, int kind, int q, int center,
                 const double *coeffs, const double *f, double *u) {
    or_op op = {kind, q, center, coeffs, g_flags, g_fcoef};
    int64_t nu = or_num_unique(M, N);
    int64_t vb = vol_base(M, N);
    int64_t V = n_vol_int(N);
    if (g_gs_order == 2) {
        for (int64_t v = 0; v < nu; v++) gs_node_seq(M, N, &op, f, u, v);
        return;
    }
    double *nw = malloc(sizeof(double) * nu);
    for (int p = 0; p < 10; p++) {
        if (g_gs_order == 1 && p < 6) {
            if (p == 0)
                for (int64_t v = 0; v < vb; v++) gs_node_seq(M, N, &op, f, u, v);
            continue;
        }
        rows_ctx c = {u, f, nw};
        for_rows(M, N, &op, u, p, cb_gs, &c);
        if (p < 6) {
            for (int64_t v = 0; v < vb; v++)
                if (!or_is_dirichlet(M, N, v) && or_gs_phase(M, N, v) == p) u[v] = nw[v];
        } else {
            for (int64_t t = 0; t < M->nt; t++) {
                int64_t v = vb + t * V;
                for (int k = 1; k <= N - 3; k++)
                    for (int j = 1; j <= N - 2 - k; j++)
                        for (int i = 1; i <= N - 1 - j - k; i++, v++)
                            if (6 + (i + 2 * j + 3 * k) % 4 == p) u[v] = nw[v];
            }
        }
    }
    free(nw);
}

/* ------------------------------------------------------------------------ */
/* grid transfer: linear interpolation in index space, R = P^T               */
/* ------------------------------------------------------------------------ */

/* parents of the fine node u (N fine intervals): coarse ids and weights */
static int parents(const or_mesh *M, int N, int64_t u, int64_t *pc, double *pw) {
    int64_t ct[256];
    int cijk[256][3];
    copies(M, N, u, ct, cijk, 256);
    int *p = cijk[0];
    int64_t t = ct[0];
    int Nc = N / 2;
    int par[3] = {p[0] & 1, p[1] & 1, p[2] & 1};
    if (!par[0] && !par[1] && !par[2]) {
        pc[0] = or_canon(M, Nc, t, p[0] / 2, p[1] / 2, p[2] / 2);
        pw[0] = 1.0;
        return 1;
    }
    /* the lattice edge direction with this parity pattern */
    int d[3];
    if (par[0] && !par[1] && !par[2]) { d[0] = 1; d[1] = 0; d[2] = 0; }
    else if (!par[0] && par[1] && !par[2]) { d[0] = 0; d[1] = 1; d[2] = 0; }
    else if (!par[0] && !par[1] && par[2]) { d[0] = 0; d[1] = 0; d[2] = 1; }
    else if (par[0] && par[1] && !par[2]) { d[0] = 1; d[1] = -1; d[2] = 0; }
    else if (par[0] && !par[1] && par[2]) { d[0] = -1; d[1] = 0; d[2] = 1; }
    else if (!par[0] && par[1] && par[2]) { d[0] = 0; d[1] = -1; d[2] = 1; }
    else { d[0] = 1; d[1] = -1; d[2] = 1; }
    int c1[3], c2[3];
    for (int a = 0; a < 3; a++) {
        c1[a] = (p[a] - d[a]) / 2;
        c2[a] = (p[a] + d[a]) / 2;
    }
    pc[0] = or_canon(M, Nc, t, c1[0], c1[1], c1[2]);
    pc[1] = or_canon(M, Nc, t, c2[0], c2[1], c2[2]);
    pw[0] = pw[1] = 0.5;
    return 2;
}

/* uf = P uc (fine N intervals), Dirichlet fine nodes set to 0 */
void or_prolongate(const or_mesh *M, int N, const double *uc, double *uf) {
    int64_t nu = or_num_unique(M, N);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < nu; u++) {
        if (or_is_dirichlet(M, N, u)) { uf[u] = 0; continue; }
        int64_t pc[2];
        double pw[2];
        int np = parents(M, N, u, pc, pw);
        double s = 0;
        for (int a = 0; a < np; a++)
            s += pw[a] * (or_is_dirichlet(M, N / 2, pc[a]) ? 0.0 : uc[pc[a]]);
        uf[u] = s;
    }
}

/* rc = P^T rf (rf on N fine intervals), Dirichlet coarse rows set to 0 */
void or_restrict(const or_mesh *M, int N, const double *rf, double *rc) {
    int64_t nf = or_num_unique(M, N), nc = or_num_unique(M, N / 2);
    for (int64_t c = 0; c < nc; c++) rc[c] = 0;
    for (int64_t u = 0; u < nf; u++) {
        if (or_is_dirichlet(M, N, u)) continue;
        int64_t pc[2];
        double pw[2];
        int np = parents(M, N, u, pc, pw);
        for (int a = 0; a < np; a++) rc[pc[a]] += pw[a] * rf[u];
    }
    for (int64_t c = 0; c < nc; c++)
        if (or_is_dirichlet(M, N / 2, c)) rc[c] = 0;
}

/* ------------------------------------------------------------------------ */
/* coarse solve: dense Cholesky of the IFEM operator at the coarsest level   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int N;
    int64_t n;        /* free nodes */
    int64_t *ids;     /* free unique ids */
    int64_t *pos;     /* unique id -> free index or -1 */
    double *L;        /* n x n lower Cholesky factor */
} or_coarse;

or_coarse *or_coarse_new(const or_mesh *M, int N) {
    int64_t nu = or_num_unique(M, N);
    or_coarse *C = calloc(1, sizeof(or_coarse));
    C->N = N;
    C->pos = malloc(sizeof(int64_t) * nu);
    C->ids = malloc(sizeof(int64_t) * nu);
    int64_t n = 0;
    for (int64_t u = 0; u < nu; u++) {
        if (or_is_dirichlet(M, N, u)) { C->pos[u] = -1; continue; }
        C->pos[u] = n;
        C->ids[n++] = u;
    }
    C->n = n;
    double *A = calloc((size_t)n * n, sizeof(double));
    double *e = calloc(nu, sizeof(double));
    double *col = malloc(sizeof(double) * nu);
    /* columns of the IFEM operator applied to unit vectors */
    for (int64_t c = 0; c < n; c++) {
        e[C->ids[c]] = 1.0;
        or_apply(M, N, 0, 0, 0, NULL, e, col);
        e[C->ids[c]] = 0.0;
        for (int64_t r = 0; r < n; r++) A[r * n + c] = col[C->ids[r]];
    }
    free(e); free(col);
    /* symmetrise the rounding, then Cholesky */
    for (int64_t r = 0; r < n; r++)
        for (int64_t c = 0; c < r; c++) {
            double m = 0.5 * (A[r * n + c] + A[c * n + r]);
            A[r * n + c] = A[c * n + r] = m;
        }
    for (int64_t j = 0; j < n; j++) {
        double s = A[j * n + j];
        for (int64_t k = 0; k < j; k++) s -= A[j * n + k] * A[j * n + k];
        A[j * n + j] = sqrt(s);
        for (int64_t i = j + 1; i < n; i++) {
            double t = A[i * n + j];
            for (int64_t k = 0; k < j; k++) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / A[j * n + j];
        }
    }
    C->L = A;
    return C;
}

void or_coarse_free(or_coarse *C) {
    if (!C) return;
    free(C->ids); free(C->pos); free(C->L); free(C);
}

int64_t or_coarse_size(const or_coarse *C) { return C->n; }

/* u = L0^{-1} f on the free nodes (canonical vectors at the coarse level) */
void or_coarse_solve(const or_coarse *C, const or_mesh *M, const double *f, double *u) {
    int64_t n = C->n, nu = or_num_unique(M, C->N);
    double *z = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; i++) {
        double s = f[C->ids[i]];
        for (int64_t k = 0; k < i; k++) s -= C->L[i * n + k] * z[k];
        z[i] = s / C->L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; i--) {
        double s = z[i];
        for (int64_t k = i + 1; k < n; k++) s -= C->L[k * n + i] * z[k];
        z[i] = s / C->L[i * n + i];
    }
    for (int64_t v = 0; v < nu; v++) u[v] = 0;
    for (int64_t i = 0; i < n; i++) u[C->ids[i]] = z[i];
    free(z);
}

/* ------------------------------------------------------------------------ */
/* V(nu1, nu2) cycle                                                         */
/* ------------------------------------------------------------------------ */

/* levels: N = 2^lam for lam = lam0 .. lamL; lam0 uses IFEM and the coarse
   solve; every finer level uses the operator (kind, q, center) with its own
   coefficients coeffs[lam - lam0] (NULL entries are allowed for IFEM).
   dd != 0 selects double discretisation (Sec. 4 introduction): the smoothing sweeps keep
   the operator (kind, q, center) while every residual r = f - L u uses the
   exact IFEM operator L. */
typedef struct {
    const or_mesh *M;
    int lam0, lamL, kind, q, center, nu1, nu2, dd;
    const double **coeffs;
    const unsigned char **flags;
    const double **fcoef;
    or_coarse *coarse;
} or_mg;

or_mg *or_mg_new(const or_mesh *M, int lam0, int lamL, int kind, int q, int center,
                 int nu1, int nu2, const double **coeffs) {
    or_mg *G = calloc(1, sizeof(or_mg));
    G->M = M; G->lam0 = lam0; G->lamL = lamL; G->kind = kind; G->q = q;
    G->center = center; G->nu1 = nu1; G->nu2 = nu2;
    int nl = lamL - lam0 + 1;
    G->coeffs = calloc(nl, sizeof(double *));
    G->flags = calloc(nl, sizeof(unsigned char *));
    G->fcoef = calloc(nl, sizeof(double *));
    for (int l = 0; l < nl; l++) G->coeffs[l] = coeffs ? coeffs[l] : NULL;
    G->coarse = or_coarse_new(M, 1 << lam0);
    return G;
}

void or_mg_set_flags(or_mg *G, int lam, const unsigned char *flags) {
    G->flags[lam - G->lam0] = flags;
}

void or_mg_set_dd(or_mg *G, int dd) { G->dd = dd; }

void or_mg_set_face_coeffs(or_mg *G, int lam, const double *fcoef) {
    G->fcoef[lam - G->lam0] = fcoef;
}

void or_mg_free(or_mg *G) {
    if (!G) return;
    or_coarse_free(G->coarse);
    free(G->coeffs);
    free(G->flags);
    free(G->fcoef);
    free(G);
}

static void vcycle_rec(const or_mg *G, int lam, const double *f, double *u) {
    const or_mesh *M = G->M;
    int N = 1 << lam;
    if (lam == G->lam0) {
        or_coarse_solve(G->coarse, M, f, u);
        return;
    }
    int kind = G->kind;
    const double *cf = G->coeffs[lam - G->lam0];
    or_set_ifem_flags(G->flags[lam - G->lam0]);
    or_set_face_coeffs(G->fcoef[lam - G->lam0]);
    for (int s = 0; s < G->nu1; s++) or_gs_sweep(M, N, kind, G->q, G->center, cf, f, u);
    int64_t nf = or_num_unique(M, N), nc = or_num_unique(M, N / 2);
    double *r = malloc(sizeof(double) * nf);
    double *fc = malloc(sizeof(double) * nc);
    double *uc = calloc(nc, sizeof(double));
    double *e = malloc(sizeof(double) * nf);
    if (G->dd)
        or_residual(M, N, 0, G->q, G->center, NULL, f, u, r);
    else
        or_residual(M, N, kind, G->q, G->center, cf, f, u, r);
    or_restrict(M, N, r, fc);
    vcycle_rec(G, lam - 1, fc, uc);
    or_set_ifem_flags(G->flags[lam - G->lam0]);
    or_set_face_coeffs(G->fcoef[lam - G->lam0]);
    or_prolongate(M, N, uc, e);
    for (int64_t v = 0; v < nf; v++) u[v] += e[v];
    for (int s = 0; s < G->nu2; s++) or_gs_sweep(M, N, kind, G->q, G->center, cf, f, u);
    free(r); free(fc); free(uc); free(e);
}

void or_vcycle(const or_mg *G, const double *f, double *u) {
    vcycle_rec(G, G->lamL, f, u);
}

/* ||r||_2 over free rows */
double or_norm_free(const or_mesh *M, int N, const double *r) {
    int64_t nu = or_num_unique(M, N);
    double s = 0;
    for (int64_t v = 0; v < nu; v++)
        if (!or_is_dirichlet(M, N, v)) s += r[v] * r[v];
    return sqrt(s);
}

/* FP64 solve by V-cycles until ||f - L u|| <= rtol ||f||.  Returns the number
   of cycles (or -1 when max_cycles is reached); hist gets the relative
   residual after each cycle (size max_cycles + 1). */
int or_solve(const or_mg *G, const double *f, double *u, double rtol,
             int max_cycles, double *hist) {
    const or_mesh *M = G->M;
    int N = 1 << G->lamL;
    int64_t nu = or_num_unique(M, N);
    double *r = malloc(sizeof(double) * nu);
    const double *cf = G->coeffs[G->lamL - G->lam0];
    double nf = or_norm_free(M, N, f);
    or_set_ifem_flags(G->flags[G->lamL - G->lam0]);
    or_set_face_coeffs(G->fcoef[G->lamL - G->lam0]);
    or_residual(M, N, G->kind, G->q, G->center, cf, f, u, r);
    double rel = or_norm_free(M, N, r) / nf;
    if (hist) hist[0] = rel;
    int c = 0;
    while (rel > rtol && c < max_cycles) {
        or_vcycle(G, f, u);
        or_set_ifem_flags(G->flags[G->lamL - G->lam0]);
        or_set_face_coeffs(G->fcoef[G->lamL - G->lam0]);
        or_residual(M, N, G->kind, G->q, G->center, cf, f, u, r);
        rel = or_norm_free(M, N, r) / nf;
        c++;
        if (hist) hist[c] = rel;
    }
    free(r);
    return rel <= rtol ? c : -1;
}

/* Double-discretisation solve (Sec. 4 introduction): with two operators in the cycle the
   residual does not go to zero, so the stop test is on the update instead,
   ||u_c - u_{c-1}||_2 <= rtol ||u_c||_2 over the free rows.  Returns the
   number of cycles (or -1 when max_cycles is reached); hist[c - 1] gets the
   relative update of cycle c (size max_cycles). */
int or_solve_dd(const or_mg *G, const double *f, double *u, double rtol,
                int max_cycles, double *hist) {
    const or_mesh *M = G->M;
    int N = 1 << G->lamL;
    int64_t nu = or_num_unique(M, N);
    double *prev = malloc(sizeof(double) * nu);
    double *d = malloc(sizeof(double) * nu);
    double rel = INFINITY;
    int c = 0;
    while (c < max_cycles) {
        memcpy(prev, u, sizeof(double) * nu);
        or_vcycle(G, f, u);
        for (int64_t v = 0; v < nu; v++) d[v] = u[v] - prev[v];
        double nu_ = or_norm_free(M, N, u);
        rel = nu_ > 0 ? or_norm_free(M, N, d) / nu_ : 0.0;
        if (hist) hist[c] = rel;
        c++;
        if (rel <= rtol) break;
    }
    free(prev);
    free(d);
    return rel <= rtol ? c : -1;
}

/* ------------------------------------------------------------------------ */
/* right-hand side: f = M I f with the consistent P1 mass matrix             */
/* ------------------------------------------------------------------------ */

/* kind 0: f = -Laplace(u) for u = sin(pi (r - r1)/(r2 - r1)) x y z,
           params = {r1, r2}
   kind 1: sum of Gaussian bumps, params = records (cx, cy, cz, sigma, amp)
   kind 2: f = 1 */
static double rhs_point(int kind, const double *par, int np, const double x[3]) {
    if (kind == 0) {
        double r1 = par[0], r2 = par[1], d = r2 - r1;
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        double th = M_PI * (r - r1) / d;
        double h = x[0] * x[1] * x[2];
        double k = M_PI / d;
        return h * (k * k * sin(th) - (8.0 / r) * k * cos(th));
    }
    if (kind == 1) {
        double s = 0;
        for (int b = 0; b + 5 <= np; b += 5) {
            double dx = x[0] - par[b], dy = x[1] - par[b + 1], dz = x[2] - par[b + 2];
            double sg = par[b + 3];
            s += par[b + 4] * exp(-(dx * dx + dy * dy + dz * dz) / (2 * sg * sg));
        }
        return s;
    }
    return 1.0;
}

double or_exact_manufactured(double r1, double r2, const double *x) {
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    return sin(M_PI * (r - r1) / (r2 - r1)) * x[0] * x[1] * x[2];
}

void or_rhs(const or_mesh *M, int N, int kind, const double *par, int np, double *f) {
    int64_t nu = or_num_unique(M, N);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < nu; u++) {
        if (or_is_dirichlet(M, N, u)) { f[u] = 0; continue; }
        int64_t ct[256];
        int cijk[256][3];
        int nc = copies(M, N, u, ct, cijk, 256);
        double s = 0;
        for (int c = 0; c < nc; c++) {
            int tl[32][4][3];
            int nt = tets_at(N, cijk[c], tl);
            for (int q = 0; q < nt; q++) {
                double xx[4][3], K[4], vol, fv[4];
                for (int v = 0; v < 4; v++) {
                    node_xyz(M, N, ct[c], tl[q][v][0], tl[q][v][1], tl[q][v][2], xx[v]);
                    fv[v] = rhs_point(kind, par, np, xx[v]);
                }
                stiff_row0(xx, K, &vol);
                /* consistent mass: |T|/20 (1 + delta_ab) */
                s += vol / 20.0 * (2 * fv[0] + fv[1] + fv[2] + fv[3]);
            }
        }
        f[u] = s;
    }
}

/* V_I = sum over the fine tetrahedra at I of |T| / 4 */
void or_node_volumes(const or_mesh *M, int N, double *vol_out) {
    int64_t nu = or_num_unique(M, N);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < nu; u++) {
        int64_t ct[256];
        int cijk[256][3];
        int nc = copies(M, N, u, ct, cijk, 256);
        double s = 0;
        for (int c = 0; c < nc; c++) {
            int tl[32][4][3];
            int nt = tets_at(N, cijk[c], tl);
            for (int q = 0; q < nt; q++) {
                double xx[4][3], K[4], vol;
                for (int v = 0; v < 4; v++)
                    node_xyz(M, N, ct[c], tl[q][v][0], tl[q][v][1], tl[q][v][2], xx[v]);
                stiff_row0(xx, K, &vol);
                s += vol / 4.0;
            }
        }
        vol_out[u] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* block layout                                                              */
/* ------------------------------------------------------------------------ */

int64_t or_block_size(int N) { return (int64_t)(N + 1) * (N + 2) * (N + 3) / 6; }

/* block position of local node (i, j, k): k outer, j, i inner */
int64_t or_block_index(int N, int i, int j, int k) {
    int64_t o = 0;
    for (int kk = 0; kk < k; kk++) o += (int64_t)(N + 1 - kk) * (N + 2 - kk) / 2;
    for (int jj = 0; jj < j; jj++) o += N + 1 - k - jj;
    return o + i;
}

/* canonical -> block; Dirichlet entries become 0 */
void or_canon_to_block(const or_mesh *M, int N, const double *c, double *b) {
    int64_t B = or_block_size(N);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < M->nt; t++) {
        int64_t p = 0;
        for (int k = 0; k <= N; k++)
            for (int j = 0; j + k <= N; j++)
                for (int i = 0; i + j + k <= N; i++) {
                    int64_t u = or_canon(M, N, t, i, j, k);
                    b[t * B + p] = or_is_dirichlet(M, N, u) ? 0.0 : c[u];
                    p++;
                }
    }
}

/* block -> canonical (first copy of each node); returns the largest
   difference between copies of one node (0 for a consistent block vector) */
double or_block_to_canon(const or_mesh *M, int N, const double *b, double *c) {
    int64_t nu = or_num_unique(M, N);
    int64_t B = or_block_size(N);
    double worst = 0;
    for (int64_t u = 0; u < nu; u++) {
        int64_t ct[256];
        int cijk[256][3];
        int nc = copies(M, N, u, ct, cijk, 256);
        double v0 = b[ct[0] * B + or_block_index(N, cijk[0][0], cijk[0][1], cijk[0][2])];
        c[u] = v0;
        for (int q = 1; q < nc; q++) {
            double v = b[ct[q] * B + or_block_index(N, cijk[q][0], cijk[q][1], cijk[q][2])];
            double d = fabs(v - v0);
            if (d > worst) worst = d;
        }
    }
    return worst;
}

/* canonical ids of every block slot (for building sample maps in tests) */
void or_block_canon_ids(const or_mesh *M, int N, int64_t *ids) {
    int64_t B = or_block_size(N);
    for (int64_t t = 0; t < M->nt; t++) {
        int64_t p = 0;
        for (int k = 0; k <= N; k++)
            for (int j = 0; j + k <= N; j++)
                for (int i = 0; i + j + k <= N; i++) ids[t * B + p++] = or_canon(M, N, t, i, j, k);
    }
}

void or_dirichlet_mask(const or_mesh *M, int N, unsigned char *mask) {
    int64_t nu = or_num_unique(M, N);
    for (int64_t u = 0; u < nu; u++) mask[u] = (unsigned char)or_is_dirichlet(M, N, u);
}

void or_gs_phases_all(const or_mesh *M, int N, int *ph) {
    int64_t nu = or_num_unique(M, N);
    for (int64_t u = 0; u < nu; u++) ph[u] = or_gs_phase(M, N, u);
}

/* Least-squares (or interpolation) fit of given sample values: vals is
   ns x 15 at the sampling points of (N, method, jsamp); coeffs 15 x m_q. */
int or_fit_values(int N, int method, int q, int jsamp, const double *vals, double *coeffs) {
    int mq = or_num_coeffs(q);
    int64_t ns = or_sample_points(N, method, jsamp, NULL);
    int *pts = malloc(sizeof(int) * 3 * ns);
    or_sample_points(N, method, jsamp, pts);
    double *A = malloc(sizeof(double) * ns * mq);
    double *B = malloc(sizeof(double) * ns * NW);
    double *X = malloc(sizeof(double) * mq * NW);
    for (int64_t s = 0; s < ns; s++) basis_row(q, N, pts[3 * s], pts[3 * s + 1], pts[3 * s + 2], A + s * mq);
    memcpy(B, vals, sizeof(double) * ns * NW);
    int err = householder_lsq((int)ns, mq, A, B, NW, X);
    for (int w = 0; w < NW; w++)
        for (int c = 0; c < mq; c++) coeffs[w * mq + c] = X[c * NW + w];
    free(pts); free(A); free(B); free(X);
    return err;
}

/* The fine tetrahedra of a macro at local node (i,j,k): out is cnt x 4 x 3
   index triples (the node first).  Returns cnt. */
int or_tets_at_list(int N, int i, int j, int k, int *out) {
    int p[3] = {i, j, k};
    int tl[32][4][3];
    int n = tets_at(N, p, tl);
    memcpy(out, tl, sizeof(int) * 12 * n);
    return n;
}

/* Selective surrogate (remark in Sec. 3.4: the surrogate can be switched off
   per macro depending on its shape): a macro keeps IFEM rows on this level if
   at any of the check points (1,1,1), (N-3,1,1), (1,N-3,1), (1,1,N-3) and
   (N/4,N/4,N/4) the surrogate centre weight is not positive or differs from
   the exact one by more than tol times the exact one.  tol <= 0 disables the
   check (all flags 0). */
void or_fallback_flags(const or_mesh *M, int N, int q, const double *coeffs, double tol,
                       unsigned char *flags) {
    int mq = or_num_coeffs(q);
    for (int64_t t = 0; t < M->nt; t++) {
        flags[t] = 0;
        if (tol <= 0) continue;
        int P[5][3] = {{1, 1, 1}, {N - 3, 1, 1}, {1, N - 3, 1}, {1, 1, N - 3}, {N / 4, N / 4, N / 4}};
        for (int c = 0; c < 5; c++) {
            double s[NW];
            or_ifem_stencil(M, N, t, P[c][0], P[c][1], P[c][2], s);
            double e = or_poly_eval(q, N, coeffs + t * NW * mq, P[c][0], P[c][1], P[c][2]);
            if (!(e > 0) || fabs(e - s[0]) > tol * s[0]) flags[t] = 1;
        }
    }
}
