// Stencil kernels for gfx950 besides the surrogate volume kernel: IFEM
// volume rows (Sec. 2.3, element-wise assembly from the 24 fine tetrahedra
// at a node; the comparison path), lower-primitive rows (faces, edges,
// vertices: element-wise assembly over all adjacent macros, with the
// per-copy partial stencils stored once per level), and the dispatch of the
// surrogate volume kernel.  Each kernel serves y = L x, r = f - L x and the
// Gauss-Seidel update u_I = (f_I - sum_{w != mc} s_w u_{I_w}) / s_mc
// (eq. iteration-scheme).
#include "ts_face.h"
#include "ts_surrogate.h"

namespace ts {

// lanes per node of the general lower-primitive path (a power of two <= 64)
constexpr int IFACE_LANES = 8;

// Lower primitives -------------------------------------------------------------
// General path: eight lanes per listed free face/edge/vertex node (32 nodes
// per workgroup; an edge has 3-7 copies, a vertex up to about 20).  The
// lanes take the node's copies (the stored element-wise partial stencil of
// each adjacent macro), the partial sums are reduced across the eight lanes
// in a fixed tree order, and the lanes write the copies.  MODE 0: y = L x; 1: y = f - L x, written to every copy; 2:
// Gauss-Seidel value (f - off) / diag, written to every copy for t <
// n_direct, else into tmp[t - n_direct].
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_iface(
    const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ f,
    const int* __restrict__ off, const int4* __restrict__ cp, const int* __restrict__ rc_base,
    const double* __restrict__ sten, int n_rc, const int* __restrict__ list, int n, int N,
    int64_t B, double* __restrict__ tmp, int n_direct) {
    constexpr int LPN = IFACE_LANES;
    const int t = blockIdx.x * (256 / LPN) + (int)(threadIdx.x / LPN);
    const int lane = (int)(threadIdx.x % LPN);
    if (t >= n) return;  // the node's whole lane group
    const int node = list[t];
    const int c0 = off[node], c1 = off[node + 1];
    const int rb = rc_base[node] - c0;
    double dg = 0.0, of = 0.0;
    for (int c = c0 + lane; c < c1; c += LPN) {
        const int4 q = cp[c];
        const double* sw = sten + rb + c;
        const T* xm = x + (size_t)q.x * B;
        int o[NW];
        nbr_index((int)bidx(N, q.y, q.z, q.w), N + 1 - q.w, q.z, o);
        dg += sw[0];
#pragma unroll
        for (int w = 1; w < NW; w++)
            if (inside(N, q.y + dir_i(w), q.z + dir_j(w), q.w + dir_k(w)))
                of += sw[(size_t)w * n_rc] * (double)xm[o[w]];
    }
#pragma unroll
    for (int m = LPN / 2; m > 0; m >>= 1) {
        dg += __shfl_xor(dg, m, LPN);
        of += __shfl_xor(of, m, LPN);
    }
    const int4 q0 = cp[c0];
    const size_t s0 = (size_t)q0.x * B + bidx(N, q0.y, q0.z, q0.w);
    if (MODE == 2) {
        const double g = ((double)f[s0] - of) / dg;
        if (t >= n_direct) {
            if (lane == 0) tmp[t - n_direct] = g;
            return;
        }
        for (int c = c0 + lane; c < c1; c += LPN) {
            const int4 q = cp[c];
            y[(size_t)q.x * B + bidx(N, q.y, q.z, q.w)] = (T)g;
        }
        return;
    }
    double v = dg * (double)x[s0] + of;
    if (MODE == 1) v = (double)f[s0] - v;
    for (int c = c0 + lane; c < c1; c += LPN) {
        const int4 q = cp[c];
        y[(size_t)q.x * B + bidx(N, q.y, q.z, q.w)] = (T)v;
    }
}

// element-wise partial stencils of listed copies, stored as [15][n]
__global__ __launch_bounds__(128) void k_copy_stencils(const int4* __restrict__ cp, int n,
                                                       const MacroGeom* __restrict__ geom, int N,
                                                       double* __restrict__ sten) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int4 c = cp[t];
    double s[NW];
    ifem_partial_stencil(geom[c.x], N, c.y, c.z, c.w, s);
#pragma unroll
    for (int w = 0; w < NW; w++) sten[(size_t)w * n + t] = s[w];
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_slots(T* __restrict__ y,
                                                    const int64_t* __restrict__ slots, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[slots[t]] = (T)0;
}

// Same modes as k_iface; list (optional) selects positions; FQ > 0 takes
// the face fits of that degree instead of the stored rows.
template <typename T, int MODE, int FQ>
__global__ __launch_bounds__(256) void k_face2(
    const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ f,
    const int4* __restrict__ cp, const T* __restrict__ sten,
    const double* __restrict__ fcoef, int n2, const int* __restrict__ list, int n, int N,
    int64_t B, double* __restrict__ tmp, int n_direct) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    face2_node<T, MODE, FQ>(x, y, f, cp, sten, fcoef, n2, list, t, N, B, tmp, n_direct);
}

// Least-squares fit of the face rows of one interior face per workgroup: the
// exact combined rows at the sampling lattice (the face nodes whose
// barycentric weights are all multiples of st = N / Ns, Ns = 2^(m+2)) are
// staged in LDS in chunks; each thread accumulates entries of the normal
// equations (Gram matrix of the face basis, and its products with the 15
// entries); one thread then solves them by Cholesky.  Sample s runs over the
// Ns lattice by b' = 1 .. Ns-2, a' = 1 .. Ns-1-b' in the face frame, where
// the node (a, b) = (a' st, b' st) sits at (b-1)(N-1) - (b-1) b / 2 + a-1 in
// the face's range.
template <int FQ>
__global__ __launch_bounds__(256) void k_face_fit(const int4* __restrict__ cp,
                                                  const double* __restrict__ sten, int n2,
                                                  const int* __restrict__ foff, int N, int Ns,
                                                  double* __restrict__ fcoef) {
    constexpr int M2 = FaceBasis<FQ>::M2;
    constexpr int NG = M2 * (M2 + 1) / 2, NE = NG + M2 * NW;
    constexpr int CH = 128, PER = (NE + 255) / 256;
    __shared__ double sphi[CH][M2];
    __shared__ double sw[CH][NW];
    __shared__ double sys[NE];
    __shared__ double R[M2][M2], X[M2][NW];
    const int tid = (int)threadIdx.x;
    const int off = foff[blockIdx.x];
    const int st = N / Ns, ns = (Ns - 1) * (Ns - 2) / 2;
    // entry e < NG: Gram (r, c), r <= c; else right-hand side (r, w)
    int er[PER], ec[PER];
#pragma unroll
    for (int p = 0; p < PER; p++) {
        const int e = tid + p * 256;
        er[p] = -1;
        ec[p] = 0;
        if (e < NG) {
            int r = 0, rem = e;
            while (rem >= M2 - r) {
                rem -= M2 - r;
                r++;
            }
            er[p] = r;
            ec[p] = r + rem;
        } else if (e < NE) {
            er[p] = (e - NG) / NW;
            ec[p] = M2 + (e - NG) % NW;
        }
    }
    // Pass 0 forms the normal equations and solves them; pass 1 forms A^T of
    // the FP64 residual b - A x of that solution and adds the correction
    // (one step of iterative refinement: the squared condition number of the
    // normal equations no longer limits the accuracy of x).
    for (int pass = 0; pass < 2; pass++) {
        double acc[PER];
#pragma unroll
        for (int p = 0; p < PER; p++) acc[p] = 0.0;
        for (int c0 = 0; c0 < ns; c0 += CH) {
            const int sidx = c0 + tid;
            if (tid < CH && sidx < ns) {
                int bq = 1, r = sidx;
                while (r >= Ns - 1 - bq) {
                    r -= Ns - 1 - bq;
                    bq++;
                }
                const int a = (r + 1) * st, b = bq * st;
                const int q = off + (b - 1) * (N - 1) - (b - 1) * b / 2 + a - 1;
                const int4 ca = cp[q];
                const int fa = face_type(N, ca.y, ca.z, ca.w);
                const double invN = 1.0 / (double)N;
                const double u = (double)(fa == 0 ? ca.z : ca.y) * invN - 1.0 / 3.0;
                const double v = (double)(fa <= 1 ? ca.w : ca.z) * invN - 1.0 / 3.0;
                double phi[M2];
                face_phi<FQ>(u, v, phi);
#pragma unroll
                for (int c = 0; c < M2; c++) sphi[tid][c] = phi[c];
                for (int e = 0; e < NW; e++) {
                    double bv = sten[(size_t)e * n2 + q];
                    if (pass == 1)
                        for (int c = 0; c < M2; c++) bv -= phi[c] * X[c][e];
                    sw[tid][e] = bv;
                }
            }
            __syncthreads();
            const int nc = min(CH, ns - c0);
#pragma unroll
            for (int p = 0; p < PER; p++) {
                if (er[p] < 0 || (pass == 1 && ec[p] < M2)) continue;
                double a = acc[p];
                for (int k = 0; k < nc; k++)
                    a += sphi[k][er[p]] * (ec[p] < M2 ? sphi[k][ec[p]] : sw[k][ec[p] - M2]);
                acc[p] = a;
            }
            __syncthreads();
        }
#pragma unroll
        for (int p = 0; p < PER; p++)
            if (er[p] >= 0) sys[tid + p * 256] = acc[p];
        __syncthreads();
        if (tid == 0) {
            if (pass == 0) {
                // Gram G (upper triangle, row-packed) -> Cholesky G = R^T R
                for (int r = 0, e = 0; r < M2; r++)
                    for (int c = r; c < M2; c++, e++) R[r][c] = sys[e];
                for (int r = 0; r < M2; r++) {
                    double d = R[r][r];
                    for (int k = 0; k < r; k++) d -= R[k][r] * R[k][r];
                    d = sqrt(d);
                    R[r][r] = d;
                    for (int c = r + 1; c < M2; c++) {
                        double v = R[r][c];
                        for (int k = 0; k < r; k++) v -= R[k][r] * R[k][c];
                        R[r][c] = v / d;
                    }
                }
            }
            // R^T z = rhs, then R dx = z, for the 15 entries; x (+)= dx
            for (int w = 0; w < NW; w++) {
                double z[M2];
                for (int r = 0; r < M2; r++) {
                    double v = sys[NG + r * NW + w];
                    for (int k = 0; k < r; k++) v -= R[k][r] * z[k];
                    z[r] = v / R[r][r];
                }
                for (int r = M2 - 1; r >= 0; r--) {
                    double v = z[r];
                    for (int k = r + 1; k < M2; k++) v -= R[r][k] * z[k];
                    z[r] = v / R[r][r];
                }
                for (int r = 0; r < M2; r++) X[r][w] = pass == 0 ? z[r] : X[r][w] + z[r];
            }
        }
        __syncthreads();
    }
    if (tid != 0) return;
    const int4 c0 = cp[off];
    double* out = fcoef + ((size_t)c0.x * 4 + face_type(N, c0.y, c0.z, c0.w)) * (NW * M2);
    for (int w = 0; w < NW; w++)
        for (int c = 0; c < M2; c++) out[w * M2 + c] = X[c][w];
}

void launch_face_fit(const Level& L, const double* f2sten, int q, int jsamp, int nt, double* fcoef,
                     hipStream_t s) {
    const int N = L.N;
    int l = 0;
    while ((4 << l) < N) l++;
    const int m = std::min(l, std::max(1, jsamp));
    const int Ns = 4 << m;
    TS_REQUIRE((Ns - 1) * (Ns - 2) / 2 >= (q + 1) * (q + 2) / 2, TS_EINVAL,
               "face sampling set smaller than the polynomial space");
    TS_HIP(hipMemsetAsync(fcoef, 0, (size_t)nt * 4 * NW * ((q + 1) * (q + 2) / 2) * sizeof(double), s));
    if (L.n_f2_faces == 0) return;
    const unsigned g = (unsigned)L.n_f2_faces;
#define TS_FF(Q) k_face_fit<Q><<<g, 256, 0, s>>>(L.f2_cp.p, f2sten, L.n_f2, L.f2_face_off.p, N, Ns, fcoef)
    switch (q) {
        case 1: TS_FF(1); break;
        case 2: TS_FF(2); break;
        case 3: TS_FF(3); break;
        case 4: TS_FF(4); break;
        default: throw Error{TS_EINVAL, "unsupported surrogate degree"};
    }
#undef TS_FF
    TS_HIP(hipGetLastError());
}

// Combined face stencils: the element-wise partial stencils of both copies,
// with each in-face direction of A matched to the direction of B that reaches
// the same global node (through the barycentric coordinates over the shared
// vertices).
__global__ __launch_bounds__(128) void k_face2_stencils(const int4* __restrict__ cp, int n2,
                                                        const MacroGeom* __restrict__ geom,
                                                        const MacroTopo* __restrict__ topo, int N,
                                                        double* __restrict__ sten) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n2) return;
    const int4 ca = cp[q], cb = cp[(size_t)n2 + q];
    double sa[NW], sb[NW];
    ifem_partial_stencil(geom[ca.x], N, ca.y, ca.z, ca.w, sa);
    ifem_partial_stencil(geom[cb.x], N, cb.y, cb.z, cb.w, sb);
    const int fa = face_type(N, ca.y, ca.z, ca.w), fb = face_type(N, cb.y, cb.z, cb.w);
    const MacroTopo& TA = topo[ca.x];
    const MacroTopo& TB = topo[cb.x];
    for (int e = 0; e < 11; e++) {
        const int w = kFaceDirs.a[fa][e];
        double v = sa[w];
        if (face_side(fa, w) == 0) {
            const int i = ca.y + kDI[w], j = ca.z + kDJ[w], k = ca.w + kDK[w];
            const int mu[4] = {N - i - j - k, i, j, k};
            int mb[4] = {0, 0, 0, 0};
            for (int b = 0; b < 4; b++)
                for (int a = 0; a < 4; a++)
                    if (TB.vg[b] == TA.vg[a]) mb[b] = mu[a];
            const int wb = dir_index(mb[1] - cb.y, mb[2] - cb.z, mb[3] - cb.w);
            if (wb >= 0) v += sb[wb];
        }
        sten[(size_t)e * n2 + q] = v;
    }
    for (int e = 0; e < 4; e++) sten[(size_t)(11 + e) * n2 + q] = sb[kFaceDirs.b[fb][e]];
}
// Stored stencils of a level's interface nodes (built on first use, and
// again after the vertex coordinates change): the combined row of every face
// fast-path node ([15][n_f2]) and the partial stencil of every copy of the
// other free lower-primitive nodes ([15][n_rc]).
const double* face_stencils(Mesh& M, int lam, hipStream_t s) {
    const Level& L = M.level(lam);
    LevelGeo& G = M.level_geo(lam);
    if (G.sten_gen == M.geo_gen) return G.f2_sten.p;
    if (L.n_f2) {
        if (!G.f2_sten.p) G.f2_sten.alloc((size_t)NW * L.n_f2);
        if (!G.f2g_sten.p) G.f2g_sten.alloc((size_t)NW * L.n_f2);
        k_face2_stencils<<<(L.n_f2 + 127) / 128, 128, 0, s>>>(L.f2_cp.p, L.n_f2, M.d_geom.p,
                                                              M.d_topo.p, L.N, G.f2_sten.p);
        k_face2_stencils<<<(L.n_f2 + 127) / 128, 128, 0, s>>>(L.f2g_cp.p, L.n_f2, M.d_geom.p,
                                                              M.d_topo.p, L.N, G.f2g_sten.p);
        TS_HIP(hipGetLastError());
    }
    if (L.n_rc) {
        if (!G.rest_sten.p) G.rest_sten.alloc((size_t)NW * L.n_rc);
        k_copy_stencils<<<(L.n_rc + 127) / 128, 128, 0, s>>>(L.rc_cp.p, L.n_rc, M.d_geom.p, L.N,
                                                             G.rest_sten.p);
        TS_HIP(hipGetLastError());
    }
    G.sten_gen = M.geo_gen;
    return G.f2_sten.p;
}

const float* face_stencils32(Mesh& M, int lam, hipStream_t s) {
    const Level& L = M.level(lam);
    LevelGeo& G = M.level_geo(lam);
    face_stencils(M, lam, s);
    if (G.sten32_gen == M.geo_gen) return G.f2_sten32.p;
    if (L.n_f2) {
        const int64_t n = (int64_t)NW * L.n_f2;
        if (!G.f2_sten32.p) G.f2_sten32.alloc(n);
        if (!G.f2g_sten32.p) G.f2g_sten32.alloc(n);
        launch_cast(G.f2_sten.p, TS_F64, G.f2_sten32.p, TS_F32, n, s);
        launch_cast(G.f2g_sten.p, TS_F64, G.f2g_sten32.p, TS_F32, n, s);
    }
    G.sten32_gen = M.geo_gen;
    return G.f2_sten32.p;
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
    const int q = list ? list[t] : t;
    const T v = (T)tmp[t];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        const int4 c = cp[(size_t)r * n2 + q];
        u[(size_t)c.x * B + bidx(N, c.y, c.z, c.w)] = v;
    }
}

// Launchers --------------------------------------------------------------------

#define TS_DECL(Q, K)                                                                     \
    void launch_surr_q##Q##_k##K(const Level& L, int nt, const LevelOp& lo, int dtype,    \
                                 int center, int mode, const void* x, void* y,            \
                                 const void* f, int colour, hipStream_t s,                \
                                 const void* f2sten, const double* f2coef);
TS_DECL(0, 2) TS_DECL(0, 4) TS_DECL(0, 8)
TS_DECL(1, 2) TS_DECL(1, 4) TS_DECL(1, 8)
TS_DECL(2, 2) TS_DECL(2, 4) TS_DECL(2, 8)
TS_DECL(3, 2) TS_DECL(3, 4) TS_DECL(3, 8)
TS_DECL(4, 2) TS_DECL(4, 4) TS_DECL(4, 8)
#undef TS_DECL

void launch_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                   const void* f, int colour, hipStream_t s, bool fuse_face) {
    Mesh& M = op->mesh->m;
    const Level& L = M.level(lam);
    const LevelOp& lo = *op->lv.at(lam);
    const int nt = (int)M.nt, q = op->p.q, c = op->p.center;
    if (lo.n_ifem)  // selective surrogate: these macros keep IFEM rows
        launch_ifem_volume(op, lam, dtype == TS_F16W ? TS_F32 : dtype, mode, x, y, f, colour, s,
                           lo.ifem_list.p, lo.n_ifem);
    if (lo.n_sur == 0) return;
    const int kpt = L.lds_kpt <= 2 ? 2 : L.lds_kpt <= 4 ? 4 : 8;
    TS_REQUIRE(L.lds_kpt <= 8, TS_EINVAL, "level too large for the surrogate volume kernel");
    // face rows fused into the launch (apply / residual); built on first use
    const void* f2 = nullptr;
    if (fuse_face && mode != 2 && L.n_f2)
        f2 = dtype == TS_F64 ? (const void*)face_stencils(M, lam, s)
                             : (const void*)face_stencils32(M, lam, s);
    const double* fc = f2 && lo.face_fit ? lo.fcoef.p : nullptr;
#define TS_GO(Q, K) launch_surr_q##Q##_k##K(L, nt, lo, dtype, c, mode, x, y, f, colour, s, f2, fc)
    switch (q * 16 + kpt) {
        case 2: TS_GO(0, 2); break;
        case 4: TS_GO(0, 4); break;
        case 8: TS_GO(0, 8); break;
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

void launch_ifem_k2(const Level& L, const double* xyz, int nt, const int* mlist, int dtype,
                    int mode, const void* x, void* y, const void* f, int colour, hipStream_t s);
void launch_ifem_k4(const Level& L, const double* xyz, int nt, const int* mlist, int dtype,
                    int mode, const void* x, void* y, const void* f, int colour, hipStream_t s);

// blended coordinates of every slot of a level, computed on first use
static const double* level_coords(Mesh& M, int lam, hipStream_t s) {
    const Level& L = M.level(lam);
    LevelGeo& G = M.level_geo(lam);
    if (G.xyz_gen != M.geo_gen) {
        if (!G.xyz.p) G.xyz.alloc((size_t)3 * L.len);
        launch_coords(M, lam, G.xyz.p, s);
        G.xyz_gen = M.geo_gen;
    }
    return G.xyz.p;
}

// builds (once per geometry) what the operator's rows read on level lam: the
// stored interface stencils and, if element-wise volume rows are needed
// there, the stored coordinates
void warm_level(const ts_op* op, int lam, bool ifem_rows, hipStream_t s) {
    Mesh& M = op->mesh->m;
    face_stencils(M, lam, s);
    if (ifem_rows && M.level(lam).lds_kpt <= 4) level_coords(M, lam, s);
}

void launch_ifem_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                        const void* f, int colour, hipStream_t s, const int* mlist, int n_list) {
    Mesh& M = op->mesh->m;
    const Level& L = M.level(lam);
    const int nt = n_list >= 0 ? n_list : (int)M.nt;
    if (nt == 0 || L.n_lds_tiles == 0) return;
    TS_REQUIRE(L.lds_kpt <= 4, TS_EINVAL,
               "element-wise (IFEM) volume rows are supported up to level 8");
    const double* xyz = level_coords(M, lam, s);
    if (L.lds_kpt <= 2)
        launch_ifem_k2(L, xyz, nt, mlist, dtype, mode, x, y, f, colour, s);
    else
        launch_ifem_k4(L, xyz, nt, mlist, dtype, mode, x, y, f, colour, s);
    TS_HIP(hipGetLastError());
}

// Lower-primitive rows: phase < 0 handles every node (apply / residual);
// phase >= 0 computes the Gauss-Seidel values of that phase into tmp (face
// fast path first, then the general nodes after it in tmp).
void launch_iface(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                  const void* f, int phase, double* tmp, hipStream_t s, bool skip_face,
                  bool exact) {
    Mesh& M = op->mesh->m;
    const Level& L = M.level(lam);
    face_stencils(M, lam, s);
    const LevelOp* lo = op->lv.count(lam) ? op->lv.at(lam).get() : nullptr;
    const int fq = !exact && lo && lo->face_fit ? op->p.q : 0;
    const double* fc = fq ? lo->fcoef.p : nullptr;
    // apply / residual: canonical order; Gauss-Seidel phase: its contiguous
    // range of the phase-grouped copy
    const int go = phase >= 0 ? L.f2g_off[phase] : 0;
    const int4* cp2 = phase >= 0 ? L.f2g_cp.p + go : L.f2_cp.p;
    const LevelGeo& G = M.level_geo(lam);
    const double* sten = phase >= 0 ? G.f2g_sten.p + go : G.f2_sten.p;
    const float* sten32 = nullptr;
    if (dtype != TS_F64 && L.n_f2) {
        face_stencils32(M, lam, s);
        sten32 = phase >= 0 ? G.f2g_sten32.p + go : G.f2_sten32.p;
    }
    const int n2 = skip_face ? 0 : phase >= 0 ? L.n_f2_phase[phase] : L.n_f2;
    const int* lr = phase >= 0 ? L.rest_phase[phase].p : L.rest.p;
    const int nr = phase >= 0 ? L.n_rest_phase[phase] : L.n_rest;
    // Gauss-Seidel: the uncoupled nodes of the phase are written in place,
    // the coupled ones go to tmp (face nodes first, then the general ones)
    const int d2 = phase >= 0 ? L.n_f2_direct[phase] : 0;
    const int dr = phase >= 0 ? L.n_rest_direct[phase] : 0;
    double* tmp_r = tmp ? tmp + (n2 - d2) : nullptr;
#define TS_F2Q(T_, M_, Q_)                                                                    \
    k_face2<T_, M_, Q_><<<(n2 + 255) / 256, 256, 0, s>>>((const T_*)x, (T_*)y, (const T_*)f,   \
                                                         cp2, sizeof(T_) == 8 ? (const T_*)sten   \
                                                         : (const T_*)sten32, fc, L.n_f2,     \
                                                         nullptr, n2,                         \
                                                         L.N, L.B, tmp, d2)
#define TS_F2(T_, M_)                                                                         \
    do {                                                                                      \
        switch (fq) {                                                                         \
            case 0: TS_F2Q(T_, M_, 0); break;                                                 \
            case 1: TS_F2Q(T_, M_, 1); break;                                                 \
            case 2: TS_F2Q(T_, M_, 2); break;                                                 \
            case 3: TS_F2Q(T_, M_, 3); break;                                                 \
            default: TS_F2Q(T_, M_, 4); break;                                                \
        }                                                                                     \
    } while (0)
#define TS_IF(T_, M_)                                                                         \
    k_iface<T_, M_><<<(nr + 256 / IFACE_LANES - 1) / (256 / IFACE_LANES), 256, 0, s>>>(        \
                                                     (const T_*)x, (T_*)y, (const T_*)f,      \
                                                     L.if_off.p, L.if_copy.p, L.rc_base.p,    \
                                                     G.rest_sten.p, L.n_rc, lr, nr, L.N, L.B, \
                                                     tmp_r, dr)
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
    if (phase < 0 && L.n_dir_slots) {  // Dirichlet rows are zero
        const unsigned g = (unsigned)((L.n_dir_slots + 255) / 256);
        if (dtype == TS_F64)
            k_zero_slots<double><<<g, 256, 0, s>>>((double*)y, L.dir_slots.p, L.n_dir_slots);
        else
            k_zero_slots<float><<<g, 256, 0, s>>>((float*)y, L.dir_slots.p, L.n_dir_slots);
    }
#undef TS_F2
#undef TS_F2Q
#undef TS_IF
    TS_HIP(hipGetLastError());
}

// the coupled nodes of a phase (after the uncoupled ones in each list) take
// their values from tmp once every node of the phase is computed
void launch_iface_scatter(const ts_op* op, int lam, int dtype, int phase, const double* tmp,
                          void* u, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const int d2 = L.n_f2_direct[phase], dr = L.n_rest_direct[phase];
    const int n2 = L.n_f2_phase[phase] - d2, nr = L.n_rest_phase[phase] - dr;
    const int4* cp2 = L.f2g_cp.p + L.f2g_off[phase] + d2;
    const int* lr = L.rest_phase[phase].p + dr;
    if (n2) {
        if (dtype == TS_F64)
            k_face2_scatter<double><<<(n2 + 255) / 256, 256, 0, s>>>((double*)u, tmp, cp2, L.n_f2, nullptr, n2, L.N, L.B);
        else
            k_face2_scatter<float><<<(n2 + 255) / 256, 256, 0, s>>>((float*)u, tmp, cp2, L.n_f2, nullptr, n2, L.N, L.B);
    }
    if (nr) {
        if (dtype == TS_F64)
            k_iface_scatter<double><<<(nr + 255) / 256, 256, 0, s>>>((double*)u, tmp + n2, L.if_off.p, L.if_copy.p, lr, nr, L.N, L.B);
        else
            k_iface_scatter<float><<<(nr + 255) / 256, 256, 0, s>>>((float*)u, tmp + n2, L.if_off.p, L.if_copy.p, lr, nr, L.N, L.B);
    }
    TS_HIP(hipGetLastError());
}

}  // namespace ts
