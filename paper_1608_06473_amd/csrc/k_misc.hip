// Kernels around the stencils: grid transfer (linear interpolation in
// index space and its transpose), deterministic norms, element-wise vector
// work, canonical <-> block conversion, node coordinates, load vectors with
// the consistent P1 mass matrix, the surrogate setup (exact stencils at the
// sampling points and the FP64 normal equations, Sec. 3.1-3.2) and the
// coarsest-level dense inverse (Gauss-Jordan) with its solve.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "ts_internal.h"
#include "ts_face.h"

namespace ts {

// ---------------------------------------------------------------- helpers

// slot (position r in plane k) -> (i, j): row j has A - j slots, A = N+1-k.
// The FP32 estimate is exact enough (operands below 2^24) for the integer
// fix-up to need at most one step.
__device__ __forceinline__ void plane_pos_to_ij(int r, int A, int& i, int& j) {
    const float a = 2.0f * (float)A + 1.0f;
    int J = (int)((a - sqrtf(a * a - 8.0f * (float)r)) * 0.5f);
    if (J < 0) J = 0;
    while (J > 0 && J * (2 * A - J + 1) / 2 > r) J--;
    while ((J + 1) * (2 * A - J) / 2 <= r) J++;
    j = J;
    i = r - J * (2 * A - J + 1) / 2;
}

// 32-bit block indices for the slot and transfer kernels: levels go up to 9
// (N <= 512), where every index of a block stays below 2^25 and
// n (n + 1) (n + 2) below 2^28, so no 64-bit products or divisions are needed
__device__ __forceinline__ unsigned tet32(unsigned n) { return n * (n + 1u) * (n + 2u) / 6u; }
__device__ __forceinline__ int plane_off32(int N, int k) {
    return (int)(tet32((unsigned)N + 1u) - tet32((unsigned)(N + 1 - k)));
}
__device__ __forceinline__ int bidx32(int N, int i, int j, int k) {
    const unsigned a = (unsigned)(N + 1 - k), uj = (unsigned)j;
    return plane_off32(N, k) + (int)(uj * a - (uj * (uj - 1u)) / 2u) + i;
}

// all-slot kernels: grid = n_macros x n_slot_tiles (tiles of plane k)
#define TS_SLOT_DECODE(L_ARGS)                                                       \
    const int macro = blockIdx.y;                                                    \
    const int2 td = slot_tiles[blockIdx.x];                                          \
    const int k = td.x;                                                              \
    const int A = N + 1 - k;                                                         \
    const int r = td.y + (int)threadIdx.x;                                           \
    if (r >= A * (A + 1) / 2) return;                                                \
    int i, j;                                                                        \
    plane_pos_to_ij(r, A, i, j);                                                     \
    const size_t slot = (size_t)macro * B + (size_t)(plane_off32(N, k) + r);

// ---------------------------------------------------------------- transfers

// coarse interior nodes: r_c = r_f(2c) + 1/2 sum_w r_f(2c + w) (R = P^T;
// every fine midpoint around an interior coarse node is interior to the
// macro)
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_volume(
    const T* __restrict__ rf, T* __restrict__ rc, const int2* __restrict__ slot_tiles, int Nc,
    int64_t Bf, int64_t Bc) {
    const int N = Nc;
    const int64_t B = Bc;
    TS_SLOT_DECODE();
    if (i < 1 || j < 1 || k < 1 || i + j + k > Nc - 1) return;
    const int Nf = 2 * Nc;
    const T* fm = rf + (size_t)macro * Bf;
    T s = fm[bidx32(Nf, 2 * i, 2 * j, 2 * k)];
    T h = (T)0;
#pragma unroll
    for (int w = 1; w < NW; w++)
        h += fm[bidx32(Nf, 2 * i + dir_i(w), 2 * j + dir_j(w), 2 * k + dir_k(w))];
    rc[slot] = s + (T)0.5 * h;
}

// number of macros containing the primitive of fine node p in macro t
__device__ __forceinline__ int node_mult(const MacroTopo& T, int N, int i, int j, int k) {
    const int mu[4] = {N - i - j - k, i, j, k};
    int z[4], nz = 0;
    for (int a = 0; a < 4; a++)
        if (mu[a] == 0) z[nz++] = a;
    if (nz == 0) return 1;
    if (nz == 1) return T.fmult[z[0]];
    // edge: the two local vertices that are not zero
    int a = -1, b = -1;
    for (int q = 0; q < 4; q++)
        if (mu[q] != 0) {
            if (a < 0) a = q; else b = q;
        }
    const int EL[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int e = 0; e < 6; e++)
        if (EL[e][0] == a && EL[e][1] == b) return T.emult[e];
    return 1;
}

// coarse lower-primitive nodes: sum over the node's copies of the fine
// midpoints in that macro, each divided by the number of macros that hold it
// sum over the 14 neighbours w of coarse copy q of the fine values at the
// midpoints 2q + w, each shared by the fine node's copies (the restriction
// R = P^T accumulated once over all copies)
template <typename T>
__device__ __forceinline__ double restrict_copy(const T* __restrict__ rf, int4 q,
                                                const MacroTopo& TP, int Nc, int64_t Bf) {
    const int Nf = 2 * Nc;
    const T* fm = rf + (size_t)q.x * Bf;
    double v = 0.0;
#pragma unroll
    for (int w = 1; w < NW; w++) {
        if (!inside(Nc, q.y + dir_i(w), q.z + dir_j(w), q.w + dir_k(w))) continue;
        const int a = 2 * q.y + dir_i(w), b = 2 * q.z + dir_j(w), cc = 2 * q.w + dir_k(w);
        v += 0.5 * (double)fm[bidx32(Nf, a, b, cc)] / (double)node_mult(TP, Nf, a, b, cc);
    }
    return v;
}

// coarse face nodes with two copies: one thread per node
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_face2(
    const T* __restrict__ rf, T* __restrict__ rc, const int4* __restrict__ cp, int n2,
    const MacroTopo* __restrict__ topo, int Nc, int64_t Bf, int64_t Bc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2) return;
    const int4 qa = cp[t], qb = cp[(size_t)n2 + t];
    double v = (double)rf[(size_t)qa.x * Bf + bidx32(2 * Nc, 2 * qa.y, 2 * qa.z, 2 * qa.w)];
    v += restrict_copy(rf, qa, topo[qa.x], Nc, Bf);
    v += restrict_copy(rf, qb, topo[qb.x], Nc, Bf);
    rc[(size_t)qa.x * Bc + bidx32(Nc, qa.y, qa.z, qa.w)] = (T)v;
    rc[(size_t)qb.x * Bc + bidx32(Nc, qb.y, qb.z, qb.w)] = (T)v;
}

// other free coarse interface nodes (edges, vertices): eight lanes per node
// (32 nodes per workgroup), copies across the lanes, fixed-order reduction
constexpr int REST_LANES = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_restrict_rest(
    const T* __restrict__ rf, T* __restrict__ rc, const int* __restrict__ off,
    const int4* __restrict__ cp, const int* __restrict__ list, int n,
    const MacroTopo* __restrict__ topo, int Nc, int64_t Bf, int64_t Bc) {
    constexpr int LPN = REST_LANES;
    const int t = blockIdx.x * (256 / LPN) + (int)(threadIdx.x / LPN);
    const int lane = (int)(threadIdx.x % LPN);
    if (t >= n) return;  // the node's whole lane group
    const int node = list[t];
    const int c0 = off[node], c1 = off[node + 1];
    double v = 0.0;
    for (int c = c0 + lane; c < c1; c += LPN) v += restrict_copy(rf, cp[c], topo[cp[c].x], Nc, Bf);
#pragma unroll
    for (int m = LPN / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, LPN);
    const int4 q0 = cp[c0];
    v += (double)rf[(size_t)q0.x * Bf + bidx32(2 * Nc, 2 * q0.y, 2 * q0.z, 2 * q0.w)];
    for (int c = c0 + lane; c < c1; c += LPN) {
        const int4 q = cp[c];
        rc[(size_t)q.x * Bc + bidx32(Nc, q.y, q.z, q.w)] = (T)v;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_slots_misc(T* __restrict__ y,
                                                         const int64_t* __restrict__ slots,
                                                         int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[slots[t]] = (T)0;
}

// u_f += P u_c over every fine slot: even nodes copy the coarse node, odd
// nodes average the two ends of the coarse edge they bisect
template <typename T>
__global__ __launch_bounds__(256) void k_prolongate_add(
    const T* __restrict__ uc, T* __restrict__ uf, const int2* __restrict__ slot_tiles, int N,
    int64_t B, int64_t Bc) {
    TS_SLOT_DECODE();
    const int Nc = N / 2;
    const T* cm = uc + (size_t)macro * Bc;
    const int pi = i & 1, pj = j & 1, pk = k & 1;
    T v;
    if (!(pi | pj | pk)) {
        v = cm[bidx32(Nc, i / 2, j / 2, k / 2)];
    } else {
        // the lattice edge direction with this parity pattern
        int di, dj, dk;
        if (pi && !pj && !pk) { di = 1; dj = 0; dk = 0; }
        else if (!pi && pj && !pk) { di = 0; dj = 1; dk = 0; }
        else if (!pi && !pj && pk) { di = 0; dj = 0; dk = 1; }
        else if (pi && pj && !pk) { di = 1; dj = -1; dk = 0; }
        else if (pi && !pj && pk) { di = -1; dj = 0; dk = 1; }
        else if (!pi && pj && pk) { di = 0; dj = -1; dk = 1; }
        else { di = 1; dj = -1; dk = 1; }
        const T a = cm[bidx32(Nc, (i - di) / 2, (j - dj) / 2, (k - dk) / 2)];
        const T b = cm[bidx32(Nc, (i + di) / 2, (j + dj) / 2, (k + dk) / 2)];
        v = (T)0.5 * (a + b);
    }
    uf[slot] += v;
}

void launch_restrict(const Mesh& M, int lam_f, int dtype, const void* rf, void* rc,
                     hipStream_t s) {
    Mesh& MM = const_cast<Mesh&>(M);
    const Level& Lf = MM.level(lam_f);
    const Level& Lc = MM.level(lam_f - 1);
    const dim3 g1(Lc.n_slot_tiles, (unsigned)M.nt), b1(256);
    const unsigned g2 = (unsigned)((Lc.n_f2 + 255) / 256), g3 = (unsigned)((Lc.n_rest + 256 / REST_LANES - 1) / (256 / REST_LANES));
    const unsigned g4 = (unsigned)((Lc.n_dir_slots + 255) / 256);
#define TS_R(T_)                                                                                  \
    k_restrict_volume<T_><<<g1, b1, 0, s>>>((const T_*)rf, (T_*)rc, Lc.slot_tiles.p, Lc.N, Lf.B,  \
                                            Lc.B);                                                \
    if (g2) k_restrict_face2<T_><<<g2, 256, 0, s>>>((const T_*)rf, (T_*)rc, Lc.f2_cp.p, Lc.n_f2,  \
                                                    M.d_topo.p, Lc.N, Lf.B, Lc.B);                \
    if (g3) k_restrict_rest<T_><<<g3, 256, 0, s>>>((const T_*)rf, (T_*)rc, Lc.if_off.p,           \
                                                   Lc.if_copy.p, Lc.rest.p, Lc.n_rest,            \
                                                   M.d_topo.p, Lc.N, Lf.B, Lc.B);                 \
    if (g4) k_zero_slots_misc<T_><<<g4, 256, 0, s>>>((T_*)rc, Lc.dir_slots.p, Lc.n_dir_slots)
    if (dtype == TS_F64) {
        TS_R(double);
    } else {
        TS_R(float);
    }
#undef TS_R
    TS_HIP(hipGetLastError());
}

void launch_prolongate_add(const Mesh& M, int lam_f, int dtype, const void* uc, void* uf,
                           hipStream_t s) {
    Mesh& MM = const_cast<Mesh&>(M);
    const Level& Lf = MM.level(lam_f);
    const Level& Lc = MM.level(lam_f - 1);
    const dim3 g(Lf.n_slot_tiles, (unsigned)M.nt), b(256);
    if (dtype == TS_F64)
        k_prolongate_add<double><<<g, b, 0, s>>>((const double*)uc, (double*)uf, Lf.slot_tiles.p, Lf.N, Lf.B, Lc.B);
    else
        k_prolongate_add<float><<<g, b, 0, s>>>((const float*)uc, (float*)uf, Lf.slot_tiles.p, Lf.N, Lf.B, Lc.B);
    TS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- vectors

template <typename T>
__global__ void k_fill(T* x, int64_t n, T v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        x[t] = v;
}
template <typename S, typename D>
__global__ void k_cast(const S* __restrict__ a, D* __restrict__ b, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        b[t] = (D)a[t];
}
template <typename S>
__global__ void k_axpy(double a, const S* __restrict__ x, double* __restrict__ y, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        y[t] += a * (double)x[t];
}

static dim3 ew_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

void launch_fill(void* x, int dtype, int64_t n, double v, hipStream_t s) {
    if (dtype == TS_F64)
        k_fill<double><<<ew_grid(n), 256, 0, s>>>((double*)x, n, v);
    else
        k_fill<float><<<ew_grid(n), 256, 0, s>>>((float*)x, n, (float)v);
    TS_HIP(hipGetLastError());
}
void launch_cast(const void* src, int dsrc, void* dst, int ddst, int64_t n, hipStream_t s) {
    const bool s64 = dsrc == TS_F64, d64 = ddst == TS_F64;
    if (s64 && !d64) k_cast<double, float><<<ew_grid(n), 256, 0, s>>>((const double*)src, (float*)dst, n);
    else if (!s64 && d64) k_cast<float, double><<<ew_grid(n), 256, 0, s>>>((const float*)src, (double*)dst, n);
    else if (s64) k_cast<double, double><<<ew_grid(n), 256, 0, s>>>((const double*)src, (double*)dst, n);
    else k_cast<float, float><<<ew_grid(n), 256, 0, s>>>((const float*)src, (float*)dst, n);
    TS_HIP(hipGetLastError());
}
void launch_axpy(double a, const void* x, int dx, double* y, int64_t n, hipStream_t s) {
    if (dx == TS_F64)
        k_axpy<double><<<ew_grid(n), 256, 0, s>>>(a, (const double*)x, y, n);
    else
        k_axpy<float><<<ew_grid(n), 256, 0, s>>>(a, (const float*)x, y, n);
    TS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- norms
// Deterministic: fixed per-block tree sums into partial[], then one block
// sums partial[] in a fixed order.

template <int NT = 256>
__device__ __forceinline__ double block_sum(double v) {
    // NT threads; the part above the largest power of two P <= NT is folded
    // onto the first NT - P entries first
    constexpr int P = NT >= 1024 ? 1024 : NT >= 512 ? 512 : NT >= 256 ? 256 : NT >= 128 ? 128 : 64;
    __shared__ double sh[NT];
    sh[threadIdx.x] = v;
    __syncthreads();
    if constexpr (NT > P) {
        if ((int)threadIdx.x < NT - P) sh[threadIdx.x] += sh[threadIdx.x + P];
        __syncthreads();
    }
    for (int st = P / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    return sh[0];
}

// one workgroup per (volume tile, macro): each lane sums the squares of its
// column's interior nodes in the tile's slab (the columns of the volume
// kernel, in its apply order)
template <typename T>
__global__ __launch_bounds__(VOL_THREADS) void k_norm_volume(const T* __restrict__ x,
                                                     const int4* __restrict__ tiles,
                                                     const unsigned* __restrict__ lanes, int N,
                                                     int64_t B, double* __restrict__ partial) {
    const int tile = blockIdx.x, macro = blockIdx.y;
    const int k0 = tiles[tile].x;
    const unsigned e = lanes[(size_t)tile * VOL_THREADS + threadIdx.x];
    double v = 0.0;
    if (e != 0xFFFFFFFFu) {
        const int i = (int)(e & 0xFFFFu), j = (int)(e >> 16);
        const int nlive = min(N - 1 - i - j, k0 + VOL_R - 1) - k0 + 1;
        const T* xm = x + (size_t)macro * B;
        int idx = (int)bidx(N, i, j, k0);
        for (int r = 0; r < nlive; r++) {
            const double a = (double)xm[idx];
            v += a * a;
            const int Ak = N + 1 - (k0 + r);
            idx += Ak * (Ak + 1) / 2 - j;
        }
    }
    const double s = block_sum<VOL_THREADS>(v);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_norm_iface(const T* __restrict__ x, const int* __restrict__ list,
                                                    int n, const int* __restrict__ off,
                                                    const int4* __restrict__ cp, int N, int64_t B,
                                                    double* __restrict__ partial) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (t < n) {
        const int4 q = cp[off[list[t]]];
        const double a = (double)x[(size_t)q.x * B + bidx(N, q.y, q.z, q.w)];
        v = a * a;
    }
    const double s = block_sum(v);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// tree reduction of partial sums in a fixed order: workgroup b sums
// p[b * 4096 .. b * 4096 + 4095] (sqrt of the total when `root` and a single
// workgroup)
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ p, int64_t n,
                                                      double* out, int root) {
    const int64_t b0 = (int64_t)blockIdx.x * 4096;
    double v = 0.0;
    for (int t = threadIdx.x; t < 4096; t += 256)
        if (b0 + t < n) v += p[b0 + t];
    const double s = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = root ? sqrt(s) : s;
}

// ---------------------------------------------------------------- norm
// without allocation
//
// The partial sums of the allocation-free norm live in a fixed device array
// of this file, one copy per GPU that loads the library (held until the
// process ends).  Host code never passes the array's name to a kernel (in
// host code it is only a stand-in for the symbol): the device address of each
// GPU's copy is looked up once, with that GPU current, and kept per device.
constexpr int64_t kNormScratch = (int64_t)1 << 20;  // doubles (8 MiB)
static __device__ __align__(256) double scratch[kNormScratch];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[64] = {};

static double* scratch_ptr(int dev) {
    TS_REQUIRE(dev >= 0 && dev < 64, TS_EINVAL, "device id out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        TS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        TS_REQUIRE(p != nullptr, TS_EHIP, "no device address for the norm scratch array");
        g_scratch_ptr[dev] = (double*)p;
    }
    return g_scratch_ptr[dev];
}

// the same kernels as ts_norm2 (so bitwise the same result), their partial
// sums in the fixed array; the norm goes to the device double *out
void norm2_noalloc(const Mesh& M, int lam, int dtype, const void* x, double* out,
                   hipStream_t s) {
    int dev = -1;
    TS_HIP(hipGetDevice(&dev));
    TS_REQUIRE(dev == M.device, TS_EINVAL, "the mesh's device must be the current device");
    TS_REQUIRE(M.levels.count(lam), TS_EINVAL,
               "level not built on this mesh (ts_layout builds it; this call allocates nothing)");
    const int64_t need = norm_partial_count(M, lam);
    TS_REQUIRE(need <= kNormScratch, TS_EINVAL,
               "the norm needs " + std::to_string(need) + " partial sums, more than the " +
                   std::to_string(kNormScratch) + " of the allocation-free variant");
    launch_norm2_free(M, lam, dtype, x, scratch_ptr(dev), out, s);
}

static int64_t volume_partials(const Mesh& M, int lam) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    return (int64_t)L.n_lds_tiles * M.nt;
}

int64_t norm_partial_count(const Mesh& M, int lam) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const int64_t n = volume_partials(M, lam) + (L.n_if_free + 255) / 256;
    // partials, then the sums of up to 4096 partials each, then their sums
    return n + (n + 4095) / 4096 + 2;
}

void launch_norm2_free(const Mesh& M, int lam, int dtype, const void* x, double* partial,
                       double* out, hipStream_t s) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const int64_t n1 = volume_partials(M, lam);
    const int n2 = (L.n_if_free + 255) / 256;
    if (n1) {
        const dim3 g1((unsigned)L.n_lds_tiles, (unsigned)M.nt);
        if (dtype == TS_F64)
            k_norm_volume<double><<<g1, VOL_THREADS, 0, s>>>((const double*)x, L.lds_tiles.p, L.ap_lanes.p, L.N, L.B, partial);
        else
            k_norm_volume<float><<<g1, VOL_THREADS, 0, s>>>((const float*)x, L.lds_tiles.p, L.ap_lanes.p, L.N, L.B, partial);
    }
    if (n2) {
        if (dtype == TS_F64)
            k_norm_iface<double><<<n2, 256, 0, s>>>((const double*)x, L.if_free.p, L.n_if_free, L.if_off.p, L.if_copy.p, L.N, L.B, partial + n1);
        else
            k_norm_iface<float><<<n2, 256, 0, s>>>((const float*)x, L.if_free.p, L.n_if_free, L.if_off.p, L.if_copy.p, L.N, L.B, partial + n1);
    }
    const int64_t n = n1 + n2;
    const int64_t m = (n + 4095) / 4096;
    double* mid = partial + n;
    // n <= 4096^2 for every supported level and mesh of up to a few
    // thousand macros, so two stages suffice
    TS_REQUIRE(m <= 4096, TS_EINVAL, "too many partial sums for the norm");
    k_sum_partials<<<(unsigned)m, 256, 0, s>>>(partial, n, mid, 0);
    k_sum_partials<<<1, 256, 0, s>>>(mid, m, out, 1);
    TS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- canonical

__device__ __forceinline__ int64_t canon_of(const MacroTopo& T, int64_t m, int N, int64_t nv,
                                            int64_t ne, int64_t nf, int i, int j, int k,
                                            int* dir) {
    const int mu[4] = {N - i - j - k, i, j, k};
    int nz = 0, zero_at = -1;
    for (int a = 0; a < 4; a++) {
        if (mu[a] != 0) nz++;
        else zero_at = a;
    }
    const int64_t F = (int64_t)(N - 1) * (N - 2) / 2;
    if (nz == 1) {
        for (int a = 0; a < 4; a++)
            if (mu[a] == N) {
                *dir = T.vdir[a];
                return T.vg[a];
            }
    }
    if (nz == 2) {
        for (int e = 0; e < 6; e++)
            if (mu[T.elo[e]] != 0 && mu[T.ehi[e]] != 0) {
                *dir = T.edir[e];
                return nv + T.e[e] * (N - 1) + (mu[T.ehi[e]] - 1);
            }
    }
    if (nz == 3) {
        const int o = zero_at;
        const int a = mu[T.fs[o][1]], b = mu[T.fs[o][2]];
        *dir = T.fdir[o];
        const int64_t fo = (int64_t)(b - 1) * (N - 1) - (int64_t)(b - 1) * b / 2 + (a - 1);
        return nv + ne * (N - 1) + T.f[o] * F + fo;
    }
    *dir = 0;
    const int64_t V = (int64_t)(N - 1) * (N - 2) * (N - 3) / 6;
    const int64_t vo = tet_n(N - 3) - tet_n(N - 2 - k) + (int64_t)(j - 1) * (N - 1 - k) -
                       (int64_t)(j - 1) * j / 2 + (i - 1);
    return nv + ne * (N - 1) + nf * F + m * V + vo;
}

__global__ __launch_bounds__(256) void k_canon_to_block(const double* __restrict__ c, double* __restrict__ b,
                                                        const MacroTopo* __restrict__ topo,
                                                        const int2* __restrict__ slot_tiles, int N,
                                                        int64_t B, int64_t nv, int64_t ne, int64_t nf) {
    TS_SLOT_DECODE();
    int dir;
    const int64_t id = canon_of(topo[macro], macro, N, nv, ne, nf, i, j, k, &dir);
    b[slot] = dir ? 0.0 : c[id];
}

__global__ __launch_bounds__(256) void k_block_to_canon(const double* __restrict__ b, double* __restrict__ c,
                                                        const MacroTopo* __restrict__ topo,
                                                        const int2* __restrict__ slot_tiles, int N,
                                                        int64_t B, int64_t nv, int64_t ne, int64_t nf,
                                                        const int* __restrict__ off,
                                                        const int4* __restrict__ cp) {
    TS_SLOT_DECODE();
    int dir;
    const int64_t id = canon_of(topo[macro], macro, N, nv, ne, nf, i, j, k, &dir);
    const bool interior = i >= 1 && j >= 1 && k >= 1 && i + j + k <= N - 1;
    if (interior) {
        c[id] = b[slot];
    } else {
        // only the first copy writes
        const int4 q = cp[off[id]];
        if (q.x == macro && q.y == i && q.z == j && q.w == k) c[id] = b[slot];
    }
}

void launch_canon_to_block(const Mesh& M, int lam, const double* c, double* b, hipStream_t s) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const dim3 g(L.n_slot_tiles, (unsigned)M.nt);
    k_canon_to_block<<<g, 256, 0, s>>>(c, b, M.d_topo.p, L.slot_tiles.p, L.N, L.B, M.nv, M.ne, M.nf);
    TS_HIP(hipGetLastError());
}
void launch_block_to_canon(const Mesh& M, int lam, const double* b, double* c, hipStream_t s) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const dim3 g(L.n_slot_tiles, (unsigned)M.nt);
    k_block_to_canon<<<g, 256, 0, s>>>(b, c, M.d_topo.p, L.slot_tiles.p, L.N, L.B, M.nv, M.ne, M.nf, L.if_off.p, L.if_copy.p);
    TS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_coords(double* __restrict__ xyz, const MacroGeom* __restrict__ geom,
                                                const int2* __restrict__ slot_tiles, int N, int64_t B) {
    TS_SLOT_DECODE();
    double x[3];
    node_xyz(geom[macro], N, i, j, k, x);
    xyz[3 * slot] = x[0];
    xyz[3 * slot + 1] = x[1];
    xyz[3 * slot + 2] = x[2];
}

void launch_coords(const Mesh& M, int lam, double* xyz, hipStream_t s) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const dim3 g(L.n_slot_tiles, (unsigned)M.nt);
    k_coords<<<g, 256, 0, s>>>(xyz, M.d_geom.p, L.slot_tiles.p, L.N, L.B);
    TS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- load vector

__device__ __forceinline__ double rhs_point(int kind, const double* par, int np, const double* x) {
    if (kind == TS_RHS_MANUFACTURED) {
        const double r1 = par[0], r2 = par[1], d = r2 - r1;
        const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double kk = M_PI / d;
        const double th = kk * (r - r1);
        const double h = x[0] * x[1] * x[2];
        return h * (kk * kk * sin(th) - (8.0 / r) * kk * cos(th));
    }
    if (kind == TS_RHS_BUMPS) {
        double s = 0.0;
        for (int b = 0; b + 5 <= np; b += 5) {
            const double dx = x[0] - par[b], dy = x[1] - par[b + 1], dz = x[2] - par[b + 2];
            const double sg = par[b + 3];
            s += par[b + 4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * sg * sg));
        }
        return s;
    }
    return 1.0;
}

// f at every slot of every macro block, from that macro's blended
// coordinates: each point is evaluated once, and the mass rows below read
// these values instead of evaluating f at all 15 points of every row
__global__ __launch_bounds__(256) void k_rhs_nodal(double* __restrict__ fv,
                                                   const MacroGeom* __restrict__ geom,
                                                   const int2* __restrict__ slot_tiles, int N,
                                                   int64_t B, int kind,
                                                   const double* __restrict__ par, int np) {
    TS_SLOT_DECODE();
    double x[3];
    node_xyz(geom[macro], N, i, j, k, x);
    fv[slot] = rhs_point(kind, par, np, x);
}

// partial consistent-mass row of local node (i,j,k) of one macro applied to
// the nodal values of f (fvb: that macro's block of them):
// sum_T |T|/20 (2 f_I + sum_{J in T, J != I} f_J).  Both loops are unrolled
// so that the points stay in registers.
__device__ __forceinline__ double mass_partial(const MacroGeom& g, int N, int i, int j, int k,
                                               const double* __restrict__ fvb) {
    double xs[NW][3], fv[NW];
    unsigned valid = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const int a = i + dir_i(w), b = j + dir_j(w), c = k + dir_k(w);
        xs[w][0] = xs[w][1] = xs[w][2] = 0.0;
        fv[w] = 0.0;
        if (inside(N, a, b, c)) {
            valid |= 1u << w;
            node_xyz(g, N, a, b, c, xs[w]);
            fv[w] = fvb[bidx(N, a, b, c)];
        }
    }
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 24; t++) {
        const int w0 = kTets24.t[t][0], w1 = kTets24.t[t][1], w2 = kTets24.t[t][2],
                  w3 = kTets24.t[t][3];
        const unsigned need = (1u << w0) | (1u << w1) | (1u << w2) | (1u << w3);
        if ((valid & need) != need) continue;
        double K[4];
        const double vol = stiffness_row0(xs[w0], xs[w1], xs[w2], xs[w3], K);
        s += vol / 20.0 * (2.0 * fv[w0] + fv[w1] + fv[w2] + fv[w3]);
    }
    return s;
}

__global__ __launch_bounds__(256) void k_rhs_volume(double* __restrict__ f, const MacroGeom* __restrict__ geom,
                                                    const int2* __restrict__ slot_tiles,
                                                    int N, int64_t B,
                                                    const double* __restrict__ fv) {
    TS_SLOT_DECODE();
    if (i < 1 || j < 1 || k < 1 || i + j + k > N - 1) return;
    f[slot] = mass_partial(geom[macro], N, i, j, k, fv + (size_t)macro * B);
}

__global__ __launch_bounds__(256) void k_rhs_iface(double* __restrict__ f, const MacroGeom* __restrict__ geom,
                                                   const int* __restrict__ off,
                                                   const int4* __restrict__ cp,
                                                   const unsigned char* __restrict__ flag, int n, int N,
                                                   int64_t B, const double* __restrict__ fv) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double v = 0.0;
    if (!(flag[t] & 1))
        for (int c = off[t]; c < off[t + 1]; c++) {
            const int4 q = cp[c];
            v += mass_partial(geom[q.x], N, q.y, q.z, q.w, fv + (size_t)q.x * B);
        }
    for (int c = off[t]; c < off[t + 1]; c++) {
        const int4 q = cp[c];
        f[(size_t)q.x * B + bidx(N, q.y, q.z, q.w)] = v;
    }
}

void launch_rhs(const Mesh& M, int lam, int kind, const double* dpar, int npar, double* f,
                hipStream_t s) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    const dim3 g(L.n_slot_tiles, (unsigned)M.nt);
    SBuf<double> fv((size_t)L.len, s);
    k_rhs_nodal<<<g, 256, 0, s>>>(fv.p, M.d_geom.p, L.slot_tiles.p, L.N, L.B, kind, dpar, npar);
    k_rhs_volume<<<g, 256, 0, s>>>(f, M.d_geom.p, L.slot_tiles.p, L.N, L.B, fv.p);
    const int n = (int)L.n_if;
    if (n) k_rhs_iface<<<(n + 255) / 256, 256, 0, s>>>(f, M.d_geom.p, L.if_off.p, L.if_copy.p, L.if_flag.p, n, L.N, L.B, fv.p);
    TS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- setup

// exact (IFEM) stencils at the sampling points of every macro: B[m][s][15]
__global__ __launch_bounds__(128) void k_sample(double* __restrict__ Bout, const MacroGeom* __restrict__ geom,
                                                const int* __restrict__ pts, int npts, int N) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (s >= npts) return;
    double st[NW];
    ifem_partial_stencil(geom[m], N, pts[3 * s], pts[3 * s + 1], pts[3 * s + 2], st);
    double* o = Bout + ((size_t)m * npts + s) * NW;
    for (int w = 0; w < NW; w++) o[w] = st[w];
}

__device__ __forceinline__ int basis_row(int q, int N, int i, int j, int k, double* row);

// Constant stencils (the volume rows of the unmapped macro, Phi = Id; the
// paper's constant-stencil lower bound, Tab. flops): the exact stencil of the
// affine macro's fine tetrahedra at its interior node (1, 1, 1), which is the
// stencil of every interior node.  One thread per macro: coef[m][15].
__global__ __launch_bounds__(64) void k_cons_stencils(double* __restrict__ coef,
                                                      const MacroGeom* __restrict__ geom, int nt,
                                                      int N) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nt) return;
    MacroGeom g = geom[m];
    g.affine = 1;
    double st[NW];
    ifem_partial_stencil(g, N, 1, 1, 1, st);
    for (int w = 0; w < NW; w++) coef[(size_t)m * NW + w] = st[w];
}

void launch_cons_stencils(const Mesh& M, int lam, double* coef, hipStream_t s) {
    const int nt = (int)M.nt;
    k_cons_stencils<<<(nt + 63) / 64, 64, 0, s>>>(coef, M.d_geom.p, nt, 1 << lam);
    TS_HIP(hipGetLastError());
}

// Selective surrogate check (remark in Sec. 3.4): one thread per macro
// compares the exact centre weight with the surrogate's centre polynomial at
// five interior points near the macro's vertices and centre.
__global__ __launch_bounds__(64) void k_fallback_check(unsigned char* __restrict__ flags,
                                                       const MacroGeom* __restrict__ geom,
                                                       const double* __restrict__ coef, int nt,
                                                       int N, int q, int mq, double tol) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nt) return;
    const int P[5][3] = {{1, 1, 1}, {N - 3, 1, 1}, {1, N - 3, 1}, {1, 1, N - 3}, {N / 4, N / 4, N / 4}};
    const double* c0 = coef + (size_t)m * NW * mq;  // direction 0 (centre)
    unsigned char bad = 0;
    for (int c = 0; c < 5; c++) {
        double st[NW], row[35];
        ifem_partial_stencil(geom[m], N, P[c][0], P[c][1], P[c][2], st);
        basis_row(q, N, P[c][0], P[c][1], P[c][2], row);
        double e = 0.0;
        for (int a = 0; a < mq; a++) e += c0[a] * row[a];
        if (!(e > 0.0) || fabs(e - st[0]) > tol * st[0]) bad = 1;
    }
    flags[m] = bad;
}

void launch_fallback_check(const Mesh& M, int lam, int q, const double* coef, double tol,
                           unsigned char* flags, hipStream_t s) {
    const int nt = (int)M.nt, mq = (q + 1) * (q + 2) * (q + 3) / 6;
    k_fallback_check<<<(nt + 63) / 64, 64, 0, s>>>(flags, M.d_geom.p, coef, nt, 1 << lam, q, mq,
                                                   tol);
    TS_HIP(hipGetLastError());
}

// FP32 and FP16-weight (pre-scaled by N) copies of a level's coefficients;
// bad[0] is set when a coefficient is not finite
__global__ __launch_bounds__(256) void k_coef_variants(const double* __restrict__ c, int64_t n,
                                                       int N, float* __restrict__ c32,
                                                       float* __restrict__ c16s,
                                                       int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = c[i];
    c32[i] = (float)v;
    c16s[i] = (float)(v * N);
    if (!isfinite(v)) bad[0] = 1;
}

void launch_coef_variants(const double* c, int64_t n, int N, float* c32, float* c16s, int* bad,
                          hipStream_t s) {
    if (n == 0) return;
    k_coef_variants<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(c, n, N, c32, c16s, bad);
    TS_HIP(hipGetLastError());
}

void launch_sample(const Mesh& M, int lam, const int* pts, int npts, double* B, hipStream_t s) {
    const dim3 g((npts + 127) / 128, (unsigned)M.nt);
    k_sample<<<g, 128, 0, s>>>(B, M.d_geom.p, pts, npts, 1 << lam);
    TS_HIP(hipGetLastError());
}

// monomial basis of the centred, scaled coordinates (degree, then l, then m
// descending)
__device__ __forceinline__ int basis_row(int q, int N, int i, int j, int k, double* row) {
    const double xi = (double)i / N - 0.25, eta = (double)j / N - 0.25, ze = (double)k / N - 0.25;
    int c = 0;
    for (int d = 0; d <= q; d++)
        for (int l = d; l >= 0; l--)
            for (int m = d - l; m >= 0; m--) {
                const int n = d - l - m;
                double v = 1.0;
                for (int a = 0; a < l; a++) v *= xi;
                for (int a = 0; a < m; a++) v *= eta;
                for (int a = 0; a < n; a++) v *= ze;
                row[c++] = v;
            }
    return c;
}

// The least-squares matrix of a level's fit, A[p][c] = c-th basis function
// at sampling point p (npts x mq); it depends on the level and the sampling
// set only, not on the geometry
__global__ __launch_bounds__(256) void k_fit_basis(int N, int q, const int* __restrict__ pts,
                                                   int npts, double* __restrict__ Ab) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const int mq = (q + 1) * (q + 2) * (q + 3) / 6;
    double row[35];
    basis_row(q, N, pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], row);
    for (int c = 0; c < mq; c++) Ab[(size_t)p * mq + c] = row[c];
}

// G = A^T A and its Cholesky factor (lower, row-major) into Lf[0..mq*mq)
__global__ __launch_bounds__(256) void k_fit_gram(int q, const double* __restrict__ Ab, int npts,
                                                  double* __restrict__ Lf) {
    __shared__ double G[35 * 35];
    const int mq = (q + 1) * (q + 2) * (q + 3) / 6;
    for (int e = threadIdx.x; e < mq * mq; e += blockDim.x) {
        const int a = e / mq, b = e % mq;
        double s = 0.0;
        for (int p = 0; p < npts; p++) s += Ab[(size_t)p * mq + a] * Ab[(size_t)p * mq + b];
        G[e] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int jj = 0; jj < mq; jj++) {
            double d = G[jj * mq + jj];
            for (int kk = 0; kk < jj; kk++) d -= G[jj * mq + kk] * G[jj * mq + kk];
            d = sqrt(d);
            G[jj * mq + jj] = d;
            for (int ii = jj + 1; ii < mq; ii++) {
                double t = G[ii * mq + jj];
                for (int kk = 0; kk < jj; kk++) t -= G[ii * mq + kk] * G[jj * mq + kk];
                G[ii * mq + jj] = t / d;
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < mq * mq; e += blockDim.x) Lf[e] = G[e];
}

// per macro: rhs = A^T B_m, then (L L^T) a = rhs; then one step of
// iterative refinement, rhs = A^T (B_m - A a) in FP64 and (L L^T) d = rhs,
// a += d, so that the accuracy of a is no longer limited by the squared
// condition number of the normal equations.  coef[m][w][c].  Thread (c, w)
// walks the sampling points in order.
__global__ __launch_bounds__(256) void k_fit_solve(int q, const double* __restrict__ Ab, int npts,
                                                   const double* __restrict__ Bv, const double* __restrict__ Lf,
                                                   double* __restrict__ coef) {
    __shared__ double R[35 * NW];
    __shared__ double Z[35 * NW];
    const int m = blockIdx.x;
    const int mq = (q + 1) * (q + 2) * (q + 3) / 6;
    const double* Bm = Bv + (size_t)m * npts * NW;
    for (int pass = 0; pass < 2; pass++) {
        for (int e = threadIdx.x; e < mq * NW; e += blockDim.x) {
            const int c = e / NW, w = e % NW;
            double s = 0.0;
            for (int p = 0; p < npts; p++) {
                const double* row = Ab + (size_t)p * mq;
                double b = Bm[(size_t)p * NW + w];
                if (pass == 1)
                    for (int c2 = 0; c2 < mq; c2++) b -= row[c2] * Z[c2 * NW + w];
                s += row[c] * b;
            }
            R[c * NW + w] = s;
        }
        __syncthreads();
        const int w = threadIdx.x;
        if (w < NW) {
            double z[35];
            for (int ii = 0; ii < mq; ii++) {
                double t = R[ii * NW + w];
                for (int kk = 0; kk < ii; kk++) t -= Lf[ii * mq + kk] * z[kk];
                z[ii] = t / Lf[ii * mq + ii];
            }
            for (int ii = mq - 1; ii >= 0; ii--) {
                double t = z[ii];
                for (int kk = ii + 1; kk < mq; kk++) t -= Lf[kk * mq + ii] * z[kk];
                z[ii] = t / Lf[ii * mq + ii];
            }
            for (int c = 0; c < mq; c++) Z[c * NW + w] = pass == 0 ? z[c] : Z[c * NW + w] + z[c];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < mq * NW; e += blockDim.x) {
        const int c = e / NW, w = e % NW;
        coef[((size_t)m * NW + w) * mq + c] = Z[c * NW + w];
    }
}

void launch_fit_basis(int N, int q, const int* pts, int npts, double* Ab, double* Lf,
                      hipStream_t s) {
    k_fit_basis<<<(npts + 255) / 256, 256, 0, s>>>(N, q, pts, npts, Ab);
    k_fit_gram<<<1, 256, 0, s>>>(q, Ab, npts, Lf);
    TS_HIP(hipGetLastError());
}

void launch_fit(int q, const double* Ab, int npts, const double* Lf, const double* B, int nt,
                double* coef, hipStream_t s) {
    k_fit_solve<<<nt, 256, 0, s>>>(q, Ab, npts, B, Lf, coef);
    TS_HIP(hipGetLastError());
}

// Symmetric surrogate (the remark at the end of Sec. 3.4): one polynomial
// per edge direction pair (w, wo), fitted to the exact weights of both
// directions at the edge midpoints.  A midpoint i + w/2 is an integer point
// of the level with 2N intervals, so the pair's points are given in doubled
// coordinates and the ordinary basis rows of that level apply.  Right-hand
// side of pair p: the first np points carry the weight of w at the samples,
// the next np that of wo; Ab holds the basis rows of the 2 np points and Lf
// the Cholesky factor of their Gram matrix.  coef7[m][p][c].
__global__ __launch_bounds__(64) void k_fit_solve_pair(int q, const double* __restrict__ Ab,
                                                       int np, const double* __restrict__ Bv,
                                                       const double* __restrict__ Lf, int w,
                                                       int wo, int p,
                                                       double* __restrict__ coef7) {
    __shared__ double R[35];
    __shared__ double Z[35];
    const int m = blockIdx.x;
    const int mq = (q + 1) * (q + 2) * (q + 3) / 6;
    const double* Bm = Bv + (size_t)m * np * NW;
    // normal equations, then one step of iterative refinement on the FP64
    // residual (as in k_fit_solve)
    for (int pass = 0; pass < 2; pass++) {
        for (int c = threadIdx.x; c < mq; c += blockDim.x) {
            double sum = 0.0;
            for (int t = 0; t < 2 * np; t++) {
                const double* row = Ab + (size_t)t * mq;
                double b = Bm[(size_t)(t < np ? t : t - np) * NW + (t < np ? w : wo)];
                if (pass == 1)
                    for (int c2 = 0; c2 < mq; c2++) b -= row[c2] * Z[c2];
                sum += row[c] * b;
            }
            R[c] = sum;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double z[35];
            for (int ii = 0; ii < mq; ii++) {
                double t = R[ii];
                for (int kk = 0; kk < ii; kk++) t -= Lf[ii * mq + kk] * z[kk];
                z[ii] = t / Lf[ii * mq + ii];
            }
            for (int ii = mq - 1; ii >= 0; ii--) {
                double t = z[ii];
                for (int kk = ii + 1; kk < mq; kk++) t -= Lf[kk * mq + ii] * z[kk];
                z[ii] = t / Lf[ii * mq + ii];
            }
            for (int c = 0; c < mq; c++) Z[c] = pass == 0 ? z[c] : Z[c] + z[c];
        }
        __syncthreads();
    }
    for (int c = threadIdx.x; c < mq; c += blockDim.x) coef7[((size_t)m * 7 + p) * mq + c] = Z[c];
}

__device__ __forceinline__ double binom_small(int n, int k) {
    double r = 1.0;
    for (int a = 1; a <= k; a++) r = r * (n - k + a) / a;
    return r;
}
__device__ __forceinline__ double pow_small(double x, int n) {
    double r = 1.0;
    for (int a = 0; a < n; a++) r *= x;
    return r;
}

// Per macro and direction w = 1..14: the pair polynomial of w translated by
// half an edge, Q_w(xi) = P_pair(w)(xi + w / (2N)), so that its value at a
// node is the pair polynomial at the midpoint of the node's edge in direction
// w; the monomials are expanded binomially (same basis order as basis_row).
__global__ __launch_bounds__(64) void k_sym_shift(const double* __restrict__ coef7,
                                                  const int* __restrict__ pair_of, int nt, int q,
                                                  int N, double* __restrict__ coef15) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nt * 14) return;
    const int m = idx / 14, w = 1 + idx % 14;
    const int mq = (q + 1) * (q + 2) * (q + 3) / 6;
    const double* P = coef7 + ((size_t)m * 7 + pair_of[w]) * mq;
    const double dx = 0.5 * kDI[w] / N, dy = 0.5 * kDJ[w] / N, dz = 0.5 * kDK[w] / N;
    double* out = coef15 + ((size_t)m * NW + w) * mq;
    int b = 0;
    for (int d = 0; d <= q; d++)
        for (int l = d; l >= 0; l--)
            for (int mm = d - l; mm >= 0; mm--) {
                const int n = d - l - mm;  // output monomial xi^l eta^mm zeta^n
                double v = 0.0;
                int a = 0;
                for (int d2 = 0; d2 <= q; d2++)
                    for (int l2 = d2; l2 >= 0; l2--)
                        for (int m2 = d2 - l2; m2 >= 0; m2--, a++) {
                            const int n2 = d2 - l2 - m2;
                            if (l2 < l || m2 < mm || n2 < n) continue;
                            v += P[a] * binom_small(l2, l) * binom_small(m2, mm) *
                                 binom_small(n2, n) * pow_small(dx, l2 - l) *
                                 pow_small(dy, m2 - mm) * pow_small(dz, n2 - n);
                        }
                out[b++] = v;
            }
}
// centre polynomial: minus the sum of the 14 translated ones (row sum zero)
__global__ void k_sym_centre(double* __restrict__ coef15, int nt, int mq) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nt * mq) return;
    const int m = idx / mq, c = idx % mq;
    double s = 0.0;
    for (int w = 1; w < NW; w++) s += coef15[((size_t)m * NW + w) * mq + c];
    coef15[(size_t)m * NW * mq + c] = -s;
}

void launch_fit_sym(int N, int q, const std::vector<int>& pts, const double* Bv, int nt,
                    double* coef15, hipStream_t s) {
    const int np = (int)pts.size() / 3;
    const int mq = (q + 1) * (q + 2) * (q + 3) / 6;
    // the seven pairs (w < opposite(w)) and the pair of every direction
    int pw[7][2], pair_of[NW] = {0};
    int np7 = 0;
    for (int w = 1; w < NW; w++)
        for (int o = w + 1; o < NW; o++)
            if (kDI[o] == -kDI[w] && kDJ[o] == -kDJ[w] && kDK[o] == -kDK[w]) {
                pair_of[w] = pair_of[o] = np7;
                pw[np7][0] = w;
                pw[np7][1] = o;
                np7++;
            }
    TS_REQUIRE(np7 == 7, TS_EINVAL, "direction table without seven opposite pairs");
    SBuf<double> c7((size_t)nt * 7 * mq, s), work((size_t)mq * mq, s);
    const std::vector<int> hpair(pair_of, pair_of + NW);
    SBuf<int> dpair(hpair, s), d2((size_t)6 * np, s);
    SBuf<double> ab2((size_t)2 * np * mq, s);
    for (int p = 0; p < 7; p++) {
        std::vector<int> p2((size_t)6 * np);
        for (int h = 0; h < 2; h++) {
            const int w = pw[p][h];
            for (int t = 0; t < np; t++) {
                p2[3 * ((size_t)h * np + t)] = 2 * pts[3 * t] + kDI[w];
                p2[3 * ((size_t)h * np + t) + 1] = 2 * pts[3 * t + 1] + kDJ[w];
                p2[3 * ((size_t)h * np + t) + 2] = 2 * pts[3 * t + 2] + kDK[w];
            }
        }
        TS_HIP(hipMemcpyAsync(d2.p, p2.data(), p2.size() * sizeof(int), hipMemcpyHostToDevice, s));
        k_fit_basis<<<(2 * np + 255) / 256, 256, 0, s>>>(2 * N, q, d2.p, 2 * np, ab2.p);
        k_fit_gram<<<1, 256, 0, s>>>(q, ab2.p, 2 * np, work.p);
        k_fit_solve_pair<<<nt, 64, 0, s>>>(q, ab2.p, np, Bv, work.p, pw[p][0], pw[p][1], p,
                                          c7.p);
        TS_HIP(hipStreamSynchronize(s));  // p2, d2 and work are reused by the next pair
    }
    k_sym_shift<<<(nt * 14 + 63) / 64, 64, 0, s>>>(c7.p, dpair.p, nt, q, N, coef15);
    k_sym_centre<<<(nt * mq + 255) / 256, 256, 0, s>>>(coef15, nt, mq);
    TS_HIP(hipGetLastError());
    TS_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- coarse level

// dense IFEM matrix of the free nodes: thread per free row r with copies
// cp[off[r] .. off[r+1]); slot_free maps block slots to free indices (-1:
// Dirichlet)
__global__ __launch_bounds__(64) void k_dense_assemble(const MacroGeom* __restrict__ geom,
                                                       const int* __restrict__ off,
                                                       const int4* __restrict__ cp, int nfree,
                                                       const int* __restrict__ slot_free, int N,
                                                       int64_t B, double* __restrict__ A) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nfree) return;
    double* row = A + (size_t)r * nfree;
    for (int c = off[r]; c < off[r + 1]; c++) {
        const int4 q = cp[c];
        double s[NW];
        ifem_partial_stencil(geom[q.x], N, q.y, q.z, q.w, s);
        for (int w = 0; w < NW; w++) {
            const int a = q.y + dir_i(w), b = q.z + dir_j(w), cc = q.w + dir_k(w);
            if (!inside(N, a, b, cc)) continue;
            const int col = slot_free[(size_t)q.x * B + bidx(N, a, b, cc)];
            if (col >= 0) row[col] += s[w];
        }
    }
}

// Blocked in-place Gauss-Jordan inversion of the SPD coarse matrix (row-major
// n x n), pivot blocks K = k0 .. k0+b-1 of at most GJB rows in order:
//   D = A[K,K]^-1;  P = D A[K,:];  A[i,j] -= A[i,K] P[:,j] (i, j outside K);
//   A[i,K] = -A[i,K] D (i outside K);  A[K,j] = P[:,j] (j outside K);  A[K,K] = D.
constexpr int GJB = 64;

// D = A[K,K]^-1 by unblocked Gauss-Jordan in LDS (one workgroup of four
// wavefronts): thread (r, j) owns column j of rows r, r + 4, ...; per pivot
// k the scaled pivot row and the old pivot column are published first, then
// every entry is updated independently
__global__ __launch_bounds__(256) void k_bgj_diag(const double* __restrict__ A, int n, int k0,
                                                  int b, double* __restrict__ D) {
    __shared__ double M[GJB][GJB + 1];
    __shared__ double col[GJB];
    __shared__ double prow[GJB];
    const int j = (int)threadIdx.x & 63, r0 = (int)threadIdx.x >> 6;
    for (int i = r0; i < GJB; i += 4) M[i][j] = (i < b && j < b) ? A[(size_t)(k0 + i) * n + k0 + j] : 0.0;
    __syncthreads();
    for (int k = 0; k < b; k++) {
        if (r0 == 0 && j < b) {
            const double piv = M[k][k];
            col[j] = M[j][k];
            prow[j] = (j == k) ? 1.0 / piv : M[k][j] / piv;
        }
        __syncthreads();
        if (j < b) {
            const double nk = prow[j];
#pragma unroll
            for (int q = 0; q < GJB / 4; q++) {
                const int i = r0 + 4 * q;
                if (i < b) M[i][j] = (i == k) ? nk : (j == k ? 0.0 : M[i][j]) - col[i] * nk;
            }
        }
        __syncthreads();
    }
    for (int e = (int)threadIdx.x; e < b * b; e += 256) D[e] = M[e / b][e % b];
}

// P[r][j] = sum_s D[r][s] A[k0+s][j] for every column j (b x n)
__global__ __launch_bounds__(256) void k_bgj_panel(const double* __restrict__ A, int n, int k0,
                                                   int b, const double* __restrict__ D,
                                                   double* __restrict__ P) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= n) return;
    double v = 0.0;
    for (int q = 0; q < b; q++) v += D[r * b + q] * A[(size_t)(k0 + q) * n + j];
    P[(size_t)r * n + j] = v;
}

// A[i][j] -= sum_s A[i][k0+s] P[s][j] for i, j outside the pivot block:
// 64 x 64 output tiles, 4 x 4 per thread, operands staged in LDS
__global__ __launch_bounds__(256) void k_bgj_update(double* __restrict__ A, int n, int k0, int b,
                                                    const double* __restrict__ P) {
    __shared__ double Ls[GJB][GJB + 1];  // A[i0 + r][k0 + s]
    __shared__ double Ps[GJB][GJB + 1];  // P[s][j0 + c]
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    for (int e = threadIdx.x; e < 64 * GJB; e += 256) {
        const int r = e / GJB, q = e % GJB;
        Ls[r][q] = (i0 + r < n && q < b) ? A[(size_t)(i0 + r) * n + k0 + q] : 0.0;
        const int c = e % 64, q2 = e / 64;
        Ps[q2][c] = (j0 + c < n && q2 < b) ? P[(size_t)q2 * n + j0 + c] : 0.0;
    }
    __syncthreads();
    const int tr = (threadIdx.x / 16) * 4, tc = (threadIdx.x % 16) * 4;
    double acc[4][4] = {};
    for (int q = 0; q < b; q++) {
        double a[4], p[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            a[u] = Ls[tr + u][q];
            p[u] = Ps[q][tc + u];
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int v = 0; v < 4; v++) acc[u][v] += a[u] * p[v];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int i = i0 + tr + u;
        if (i >= n || (i >= k0 && i < k0 + b)) continue;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int j = j0 + tc + v;
            if (j >= n || (j >= k0 && j < k0 + b)) continue;
            A[(size_t)i * n + j] -= acc[u][v];
        }
    }
}

// A[i][K] = -A[i][K] D for rows outside K (four rows per workgroup, one
// column per lane); then the pivot rows and block
__global__ __launch_bounds__(256) void k_bgj_cols(double* __restrict__ A, int n, int k0, int b,
                                                  const double* __restrict__ D) {
    __shared__ double Ds[GJB][GJB + 1];
    __shared__ double R[4][GJB];
    const int c = (int)threadIdx.x & 63, rr = (int)threadIdx.x >> 6;
    const int i = (int)blockIdx.x * 4 + rr;
    for (int e = (int)threadIdx.x; e < b * b; e += 256) Ds[e / b][e % b] = D[e];
    const bool act = i < n && !(i >= k0 && i < k0 + b) && c < b;
    if (act) R[rr][c] = A[(size_t)i * n + k0 + c];
    __syncthreads();
    if (act) {
        double v = 0.0;
        for (int q = 0; q < b; q++) v += R[rr][q] * Ds[q][c];
        A[(size_t)i * n + k0 + c] = -v;
    }
}
__global__ __launch_bounds__(256) void k_bgj_rows(double* __restrict__ A, int n, int k0, int b,
                                                  const double* __restrict__ P,
                                                  const double* __restrict__ D) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (j >= n) return;
    A[(size_t)(k0 + r) * n + j] = (j >= k0 && j < k0 + b) ? D[r * b + (j - k0)] : P[(size_t)r * n + j];
}

// work: at least GJB * (n + GJB) doubles
void launch_gj_blocked(double* A, int n, double* work, hipStream_t s) {
    double* D = work;
    double* P = work + GJB * GJB;
    const unsigned gt = (unsigned)((n + 63) / 64), gc = (unsigned)((n + 255) / 256);
    for (int k0 = 0; k0 < n; k0 += GJB) {
        const int b = std::min(GJB, n - k0);
        k_bgj_diag<<<1, 256, 0, s>>>(A, n, k0, b, D);
        k_bgj_panel<<<dim3(gc, b), 256, 0, s>>>(A, n, k0, b, D, P);
        k_bgj_update<<<dim3(gt, gt), 256, 0, s>>>(A, n, k0, b, P);
        k_bgj_cols<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(A, n, k0, b, D);
        k_bgj_rows<<<dim3(gc, b), 256, 0, s>>>(A, n, k0, b, P, D);
    }
    TS_HIP(hipGetLastError());
}

// u = Ainv f on the coarsest level: gather f at the first copy of each free
// node, dense product (A^-1 stored transposed: coalesced columns), scatter to
// every copy
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gather(const T* __restrict__ f, const int* __restrict__ off,
                                                       const int64_t* __restrict__ slot, int n,
                                                       double* __restrict__ fb) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) fb[r] = (double)f[slot[off[r]]];
}
// ub = A^{-1} fb with the transposed inverse: workgroup (x, y) takes rows
// 64x .. 64x+63 and the columns of split y (KSPLIT splits, 4 interleaved
// column lanes each), partial sums summed in a fixed order afterwards
constexpr int KSPLIT = 16;
__global__ __launch_bounds__(256) void k_coarse_matvec(const double* __restrict__ AinvT,
                                                       const double* __restrict__ fb, int n,
                                                       double* __restrict__ part) {
    const int r = blockIdx.x * 64 + (threadIdx.x & 63);
    const int lane = threadIdx.x >> 6;
    const int per = (n + KSPLIT - 1) / KSPLIT;
    const int c0 = blockIdx.y * per, c1 = min(n, c0 + per);
    double s = 0.0;
    if (r < n)
        for (int c = c0 + lane; c < c1; c += 4) s += AinvT[(size_t)c * n + r] * fb[c];
    if (r < n) part[((size_t)blockIdx.y * 4 + lane) * n + r] = s;
}
__global__ __launch_bounds__(256) void k_coarse_matvec_sum(const double* __restrict__ part, int n,
                                                           double* __restrict__ ub) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double s = 0.0;
    for (int q = 0; q < KSPLIT * 4; q++) s += part[(size_t)q * n + r];
    ub[r] = s;
}
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_scatter(T* __restrict__ u, const int* __restrict__ off,
                                                        const int64_t* __restrict__ slot, int n,
                                                        const double* __restrict__ ub) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const T v = (T)ub[r];
    for (int c = off[r]; c < off[r + 1]; c++) u[slot[c]] = v;
}

void launch_coarse_solve(const double* AinvT, int n, const int* free_first, const int* cp_off,
                         const int64_t* cp_slot, int dtype, const void* f, void* u,
                         double* work, hipStream_t s) {
    (void)free_first;
    const int g = (n + 255) / 256;
    double* fb = work;
    double* ub = work + n;
    double* part = work + 2 * (size_t)n;
    const dim3 gm((unsigned)((n + 63) / 64), KSPLIT);
    if (dtype == TS_F64)
        k_coarse_gather<double><<<g, 256, 0, s>>>((const double*)f, cp_off, cp_slot, n, fb);
    else
        k_coarse_gather<float><<<g, 256, 0, s>>>((const float*)f, cp_off, cp_slot, n, fb);
    k_coarse_matvec<<<gm, 256, 0, s>>>(AinvT, fb, n, part);
    k_coarse_matvec_sum<<<g, 256, 0, s>>>(part, n, ub);
    if (dtype == TS_F64)
        k_coarse_scatter<double><<<g, 256, 0, s>>>((double*)u, cp_off, cp_slot, n, ub);
    else
        k_coarse_scatter<float><<<g, 256, 0, s>>>((float*)u, cp_off, cp_slot, n, ub);
    TS_HIP(hipGetLastError());
}

// exported for the solver: dense assembly with explicit copies
void launch_dense_assemble_cp(const Mesh& M, int lam, const int* off, const int4* cp, int nfree,
                              const int* slot_free, double* A, hipStream_t s) {
    const Level& L = const_cast<Mesh&>(M).level(lam);
    k_dense_assemble<<<(nfree + 63) / 64, 64, 0, s>>>(M.d_geom.p, off, cp, nfree, slot_free, L.N, L.B, A);
    TS_HIP(hipGetLastError());
}

template <typename T>
__global__ void k_transpose(const T* __restrict__ a, T* __restrict__ b, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c < n) b[(size_t)c * n + r] = a[(size_t)r * n + c];
}
void launch_transpose(const double* a, double* b, int n, hipStream_t s) {
    k_transpose<double><<<dim3((n + 255) / 256, n), 256, 0, s>>>(a, b, n);
    TS_HIP(hipGetLastError());
}

}  // namespace ts
