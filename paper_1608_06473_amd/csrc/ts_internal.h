// Internal data structures of the two-scale library (host side) and the
// kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <atomic>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "ts_geom.h"
#include "../../include/twoscale.h"

namespace ts {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
struct Error {
    int code;
    std::string msg;
};
#define TS_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            throw ::ts::Error{TS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)
#define TS_REQUIRE(cond, code, msg)                        \
    do {                                                   \
        if (!(cond)) throw ::ts::Error{(code), (msg)};     \
    } while (0)

// ------------------------------------------------------------ device buffer
// device bytes held by all library objects of the process
inline std::atomic<int64_t> g_dev_bytes{0};

template <typename X>
struct DBuf {
    X* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { reset(); }
    void reset() {
        if (p) {
            (void)hipFree(p);
            g_dev_bytes -= (int64_t)(n * sizeof(X));
        }
        p = nullptr;
        n = 0;
    }
    // keeps the buffer when it already holds count elements (rebuilds of
    // geometry-dependent data reuse their memory); contents are undefined
    void alloc(size_t count) {
        if (p && n == count) return;
        reset();
        if (count == 0) return;
        hipError_t e = hipMalloc(&p, count * sizeof(X));
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{TS_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(X)) + " bytes failed"};
        }
        n = count;
        g_dev_bytes += (int64_t)(count * sizeof(X));
    }
    void upload(const std::vector<X>& h) {
        alloc(h.size());
        if (!h.empty()) TS_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice));
    }
};

// Stream-ordered temporary device buffer: allocated and freed in the order of
// stream s (hipMallocAsync / hipFreeAsync), so releasing it waits for nothing
// but s, where a plain hipFree would wait for the whole device (set-up work of
// one request then stalls behind every other request's queued kernels).
// Every use must be ordered on s; upload() copies asynchronously on s, so the
// host vector must outlive the next synchronisation of s.
template <class X>
struct SBuf {
    X* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    SBuf(size_t count, hipStream_t st) : n(count), s(st) {
        if (!count) return;
        if (hipMallocAsync((void**)&p, count * sizeof(X), s) != hipSuccess) {
            p = nullptr;
            throw Error{TS_ENOMEM, "hipMallocAsync of " + std::to_string(count * sizeof(X)) +
                                       " bytes failed"};
        }
        g_dev_bytes += (int64_t)(count * sizeof(X));
    }
    SBuf(const std::vector<X>& h, hipStream_t st) : SBuf(h.size(), st) {
        if (n) TS_HIP(hipMemcpyAsync(p, h.data(), n * sizeof(X), hipMemcpyHostToDevice, s));
    }
    SBuf(const SBuf&) = delete;
    SBuf& operator=(const SBuf&) = delete;
    ~SBuf() {
        if (p) {
            (void)hipFreeAsync(p, s);
            g_dev_bytes -= (int64_t)(n * sizeof(X));
        }
    }
};

// Per-macro topology record on the device: global vertex ids, edge and face
// ids of the primitives (local edge order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3);
// face o is opposite local vertex o), which local vertex of each edge has the
// larger global id, the local vertices of each face sorted by global id,
// Dirichlet flags and macro multiplicities of each primitive.
struct MacroTopo {
    int64_t vg[4];
    int64_t e[6];
    int64_t f[4];
    signed char ehi[6];      // local vertex (0..3) with the larger global id
    signed char elo[6];
    signed char fs[4][3];    // face o: local vertices sorted by global id
    unsigned char vdir[4], edir[6], fdir[4];
    unsigned char emult[6], fmult[4];
    unsigned char pad[2];
};

// GS phases of the lower primitives: 0 vertices, 1-2 edges (a mod 2), 3-5
// faces ((a + 2b) mod 3 in the face frame).
constexpr int N_IF_PHASES = 6;

// Per-level layout and interface maps.
// Level data that depend only on the connectivity: index lists, tiles, lane
// orders.  Meshes with the same connectivity may share them.
struct Level {
    int lam = 0, N = 0;
    int64_t B = 0, len = 0;       // block size, vector length (n_macros * B)
    int64_t n_unique = 0, n_free = 0;
    int64_t n_if = 0;             // unique lower-primitive nodes (incl. Dirichlet)
    DBuf<int> if_off;             // n_if + 1
    DBuf<int4> if_copy;           // (macro, i, j, k)
    DBuf<unsigned char> if_flag;  // bit 0: Dirichlet; bits 1-3: GS phase
    DBuf<int> phase_list[N_IF_PHASES];
    int n_phase[N_IF_PHASES] = {0, 0, 0, 0, 0, 0};
    DBuf<int> if_free;            // free interface nodes (for norms)
    int n_if_free = 0;
    // all-slot tiles: (plane k, first slot of a chunk of plane k)
    DBuf<int2> slot_tiles;
    int n_slot_tiles = 0;
    // LDS-staged volume tiles: (k0, j0, j1, i0): rows j0..j1-1 of plane k0's
    // interior (i0 = 0), or one row j0 from i0 on (i0 >= 1, long rows)
    DBuf<int4> lds_tiles;
    int n_lds_tiles = 0;
    int lds_kpt = 0;              // staged values per thread and plane
    DBuf<unsigned> gs_lanes;      // per tile and lane: i | j << 16 (GS order)
    DBuf<unsigned> ap_lanes;      // per tile and lane: i | j << 16 (apply order)
    DBuf<int> stage_tbl;          // per tile and staged plane k0-1+st (st = 0..R+1):
                                  // first block element of rows j0-1 .. j1 (0 if none)
    // fast path for free nodes of interior faces (exactly two copies): node
    // ids, both copies, and their combined rows as struct of arrays
    // [slot][face node] so that lane loads are coalesced; the remaining free
    // lower-primitive nodes (edges, vertices) go through the general copy
    // lists
    int n_f2 = 0;
    DBuf<int> f2_node;
    DBuf<int4> f2_cp;             // [2][n_f2]
    DBuf<int> rest;               // other free lower-primitive nodes (node ids)
    int n_rest = 0;
    // stored partial stencils of the copies of the `rest` nodes: copy c of
    // node n has compact index rc_base[n] + (c - off[n]); [15][n_rc]
    DBuf<int> rc_base;
    DBuf<int4> rc_cp;
    int n_rc = 0;
    // block slots of every copy of every Dirichlet node (zero rows)
    DBuf<int64_t> dir_slots;
    int64_t n_dir_slots = 0;
    // Gauss-Seidel copy of the face fast path, grouped by phase: copies
    // [2][n_f2] and combined rows [15][n_f2]; phase p is the range
    // f2g_off[p] .. f2g_off[p] + n_f2_phase[p]
    DBuf<int4> f2g_cp;
    // face fast path grouped by face: nodes f2_face_off[f] .. f2_face_off[f+1]
    // of the canonical copy belong to the f-th interior face, in the face
    // frame order (b = 1 .. N-2, a = 1 .. N-1-b)
    DBuf<int> f2_face_off;
    int n_f2_faces = 0;
    int f2g_off[N_IF_PHASES] = {0, 0, 0, 0, 0, 0};
    int n_f2_phase[N_IF_PHASES] = {0, 0, 0, 0, 0, 0};
    // per GS phase: node ids of the general lists
    DBuf<int> rest_phase[N_IF_PHASES];
    int n_rest_phase[N_IF_PHASES] = {0, 0, 0, 0, 0, 0};
    // Within a phase the nodes that no free node of the same phase is
    // coupled to come first (the first n_f2_direct / n_rest_direct of each
    // list): they are written in place, the rest through a temporary that
    // is scattered after the phase.
    int n_f2_direct[N_IF_PHASES] = {0, 0, 0, 0, 0, 0};
    int n_rest_direct[N_IF_PHASES] = {0, 0, 0, 0, 0, 0};
};

#ifndef TS_VOL_R
#define TS_VOL_R 24
#endif
#ifndef TS_VOL_WAVES
#define TS_VOL_WAVES 2
#endif
#ifndef TS_VOL_PF
#define TS_VOL_PF 4
#endif
#ifndef TS_VOL_G
#define TS_VOL_G 2
#endif
// minimum waves per SIMD the apply- and residual-mode surrogate volume
// kernels are compiled for when q <= 2 and the staging width is 2 (levels up
// to 7): a budget of 168 VGPRs at three waves, which those instantiations meet
// without spilling (FP32 ones use under 100 anyway)
#ifndef TS_VOL_WAVES_EU
#define TS_VOL_WAVES_EU 3
#endif
constexpr int VOL_R = TS_VOL_R;  // planes per volume tile
// threads of a volume workgroup (one column each; a multiple of 64)
#ifndef TS_VOL_THREADS
#define TS_VOL_THREADS 256
#endif
constexpr int VOL_THREADS = TS_VOL_THREADS;
static_assert(VOL_THREADS % 64 == 0 && VOL_THREADS <= 1024, "bad volume workgroup size");

// Level data that depend on the vertex coordinates, owned by each mesh and
// built on first use: the blended coordinates of every slot (element-wise
// volume rows), the combined rows of the face fast path in canonical and
// phase-grouped order ([15][n_f2] each), the partial stencils of the other
// interface copies ([15][n_rc]), and single-precision copies of the face
// rows for the FP32 vectors; gens: the geometry generation they were
// computed for (-1: none).
struct LevelGeo {
    int xyz_gen = -1, sten_gen = -1, sten32_gen = -1;
    DBuf<double> xyz;
    DBuf<double> f2_sten, f2g_sten, rest_sten;
    DBuf<float> f2_sten32, f2g_sten32;
};

struct Mesh {
    int64_t nv = 0, nt = 0, ne = 0, nf = 0;
    int geom = TS_GEOM_SHELL;
    std::vector<double> vtx;
    std::vector<int64_t> tet;
    std::vector<std::array<int64_t, 2>> edges;
    std::vector<std::array<int64_t, 3>> faces;
    std::vector<unsigned char> vdir, edir, fdir;
    std::vector<std::vector<int64_t>> v_tets, e_tets, f_tets;
    std::vector<MacroTopo> topo;
    std::vector<MacroGeom> geomh;
    DBuf<MacroGeom> d_geom;
    DBuf<MacroTopo> d_topo;
    std::map<int, std::shared_ptr<Level>> levels;
    std::map<int, std::unique_ptr<LevelGeo>> geo;
    int device = 0;
    int geo_gen = 0;  // bumped whenever the vertex coordinates change

    LevelGeo& level_geo(int lam) {
        auto& g = geo[lam];
        if (!g) g = std::make_unique<LevelGeo>();
        return *g;
    }
    Level& level(int lam);
    int64_t num_unique(int N) const {
        return nv + ne * (N - 1) + nf * (int64_t)(N - 1) * (N - 2) / 2 +
               nt * (int64_t)(N - 1) * (N - 2) * (N - 3) / 6;
    }
};

void build_topology(Mesh& M);
// macro geometry records (host and device) from the vertex coordinates
void build_geometry(Mesh& M);
const double* face_stencils(Mesh& M, int lam, hipStream_t s);
// the face rows rounded to FP32 (canonical order), built on first use
const float* face_stencils32(Mesh& M, int lam, hipStream_t s);
void warm_level(const ts_op* op, int lam, bool ifem_rows, hipStream_t s);

// ------------------------------------------------------------ operators
struct LevelOp {
    int lam = 0;
    DBuf<double> coef64;   // [nt][15][mq]
    DBuf<float> coef32;
    DBuf<float> coef16s;   // FP16-weight variant: coefficients pre-scaled by N
    // selective surrogate: macros with surrogate volume rows / with IFEM rows
    std::vector<unsigned char> flags;
    DBuf<int> sur_list, ifem_list;
    int n_sur = 0, n_ifem = 0;
    bool has_coef = false;
    DBuf<double> gs_tmp;   // interface Gauss-Seidel values of one phase
    // surrogate rows of interior faces: [nt][4][15][m2] by (first macro of
    // the face, its face type); face_fit: used on this level
    DBuf<double> fcoef;
    bool face_fit = false;
    // the fit's sampling points, least-squares matrix and Gram factor
    // (geometry-independent: kept when the level is rebuilt for new vertices)
    DBuf<int> fit_pts;
    DBuf<double> fit_basis, fit_gram;
    // set-up results read back once for all levels: the fallback check's
    // per-macro flags and the non-finite-coefficient flag
    DBuf<unsigned char> d_flags;
    DBuf<int> d_bad;
};

}  // namespace ts

struct ts_mesh {
    ts::Mesh m;
    std::atomic<int> ops{0};  // operators created on this mesh and not destroyed
};

struct ts_op {
    ts_mesh* mesh = nullptr;
    ts_op_params p{};
    int max_level = 0;
    int mq = 0;
    std::map<int, std::unique_ptr<ts::LevelOp>> lv;
    // side stream for the lower-primitive rows, run beside the volume kernel
    // (fork / join through events on the caller's stream)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    ~ts_op() {
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
    }
};

namespace ts {

// ------------------------------------------------------------ kernel launchers
// vector dtype codes follow TS_F64 / TS_F32 / TS_F16W (the last two use
// float vectors).
void launch_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                   const void* f, int colour, hipStream_t s, bool fuse_face = false);
// exact: the face rows take the stored exact stencils even where the
// operator has face fits (exact residuals)
void launch_iface(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                  const void* f, int phase, double* tmp, hipStream_t s, bool skip_face = false,
                  bool exact = false);
// least-squares fits of the face rows of a level (one workgroup per interior
// face) into fcoef [nt][4][15][m2]; the exact face rows must exist
void launch_face_fit(const Level& L, const double* f2sten, int q, int jsamp, int nt, double* fcoef,
                     hipStream_t s);
void launch_iface_scatter(const ts_op* op, int lam, int dtype, int phase, const double* tmp,
                          void* u, hipStream_t s);
void launch_ifem_volume(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                        const void* f, int colour, hipStream_t s, const int* mlist = nullptr,
                        int n_list = -1);
void launch_coef_variants(const double* c, int64_t n, int N, float* c32, float* c16s, int* bad,
                          hipStream_t s);
void launch_fallback_check(const Mesh& M, int lam, int q, const double* coef, double tol,
                           unsigned char* flags, hipStream_t s);
void launch_restrict(const Mesh& M, int lam_f, int dtype, const void* rf, void* rc, hipStream_t s);
void launch_prolongate_add(const Mesh& M, int lam_f, int dtype, const void* uc, void* uf,
                           hipStream_t s);
void launch_fill(void* x, int dtype, int64_t n, double v, hipStream_t s);
void launch_cast(const void* src, int dsrc, void* dst, int ddst, int64_t n, hipStream_t s);
void launch_axpy(double a, const void* x, int dx, double* y, int64_t n, hipStream_t s);
double norm2_free(const Mesh& M, int lam, int dtype, const void* x, double* partial,
                  hipStream_t s);  // synchronising
int64_t norm_partial_count(const Mesh& M, int lam);
void norm2_noalloc(const Mesh& M, int lam, int dtype, const void* x, double* out, hipStream_t s);
void launch_norm2_free(const Mesh& M, int lam, int dtype, const void* x, double* partial,
                       double* out, hipStream_t s);
void launch_canon_to_block(const Mesh& M, int lam, const double* c, double* b, hipStream_t s);
void launch_block_to_canon(const Mesh& M, int lam, const double* b, double* c, hipStream_t s);
void launch_coords(const Mesh& M, int lam, double* xyz, hipStream_t s);
void launch_rhs(const Mesh& M, int lam, int kind, const double* dpar, int npar, double* f,
                hipStream_t s);
void launch_sample(const Mesh& M, int lam, const int* pts, int npts, double* B, hipStream_t s);
void launch_cons_stencils(const Mesh& M, int lam, double* coef, hipStream_t s);
// symmetric surrogate: pair fits at the edge midpoints, translated to the 15
// per-direction polynomials [nt][15][mq] (centre: minus the sum)
void launch_fit_sym(int N, int q, const std::vector<int>& pts, const double* B, int nt,
                    double* coef15, hipStream_t s);
// least-squares matrix of a level's fit (npts x mq) and the Cholesky factor
// of its Gram matrix (mq x mq); they depend on the level and sampling set only
void launch_fit_basis(int N, int q, const int* pts, int npts, double* Ab, double* Lf,
                      hipStream_t s);
void launch_fit(int q, const double* Ab, int npts, const double* Lf, const double* B, int nt,
                double* coef, hipStream_t s);
void launch_dense_assemble_cp(const Mesh& M, int lam, const int* off, const int4* cp, int nfree,
                              const int* slot_free, double* A, hipStream_t s);
void launch_transpose(const double* a, double* b, int n, hipStream_t s);
void launch_gj_blocked(double* A, int n, double* work, hipStream_t s);
void launch_coarse_solve(const double* Ainv, int n, const int* free_first, const int* cp_off,
                         const int64_t* cp_slot, int dtype, const void* f, void* u,
                         double* work, hipStream_t s);

}  // namespace ts
