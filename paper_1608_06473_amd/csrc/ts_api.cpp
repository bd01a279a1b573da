// C ABI of the two-scale library: host orchestration of the kernels.
// Setup of the surrogate (Sec. 3.1-3.3), operator application and smoothing
// (Sec. 3.4, eq. iteration-scheme), V(nu1, nu2) multigrid (Sec. 4 introduction) with an
// exact FP64 coarsest level, and the FP64 / mixed-precision solve.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "ts_internal.h"

namespace ts {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

template <class F>
static int guarded(F&& f) {
    try {
        f();
        return TS_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return TS_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return TS_EINVAL;
    }
}

static hipStream_t S(ts_stream s) { return (hipStream_t)s; }

static int mq_of(int q) { return (q + 1) * (q + 2) * (q + 3) / 6; }

// Sampling points of a level (N intervals): LSQP uses the interior nodes of
// the level-m lattice, m = min(l, max(1, j)) with l = log2(N) - 2, embedded
// at stride N / 2^(m+2) (eq. samplingSetFunctions); IPOLY the ten quadratic
// nodes of the shrunk macro, a = N - 3, b = N/2 - 1 (Sec. 3.1).
static std::vector<int> sample_points(int N, int method, int jsamp) {
    std::vector<int> p;
    if (method == TS_IPOLY) {
        const int a = N - 3, b = N / 2 - 1;
        const int P[10][3] = {{1, 1, 1}, {1, 1, a}, {1, a, 1}, {a, 1, 1}, {1, 1, b},
                              {1, b, 1}, {b, 1, 1}, {1, b, b}, {b, 1, b}, {b, b, 1}};
        for (auto& r : P) p.insert(p.end(), r, r + 3);
        return p;
    }
    int l = 0;
    while ((4 << l) < N) l++;
    int m = std::min(l, std::max(1, jsamp));
    const int Ns = 4 << m, st = N / Ns;
    for (int k = 1; k <= Ns - 3; k++)
        for (int j = 1; j <= Ns - 2 - k; j++)
            for (int i = 1; i <= Ns - 1 - j - k; i++) {
                p.push_back(i * st);
                p.push_back(j * st);
                p.push_back(k * st);
            }
    return p;
}

static bool uses_surrogate(const ts_op* op, int lam) {
    return op->p.method != TS_IFEM && lam >= 3 && op->lv.count(lam) && op->lv.at(lam)->has_coef;
}

// Per-macro split of the volume rows (selective surrogate): run the check on
// the device coefficients, then upload the surrogate and IFEM macro lists.
static void split_macros(ts_op* op, LevelOp& lo, int lam, hipStream_t s) {
    const Mesh& M = op->mesh->m;
    const int nt = (int)M.nt;
    lo.flags.assign(nt, 0);
    if (op->p.fallback_tol > 0) {
        SBuf<unsigned char> d(nt, s);
        launch_fallback_check(M, lam, op->p.q, lo.coef64.p, op->p.fallback_tol, d.p, s);
        TS_HIP(hipMemcpyAsync(lo.flags.data(), d.p, nt, hipMemcpyDeviceToHost, s));
        TS_HIP(hipStreamSynchronize(s));
    }
    std::vector<int> sur, ifem;
    for (int t = 0; t < nt; t++) (lo.flags[t] ? ifem : sur).push_back(t);
    lo.n_sur = (int)sur.size();
    lo.n_ifem = (int)ifem.size();
    if (lo.n_sur) lo.sur_list.upload(sur); else lo.sur_list.reset();
    if (lo.n_ifem) lo.ifem_list.upload(ifem); else lo.ifem_list.reset();
    // face fits: only where every volume keeps its surrogate
    lo.face_fit = lo.fcoef.p && lo.n_ifem == 0;
}

static void upload_coef_variants(ts_op* op, LevelOp& lo, int lam, const std::vector<double>& h) {
    const int N = 1 << lam;
    std::vector<float> f32(h.size()), f16s(h.size());
    for (size_t i = 0; i < h.size(); i++) {
        f32[i] = (float)h[i];
        f16s[i] = (float)(h[i] * N);
    }
    lo.coef32.upload(f32);
    lo.coef16s.upload(f16s);
    lo.has_coef = true;
}

// Enqueues on s the level's geometry-dependent operator data (fits or
// constant stencils, their FP32 / FP16-weight copies, face fits, the
// fallback check); a level built before (new vertex coordinates) is rebuilt
// in the buffers it has.  finish_levels reads the checks back.
static void enqueue_level(ts_op* op, int lam, hipStream_t s) {
    Mesh& M = op->mesh->m;
    std::unique_ptr<LevelOp> lo;
    auto it = op->lv.find(lam);
    if (it != op->lv.end()) {
        lo = std::move(it->second);
        op->lv.erase(it);
    } else {
        lo = std::make_unique<LevelOp>();
    }
    lo->lam = lam;
    lo->has_coef = false;
    M.level(lam);
    const bool cons = op->p.method == TS_CONS && lam >= 3;
    const bool sur = op->p.method != TS_IFEM && op->p.method != TS_CONS && lam >= 3;
    if (cons) {
        // one stencil per macro: the exact stencil of its unmapped fine
        // tetrahedra, the same at every interior node (degree-0 coefficients)
        lo->coef64.alloc((size_t)M.nt * NW);
        launch_cons_stencils(M, lam, lo->coef64.p, s);
    } else if (sur) {
        const int N = 1 << lam, q = op->p.q, mq = op->mq;
        lo->coef64.alloc((size_t)M.nt * NW * mq);
        if (op->p.coarse_from_finest && lam < op->max_level) {
            // the finest level's polynomials (same reference coordinates),
            // scaled by the mesh-size ratio: exact, a power of two
            const LevelOp& fine = *op->lv.at(op->max_level);
            const int64_t n = (int64_t)lo->coef64.n;
            launch_fill(lo->coef64.p, TS_F64, n, 0.0, s);
            launch_axpy(ldexp(1.0, op->max_level - lam), fine.coef64.p, TS_F64, lo->coef64.p,
                        n, s);
        } else {
            std::vector<int> pts = sample_points(N, op->p.method, op->p.sample_j);
            const int np = (int)pts.size() / 3;
            TS_REQUIRE(np >= mq, TS_EINVAL, "sampling set smaller than the polynomial space");
            if (!lo->fit_pts.p) {
                lo->fit_pts.upload(pts);
                if (op->p.method != TS_LSQP_SYM) {
                    lo->fit_basis.alloc((size_t)np * mq);
                    lo->fit_gram.alloc((size_t)mq * mq);
                    launch_fit_basis(N, q, lo->fit_pts.p, np, lo->fit_basis.p, lo->fit_gram.p,
                                     s);
                }
            }
            SBuf<double> Bv((size_t)M.nt * np * NW, s);
            launch_sample(M, lam, lo->fit_pts.p, np, Bv.p, s);
            if (op->p.method == TS_LSQP_SYM)
                launch_fit_sym(N, q, pts, Bv.p, (int)M.nt, lo->coef64.p, s);
            else
                launch_fit(q, lo->fit_basis.p, np, lo->fit_gram.p, Bv.p, (int)M.nt,
                           lo->coef64.p, s);
        }
    }
    if (cons || sur) {
        const size_t n = lo->coef64.n;
        lo->coef32.alloc(n);
        lo->coef16s.alloc(n);
        lo->d_bad.alloc(1);
        TS_HIP(hipMemsetAsync(lo->d_bad.p, 0, sizeof(int), s));
        launch_coef_variants(lo->coef64.p, (int64_t)n, 1 << lam, lo->coef32.p, lo->coef16s.p,
                             lo->d_bad.p, s);
        if (sur && op->p.face_surrogate) {
            const double* f2sten = face_stencils(M, lam, s);
            const int m2 = (op->p.q + 1) * (op->p.q + 2) / 2;
            lo->fcoef.alloc((size_t)M.nt * 4 * NW * m2);
            launch_face_fit(M.level(lam), f2sten, op->p.q, op->p.sample_j, (int)M.nt,
                            lo->fcoef.p, s);
        }
        if (op->p.fallback_tol > 0) {
            lo->d_flags.alloc((size_t)M.nt);
            launch_fallback_check(M, lam, op->p.q, lo->coef64.p, op->p.fallback_tol,
                                  lo->d_flags.p, s);
        }
    }
    op->lv[lam] = std::move(lo);
}

// One read-back for all levels: the non-finite flags (TS_ENONFINITE) and the
// fallback flags, from which the surrogate and IFEM macro lists are built.
static void finish_levels(ts_op* op, hipStream_t s) {
    const int nt = (int)op->mesh->m.nt;
    std::vector<LevelOp*> los;
    for (auto& kv : op->lv)
        if (kv.second->d_bad.p) los.push_back(kv.second.get());
    std::vector<int> bad(los.size(), 0);
    std::vector<std::vector<unsigned char>> fl(los.size());
    for (size_t a = 0; a < los.size(); a++) {
        TS_HIP(hipMemcpyAsync(&bad[a], los[a]->d_bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        fl[a].assign(nt, 0);
        if (op->p.fallback_tol > 0)
            TS_HIP(hipMemcpyAsync(fl[a].data(), los[a]->d_flags.p, nt, hipMemcpyDeviceToHost, s));
    }
    TS_HIP(hipStreamSynchronize(s));
    for (size_t a = 0; a < los.size(); a++) {
        LevelOp& lo = *los[a];
        TS_REQUIRE(!bad[a], TS_ENONFINITE,
                   op->p.method == TS_CONS ? "non-finite constant stencil"
                                           : "non-finite surrogate coefficient");
        lo.flags.swap(fl[a]);
        std::vector<int> sur, ifem;
        for (int t = 0; t < nt; t++) (lo.flags[t] ? ifem : sur).push_back(t);
        lo.n_sur = (int)sur.size();
        lo.n_ifem = (int)ifem.size();
        if (lo.n_sur) lo.sur_list.upload(sur); else lo.sur_list.reset();
        if (lo.n_ifem) lo.ifem_list.upload(ifem); else lo.ifem_list.reset();
        lo.face_fit = lo.fcoef.p && lo.n_ifem == 0;
        lo.has_coef = true;
    }
}

// every level of the operator, built (or rebuilt) on s; synchronous
static void setup_levels(ts_op* op, hipStream_t s) {
    // with coarse_from_finest the finest level is fitted first: the coarser
    // ones scale its coefficients
    if (op->p.coarse_from_finest) enqueue_level(op, op->max_level, s);
    for (int lam = 2; lam <= op->max_level; lam++)
        if (!(op->p.coarse_from_finest && lam == op->max_level)) enqueue_level(op, lam, s);
    finish_levels(op, s);
}

// Interface Gauss-Seidel values of one phase (sized for the largest phase),
// owned by the operator's level.
static double* iface_tmp(const ts_op* op, int lam) {
    LevelOp& lo = *op->lv.at(lam);
    if (!lo.gs_tmp.p) {
        const Level& L = op->mesh->m.level(lam);
        int mx = 1;
        for (int p = 0; p < N_IF_PHASES; p++) mx = std::max(mx, L.n_f2_phase[p] + L.n_rest_phase[p]);
        lo.gs_tmp.alloc(mx);
    }
    return lo.gs_tmp.p;
}

// levels from which the lower-primitive rows run on the side stream
constexpr int kForkLevel = 6;
// face rows inside the surrogate volume launch (1) or as their own launch (0)
#ifndef TS_FUSE_FACE
#define TS_FUSE_FACE 1
#endif

// y = L x (mode 0) or y = f - L x (mode 1).  The lower-primitive rows and the
// volume rows write disjoint slots, so on large levels the former run on the
// operator's side stream while the volume kernel runs on s.  exact: the
// volume rows take the element-wise IFEM stencils even on surrogate levels.
static void op_rows(const ts_op* op, int lam, int dtype, int mode, const void* x, void* y,
                    const void* f, hipStream_t s, bool exact = false) {
    const bool sur = !exact && uses_surrogate(op, lam);
    // the face rows run inside the surrogate volume launch when it has work
    const bool fuse = TS_FUSE_FACE && sur && op->lv.at(lam)->n_sur > 0;
    const bool fork = lam >= kForkLevel && op->side;
    // stored interface rows are built (once) on s, before either stream reads them
    face_stencils(op->mesh->m, lam, s);
    if (dtype != TS_F64) face_stencils32(op->mesh->m, lam, s);
    if (fork) {
        TS_HIP(hipEventRecord(op->ev_fork, s));
        TS_HIP(hipStreamWaitEvent(op->side, op->ev_fork, 0));
        launch_iface(op, lam, dtype, mode, x, y, f, -1, nullptr, op->side, fuse, exact);
        TS_HIP(hipEventRecord(op->ev_join, op->side));
    } else {
        launch_iface(op, lam, dtype, mode, x, y, f, -1, nullptr, s, fuse, exact);
    }
    if (sur)
        launch_volume(op, lam, dtype, mode, x, y, f, 0, s, fuse);
    else
        launch_ifem_volume(op, lam, dtype == TS_F16W ? TS_F32 : dtype, mode, x, y, f, 0, s);
    if (fork) TS_HIP(hipStreamWaitEvent(s, op->ev_join, 0));
}

static void gs_sweep(const ts_op* op, int lam, int dtype, const void* f, void* u, hipStream_t s) {
    double* tmp = iface_tmp(op, lam);
    const int vd = dtype == TS_F16W ? TS_F32 : dtype;
    for (int p = 0; p < N_IF_PHASES; p++) {
        launch_iface(op, lam, vd, 2, u, u, f, p, tmp, s);
        launch_iface_scatter(op, lam, vd, p, tmp, u, s);
    }
    const bool sur = uses_surrogate(op, lam);
    for (int c = 0; c < 4; c++) {
        if (sur)
            launch_volume(op, lam, dtype, 2, u, u, f, c, s);
        else
            launch_ifem_volume(op, lam, vd, 2, u, u, f, c, s);
    }
}

}  // namespace ts

using namespace ts;

// ------------------------------------------------------------------ solver

struct ts_solver {
    ts_op* op = nullptr;
    int L = 0;
    ts_solve_params p{};
    // per level vectors for the V-cycle, by dtype: 0 FP64, 1 FP32
    std::map<int, std::unique_ptr<DBuf<double>>> f64, u64, r64;
    std::map<int, std::unique_ptr<DBuf<float>>> f32, u32, r32;
    // coarsest level
    int n0 = 0;
    DBuf<double> AinvT, cwork;
    DBuf<int> c_off;
    DBuf<int64_t> c_slot;
    // copies of the coarse free nodes and the free index of every block slot
    // (connectivity only: built once, kept when the vertices change)
    DBuf<int4> c_cp;
    DBuf<int> c_sf;
    // outer iteration
    DBuf<double> r_outer;
    DBuf<float> r_in, e_in;
    DBuf<double> partial, nrm;
    // asynchronous solve: operands, stream, pinned norms ||f||, ||r|| and the
    // event of the last enqueued step
    const double* af = nullptr;
    double* au = nullptr;
    hipStream_t as = nullptr;
    double* hnrm = nullptr;
    hipEvent_t ev = nullptr;
    int state = 0;  // 0 idle, else TS_SOLVE_RUNNING / READY / DONE
    bool have_nf = false;
    double nf = 0.0, prev = 0.0;
    int ups = 0;
    ts_solve_info info{};
    ~ts_solver() {
        if (hnrm) (void)hipHostFree(hnrm);
        if (ev) (void)hipEventDestroy(ev);
    }
};

namespace ts {

template <class X>
static X* vec(std::map<int, std::unique_ptr<DBuf<X>>>& m, int lam, int64_t n) {
    auto& b = m[lam];
    if (!b) {
        b = std::make_unique<DBuf<X>>();
        b->alloc(n);
    }
    return b->p;
}

// the V-cycle vectors of every level below the solver's (restricted
// right-hand side, correction) and of the levels above 2 (residual)
static void alloc_cycle_vectors(ts_solver* sv, int vd) {
    Mesh& M = sv->op->mesh->m;
    for (int lam = sv->L; lam >= 3; lam--) {
        const int64_t nf = M.level(lam).len, nc = M.level(lam - 1).len;
        if (vd == TS_F64) {
            vec(sv->r64, lam, nf);
            vec(sv->f64, lam - 1, nc);
            vec(sv->u64, lam - 1, nc);
        } else {
            vec(sv->r32, lam, nf);
            vec(sv->f32, lam - 1, nc);
            vec(sv->u32, lam - 1, nc);
        }
    }
}

static void coarse_setup(ts_solver* sv, hipStream_t s) {
    Mesh& M = sv->op->mesh->m;
    const int lam = 2;
    Level& L = M.level(lam);
    const int N = L.N;
    if (!sv->c_cp.p) {
        // free nodes: free lower-primitive nodes (canonical order), then the
        // one interior node of every macro
        std::vector<int> off_if(L.n_if + 1);
        std::vector<int4> cp_if(L.if_copy.n);
        std::vector<unsigned char> flag(L.n_if);
        TS_HIP(hipMemcpy(off_if.data(), L.if_off.p, off_if.size() * sizeof(int), hipMemcpyDeviceToHost));
        TS_HIP(hipMemcpy(cp_if.data(), L.if_copy.p, cp_if.size() * sizeof(int4), hipMemcpyDeviceToHost));
        TS_HIP(hipMemcpy(flag.data(), L.if_flag.p, flag.size(), hipMemcpyDeviceToHost));
        std::vector<int> off{0};
        std::vector<int4> cp;
        std::vector<int64_t> slot;
        std::vector<int> slot_free(L.len, -1);
        int n = 0;
        auto add_copy = [&](int4 q) {
            cp.push_back(q);
            const int64_t sl = (int64_t)q.x * L.B + bidx(N, q.y, q.z, q.w);
            slot.push_back(sl);
            slot_free[sl] = n;
        };
        for (int64_t t = 0; t < L.n_if; t++) {
            if (flag[t] & 1) continue;
            for (int c = off_if[t]; c < off_if[t + 1]; c++) add_copy(cp_if[c]);
            n++;
            off.push_back((int)cp.size());
        }
        for (int64_t m = 0; m < M.nt; m++) {
            add_copy(make_int4((int)m, 1, 1, 1));
            n++;
            off.push_back((int)cp.size());
        }
        sv->n0 = n;
        sv->c_off.upload(off);
        sv->c_slot.upload(slot);
        sv->c_sf.upload(slot_free);
        sv->c_cp.upload(cp);
    }
    // the IFEM matrix of the free coarse nodes for the current geometry and
    // its inverse; the temporaries are released in the order of s
    const int n = sv->n0;
    SBuf<double> A((size_t)n * n, s), work((size_t)64 * (n + 64), s);
    TS_HIP(hipMemsetAsync(A.p, 0, (size_t)n * n * sizeof(double), s));
    launch_dense_assemble_cp(M, lam, sv->c_off.p, sv->c_cp.p, n, sv->c_sf.p, A.p, s);
    launch_gj_blocked(A.p, n, work.p, s);
    TS_HIP(hipGetLastError());
    sv->AinvT.alloc((size_t)n * n);
    launch_transpose(A.p, sv->AinvT.p, n, s);
    sv->cwork.alloc((2 + 4 * 16) * (size_t)n);  // fb, ub and the matvec partial sums
}

template <class X>
static void vcycle_t(ts_solver* sv, int lam, int dtype, const X* f, X* u, hipStream_t s,
                     std::map<int, std::unique_ptr<DBuf<X>>>& F,
                     std::map<int, std::unique_ptr<DBuf<X>>>& U,
                     std::map<int, std::unique_ptr<DBuf<X>>>& R) {
    Mesh& M = sv->op->mesh->m;
    const int vd = dtype == TS_F64 ? TS_F64 : TS_F32;
    if (lam == 2) {
        launch_fill(u, vd, M.level(2).len, 0.0, s);
        launch_coarse_solve(sv->AinvT.p, sv->n0, nullptr, sv->c_off.p, sv->c_slot.p, vd, f, u,
                            sv->cwork.p, s);
        return;
    }
    const Level& Lf = M.level(lam);
    const Level& Lc = M.level(lam - 1);
    for (int k = 0; k < sv->p.nu1; k++) gs_sweep(sv->op, lam, dtype, f, u, s);
    X* r = vec(R, lam, Lf.len);
    op_rows(sv->op, lam, dtype, 1, u, r, f, s, sv->p.dd != 0);
    X* fc = vec(F, lam - 1, Lc.len);
    X* uc = vec(U, lam - 1, Lc.len);
    launch_restrict(M, lam, vd, r, fc, s);
    launch_fill(uc, vd, Lc.len, 0.0, s);  // zero initial coarse correction
    vcycle_t<X>(sv, lam - 1, dtype, fc, uc, s, F, U, R);
    launch_prolongate_add(M, lam, vd, uc, u, s);
    for (int k = 0; k < sv->p.nu2; k++) gs_sweep(sv->op, lam, dtype, f, u, s);
}

static void vcycle(ts_solver* sv, int dtype, const void* f, void* u, hipStream_t s) {
    if (dtype == TS_F64)
        vcycle_t<double>(sv, sv->L, dtype, (const double*)f, (double*)u, s, sv->f64, sv->u64, sv->r64);
    else
        vcycle_t<float>(sv, sv->L, dtype, (const float*)f, (float*)u, s, sv->f32, sv->u32, sv->r32);
}

}  // namespace ts

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* ts_last_error(void) { return g_last_error.c_str(); }

int ts_mesh_create(const double* vtx, int64_t nv, const int64_t* tet, int64_t nt, int geom,
                   ts_mesh** out) {
    return guarded([&] {
        TS_REQUIRE(vtx && tet && out && nv >= 4 && nt >= 1, TS_EINVAL, "bad mesh arguments");
        TS_REQUIRE(geom == TS_GEOM_SHELL || geom == TS_GEOM_AFFINE, TS_EINVAL, "bad geometry kind");
        auto* m = new ts_mesh();
        try {
            m->m.nv = nv;
            m->m.nt = nt;
            m->m.geom = geom;
            m->m.vtx.assign(vtx, vtx + 3 * nv);
            m->m.tet.assign(tet, tet + 4 * nt);
            TS_HIP(hipGetDevice(&m->m.device));
            build_topology(m->m);
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

int ts_mesh_check_shell(const ts_mesh* mesh, double r_in, double r_out, double tol) {
    return guarded([&] {
        TS_REQUIRE(mesh, TS_EINVAL, "null mesh");
        TS_REQUIRE(std::isfinite(r_in) && std::isfinite(r_out) && 0.0 < r_in && r_in < r_out,
                   TS_EINVAL, "radii must satisfy 0 < r_in < r_out");
        TS_REQUIRE(tol >= 0.0 && tol < 0.5 * (r_out - r_in), TS_EINVAL, "bad tolerance");
        const Mesh& M = mesh->m;
        auto radius = [&](int64_t v) {
            const double* p = &M.vtx[3 * v];
            return sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        };
        for (int64_t v = 0; v < M.nv; v++) {
            const double r = radius(v);
            if (r < r_in - tol || r > r_out + tol)
                throw Error{TS_EINVAL, "vertex " + std::to_string(v) + " at radius " +
                                           std::to_string(r) + " lies outside the shell"};
        }
        // every face of the mesh boundary (one adjacent macro) lies on one of
        // the two spheres: all three vertices at r_in, or all three at r_out
        for (int64_t f = 0; f < M.nf; f++) {
            if (M.f_tets[f].size() != 1) continue;
            int on_in = 0, on_out = 0;
            for (int a = 0; a < 3; a++) {
                const double r = radius(M.faces[f][a]);
                on_in += fabs(r - r_in) <= tol;
                on_out += fabs(r - r_out) <= tol;
            }
            if (on_in != 3 && on_out != 3)
                throw Error{TS_EINVAL, "boundary face " + std::to_string(f) + " (vertices " +
                                           std::to_string(M.faces[f][0]) + ", " +
                                           std::to_string(M.faces[f][1]) + ", " +
                                           std::to_string(M.faces[f][2]) +
                                           ") does not lie on the sphere r_in or r_out"};
        }
    });
}

int ts_mesh_destroy(ts_mesh* mesh) {
    return guarded([&] { delete mesh; });
}

int ts_mesh_create_like(const ts_mesh* like, const double* vtx, ts_mesh** out) {
    return guarded([&] {
        TS_REQUIRE(like && vtx && out, TS_EINVAL, "null argument");
        const Mesh& A = like->m;
        auto* m = new ts_mesh();
        try {
            Mesh& M = m->m;
            M.nv = A.nv; M.nt = A.nt; M.ne = A.ne; M.nf = A.nf;
            M.geom = A.geom;
            M.vtx.assign(vtx, vtx + 3 * A.nv);
            M.tet = A.tet;
            M.edges = A.edges;
            M.faces = A.faces;
            M.vdir = A.vdir; M.edir = A.edir; M.fdir = A.fdir;
            M.v_tets = A.v_tets; M.e_tets = A.e_tets; M.f_tets = A.f_tets;
            M.topo = A.topo;
            M.device = A.device;
            M.d_topo.alloc(M.topo.size());
            TS_HIP(hipMemcpy(M.d_topo.p, A.d_topo.p, M.topo.size() * sizeof(MacroTopo),
                             hipMemcpyDeviceToDevice));
            build_geometry(M);
            M.levels = A.levels;  // connectivity-only level data, shared
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

int ts_mesh_set_vertices(ts_mesh* mesh, const double* vtx) {
    return guarded([&] {
        TS_REQUIRE(mesh && vtx, TS_EINVAL, "null argument");
        TS_REQUIRE(mesh->ops.load() == 0, TS_EINVAL,
                   "operators created on this mesh must be destroyed first");
        Mesh& M = mesh->m;
        std::vector<double> old(M.vtx);
        M.vtx.assign(vtx, vtx + 3 * M.nv);
        try {
            build_geometry(M);
        } catch (...) {
            M.vtx.swap(old);
            throw;
        }
        M.geo_gen++;  // stored coordinates and interface stencils are rebuilt on use
    });
}

int ts_layout(ts_mesh* mesh, int level, ts_layout_info* out) {
    return guarded([&] {
        TS_REQUIRE(mesh && out, TS_EINVAL, "null argument");
        Level& L = mesh->m.level(level);
        out->level = level;
        out->N = L.N;
        out->n_macros = mesh->m.nt;
        out->block_size = L.B;
        out->vec_len = L.len;
        out->n_unique = L.n_unique;
        out->n_free = L.n_free;
        out->n_volume = mesh->m.nt * (int64_t)(L.N - 1) * (L.N - 2) * (L.N - 3) / 6;
    });
}

int ts_canon_to_block(ts_mesh* mesh, int level, const double* canon, double* block, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(mesh && canon && block, TS_EINVAL, "null argument");
        launch_canon_to_block(mesh->m, level, canon, block, S(s));
    });
}

int ts_block_to_canon(ts_mesh* mesh, int level, const double* block, double* canon, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(mesh && canon && block, TS_EINVAL, "null argument");
        launch_block_to_canon(mesh->m, level, block, canon, S(s));
    });
}

int ts_node_coords(ts_mesh* mesh, int level, double* xyz, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(mesh && xyz, TS_EINVAL, "null argument");
        launch_coords(mesh->m, level, xyz, S(s));
    });
}

int ts_rhs(ts_mesh* mesh, int level, int kind, const double* params, int nparams, double* f,
           ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(mesh && f, TS_EINVAL, "null argument");
        TS_REQUIRE(kind >= 0 && kind <= 2, TS_EINVAL, "bad rhs kind");
        TS_REQUIRE(kind != TS_RHS_MANUFACTURED || (params && nparams >= 2), TS_EINVAL,
                   "manufactured rhs needs {r1, r2}");
        TS_REQUIRE(nparams >= 0 && nparams <= 4096, TS_EINVAL, "bad parameter count");
        for (int i = 0; i < nparams; i++)
            TS_REQUIRE(std::isfinite(params[i]), TS_ENONFINITE, "non-finite rhs parameter");
        std::vector<double> h(params ? params : nullptr, params ? params + nparams : nullptr);
        if (h.empty()) h.push_back(0.0);
        SBuf<double> d(h, S(s));
        launch_rhs(mesh->m, level, kind, d.p, nparams, f, S(s));
        TS_HIP(hipStreamSynchronize(S(s)));
    });
}

int ts_op_create(ts_mesh* mesh, int max_level, const ts_op_params* p, ts_stream s, ts_op** out) {
    return guarded([&] {
        TS_REQUIRE(mesh && p && out, TS_EINVAL, "null argument");
        TS_REQUIRE(max_level >= 2 && max_level <= 9, TS_EINVAL, "max_level must be in 2..9");
        TS_REQUIRE(p->method == TS_IFEM || p->method == TS_LSQP || p->method == TS_IPOLY ||
                       p->method == TS_LSQP_SYM || p->method == TS_CONS,
                   TS_EINVAL, "bad method");
        if (p->method == TS_CONS) {
            TS_REQUIRE(p->center == TS_CENTER_POLY || p->center == TS_CENTER_ROWSUM, TS_EINVAL,
                       "bad centre mode");
            TS_REQUIRE(!p->face_surrogate && !(p->fallback_tol > 0), TS_EINVAL,
                       "the constant stencil takes no face surrogate and no fallback check");
        } else if (p->method != TS_IFEM) {
            TS_REQUIRE(p->q >= 1 && p->q <= 4, TS_EINVAL, "degree q must be in 1..4");
            TS_REQUIRE(p->method != TS_IPOLY || p->q == 2, TS_EINVAL, "IPOLY is defined for q = 2");
            TS_REQUIRE(p->center == TS_CENTER_POLY || p->center == TS_CENTER_ROWSUM, TS_EINVAL,
                       "bad centre mode");
            TS_REQUIRE(!std::isnan(p->fallback_tol), TS_EINVAL, "fallback_tol is NaN");
            // the symmetric surrogate's node coefficients carry a shift of
            // half a mesh step, different on every level
            TS_REQUIRE(!(p->coarse_from_finest && p->method == TS_LSQP_SYM), TS_EINVAL,
                       "coarse_from_finest is defined for TS_LSQP and TS_IPOLY");
        }
        auto* op = new ts_op();
        try {
            op->mesh = mesh;
            op->p = *p;
            // the symmetric surrogate defines the centre weight by the row sum
            if (p->method == TS_LSQP_SYM) op->p.center = TS_CENTER_ROWSUM;
            op->max_level = max_level;
            if (p->method == TS_CONS) op->p.q = 0;  // degree-0 "polynomials"
            if (p->method == TS_IFEM || p->method == TS_CONS) op->p.coarse_from_finest = 0;
            op->mq = p->method == TS_IFEM ? 0 : mq_of(op->p.q);
            setup_levels(op, S(s));
            TS_HIP(hipStreamCreateWithFlags(&op->side, hipStreamNonBlocking));
            TS_HIP(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming));
            TS_HIP(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming));
        } catch (...) {
            delete op;
            throw;
        }
        mesh->ops++;
        *out = op;
    });
}

int ts_op_destroy(ts_op* op) {
    return guarded([&] {
        if (op && op->mesh) op->mesh->ops--;
        delete op;
    });
}

int ts_op_coeffs_export(ts_op* op, int level, double* host, size_t n) {
    return guarded([&] {
        TS_REQUIRE(op && host, TS_EINVAL, "null argument");
        TS_REQUIRE(uses_surrogate(op, level), TS_EINVAL, "no surrogate coefficients on this level");
        const size_t need = (size_t)op->mesh->m.nt * NW * op->mq;
        TS_REQUIRE(n >= need, TS_EINVAL, "buffer too small");
        TS_HIP(hipMemcpy(host, op->lv[level]->coef64.p, need * sizeof(double), hipMemcpyDeviceToHost));
    });
}

int ts_op_coeffs_import(ts_op* op, int level, const double* host, size_t n) {
    return guarded([&] {
        TS_REQUIRE(op && host, TS_EINVAL, "null argument");
        TS_REQUIRE(uses_surrogate(op, level), TS_EINVAL, "no surrogate coefficients on this level");
        const size_t need = (size_t)op->mesh->m.nt * NW * op->mq;
        TS_REQUIRE(n == need, TS_EINVAL, "coefficient count mismatch");
        std::vector<double> h(host, host + need);
        for (double v : h) TS_REQUIRE(std::isfinite(v), TS_ENONFINITE, "non-finite coefficient");
        LevelOp& lo = *op->lv[level];
        TS_HIP(hipMemcpy(lo.coef64.p, h.data(), need * sizeof(double), hipMemcpyHostToDevice));
        upload_coef_variants(op, lo, level, h);
        split_macros(op, lo, level, nullptr);
    });
}

int ts_op_macro_flags(ts_op* op, int level, unsigned char* host, size_t n) {
    return guarded([&] {
        TS_REQUIRE(op && host, TS_EINVAL, "null argument");
        TS_REQUIRE(level >= 2 && level <= op->max_level, TS_EINVAL,
                   "level outside the operator's range");
        const int64_t nt = op->mesh->m.nt;
        TS_REQUIRE(n >= (size_t)nt, TS_EINVAL, "buffer too small");
        const LevelOp& lo = *op->lv.at(level);
        for (int64_t t = 0; t < nt; t++)
            host[t] = uses_surrogate(op, level) && !lo.flags.empty() ? lo.flags[t] : 0;
    });
}

static void check_level(ts_op* op, int level) {
    TS_REQUIRE(op, TS_EINVAL, "null operator");
    TS_REQUIRE(level >= 2 && level <= op->max_level, TS_EINVAL, "level outside the operator's range");
}
static void check_dtype(int dt) {
    TS_REQUIRE(dt == TS_F64 || dt == TS_F32 || dt == TS_F16W, TS_EINVAL, "bad dtype");
}

int ts_apply(ts_op* op, int level, int dtype, const void* x, void* y, ts_stream s) {
    return guarded([&] {
        check_level(op, level);
        check_dtype(dtype);
        TS_REQUIRE(x && y && x != y, TS_EINVAL, "x and y must be distinct device vectors");
        op_rows(op, level, dtype, 0, x, y, nullptr, S(s));
    });
}

int ts_apply_volume(ts_op* op, int level, int dtype, const void* x, void* y, ts_stream s) {
    return guarded([&] {
        check_level(op, level);
        check_dtype(dtype);
        TS_REQUIRE(x && y && x != y, TS_EINVAL, "x and y must be distinct device vectors");
        if (uses_surrogate(op, level))
            launch_volume(op, level, dtype, 0, x, y, nullptr, 0, S(s));
        else
            launch_ifem_volume(op, level, dtype == TS_F16W ? TS_F32 : dtype, 0, x, y, nullptr, 0, S(s));
    });
}

int ts_residual(ts_op* op, int level, int dtype, const void* f, const void* u, void* r, ts_stream s) {
    return guarded([&] {
        check_level(op, level);
        check_dtype(dtype);
        TS_REQUIRE(f && u && r && r != u && r != f, TS_EINVAL, "bad vectors");
        op_rows(op, level, dtype, 1, u, r, f, S(s));
    });
}

int ts_smooth(ts_op* op, int level, int dtype, const void* f, void* u, int sweeps, ts_stream s) {
    return guarded([&] {
        check_level(op, level);
        check_dtype(dtype);
        TS_REQUIRE(f && u && f != u && sweeps >= 0, TS_EINVAL, "bad arguments");
        for (int k = 0; k < sweeps; k++) gs_sweep(op, level, dtype, f, u, S(s));
    });
}

int ts_restrict(ts_op* op, int level, int dtype, const void* rf, void* rc, ts_stream s) {
    return guarded([&] {
        check_level(op, level);
        TS_REQUIRE(level >= 3, TS_EINVAL, "no coarser level");
        check_dtype(dtype);
        launch_restrict(op->mesh->m, level, dtype == TS_F64 ? TS_F64 : TS_F32, rf, rc, S(s));
    });
}

int ts_prolongate_add(ts_op* op, int level, int dtype, const void* uc, void* uf, ts_stream s) {
    return guarded([&] {
        check_level(op, level);
        TS_REQUIRE(level >= 3, TS_EINVAL, "no coarser level");
        check_dtype(dtype);
        launch_prolongate_add(op->mesh->m, level, dtype == TS_F64 ? TS_F64 : TS_F32, uc, uf, S(s));
    });
}

int ts_norm2(ts_mesh* mesh, int level, int dtype, const void* x, double* out, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(mesh && x && out, TS_EINVAL, "null argument");
        check_dtype(dtype);
        SBuf<double> part(norm_partial_count(mesh->m, level), S(s)), r(1, S(s));
        launch_norm2_free(mesh->m, level, dtype == TS_F64 ? TS_F64 : TS_F32, x, part.p, r.p, S(s));
        TS_HIP(hipMemcpyAsync(out, r.p, sizeof(double), hipMemcpyDeviceToHost, S(s)));
        TS_HIP(hipStreamSynchronize(S(s)));
    });
}

int ts_norm2_noalloc(ts_mesh* mesh, int level, int dtype, const void* x, double* out,
                     ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(mesh && x && out, TS_EINVAL, "null argument");
        check_dtype(dtype);
        norm2_noalloc(mesh->m, level, dtype == TS_F64 ? TS_F64 : TS_F32, x, out, S(s));
    });
}

namespace ts {

// element-wise volume rows stop at level 8: a solve above it must keep
// surrogate rows everywhere and take no exact residuals
static void check_exact_rows(const ts_op* op, int level, bool dd) {
    for (int lam = 9; lam <= level; lam++) {
        TS_REQUIRE(!dd, TS_EINVAL, "double discretisation needs IFEM rows: level 8 at most");
        TS_REQUIRE(uses_surrogate(op, lam) && op->lv.at(lam)->n_ifem == 0, TS_EINVAL,
                   "IFEM volume rows (method or selective surrogate) are supported up to level 8");
    }
}

// the solver's geometry-dependent data on s: the coarse inverse, and the
// stored rows, coordinates and Gauss-Seidel scratch of every level the cycle
// visits (built now rather than in a step); synchronous
static void solver_geometry(ts_solver* sv, hipStream_t s) {
    ts_op* op = sv->op;
    coarse_setup(sv, s);
    for (int lam = 3; lam <= sv->L; lam++) {
        const bool ifem = sv->p.dd || !uses_surrogate(op, lam) || op->lv.at(lam)->n_ifem > 0;
        warm_level(op, lam, ifem, s);
        if (sv->p.precision != TS_F64) face_stencils32(op->mesh->m, lam, s);
        iface_tmp(op, lam);
    }
    TS_HIP(hipStreamSynchronize(s));
}

}  // namespace ts

int ts_solver_create(ts_op* op, int level, const ts_solve_params* p, ts_solver** out) {
    return guarded([&] {
        check_level(op, level);
        TS_REQUIRE(p && out, TS_EINVAL, "null argument");
        TS_REQUIRE(level >= 3, TS_EINVAL, "the solver needs at least one level above level 2");
        TS_REQUIRE(p->nu1 >= 0 && p->nu2 >= 0 && p->nu1 + p->nu2 > 0, TS_EINVAL, "bad smoothing counts");
        TS_REQUIRE(p->max_cycles > 0 && p->max_cycles < TS_MAX_HIST - 1, TS_EINVAL, "bad max_cycles");
        TS_REQUIRE(p->rtol > 0, TS_EINVAL, "rtol must be positive");
        check_dtype(p->precision);
        TS_REQUIRE(!p->dd || p->precision == TS_F64, TS_EINVAL,
                   "double discretisation runs in FP64 precision");
        check_exact_rows(op, level, p->dd);
        auto* sv = new ts_solver();
        try {
            sv->op = op;
            sv->L = level;
            sv->p = *p;
            if (sv->p.diverge_window <= 0) sv->p.diverge_window = 3;
            // set-up work runs on a private stream, so that it does not order
            // against other work on the device
            hipStream_t s = nullptr;
            TS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            try {
                solver_geometry(sv, s);
            } catch (...) {
                (void)hipStreamDestroy(s);
                throw;
            }
            TS_HIP(hipStreamDestroy(s));
            Mesh& M = op->mesh->m;
            sv->partial.alloc(norm_partial_count(M, level));
            sv->nrm.alloc(3);
            // every vector a solve step uses is allocated here, so that a step
            // never allocates (and cannot fail part-way on memory)
            alloc_cycle_vectors(sv, p->precision == TS_F64 ? TS_F64 : TS_F32);
            sv->r_outer.alloc(M.level(level).len);
            if (p->precision != TS_F64) {
                sv->r_in.alloc(M.level(level).len);
                sv->e_in.alloc(M.level(level).len);
            }
            TS_HIP(hipHostMalloc((void**)&sv->hnrm, 3 * sizeof(double), hipHostMallocDefault));
            TS_HIP(hipEventCreateWithFlags(&sv->ev, hipEventDisableTiming));
        } catch (...) {
            delete sv;
            throw;
        }
        *out = sv;
    });
}

int ts_solver_destroy(ts_solver* sv) {
    return guarded([&] { delete sv; });
}

int ts_solver_set_vertices(ts_solver* sv, const double* vtx, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(sv && vtx, TS_EINVAL, "null argument");
        TS_REQUIRE(sv->state == 0 || sv->state == TS_SOLVE_DONE, TS_EINVAL,
                   "a solve is in progress");
        ts_op* op = sv->op;
        ts_mesh* mesh = op->mesh;
        TS_REQUIRE(mesh->ops.load() == 1, TS_EINVAL,
                   "the mesh carries other operators than the solver's");
        Mesh& M = mesh->m;
        for (int64_t i = 0; i < 3 * M.nv; i++)
            TS_REQUIRE(std::isfinite(vtx[i]), TS_ENONFINITE, "non-finite vertex coordinate");
        std::vector<double> old(M.vtx);
        M.vtx.assign(vtx, vtx + 3 * M.nv);
        try {
            build_geometry(M);
        } catch (...) {
            M.vtx.swap(old);
            throw;
        }
        M.geo_gen++;  // stored coordinates and interface rows are rebuilt on use
        sv->state = 0;
        setup_levels(op, S(s));
        check_exact_rows(op, sv->L, sv->p.dd);
        solver_geometry(sv, S(s));
    });
}

int ts_vcycle(ts_solver* sv, int dtype, const void* f, void* u, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(sv && f && u && f != u, TS_EINVAL, "bad arguments");
        check_dtype(dtype);
        vcycle(sv, dtype, f, u, S(s));
    });
}

}  // extern "C"

namespace ts {

// residual r = f - L u on the finest level in FP64 and its norm into nrm[1]
static void outer_residual(ts_solver* sv, hipStream_t st) {
    Mesh& M = sv->op->mesh->m;
    op_rows(sv->op, sv->L, TS_F64, 1, sv->au, sv->r_outer.p, sv->af, st);
    launch_norm2_free(M, sv->L, TS_F64, sv->r_outer.p, sv->partial.p, sv->nrm.p + 1, st);
}

static void solve_begin(ts_solver* sv, const double* f, double* u, hipStream_t st) {
    Mesh& M = sv->op->mesh->m;
    const Level& L = M.level(sv->L);
    TS_REQUIRE(sv->state == 0 || sv->state == TS_SOLVE_DONE, TS_EINVAL,
               "a solve is already in progress on this solver");
    if (!sv->r_outer.p) sv->r_outer.alloc(L.len);
    if (sv->p.precision != TS_F64 && !sv->r_in.p) {
        sv->r_in.alloc(L.len);
        sv->e_in.alloc(L.len);
    }
    sv->af = f;
    sv->au = u;
    sv->as = st;
    sv->have_nf = false;
    sv->ups = 0;
    memset(&sv->info, 0, sizeof(sv->info));
    launch_norm2_free(M, sv->L, TS_F64, f, sv->partial.p, sv->nrm.p, st);
    if (!sv->p.dd) outer_residual(sv, st);
    TS_HIP(hipMemcpyAsync(sv->hnrm, sv->nrm.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    TS_HIP(hipEventRecord(sv->ev, st));
    sv->state = TS_SOLVE_RUNNING;
}

// one outer iteration: FP64 V-cycle on u, or a V-cycle on the rounded
// residual in FP32 / FP16-weight arithmetic added to u; then the new residual.
// Double discretisation: the cycle on u, then the norms of the update
// (u_prev - u, kept in r_outer) and of u.
static void solve_step(ts_solver* sv) {
    TS_REQUIRE(sv->state == TS_SOLVE_READY, TS_EINVAL, "the solver is not ready for a step");
    Mesh& M = sv->op->mesh->m;
    const Level& L = M.level(sv->L);
    hipStream_t st = sv->as;
    const int prec = sv->p.precision;
    if (sv->p.dd) {
        TS_HIP(hipMemcpyAsync(sv->r_outer.p, sv->au, (size_t)L.len * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
        vcycle(sv, TS_F64, sv->af, sv->au, st);
        launch_axpy(-1.0, sv->au, TS_F64, sv->r_outer.p, L.len, st);
        sv->info.cycles++;
        launch_norm2_free(M, sv->L, TS_F64, sv->r_outer.p, sv->partial.p, sv->nrm.p + 1, st);
        launch_norm2_free(M, sv->L, TS_F64, sv->au, sv->partial.p, sv->nrm.p + 2, st);
        TS_HIP(hipMemcpyAsync(sv->hnrm + 1, sv->nrm.p + 1, 2 * sizeof(double),
                              hipMemcpyDeviceToHost, st));
        TS_HIP(hipEventRecord(sv->ev, st));
        sv->state = TS_SOLVE_RUNNING;
        return;
    }
    if (prec == TS_F64) {
        vcycle(sv, TS_F64, sv->af, sv->au, st);
    } else {
        launch_cast(sv->r_outer.p, TS_F64, sv->r_in.p, TS_F32, L.len, st);
        launch_fill(sv->e_in.p, TS_F32, L.len, 0.0, st);
        vcycle(sv, prec, sv->r_in.p, sv->e_in.p, st);
        launch_axpy(1.0, sv->e_in.p, TS_F32, sv->au, L.len, st);
    }
    sv->info.cycles++;
    outer_residual(sv, st);
    TS_HIP(hipMemcpyAsync(sv->hnrm + 1, sv->nrm.p + 1, sizeof(double), hipMemcpyDeviceToHost, st));
    TS_HIP(hipEventRecord(sv->ev, st));
    sv->state = TS_SOLVE_RUNNING;
}

// after the last enqueued step finished: read its norms and decide
static void solve_advance(ts_solver* sv) {
    ts_solve_info& I = sv->info;
    auto finish = [&](int status) {
        I.status = status;
        sv->state = TS_SOLVE_DONE;
    };
    if (!sv->have_nf) {
        sv->have_nf = true;
        sv->nf = sv->hnrm[0];
        if (!std::isfinite(sv->nf)) return finish(TS_ENONFINITE);
        if (sv->nf == 0.0) {  // f = 0: the solution is 0
            const Level& L = sv->op->mesh->m.level(sv->L);
            launch_fill(sv->au, TS_F64, L.len, 0.0, sv->as);
            TS_HIP(hipEventRecord(sv->ev, sv->as));
            I.rel_residual = 0.0;
            return finish(TS_OK);
        }
    }
    if (sv->p.dd && I.cycles == 0) {  // nothing to test before the first cycle
        sv->state = TS_SOLVE_READY;
        return;
    }
    const double rel = !sv->p.dd ? sv->hnrm[1] / sv->nf
                       : sv->hnrm[2] > 0.0 ? sv->hnrm[1] / sv->hnrm[2] : 0.0;
    I.rel_residual = rel;
    if (I.n_hist < TS_MAX_HIST) I.hist[I.n_hist++] = rel;
    if (!std::isfinite(rel)) return finish(TS_ENONFINITE);
    if (rel <= sv->p.rtol) return finish(TS_OK);
    if (I.cycles > (sv->p.dd ? 1 : 0)) {
        sv->ups = rel > sv->prev ? sv->ups + 1 : 0;
        if (sv->ups >= sv->p.diverge_window) return finish(TS_ENOCONV);
    }
    sv->prev = rel;
    if (I.cycles >= sv->p.max_cycles) return finish(TS_ENOCONV);
    sv->state = TS_SOLVE_READY;
}

static int solve_query(ts_solver* sv) {
    if (sv->state == TS_SOLVE_RUNNING) {
        const hipError_t e = hipEventQuery(sv->ev);
        if (e == hipErrorNotReady) return TS_SOLVE_RUNNING;
        TS_HIP(e);
        solve_advance(sv);
    }
    return sv->state;
}

}  // namespace ts

extern "C" {

int ts_device_bytes(int64_t* bytes) {
    return guarded([&] {
        TS_REQUIRE(bytes, TS_EINVAL, "null argument");
        *bytes = g_dev_bytes.load();
    });
}

int ts_solve_begin(ts_solver* sv, const double* f, double* u, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(sv && f && u && (const void*)f != (const void*)u, TS_EINVAL, "bad arguments");
        solve_begin(sv, f, u, S(s));
    });
}

// A step that fails part-way (a HIP error while enqueuing) leaves part of a
// cycle applied to u: the solve ends there, DONE with the error's status.
static void step_or_finish(ts_solver* sv) {
    try {
        solve_step(sv);
    } catch (const Error& e) {
        if (sv->state == TS_SOLVE_READY) {
            sv->info.status = e.code;
            sv->state = TS_SOLVE_DONE;
        }
        throw;
    }
}

int ts_solve_step(ts_solver* sv) {
    return guarded([&] {
        TS_REQUIRE(sv, TS_EINVAL, "null solver");
        TS_REQUIRE(sv->state == TS_SOLVE_READY, TS_EINVAL, "the solver is not ready for a step");
        step_or_finish(sv);
    });
}

int ts_solve_batch_step(ts_solver* const* v, int n) {
    return guarded([&] {
        TS_REQUIRE(n >= 0 && (n == 0 || v), TS_EINVAL, "bad arguments");
        std::vector<const ts_solver*> seen(v, v + n);
        std::sort(seen.begin(), seen.end());
        TS_REQUIRE(std::adjacent_find(seen.begin(), seen.end()) == seen.end(), TS_EINVAL,
                   "a solver appears twice in the batch");
        for (int a = 0; a < n; a++) {
            TS_REQUIRE(v[a], TS_EINVAL, "null solver in the batch");
            TS_REQUIRE(v[a]->state == TS_SOLVE_READY, TS_EINVAL,
                       "a solver in the batch is not ready for a step");
        }
        for (int a = 0; a < n; a++) step_or_finish(v[a]);
    });
}

int ts_solve_query(ts_solver* sv, int* state, ts_solve_info* info) {
    return guarded([&] {
        TS_REQUIRE(sv && state, TS_EINVAL, "null argument");
        TS_REQUIRE(sv->state != 0, TS_EINVAL, "no solve was started on this solver");
        *state = solve_query(sv);
        if (info) *info = sv->info;
    });
}

int ts_solve(ts_solver* sv, const double* f, double* u, ts_solve_info* info, ts_stream s) {
    return guarded([&] {
        TS_REQUIRE(sv && f && u && info, TS_EINVAL, "null argument");
        solve_begin(sv, f, u, S(s));
        for (;;) {
            TS_HIP(hipEventSynchronize(sv->ev));
            const int st = solve_query(sv);
            if (st == TS_SOLVE_DONE) break;
            step_or_finish(sv);
        }
        TS_HIP(hipEventSynchronize(sv->ev));
        *info = sv->info;
        const int status = sv->info.status;
        if (status != TS_OK)
            throw Error{status, status == TS_ENONFINITE ? "right-hand side or iterate is not finite"
                                                        : "no convergence to the tolerance"};
    });
}

}  // extern "C"
