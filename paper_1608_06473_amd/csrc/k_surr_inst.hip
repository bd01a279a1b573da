// Instantiation unit of the surrogate volume kernel for one polynomial degree
// TS_Q and one staging width TS_KPT (compiled once per pair, in parallel).
#include <algorithm>

#include "ts_surrogate.h"

#ifndef TS_Q
#error "TS_Q must be defined"
#endif
#ifndef TS_KPT
#error "TS_KPT must be defined"
#endif

#define TS_CAT2(a, b, c, d) a##b##c##d
#define TS_CAT(a, b, c, d) TS_CAT2(a, b, c, d)

namespace ts {

template <class WP, typename T, typename W>
static void run(const Level& L, int nt, const int* ml, const float* cf, const double* cd,
                int mode, const void* x, void* y, const void* f, int colour, hipStream_t s,
                const void* f2sten_v, const double* f2coef) {
    // the stored face rows come in the vector type
    const T* f2sten = (const T*)f2sten_v;
    const dim3 grid((unsigned)(((nt + 7) / 8) * 8 * L.n_lds_tiles)), blk(VOL_THREADS);
    if (grid.x == 0 || L.n_lds_tiles == 0) return;
    const T* xp = (const T*)x;
    T* yp = (T*)y;
    const T* fp = (const T*)f;
    // fused face rows (apply / residual): per XCD, groups of two volume
    // workgroups and one face workgroup
    const int n2 = f2sten ? L.n_f2 : 0;
    dim3 gf = grid;
    if (n2 > 0) {
        const int64_t vper = grid.x / 8, fper = ((n2 + VOL_THREADS - 1) / VOL_THREADS + 7) / 8;
        const int64_t groups = std::max((vper + 1) / 2, fper);
        gf = dim3((unsigned)(groups * 3 * 8));
    }
#define TS_GO(M_, FF_)                                                                        \
    k_surr_lds<WP, T, W, M_, VOL_R, TS_KPT, FF_><<<gf, blk, 0, s>>>(                          \
        xp, yp, fp, cf, cd, L.lds_tiles.p, L.n_lds_tiles, nt, ml, L.ap_lanes.p,               \
        L.stage_tbl.p, L.N, L.B, colour, L.f2_cp.p, f2sten, f2coef, n2)
    const bool ff = n2 > 0 && f2coef;
    if (mode == 0) {
        if (ff) TS_GO(0, true); else TS_GO(0, false);
    } else if (mode == 1) {
        if (ff) TS_GO(1, true); else TS_GO(1, false);
    } else
        k_surr_lds<WP, T, W, 2, VOL_R, TS_KPT><<<grid, blk, 0, s>>>(yp, yp, fp, cf, cd, L.lds_tiles.p, L.n_lds_tiles, nt, ml, L.gs_lanes.p, L.stage_tbl.p, L.N, L.B, colour);
#undef TS_GO
}

// dtype TS_F64: FP64 vectors and weights; TS_F32: FP32; TS_F16W: FP32 vectors
// with FP16 weight evaluation (coefficients pre-scaled by N)
void TS_CAT(launch_surr_q, TS_Q, _k, TS_KPT)(const Level& L, int nt, const LevelOp& lo, int dtype,
                                              int center, int mode, const void* x, void* y,
                                              const void* f, int colour, hipStream_t s,
                                              const void* f2sten, const double* f2coef) {
    constexpr int Q = TS_Q;
    const int* ml = lo.sur_list.p;
    nt = lo.n_sur;
    if (dtype == TS_F64) {
        if (center == TS_CENTER_POLY)
            run<SurrogateW<Q, double, TS_CENTER_POLY>, double, double>(L, nt, ml, nullptr, lo.coef64.p, mode, x, y, f, colour, s, f2sten, f2coef);
        else
            run<SurrogateW<Q, double, TS_CENTER_ROWSUM>, double, double>(L, nt, ml, nullptr, lo.coef64.p, mode, x, y, f, colour, s, f2sten, f2coef);
    } else if (dtype == TS_F32) {
        if (center == TS_CENTER_POLY)
            run<SurrogateW<Q, float, TS_CENTER_POLY>, float, float>(L, nt, ml, lo.coef32.p, nullptr, mode, x, y, f, colour, s, f2sten, f2coef);
        else
            run<SurrogateW<Q, float, TS_CENTER_ROWSUM>, float, float>(L, nt, ml, lo.coef32.p, nullptr, mode, x, y, f, colour, s, f2sten, f2coef);
    } else {
        run<SurrogateHalfW<Q>, float, float>(L, nt, ml, lo.coef16s.p, nullptr, mode, x, y, f, colour, s, f2sten, f2coef);
    }
}

}  // namespace ts
