// Host side: macro-mesh topology (edges, faces, incidence, Dirichlet flags)
// and the per-level layout (lower-primitive copy maps, GS phase lists and
// volume tiles).  Sec. 2.3: nodes are grouped into vertex, edge, face and
// volume primitives; lower primitives keep element-wise assembly.
#include <math.h>

#include <algorithm>
#include <numeric>

#include "ts_internal.h"

namespace ts {

namespace {

const int EDGE_LOC[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

template <size_t K>
int64_t find_sorted(const std::vector<std::array<int64_t, K>>& v, std::array<int64_t, K> key) {
    auto it = std::lower_bound(v.begin(), v.end(), key);
    if (it == v.end() || *it != key) return -1;
    return it - v.begin();
}

}  // namespace

void build_topology(Mesh& M) {
    const int64_t nt = M.nt, nv = M.nv;
    for (int64_t i = 0; i < 4 * nt; i++)
        TS_REQUIRE(M.tet[i] >= 0 && M.tet[i] < nv, TS_EINVAL, "tetrahedron vertex id out of range");
    // edges and faces as sorted id tuples
    std::vector<std::array<int64_t, 2>> E;
    std::vector<std::array<int64_t, 3>> F;
    E.reserve(6 * nt);
    F.reserve(4 * nt);
    for (int64_t t = 0; t < nt; t++) {
        const int64_t* g = &M.tet[4 * t];
        for (int a = 0; a < 4; a++)
            for (int b = a + 1; b < 4; b++) {
                TS_REQUIRE(g[a] != g[b], TS_EINVAL, "repeated vertex in a tetrahedron");
                E.push_back({std::min(g[a], g[b]), std::max(g[a], g[b])});
            }
        for (int o = 0; o < 4; o++) {
            std::array<int64_t, 3> f;
            int c = 0;
            for (int a = 0; a < 4; a++)
                if (a != o) f[c++] = g[a];
            std::sort(f.begin(), f.end());
            F.push_back(f);
        }
    }
    std::sort(E.begin(), E.end());
    E.erase(std::unique(E.begin(), E.end()), E.end());
    std::sort(F.begin(), F.end());
    F.erase(std::unique(F.begin(), F.end()), F.end());
    M.edges = E;
    M.faces = F;
    M.ne = E.size();
    M.nf = F.size();
    M.v_tets.assign(nv, {});
    M.e_tets.assign(M.ne, {});
    M.f_tets.assign(M.nf, {});
    M.topo.assign(nt, MacroTopo{});
    for (int64_t t = 0; t < nt; t++) {
        const int64_t* g = &M.tet[4 * t];
        MacroTopo& T = M.topo[t];
        for (int a = 0; a < 4; a++) {
            T.vg[a] = g[a];
            M.v_tets[g[a]].push_back(t);
        }
        for (int e = 0; e < 6; e++) {
            int a = EDGE_LOC[e][0], b = EDGE_LOC[e][1];
            T.e[e] = find_sorted(E, {std::min(g[a], g[b]), std::max(g[a], g[b])});
            T.ehi[e] = (signed char)(g[a] > g[b] ? a : b);
            T.elo[e] = (signed char)(g[a] > g[b] ? b : a);
            M.e_tets[T.e[e]].push_back(t);
        }
        for (int o = 0; o < 4; o++) {
            int loc[3], c = 0;
            for (int a = 0; a < 4; a++)
                if (a != o) loc[c++] = a;
            std::sort(loc, loc + 3, [&](int x, int y) { return g[x] < g[y]; });
            std::array<int64_t, 3> key = {g[loc[0]], g[loc[1]], g[loc[2]]};
            T.f[o] = find_sorted(F, key);
            for (int q = 0; q < 3; q++) T.fs[o][q] = (signed char)loc[q];
            M.f_tets[T.f[o]].push_back(t);
        }
    }
    for (int64_t f = 0; f < M.nf; f++)
        TS_REQUIRE(M.f_tets[f].size() <= 2, TS_EINVAL, "a face is shared by more than two macros");
    // Dirichlet: all primitives of boundary faces (faces of one macro)
    M.vdir.assign(nv, 0);
    M.edir.assign(M.ne, 0);
    M.fdir.assign(M.nf, 0);
    for (int64_t f = 0; f < M.nf; f++) {
        if (M.f_tets[f].size() != 1) continue;
        const auto& k = F[f];
        M.fdir[f] = 1;
        for (int a = 0; a < 3; a++) M.vdir[k[a]] = 1;
        M.edir[find_sorted(E, {k[0], k[1]})] = 1;
        M.edir[find_sorted(E, {k[0], k[2]})] = 1;
        M.edir[find_sorted(E, {k[1], k[2]})] = 1;
    }
    // per-macro flags and multiplicities
    for (int64_t t = 0; t < nt; t++) {
        MacroTopo& T = M.topo[t];
        for (int a = 0; a < 4; a++) T.vdir[a] = M.vdir[T.vg[a]];
        for (int e = 0; e < 6; e++) {
            T.edir[e] = M.edir[T.e[e]];
            T.emult[e] = (unsigned char)std::min<size_t>(255, M.e_tets[T.e[e]].size());
        }
        for (int o = 0; o < 4; o++) {
            T.fdir[o] = M.fdir[T.f[o]];
            T.fmult[o] = (unsigned char)M.f_tets[T.f[o]].size();
        }
    }
    M.d_topo.upload(M.topo);
    build_geometry(M);
}

void build_geometry(Mesh& M) {
    const int64_t nt = M.nt;
    std::vector<MacroGeom> gh(nt, MacroGeom{});
    for (int64_t t = 0; t < nt; t++) {
        MacroGeom& G = gh[t];
        const int64_t* g = &M.tet[4 * t];
        for (int a = 0; a < 4; a++) {
            double r2 = 0;
            for (int d = 0; d < 3; d++) {
                G.v[a][d] = M.vtx[3 * g[a] + d];
                r2 += G.v[a][d] * G.v[a][d];
            }
            G.r[a] = sqrt(r2);
            G.ord[a] = a;
        }
        std::sort(G.ord, G.ord + 4, [&](int x, int y) { return g[x] < g[y]; });
        G.affine = M.geom == TS_GEOM_AFFINE ? 1 : 0;
        // degenerate macro check
        double e1[3], e2[3], e3[3];
        for (int d = 0; d < 3; d++) {
            e1[d] = G.v[1][d] - G.v[0][d];
            e2[d] = G.v[2][d] - G.v[0][d];
            e3[d] = G.v[3][d] - G.v[0][d];
        }
        double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                     e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
        // relative to the cube of its longest edge from vertex 0: flat (or
        // nearly flat) macros are refused
        double l2 = 0.0;
        for (const double* e : {e1, e2, e3})
            l2 = std::max(l2, e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        TS_REQUIRE(std::isfinite(det) && fabs(det) > 1e-12 * l2 * sqrt(l2), TS_EINVAL,
                   "degenerate macro tetrahedron");
    }
    M.geomh.swap(gh);
    if (M.d_geom.p && M.d_geom.n == M.geomh.size())
        TS_HIP(hipMemcpy(M.d_geom.p, M.geomh.data(), M.geomh.size() * sizeof(MacroGeom),
                         hipMemcpyHostToDevice));
    else
        M.d_geom.upload(M.geomh);
}

Level& Mesh::level(int lam) {
    auto it = levels.find(lam);
    if (it != levels.end()) return *it->second;
    TS_REQUIRE(lam >= 2 && lam <= 9, TS_EINVAL, "level must be in 2..9");
    auto L = std::make_shared<Level>();
    const int N = 1 << lam;
    L->lam = lam;
    L->N = N;
    L->B = block_size(N);
    L->len = nt * L->B;
    L->n_unique = num_unique(N);

    // lower-primitive nodes in canonical order with their copies
    const int64_t nF = (int64_t)(N - 1) * (N - 2) / 2;
    const int64_t n_if = nv + ne * (N - 1) + nf * nF;
    TS_REQUIRE(n_if < (int64_t)1 << 31, TS_EINVAL, "too many interface nodes for this level");
    std::vector<int> off;
    std::vector<int4> cp;
    std::vector<unsigned char> flag;
    off.reserve(n_if + 1);
    flag.reserve(n_if);
    off.push_back(0);
    auto push = [&](int64_t t, const int mu[4]) {
        cp.push_back(make_int4((int)t, mu[1], mu[2], mu[3]));
    };
    auto pos_in = [&](int64_t t, int64_t gid) {
        for (int a = 0; a < 4; a++)
            if (tet[4 * t + a] == gid) return a;
        return -1;
    };
    int64_t n_free_if = 0;
    for (int64_t g = 0; g < nv; g++) {
        for (int64_t t : v_tets[g]) {
            int mu[4] = {0, 0, 0, 0};
            mu[pos_in(t, g)] = N;
            push(t, mu);
        }
        off.push_back((int)cp.size());
        flag.push_back((unsigned char)(vdir[g] | (0 << 1)));
        n_free_if += !vdir[g];
    }
    for (int64_t e = 0; e < ne; e++)
        for (int a = 1; a <= N - 1; a++) {
            for (int64_t t : e_tets[e]) {
                int mu[4] = {0, 0, 0, 0};
                mu[pos_in(t, edges[e][0])] = N - a;
                mu[pos_in(t, edges[e][1])] = a;
                push(t, mu);
            }
            off.push_back((int)cp.size());
            flag.push_back((unsigned char)(edir[e] | ((1 + a % 2) << 1)));
            n_free_if += !edir[e];
        }
    for (int64_t f = 0; f < nf; f++)
        for (int b = 1; b <= N - 2; b++)
            for (int a = 1; a <= N - 1 - b; a++) {
                for (int64_t t : f_tets[f]) {
                    int mu[4] = {0, 0, 0, 0};
                    mu[pos_in(t, faces[f][0])] = N - a - b;
                    mu[pos_in(t, faces[f][1])] = a;
                    mu[pos_in(t, faces[f][2])] = b;
                    push(t, mu);
                }
                off.push_back((int)cp.size());
                flag.push_back((unsigned char)(fdir[f] | ((3 + (a + 2 * b) % 3) << 1)));
                n_free_if += !fdir[f];
            }
    L->n_if = n_if;
    L->n_free = n_free_if + nt * (int64_t)(N - 1) * (N - 2) * (N - 3) / 6;
    L->if_off.upload(off);
    L->if_copy.upload(cp);
    L->if_flag.upload(flag);
    std::vector<int> lists[N_IF_PHASES];
    std::vector<int> freel;
    for (int64_t n = 0; n < n_if; n++) {
        if (flag[n] & 1) continue;
        lists[flag[n] >> 1].push_back((int)n);
        freel.push_back((int)n);
    }
    for (int p = 0; p < N_IF_PHASES; p++) {
        L->phase_list[p].upload(lists[p]);
        L->n_phase[p] = (int)lists[p].size();
    }
    L->if_free.upload(freel);
    L->n_if_free = (int)freel.size();
    // A phase updates every node from the values at the start of the phase.
    // A free node with no fine-mesh neighbour (in any copy) among the free
    // nodes of its own phase is read by no other node of the phase and reads
    // nothing the phase changes: it can be written in place.  The others
    // are coupled to a node of their phase (face nodes next to a face's
    // edges, edge nodes next to a vertex) and keep the start-of-phase rule
    // through a temporary.
    std::vector<unsigned char> coupled(n_if, 0);
    // set if a vertex shares a fine edge with an edge node of phase 1 (never
    // on a conforming mesh: the edge nodes next to a vertex are odd, phase 2)
    bool cross01 = false;
    {
        const int64_t base_f = nv + ne * (int64_t)(N - 1);
        // interface node at the local barycentric coordinates mu of macro t
        auto node_at = [&](int64_t t, const int mu[4]) -> int64_t {
            const MacroTopo& T = topo[t];
            int nz = 0, zo = -1, a0 = -1, a1 = -1;
            for (int a = 0; a < 4; a++) {
                if (mu[a] == 0) {
                    zo = a;
                } else {
                    nz++;
                    if (a0 < 0) a0 = a; else a1 = a;
                }
            }
            if (nz == 1) return T.vg[a0];
            if (nz == 2) {
                int e = 0;
                while (!(EDGE_LOC[e][0] == a0 && EDGE_LOC[e][1] == a1)) e++;
                return nv + T.e[e] * (N - 1) + (mu[T.ehi[e]] - 1);
            }
            const int a = mu[T.fs[zo][1]], b = mu[T.fs[zo][2]];
            return base_f + T.f[zo] * nF + (int64_t)(b - 1) * (N - 1) - (int64_t)(b - 1) * b / 2 +
                   (a - 1);
        };
        for (int64_t n = 0; n < n_if; n++) {
            if (flag[n] & 1) continue;
            const int ph = flag[n] >> 1;
            // nodes of phases 0 and 1 are scanned in full (for cross01)
            auto scanning = [&] { return !coupled[n] || ph <= 1; };
            for (int c = off[n]; c < off[n + 1] && scanning(); c++) {
                const int4 q = cp[c];
                const int m0[4] = {N - q.y - q.z - q.w, q.y, q.z, q.w};
                // a face node two or more steps from its face's edges has only
                // volume nodes and nodes of its own face around it, and those
                // are of other phases (the face colouring is proper)
                int zeros = 0, mn = N;
                for (int a = 0; a < 4; a++) {
                    if (m0[a] == 0) zeros++;
                    else mn = std::min(mn, m0[a]);
                }
                if (zeros == 1 && mn >= 2) continue;
                for (int w = 1; w < NW && scanning(); w++) {
                    const int i = q.y + dir_i(w), j = q.z + dir_j(w), k = q.w + dir_k(w);
                    if (!inside(N, i, j, k)) continue;
                    const int mu[4] = {N - i - j - k, i, j, k};
                    if (mu[0] && i && j && k) continue;  // volume node
                    const int64_t m = node_at(q.x, mu);
                    if (flag[m] & 1) continue;
                    const int pm = flag[m] >> 1;
                    if (pm == ph) coupled[n] = 1;
                    if (ph <= 1 && pm <= 1 && pm != ph) cross01 = true;
                }
            }
        }
    }
    // Whether the face-frame index a (the barycentric coordinate of the
    // face's middle vertex by global id, against the smallest) runs along the
    // block's i direction in this copy: the face's two lowest vertices are
    // the copy's local vertices 0 and 1.
    auto frame_rows_along_block_rows = [&](const int4& q) {
        const int o = N - q.y - q.z - q.w == 0 ? 0 : q.y == 0 ? 1 : q.z == 0 ? 2 : 3;
        const MacroTopo& T = topo[q.x];
        return std::min(T.fs[o][0], T.fs[o][1]) == 0 && std::max(T.fs[o][0], T.fs[o][1]) == 1;
    };
    // face fast path: free nodes of interior faces (two copies)
    {
        std::vector<int> f2, rest;
        std::vector<int4> c0, c1, rcc;
        std::vector<int> f2pos(n_if, -1), rcb(n_if, -1), f2f;
        std::vector<int64_t> dslots;
        const int64_t nfi = (int64_t)(N - 1) * (N - 2) / 2;  // free nodes per face
        int64_t last_face = -1;
        for (int64_t n = 0; n < n_if; n++) {
            const bool face = n >= nv + ne * (N - 1);
            if (flag[n] & 1) {
                for (int c = off[n]; c < off[n + 1]; c++)
                    dslots.push_back((int64_t)cp[c].x * L->B + bidx(N, cp[c].y, cp[c].z, cp[c].w));
            } else if (face && off[n + 1] - off[n] == 2) {
                const int64_t fi = (n - (nv + ne * (N - 1))) / nfi;
                if (fi != last_face) {
                    f2f.push_back((int)f2.size());
                    last_face = fi;
                }
                f2pos[n] = (int)f2.size();
                f2.push_back((int)n);
                // the first copy takes eleven of the row's entries (the
                // in-face ones and its inward ones): where only the second
                // copy has the face's frame rows along its block rows, it
                // goes first, so that consecutive nodes read consecutive
                // entries there
                int4 q0 = cp[off[n]], q1 = cp[off[n] + 1];
                if (!frame_rows_along_block_rows(q0) && frame_rows_along_block_rows(q1))
                    std::swap(q0, q1);
                c0.push_back(q0);
                c1.push_back(q1);
            } else {
                rest.push_back((int)n);
                rcb[n] = (int)rcc.size();
                for (int c = off[n]; c < off[n + 1]; c++) rcc.push_back(cp[c]);
            }
        }
        L->n_rc = (int)rcc.size();
        L->rc_base.upload(rcb);
        L->rc_cp.upload(rcc);
        L->n_dir_slots = (int64_t)dslots.size();
        L->dir_slots.upload(dslots);
        std::vector<int4> c01(c0);
        c01.insert(c01.end(), c1.begin(), c1.end());
        L->n_f2 = (int)f2.size();
        f2f.push_back(L->n_f2);
        for (size_t g = 0; g + 1 < f2f.size(); g++)
            if (f2f[g + 1] - f2f[g] != nfi) throw Error{TS_EINVAL, "interior face with missing nodes"};
        L->n_f2_faces = (int)f2f.size() - 1;
        L->f2_face_off.upload(f2f);
        L->f2_node.upload(f2);
        L->f2_cp.upload(c01);
        L->n_rest = (int)rest.size();
        L->rest.upload(rest);
        // Gauss-Seidel copy of the face fast path: the same nodes grouped by
        // phase, so that phase p is the contiguous range f2g_off[p] ..
        // Phases 0 (vertices) and 1 (even edge nodes) share no fine edge, so
        // updating them together gives what updating them one after the other
        // gives: they form one list (the list of phase 1 stays empty).
        std::vector<int4> g0, g1;
        for (int p = 0; p < N_IF_PHASES; p++) {
            std::vector<int> b;
            L->f2g_off[p] = (int)g0.size();
            int n2p = 0;
            std::vector<int> ph_in = {p};
            if (!cross01 && p == 0) ph_in = {0, 1};
            if (!cross01 && p == 1) ph_in = {};
            // nodes written in place first, then the coupled ones
            for (int pass = 0; pass < 2; pass++) {
                for (int pp : ph_in) for (int n : lists[pp]) {
                    if (coupled[n] != pass) continue;
                    if (f2pos[n] >= 0) {
                        g0.push_back(c0[f2pos[n]]);
                        g1.push_back(c1[f2pos[n]]);
                        n2p++;
                    } else {
                        b.push_back(n);
                    }
                }
                if (pass == 0) {
                    L->n_f2_direct[p] = n2p;
                    L->n_rest_direct[p] = (int)b.size();
                }
            }
            L->n_f2_phase[p] = n2p;
            L->rest_phase[p].upload(b);
            L->n_rest_phase[p] = (int)b.size();
        }
        g0.insert(g0.end(), g1.begin(), g1.end());
        L->f2g_cp.upload(g0);
    }

    // LDS-staged tiles: whole rows of plane k0's interior up to 256
    // positions, long rows split; the staged range of plane p covers rows
    // j0-1 .. j1 of that plane
    std::vector<int4> lt;
    int64_t maxcnt = 1;
    auto staged = [&](int k0, int j0, int j1) {
        const int p = k0 - 1, A = N + 1 - p;
        const int jl = std::min(j1, N - p);
        int64_t c = 0;
        for (int jj = j0 - 1; jj <= jl; jj++) c += A - jj;
        return c;
    };
    for (int k0 = 1; k0 <= N - 3; k0 += VOL_R) {
        const int Mr = N - 1 - k0;
        int j = 1;
        while (j <= Mr - 1) {
            const int len = Mr - j;
            if (len > VOL_THREADS) {
                for (int i0 = 1; i0 <= len; i0 += VOL_THREADS) lt.push_back(make_int4(k0, j, j + 1, i0));
                maxcnt = std::max(maxcnt, staged(k0, j, j + 1));
                j++;
                continue;
            }
            // whole rows while the tile stays within 256 columns and no
            // colour class (i + 2j) mod 4 exceeds one wavefront of 64
            int j1 = j, tot = 0;
            int cc[4] = {0, 0, 0, 0};
            while (j1 <= Mr - 1 && tot + (Mr - j1) <= VOL_THREADS) {
                int add[4] = {0, 0, 0, 0};
                for (int i = 1; i <= Mr - j1; i++) add[(i + 2 * j1) & 3]++;
                bool fits = true;
                for (int q = 0; q < 4; q++) fits = fits && cc[q] + add[q] <= VOL_THREADS / 4;
                if (!fits && j1 > j) break;
                for (int q = 0; q < 4; q++) cc[q] += add[q];
                tot += Mr - j1;
                j1++;
            }
            lt.push_back(make_int4(k0, j, j1, 0));
            maxcnt = std::max(maxcnt, staged(k0, j, j1));
            j = j1;
        }
    }
    L->lds_tiles.upload(lt);
    L->n_lds_tiles = (int)lt.size();
    L->lds_kpt = (int)((maxcnt + VOL_THREADS - 1) / VOL_THREADS);
    // Lane orders of the columns of every tile.  Columns with i + j above
    // N - k0 - R end inside the slab; sorting them after the others (by
    // i + j) gathers the columns that have ended into whole wavefronts, which
    // then skip their weight evaluation.  Apply order: the full-length
    // columns row by row, then the ending ones.  Gauss-Seidel order: colour
    // class (i + 2j) mod 4 = q in wavefront q (lanes 64q ..), so that a
    // wavefront holds one class per plane and skips the planes where its
    // class is not updated; within a class as in the apply order.
    {
        std::vector<unsigned> am((size_t)lt.size() * VOL_THREADS, 0xFFFFFFFFu);
        std::vector<unsigned> gm((size_t)lt.size() * VOL_THREADS, 0xFFFFFFFFu);
        for (size_t t = 0; t < lt.size(); t++) {
            const int4 d = lt[t];
            const int Mr = N - 1 - d.x;
            const int full = N - d.x - VOL_R;  // i + j <= full: column spans the slab
            std::vector<std::pair<int, int>> pos;
            if (d.w > 0) {
                for (int i = d.w; i <= std::min(d.w + VOL_THREADS - 1, Mr - d.y); i++)
                    pos.push_back({i, d.y});
            } else {
                for (int j = d.y; j < d.z; j++)
                    for (int i = 1; i <= Mr - j; i++) pos.push_back({i, j});
            }
            auto band = [&](const std::pair<int, int>& a) {
                return std::max(a.first + a.second, full);
            };
            auto cls = [](const std::pair<int, int>& a) { return (a.first + 2 * a.second) & 3; };
            std::vector<std::pair<int, int>> ap(pos), gs(pos);
            std::stable_sort(ap.begin(), ap.end(), [&](const std::pair<int, int>& a,
                                                       const std::pair<int, int>& b) {
                return band(a) < band(b);
            });
            std::stable_sort(gs.begin(), gs.end(), [&](const std::pair<int, int>& a,
                                                       const std::pair<int, int>& b) {
                return cls(a) != cls(b) ? cls(a) < cls(b) : band(a) < band(b);
            });
            int fill[4] = {0, 0, 0, 0};
            for (size_t l = 0; l < pos.size(); l++) {
                am[t * VOL_THREADS + l] = (unsigned)ap[l].first | ((unsigned)ap[l].second << 16);
                // class q takes the lanes of wavefront q (64 lanes; tiles keep
                // every class within that)
                const int q = cls(gs[l]);
                const int lane = fill[q] < VOL_THREADS / 4 ? q * (VOL_THREADS / 4) + fill[q]++ : -1;
                if (lane < 0) throw Error{TS_EINVAL, "volume tile with a colour class above 64"};
                gm[t * VOL_THREADS + lane] = (unsigned)gs[l].first | ((unsigned)gs[l].second << 16);
            }
        }
        L->ap_lanes.upload(am);
        L->gs_lanes.upload(gm);
    }
    // staged plane ranges of every tile: plane p = k0 - 1 + st holds rows
    // jb = j0 - 1 .. min(j1, N - p), starting at plane_off(p) + row_off(jb, p)
    {
        std::vector<int> sg((size_t)lt.size() * (VOL_R + 2), 0);
        for (size_t t = 0; t < lt.size(); t++) {
            const int4 d = lt[t];
            const int jb = d.y - 1;
            for (int st = 0; st < VOL_R + 2; st++) {
                const int p = d.x - 1 + st;
                const int jl = std::min(d.z, N - p);
                if (p <= N && jl >= jb)
                    sg[t * (VOL_R + 2) + st] = (int)(plane_off(N, p) + row_off(N, jb, p));
            }
        }
        L->stage_tbl.upload(sg);
    }
    // all-slot tiles: every plane k = 0..N in chunks of 256 slots
    std::vector<int2> st;
    for (int k = 0; k <= N; k++) {
        const int64_t n = tri_n(N + 1 - k);
        for (int64_t s = 0; s < n; s += 256) st.push_back(make_int2(k, (int)s));
    }
    L->slot_tiles.upload(st);
    L->n_slot_tiles = (int)st.size();

    Level& ref = *L;
    levels[lam] = std::move(L);
    return ref;
}

}  // namespace ts
