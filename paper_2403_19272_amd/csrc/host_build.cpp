// Host-side scene precompute in FP64: mesh validation, rest frames, lumped
// mass, hinge stencils and the PD system matrix H of Eq. (global):
//   H = M / h^2 + sum_t w_t G_t^T G_t + sum_e w_e k_e k_e^T   (scalar, nv x nv)
// Triangle strain: F = D_s D_m^{-1} with D_m the rest edges in an in-plane
// orthonormal frame, weight w_t = k_stretch * area.  Hinge bending: the
// cotangent stencil of quadratic bending, weight k_bend * 3 / (A_1 + A_2).
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <utility>
#include <vector>

#include "scene.hpp"

namespace cloth {

namespace {

struct V3 {
    double x, y, z;
};
V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(V3 a) { return std::sqrt(dot(a, a)); }
V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }

V3 vtx(const std::vector<double>& X, int i) { return {X[3 * i], X[3 * i + 1], X[3 * i + 2]}; }

// cot of the angle between a and b
double cotan(V3 a, V3 b) { return dot(a, b) / norm(cross(a, b)); }

}  // namespace

// Reverse Cuthill-McKee order of the mesh's vertex graph (edges of the
// triangles): order[i] is the input vertex placed at position i.  Each
// connected component starts from a pseudo-peripheral vertex (the last vertex
// reached by a breadth-first search from its lowest-degree vertex, repeated
// while the search depth grows); a search visits the unvisited neighbours of
// each vertex in increasing degree (ties by index), and the whole order is
// reversed at the end.  Neighbouring vertices get nearby positions, so the
// sweeps' gathers stay within a narrow band of the state vectors.
std::vector<int> rcm_order(int nv, int nt, const int32_t* tris) {
    std::vector<std::vector<int>> adj(nv);
    for (int t = 0; t < nt; ++t)
        for (int c = 0; c < 3; ++c) {
            const int a = tris[3 * t + c], b = tris[3 * t + (c + 1) % 3];
            adj[a].push_back(b);
            adj[b].push_back(a);
        }
    for (auto& l : adj) {
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    std::vector<int> deg(nv);
    for (int v = 0; v < nv; ++v) deg[v] = (int)adj[v].size();
    for (auto& l : adj)
        std::stable_sort(l.begin(), l.end(), [&](int a, int b) { return deg[a] < deg[b]; });
    std::vector<int> level(nv, -1), order, comp;
    order.reserve(nv);
    std::vector<char> done(nv, 0);
    // breadth-first levels from `root` over the unplaced vertices; returns the
    // depth and leaves the vertices in visiting order in `out`
    auto bfs = [&](int root, std::vector<int>& out) {
        out.clear();
        out.push_back(root);
        level[root] = 0;
        int depth = 0;
        for (size_t h = 0; h < out.size(); ++h) {
            const int v = out[h];
            for (int w : adj[v])
                if (!done[w] && level[w] < 0) {
                    level[w] = level[v] + 1;
                    depth = std::max(depth, level[w]);
                    out.push_back(w);
                }
        }
        for (int v : out) level[v] = -1;
        return depth;
    };
    std::vector<int> by_deg(nv);
    std::iota(by_deg.begin(), by_deg.end(), 0);
    std::stable_sort(by_deg.begin(), by_deg.end(), [&](int a, int b) { return deg[a] < deg[b]; });
    for (int start : by_deg) {
        if (done[start]) continue;
        int root = start;
        int depth = bfs(root, comp);
        for (int it = 0; it < 8; ++it) {
            // restart from the last vertex reached
            int far = comp.back();
            const int d2 = bfs(far, comp);
            if (d2 <= depth) {
                bfs(root, comp);
                break;
            }
            root = far;
            depth = d2;
        }
        for (int v : comp) {
            done[v] = 1;
            order.push_back(v);
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

std::string build_scene(Scene& s, const cloth_mesh* mesh, const float* rest, double dt,
                        const cloth_material* mat, const cloth_solver_params* prm) {
    const int nv = mesh->nv, nt = mesh->nt;
    if (nv <= 0 || nt <= 0 || !mesh->tris || !rest) return "empty mesh or missing rest shape";
    if (dt <= 0) return "dt must be positive";
    s.nv = nv;
    s.nt = nt;
    s.h = dt;
    s.density = mat->density;
    s.ks = mat->k_stretch;
    s.kb = mat->k_bend;
    s.Kb = mat->K_base > 0 ? mat->K_base : 2.0;
    s.amax = mat->a_max > 0 ? mat->a_max : 20;
    s.dhat = mat->d_hat;
    s.alpha = mat->alpha > 0 ? mat->alpha : 0.8;
    s.mu = mat->friction > 0 ? mat->friction : 0.0;
    s.feps = (mat->friction_eps_v > 0 ? mat->friction_eps_v : 1e-3) * dt;
    // strain limits: 0, 0 reads as the rotation projection (1, 1)
    s.smin = (mat->sigma_min == 0 && mat->sigma_max == 0) ? 1.0 : mat->sigma_min;
    s.smax = (mat->sigma_min == 0 && mat->sigma_max == 0) ? 1.0 : mat->sigma_max;

    s.tris.assign(mesh->tris, mesh->tris + 3 * (size_t)nt);
    s.pinned.assign(nv, 0);
    if (mesh->pinned)
        for (int i = 0; i < nv; ++i) s.pinned[i] = mesh->pinned[i] ? 1 : 0;
    s.rest.resize(3 * (size_t)nv);
    for (size_t i = 0; i < 3 * (size_t)nv; ++i) s.rest[i] = (double)rest[i];

    for (int t = 0; t < nt; ++t)
        for (int c = 0; c < 3; ++c) {
            int v = s.tris[3 * t + c];
            if (v < 0 || v >= nv) return "triangle index out of range";
        }

    // rest frames, areas, gradient rows
    s.area.assign(nt, 0.0);
    s.g.assign(6 * (size_t)nt, 0.0);
    s.mass.assign(nv, 0.0);
    for (int t = 0; t < nt; ++t) {
        int i = s.tris[3 * t], j = s.tris[3 * t + 1], k = s.tris[3 * t + 2];
        if (i == j || j == k || i == k) return "triangle with repeated vertex";
        V3 e1 = sub(vtx(s.rest, j), vtx(s.rest, i));
        V3 e2 = sub(vtx(s.rest, k), vtx(s.rest, i));
        V3 n = cross(e1, e2);
        double a2 = norm(n);
        if (!(a2 > 0)) return "degenerate rest triangle";
        double l1 = norm(e1);
        V3 u1 = scale(e1, 1.0 / l1);
        V3 u2 = cross(scale(n, 1.0 / a2), u1);
        // D_m columns: rest edges in (u1, u2)
        double m00 = dot(e1, u1), m01 = dot(e2, u1), m10 = dot(e1, u2), m11 = dot(e2, u2);
        double det = m00 * m11 - m01 * m10;
        // rows of D_m^{-1}
        double i00 = m11 / det, i01 = -m01 / det, i10 = -m10 / det, i11 = m00 / det;
        double* gt = &s.g[6 * (size_t)t];
        gt[2] = i00;  // g_j = row 0
        gt[3] = i01;
        gt[4] = i10;  // g_k = row 1
        gt[5] = i11;
        gt[0] = -i00 - i10;
        gt[1] = -i01 - i11;
        s.area[t] = 0.5 * a2;
        for (int c = 0; c < 3; ++c) s.mass[s.tris[3 * t + c]] += s.density * s.area[t] / 3.0;
    }

    // edges (sorted unique) and hinges
    std::map<std::pair<int, int>, std::vector<int>> emap;  // edge -> opposite vertices
    for (int t = 0; t < nt; ++t)
        for (int c = 0; c < 3; ++c) {
            int a = s.tris[3 * t + c], b = s.tris[3 * t + (c + 1) % 3], o = s.tris[3 * t + (c + 2) % 3];
            emap[{std::min(a, b), std::max(a, b)}].push_back(o);
        }
    s.edges.clear();
    s.hinges.clear();
    for (auto& kv : emap) {
        if (kv.second.size() > 2) return "non-manifold edge";
        s.edges.push_back(kv.first.first);
        s.edges.push_back(kv.first.second);
        if (kv.second.size() == 2) {
            s.hinges.push_back(kv.first.first);
            s.hinges.push_back(kv.first.second);
            s.hinges.push_back(kv.second[0]);
            s.hinges.push_back(kv.second[1]);
        }
    }
    s.ne = (int)(s.edges.size() / 2);
    s.nh = (int)(s.hinges.size() / 4);
    s.K.assign(4 * (size_t)s.nh, 0.0);
    s.w_hinge.assign(s.nh, 0.0);
    for (int e = 0; e < s.nh; ++e) {
        const int* hg = &s.hinges[4 * (size_t)e];
        V3 p0 = vtx(s.rest, hg[0]), p1 = vtx(s.rest, hg[1]), p2 = vtx(s.rest, hg[2]),
           p3 = vtx(s.rest, hg[3]);
        double cA0 = cotan(sub(p1, p0), sub(p2, p0)), cA1 = cotan(sub(p0, p1), sub(p2, p1));
        double cB0 = cotan(sub(p1, p0), sub(p3, p0)), cB1 = cotan(sub(p0, p1), sub(p3, p1));
        double* k = &s.K[4 * (size_t)e];
        k[0] = cA1 + cB1;
        k[1] = cA0 + cB0;
        k[2] = -cA0 - cA1;
        k[3] = -cB0 - cB1;
        double aA = 0.5 * norm(cross(sub(p1, p0), sub(p2, p0)));
        double aB = 0.5 * norm(cross(sub(p1, p0), sub(p3, p0)));
        s.w_hinge[e] = s.kb * 3.0 / (aA + aB);
        // curved rest hinges would need a bending target; this build supports
        // flat rest shapes (target 0), checked at rounding level
        V3 sK = {0, 0, 0};
        double sc = 0, ext = 0;
        for (int q = 0; q < 4; ++q) {
            V3 pq = vtx(s.rest, hg[q]);
            sK = {sK.x + k[q] * pq.x, sK.y + k[q] * pq.y, sK.z + k[q] * pq.z};
            sc += std::fabs(k[q]);
            V3 d = sub(pq, p0);
            ext = std::max(ext, std::max(std::fabs(d.x), std::max(std::fabs(d.y), std::fabs(d.z))));
        }
        if (norm(sK) > 1e-12 * sc * ext) return "curved rest shape (non-flat hinge) is not supported";
    }

    // system matrix H as FP64 CSR (rows sorted, duplicates summed)
    std::vector<std::vector<std::pair<int, double>>> rows(nv);
    const double ih2 = 1.0 / (dt * dt);
    for (int v = 0; v < nv; ++v) rows[v].push_back({v, s.mass[v] * ih2});
    for (int t = 0; t < nt; ++t) {
        const double* gt = &s.g[6 * (size_t)t];
        double w = s.ks * s.area[t];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                rows[s.tris[3 * t + a]].push_back(
                    {s.tris[3 * t + c], w * (gt[2 * a] * gt[2 * c] + gt[2 * a + 1] * gt[2 * c + 1])});
    }
    for (int e = 0; e < s.nh; ++e) {
        const int* hg = &s.hinges[4 * (size_t)e];
        const double* k = &s.K[4 * (size_t)e];
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 4; ++c) rows[hg[a]].push_back({hg[c], s.w_hinge[e] * k[a] * k[c]});
    }
    s.rowptr.assign(nv + 1, 0);
    s.col.clear();
    s.val.clear();
    s.diag.assign(nv, 0.0);
    for (int v = 0; v < nv; ++v) {
        auto& rw = rows[v];
        std::sort(rw.begin(), rw.end(),
                  [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
                      return a.first < b.first;
                  });
        for (size_t i = 0; i < rw.size();) {
            int c = rw[i].first;
            double acc = 0;
            while (i < rw.size() && rw[i].first == c) acc += rw[i++].second;
            s.col.push_back(c);
            s.val.push_back(acc);
            if (c == v) s.diag[v] = acc;
        }
        s.rowptr[v + 1] = (int)s.col.size();
        std::vector<std::pair<int, double>>().swap(rw);
    }
    s.nnz = (int64_t)s.col.size();

    // Sliced ELLPACK copy of the off-diagonal entries for the sweeps: slices
    // of 64 rows (one wavefront), each as wide as its longest row; entry j of
    // row v sits at sell_ptr[v / 64] + 64 j + v % 64, so that every load of a
    // wavefront is one contiguous 256-byte run.  Padding points at the row
    // itself with value 0.
    {
        const int ns = (nv + 63) / 64;
        s.sell_ptr.assign(ns + 1, 0);
        for (int sl = 0; sl < ns; ++sl) {
            int w = 0;
            for (int v = sl * 64; v < std::min(nv, sl * 64 + 64); ++v)
                w = std::max(w, s.rowptr[v + 1] - s.rowptr[v] - 1);
            s.sell_ptr[sl + 1] = s.sell_ptr[sl] + 64 * w;
        }
        s.nsell = s.sell_ptr[ns];
        s.sell_col.assign(s.sell_ptr[ns], 0);
        s.sell_val.assign(s.sell_ptr[ns], 0.0f);
        for (int sl = 0; sl < ns; ++sl) {
            int w = (s.sell_ptr[sl + 1] - s.sell_ptr[sl]) / 64;
            for (int lane = 0; lane < 64; ++lane) {
                int v = sl * 64 + lane;
                int j = 0;
                if (v < nv)
                    for (int k = s.rowptr[v]; k < s.rowptr[v + 1]; ++k) {
                        if (s.col[k] == v) continue;
                        size_t at = (size_t)s.sell_ptr[sl] + 64 * j + lane;
                        s.sell_col[at] = s.col[k];
                        s.sell_val[at] = (float)s.val[k];
                        ++j;
                    }
                for (; j < w; ++j) s.sell_col[(size_t)s.sell_ptr[sl] + 64 * j + lane] = v < nv ? v : 0;
            }
        }
    }

    // contact constant k
    if (mat->k_contact > 0) {
        s.kc = mat->k_contact;
    } else {
        double acc = 0;
        int cnt = 0;
        for (int v = 0; v < nv; ++v)
            if (!s.pinned[v]) {
                acc += s.diag[v] - s.mass[v] * ih2;
                ++cnt;
            }
        s.kc = cnt ? acc / cnt : 1.0;
    }

    s.r = prm->r;
    s.r_warm = prm->r_warm;
    s.uu_store = prm->uu_store ? 1 : 0;
    s.smoother = prm->smoother;
    s.adapt_samples = prm->adaptive_samples ? 1 : 0;
    s.iters_in = prm->iters_inner;
    s.iters_out = prm->iters_outer;
    s.rho = prm->cheb_rho;
    s.gamma = prm->cheb_gamma;
    s.delay = prm->cheb_delay;
    s.prec = prm->precision;
    s.self_contact = prm->self_contact;
    s.pair_cap = prm->pair_capacity > 0 ? prm->pair_capacity : (int64_t)128 * nv;
    s.tol_in = prm->tol_inner > 0 ? prm->tol_inner : 0.0;
    s.tol_out = prm->tol_outer > 0 ? prm->tol_outer : 0.0;
    s.debug_tangles = prm->debug_tangles ? 1 : 0;
    s.bp_mu0 = prm->broad_margin > 0 ? prm->broad_margin : 0.25 * s.dhat;
    s.bp_kappa = prm->broad_margin_motion > 0 ? prm->broad_margin_motion : 1.0;
    s.bp_reuse = prm->broad_reuse ? 1 : 0;
    return "";
}

}  // namespace cloth
