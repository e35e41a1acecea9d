// sme_mesh.cpp -- host-side mesh checks and triangle-mesh preprocessing
// (declared in sme_mesh.h).
#include "sme_mesh.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

namespace sme {
namespace mesh {

namespace {

int error(std::string &why, int code, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    why = buf;
    return code;
}

}  // namespace

int nfields_of(int level, int kind) { return kind == SME_MESH_1D ? level + 2 : 2 * level + 3; }

int check_mesh(const sme_mesh *m, int level, int *nf, int64_t *nc)
{
    if (!m || level < 0 || level > SME_MAX_LEVEL) return SME_EINVAL;
    *nf = nfields_of(level, m->kind);
    switch (m->kind) {
    case SME_MESH_1D:
        if (m->nx < 1 || m->nx > (int64_t)1 << 30 || !(m->x1 > m->x0)) return SME_EINVAL;
        for (int s = 0; s < 2; ++s)
            if (m->bc[s] < 0 || m->bc[s] > 2) return SME_EINVAL;
        if ((m->bc[0] == SME_BC_PERIODIC) != (m->bc[1] == SME_BC_PERIODIC)) return SME_EINVAL;
        *nc = m->nx;
        return SME_OK;
    case SME_MESH_2D_STRUCT:
        if (m->nx < 1 || m->ny < 1 || m->nx > (int64_t)1 << 24 || m->ny > (int64_t)1 << 24) return SME_EINVAL;
        if (m->nx * m->ny > ((int64_t)1 << 31) - 1) return SME_EINVAL;
        if (!(m->x1 > m->x0) || !(m->y1 > m->y0)) return SME_EINVAL;
        for (int s = 0; s < 4; ++s)
            if (m->bc[s] < 0 || m->bc[s] > 2) return SME_EINVAL;
        if ((m->bc[0] == SME_BC_PERIODIC) != (m->bc[1] == SME_BC_PERIODIC)) return SME_EINVAL;
        if ((m->bc[2] == SME_BC_PERIODIC) != (m->bc[3] == SME_BC_PERIODIC)) return SME_EINVAL;
        *nc = m->nx * m->ny;
        return SME_OK;
    case SME_MESH_2D_TRI:
        if (m->n_tri < 1 || m->n_vert < 3 || !m->vert_xy || !m->tri) return SME_EINVAL;
        if (m->n_tri > kTriMaxCells) return SME_EINVAL;
        *nc = m->n_tri;
        return SME_OK;
    default:
        return SME_EINVAL;
    }
}



int build_tri(const sme_mesh *m, TriGeom &g, std::string &why)
{
    const int64_t nt = m->n_tri, nv = m->n_vert;
    g.nbr.assign(3 * nt, -1);
    g.sx.resize(3 * nt);
    g.sy.resize(3 * nt);
    g.ivol.resize(nt);
    const double *X = m->vert_xy;
    const int32_t *T = m->tri;
    for (int64_t t = 0; t < nt; ++t) {
        int32_t v[3] = {T[3 * t], T[3 * t + 1], T[3 * t + 2]};
        for (int s = 0; s < 3; ++s)
            if (v[s] < 0 || v[s] >= nv) return error(why, SME_EMESH, "triangle %lld has a bad vertex index", (long long)t);
        double ax = X[2 * v[0]], ay = X[2 * v[0] + 1];
        double bx = X[2 * v[1]], by = X[2 * v[1] + 1];
        double cx = X[2 * v[2]], cy = X[2 * v[2] + 1];
        double area = 0.5 * ((bx - ax) * (cy - ay) - (cx - ax) * (by - ay));
        if (!(area > 0.0))
            return error(why, SME_EMESH, "triangle %lld is degenerate or not counter-clockwise", (long long)t);
        g.ivol[t] = 1.0 / area;
        for (int s = 0; s < 3; ++s) {
            int32_t p0 = v[s], p1 = v[(s + 1) % 3];
            double ex = X[2 * p1] - X[2 * p0];
            double ey = X[2 * p1 + 1] - X[2 * p0 + 1];
            if (!(ex != 0.0 || ey != 0.0)) return error(why, SME_EMESH, "triangle %lld has an edge of zero length", (long long)t);
            g.sx[3 * t + s] = ey;
            g.sy[3 * t + s] = -ex;
        }
    }
    // match half-edges: key (min, max) vertex pair
    struct HE {
        uint64_t key;
        int64_t id;  // 3 * t + s
    };
    std::vector<HE> he(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int s = 0; s < 3; ++s) {
            uint64_t a = (uint32_t)T[3 * t + s], b = (uint32_t)T[3 * t + (s + 1) % 3];
            uint64_t lo = std::min(a, b), hi = std::max(a, b);
            he[3 * t + s] = HE{lo * (uint64_t)nv + hi, 3 * t + s};
        }
    std::sort(he.begin(), he.end(), [](const HE &x, const HE &y) { return x.key < y.key || (x.key == y.key && x.id < y.id); });
    for (size_t k = 0; k < he.size();) {
        size_t e = k + 1;
        while (e < he.size() && he[e].key == he[k].key) ++e;
        if (e - k > 2) return error(why, SME_EMESH, "non-manifold edge (used by %zu triangles)", e - k);
        if (e - k == 2) {
            int64_t i0 = he[k].id, i1 = he[k + 1].id;
            // consistent orientation: the two triangles traverse the edge in opposite directions
            int32_t a0 = T[i0], b0 = T[(i0 / 3) * 3 + (i0 % 3 + 1) % 3];
            int32_t a1 = T[i1], b1 = T[(i1 / 3) * 3 + (i1 % 3 + 1) % 3];
            if (!(a0 == b1 && b0 == a1)) return error(why, SME_EMESH, "inconsistently oriented neighbours");
            g.nbr[i0] = (int32_t)(i1 / 3);
            g.nbr[i1] = (int32_t)(i0 / 3);
        }
        k = e;
    }
    return SME_OK;
}


// Reverse Cuthill-McKee order of the triangle adjacency graph.
// Returns order[k] = caller cell placed at internal position k.
std::vector<int64_t> rcm_order(const std::vector<int32_t> &nbr, int64_t n)
{
    std::vector<int> deg(n, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int s = 0; s < 3; ++s) deg[i] += nbr[3 * i + s] >= 0;
    std::vector<int64_t> order;
    order.reserve(n);
    std::vector<char> seen(n, 0);
    std::vector<int64_t> level_of(n, -1);
    auto bfs_last = [&](int64_t start) {
        // plain BFS, returns a node of the last level with minimum degree
        std::vector<int64_t> q{start};
        std::vector<int64_t> mark;
        level_of[start] = 0;
        mark.push_back(start);
        size_t h = 0;
        while (h < q.size()) {
            int64_t u = q[h++];
            for (int s = 0; s < 3; ++s) {
                int32_t v = nbr[3 * u + s];
                if (v >= 0 && level_of[v] < 0) {
                    level_of[v] = level_of[u] + 1;
                    q.push_back(v);
                    mark.push_back(v);
                }
            }
        }
        int64_t best = q.back();
        int64_t L = level_of[best];
        for (auto it = q.rbegin(); it != q.rend() && level_of[*it] == L; ++it)
            if (deg[*it] < deg[best]) best = *it;
        for (int64_t m : mark) level_of[m] = -1;
        return best;
    };
    for (int64_t root = 0; root < n; ++root) {
        if (seen[root]) continue;
        int64_t start = bfs_last(bfs_last(root));  // pseudo-peripheral start
        size_t h = order.size();
        order.push_back(start);
        seen[start] = 1;
        while (h < order.size()) {
            int64_t u = order[h++];
            int64_t cand[3];
            int nc = 0;
            for (int s = 0; s < 3; ++s) {
                int32_t v = nbr[3 * u + s];
                if (v >= 0 && !seen[v]) {
                    seen[v] = 1;
                    cand[nc++] = v;
                }
            }
            std::sort(cand, cand + nc, [&](int64_t x, int64_t y) { return deg[x] < deg[y] || (deg[x] == deg[y] && x < y); });
            for (int k = 0; k < nc; ++k) order.push_back(cand[k]);
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

}  // namespace mesh
}  // namespace sme
