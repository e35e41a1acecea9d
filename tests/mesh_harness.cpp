// mesh_harness.cpp -- CPU driver of the host mesh code (sme_mesh.cpp), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by test_mesh_sanitize.py.
// Every check prints "OK <name>"; the first failure prints "FAIL <name>: why"
// and exits with status 1.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../paper_2601_04826_amd/csrc/sme_mesh.h"

using namespace sme::mesh;

static void check(bool ok, const char *name, const char *why = "")
{
    if (!ok) {
        std::printf("FAIL %s: %s\n", name, why);
        std::exit(1);
    }
}

struct Tri {
    std::vector<double> xy;
    std::vector<int32_t> t;
    sme_mesh mesh() const
    {
        sme_mesh m{};
        m.kind = SME_MESH_2D_TRI;
        m.n_vert = (int64_t)xy.size() / 2;
        m.n_tri = (int64_t)t.size() / 3;
        m.vert_xy = xy.data();
        m.tri = t.data();
        return m;
    }
};

// n x n squares of the unit square, each cut into two counter-clockwise
// triangles; inner vertices jittered by up to jit of the spacing per
// coordinate (below 0.25 no triangle turns over), vertex labels and
// triangle order shuffled, each triangle's vertex list rotated at random
static Tri grid(int n, double jit, unsigned seed, double x0 = 0.0)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    const double d = 1.0 / n;
    Tri m;
    int nv = (n + 1) * (n + 1);
    std::vector<int> label(nv);
    for (int i = 0; i < nv; ++i) label[i] = i;
    std::shuffle(label.begin(), label.end(), rng);
    m.xy.resize(2 * nv);
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
            const bool inner = i > 0 && i < n && j > 0 && j < n;
            m.xy[2 * label[j * (n + 1) + i]] = x0 + i * d + (inner ? jit * d * u(rng) : 0.0);
            m.xy[2 * label[j * (n + 1) + i] + 1] = j * d + (inner ? jit * d * u(rng) : 0.0);
        }
    std::vector<std::vector<int32_t>> tris;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int a = label[j * (n + 1) + i], b = label[j * (n + 1) + i + 1];
            int c = label[(j + 1) * (n + 1) + i + 1], e = label[(j + 1) * (n + 1) + i];
            tris.push_back({a, b, c});
            tris.push_back({a, c, e});
        }
    std::shuffle(tris.begin(), tris.end(), rng);
    for (auto &t : tris) {
        std::rotate(t.begin(), t.begin() + (int)(rng() % 3), t.end());
        m.t.insert(m.t.end(), t.begin(), t.end());
    }
    return m;
}

static void check_valid(const Tri &T, const char *name, int64_t walls_expected)
{
    sme_mesh m = T.mesh();
    int nf = 0;
    int64_t nc = 0;
    check(check_mesh(&m, 3, &nf, &nc) == SME_OK && nf == 9 && nc == m.n_tri, name, "check_mesh");
    TriGeom g;
    std::string why;
    const int rc = build_tri(&m, g, why);
    check(rc == SME_OK, name, why.c_str());
    const int64_t nt = m.n_tri;
    int64_t walls = 0;
    for (int64_t t = 0; t < nt; ++t) {
        double area = 0.5 * ((T.xy[2 * T.t[3 * t + 1]] - T.xy[2 * T.t[3 * t]]) * (T.xy[2 * T.t[3 * t + 2] + 1] - T.xy[2 * T.t[3 * t] + 1]) -
                             (T.xy[2 * T.t[3 * t + 2]] - T.xy[2 * T.t[3 * t]]) * (T.xy[2 * T.t[3 * t + 1] + 1] - T.xy[2 * T.t[3 * t] + 1]));
        check(std::fabs(g.ivol[t] * area - 1.0) < 1e-12, name, "inverse area");
        double sx = 0, sy = 0, per = 0;
        for (int s = 0; s < 3; ++s) {
            sx += g.sx[3 * t + s];
            sy += g.sy[3 * t + s];
            per += std::hypot(g.sx[3 * t + s], g.sy[3 * t + s]);
            int32_t u = g.nbr[3 * t + s];
            if (u < 0) {
                ++walls;
                continue;
            }
            check(u != t && u < nt, name, "neighbour index");
            int back = -1;
            for (int r = 0; r < 3; ++r)
                if (g.nbr[3 * u + r] == t) back = r;
            check(back >= 0, name, "neighbour relation not symmetric");
            check(g.sx[3 * u + back] == -g.sx[3 * t + s] && g.sy[3 * u + back] == -g.sy[3 * t + s], name,
                  "scaled normals of a shared face are not exact negatives");
        }
        check(std::fabs(sx) <= 1e-13 * per && std::fabs(sy) <= 1e-13 * per, name, "scaled normals do not close");
    }
    check(walls == walls_expected, name, "wall face count");
    std::vector<int64_t> order = rcm_order(g.nbr, nt);
    check((int64_t)order.size() == nt, name, "order length");
    std::vector<char> seen(nt, 0);
    for (int64_t k : order) {
        check(k >= 0 && k < nt && !seen[k], name, "order is not a permutation");
        seen[k] = 1;
    }
    std::printf("OK %s (%lld triangles)\n", name, (long long)nt);
}

static void check_error(const Tri &T, const char *name, const char *expect)
{
    sme_mesh m = T.mesh();
    TriGeom g;
    std::string why;
    const int rc = build_tri(&m, g, why);
    check(rc == SME_EMESH && why.find(expect) != std::string::npos, name, why.c_str());
    std::printf("OK %s (%s)\n", name, why.c_str());
}

int main()
{
    check_valid(grid(1, 0.0, 1), "one_square", 4);
    check_valid(grid(7, 0.2, 2), "jittered_7", 28);
    check_valid(grid(300, 0.2, 3), "jittered_300", 1200);
    {
        // two separate components: RCM must order both
        Tri a = grid(20, 0.2, 4), b = grid(13, 0.2, 5, 3.0);
        const int32_t off = (int32_t)(a.xy.size() / 2);
        a.xy.insert(a.xy.end(), b.xy.begin(), b.xy.end());
        for (int32_t v : b.t) a.t.push_back(v + off);
        check_valid(a, "two_components", 80 + 52);
    }
    {
        Tri a = grid(4, 0.0, 6);
        a.t[5] = -1;
        check_error(a, "negative_vertex", "bad vertex index");
        a = grid(4, 0.0, 6);
        a.t[7] = (int32_t)(a.xy.size() / 2);
        check_error(a, "vertex_past_end", "bad vertex index");
        a = grid(4, 0.0, 6);
        std::swap(a.t[0], a.t[1]);
        check_error(a, "clockwise", "not counter-clockwise");
        a = grid(4, 0.0, 6);
        a.t[2] = a.t[1];
        check_error(a, "repeated_vertex", "degenerate");
    }
    {
        // collinear vertices
        Tri a;
        a.xy = {0, 0, 1, 0, 2, 0};
        a.t = {0, 1, 2};
        check_error(a, "collinear", "degenerate");
        // three triangles on edge (0, 1): two above it, one below
        a.xy = {0, 0, 1, 0, 0.5, 1, 0.5, -1, 0.3, 2};
        a.t = {0, 1, 2, 1, 0, 3, 0, 1, 4};
        check_error(a, "non_manifold", "non-manifold");
        // two counter-clockwise triangles on the same side of edge (0, 1)
        a.t = {0, 1, 2, 0, 1, 4};
        check_error(a, "same_direction", "inconsistently oriented");
    }
    {
        // check_mesh argument validation
        sme_mesh m{};
        int nf;
        int64_t nc;
        m.kind = SME_MESH_2D_STRUCT;
        m.nx = 0;
        m.ny = 4;
        m.x1 = m.y1 = 1.0;
        check(check_mesh(&m, 2, &nf, &nc) == SME_EINVAL, "struct_nx0");
        m.nx = 4;
        m.bc[0] = SME_BC_PERIODIC;
        m.bc[1] = SME_BC_WALL;
        check(check_mesh(&m, 2, &nf, &nc) == SME_EINVAL, "struct_periodic_mismatch");
        m.bc[1] = SME_BC_PERIODIC;
        check(check_mesh(&m, 2, &nf, &nc) == SME_OK && nf == 7 && nc == 16, "struct_ok");
        check(check_mesh(&m, SME_MAX_LEVEL + 1, &nf, &nc) == SME_EINVAL, "level_too_high");
        check(check_mesh(nullptr, 2, &nf, &nc) == SME_EINVAL, "null_mesh");
        m.kind = SME_MESH_1D;
        m.bc[0] = 3;
        check(check_mesh(&m, 1, &nf, &nc) == SME_EINVAL, "bad_bc");
        m.kind = SME_MESH_2D_TRI;
        m.n_tri = 1;
        m.n_vert = 3;
        check(check_mesh(&m, 1, &nf, &nc) == SME_EINVAL, "tri_null_arrays");
        m.kind = 7;
        check(check_mesh(&m, 1, &nf, &nc) == SME_EINVAL, "bad_kind");
        std::printf("OK check_mesh\n");
    }
    std::printf("ALL OK\n");
    return 0;
}
