// sme_mesh.h -- host-side mesh checks and triangle-mesh preprocessing.
//
// Plain C++ (no HIP): the library calls it while binding a context, and a
// CPU-only harness runs it under AddressSanitizer and UndefinedBehaviorSanitizer.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sme.h"

namespace sme {
namespace mesh {

// Largest triangle mesh: the triangle kernel addresses a cell within a field
// by a 32-bit byte offset, and 2^28 cells keep every field under 2 GiB.
constexpr int64_t kTriMaxCells = (int64_t)1 << 28;

// number of state fields of a level on a mesh kind
int nfields_of(int level, int kind);

// Validates the mesh description and level; sets the field count and the
// number of cells.  Returns SME_OK or SME_EINVAL.
int check_mesh(const sme_mesh *m, int level, int *nf, int64_t *nc);

// Triangle geometry in caller order: neighbour (or -1 = wall) and scaled
// outward normal n |e| = (ey, -ex) for face s = edge (v_s, v_{s+1}), 1 / |V|
// per triangle.  A shared edge is traversed in opposite directions by its two
// triangles, so their scaled normals are exact negatives of each other.
struct TriGeom {
    std::vector<int32_t> nbr;
    std::vector<double> sx, sy, ivol;
};

// Neighbours, scaled normals and inverse areas of a triangle mesh (caller
// order).  Returns SME_OK, or SME_EMESH with the reason in `why` (a bad
// vertex index, a degenerate or clockwise triangle, an edge of zero length, an
// edge shared by more than two triangles, or two neighbours that traverse
// their shared edge in the same direction).
int build_tri(const sme_mesh *m, TriGeom &g, std::string &why);

// Reverse Cuthill-McKee order of the triangle adjacency graph (nbr[3 t + s],
// -1 for none): order[k] is the caller cell placed at internal position k.
// Every connected component is ordered from a pseudo-peripheral start.
std::vector<int64_t> rcm_order(const std::vector<int32_t> &nbr, int64_t n);

}  // namespace mesh
}  // namespace sme
