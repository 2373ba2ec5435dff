// Host-side embedded simplicial complex (Def. 1 of arXiv 2508.12501) and the binary and cubic
// subdivision maps (Sec. 2.2.1).  Built once per hierarchy level; the device only ever sees
// the operator arrays derived from it.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace decmg {

struct Mesh {
  int64_t nv = 0, ne = 0, nt = 0;
  std::vector<double> xyz;        // nv x 3
  std::vector<int32_t> tri;       // nt x 3 (v0, v1, v2)
  std::vector<int32_t> edge;      // ne x 2 (lo, hi): oriented from smaller to larger id
  std::vector<int32_t> tri_edge;  // nt x 3: sides (v0v1, v1v2, v2v0)
  std::vector<int8_t> tri_sign;   // nt x 3: +1 when the boundary cycle runs lo -> hi
  std::vector<double> star0;      // nv: circumcentric dual-cell area
  std::vector<double> star1;      // ne: |dual edge| / |primal edge|
  std::vector<uint8_t> bnd;       // nv: 1 on a boundary edge
  // For a level produced by subdivision: the coarse endpoints (a, b) of each vertex, with
  // a == b for a kept coarse vertex (row j of M(f)^T = (e_a + e_b) / 2).
  std::vector<int32_t> parent;    // nv x 2, binary subdivision only
  // Any subdivision: row j of M(f)^T as up to three (coarse vertex, weight) pairs; unused
  // slots repeat the first parent with weight 0.  Empty on the base level.
  int32_t scheme = 0;             // 0 base level, 1 binary (1-to-4), 2 cubic (1-to-9)
  std::vector<int32_t> parent3;   // nv x 3
  std::vector<double> pweight;    // nv x 3

  // Edge numbering by first appearance, face maps, orientation signs.  Returns "" or an
  // error message (edge in more than two triangles, duplicate triangle, ...).
  std::string build_topology();
  void build_stars();
  void build_boundary();
  std::string validate_vertices() const;   // every vertex in some triangle, finite coords
};

// Unit square with n x n cells split along the SW-NE diagonal.
Mesh square_grid(int32_t n);
// Unit icosahedron (cyclic permutations of (0, +-1, +-phi), normalised, outward faces).
Mesh icosahedron();
// One binary subdivision: kept vertex ids, midpoint of coarse edge e at nv + e, children
// (a,ab,ca), (ab,b,bc), (ca,bc,c), (ab,bc,ca) of coarse triangle t at 4t..4t+3.
Mesh subdivide(const Mesh& c, bool project_sphere);
// One cubic subdivision: kept vertex ids; the points of coarse edge e (oriented lo -> hi) at
// 1/3 and 2/3 of its length at nv + 2e (next to lo) and nv + 2e + 1; the centroid of coarse
// triangle t at nv + 2 ne + t; nine children per triangle with the parent's orientation,
// (a,ab1,ca2), (ab2,b,bc1), (ca1,bc2,c), (ab1,ab2,m), (bc1,bc2,m), (ca1,ca2,m), (ab1,m,ca2),
// (ab2,bc1,m), (bc2,ca1,m) at 9t..9t+8, where xy1 is the point of side xy next to x.
Mesh subdivide_cubic(const Mesh& c, bool project_sphere);

}  // namespace decmg
