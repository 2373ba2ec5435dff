// Host-side embedded simplicial complex (Def. 1 of arXiv 2508.12501) and the binary
// subdivision map (Sec. 2.2.1).  Built once per hierarchy level; the device only ever sees
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
  std::vector<int32_t> parent;    // nv x 2, empty on the base level

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

}  // namespace decmg
