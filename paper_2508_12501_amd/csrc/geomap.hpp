// Geometric maps between triangle meshes given by their matrices M(f) (Def. 4) in compressed
// sparse column form: checks against the target mesh, conversion into a level's interpolation
// rows, and composition M(g o f) = M(g) M(f) (Prop. 2).  Host code.
#pragma once
#include <cstdint>
#include <string>

#include "decmg.h"
#include "mesh.hpp"

namespace decmg {

// "" when every column of f is the global barycentric coordinate vector of a point of Y
// (1 to 3 distinct rows spanning one simplex of Y, finite weights >= 0 summing to 1 within
// 1e-12) and the shape is |Y| x nx; otherwise a message naming the first bad column.
std::string check_geomap(const Mesh& Y, int64_t nx, const mg_geomap& f);

// Stores column j of M(f) as row j of X's interpolation (X.parent3 / X.pweight, padded with
// the first parent at weight 0) and marks X as made by a given map.
void set_interp_from_geomap(Mesh& X, const mg_geomap& f);

// True when column j is e_j for every vertex j of the target: the map keeps coarse ids.
bool geomap_keeps_ids(const mg_geomap& f);

// M(g) M(f) with the two-call protocol of mg_geomap_compose.  Returns "" or an error.
std::string compose_geomaps(const mg_geomap& g, const mg_geomap& f, int64_t* colptr,
                            int32_t* rowval, double* nzval, int64_t* nnz);

}  // namespace decmg
