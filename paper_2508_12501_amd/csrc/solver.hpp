// Host entry points shared by the C-ABI layer.
#pragma once
#include "hier.hpp"

namespace decmg {

template <typename T>
LevelVecs<T>& vecs(Level& L);

// One V(nu1, nu2) cycle on level l for A_l x = b.  x_init == nullptr means x = 0 (the first
// pre-sweep then reads only b and the diagonal); otherwise x_init is the initial guess and
// one of its buffers.  Returns the buffer that holds the result.
template <typename T>
T* vcycle(Hierarchy& H, int l, const T* b, T* x_init, const mg_opts& o, const int* done,
          hipStream_t s);

Hierarchy* build_hierarchy(const Mesh& base, const mg_hier_opts& o);
void upload_weights(Hierarchy& H);
int run_pcg(Hierarchy& H, const mg_opts& o, const double* b_nat, double* x_nat, mg_result* res,
            hipStream_t s);
int run_mg(Hierarchy& H, const mg_opts& o, const double* b_nat, double* x_nat, mg_result* res,
           hipStream_t s);

}  // namespace decmg
