/*
 * decmg -- geometric multigrid for the discrete-exterior-calculus 0-form Laplacian on
 * MI355X (gfx950).  C ABI of libdecmg.so.
 *
 * The method (arXiv 2508.12501):
 *   - meshes are 2-D embedded simplicial complexes (Def. 1); a hierarchy is built by binary
 *     1-to-4 or cubic 1-to-9 subdivisions, or from given meshes and geometric maps, each map
 *     f encoded by its matrix M(f) of Def. 4 (composition: Prop. 2);
 *   - on every level the operator is rediscretised (Sec. 3.1): L = d0^T star1 d0, with star1
 *     the circumcentric |dual edge|/|primal edge| ratio and star0 the dual-cell area
 *     (Eq. hodge0-laplacian; the paper's Delta_0 equals -star0^{-1} L);
 *   - interpolation is P = M(f)^T (Def. 5); restriction is R = P^T, the stiffness-form
 *     counterpart of the row-normalised operator of Def. 6;
 *   - V-, W- or F-cycles with weighted-Jacobi, multicolour Gauss-Seidel or CG smoothing and
 *     an exact coarsest solve are used as a solver and as a (flexible) CG preconditioner
 *     (Sec. 2, Sec. 3.1); the Darcy pressure step of porous convection solves
 *     d0^T star1 K d0 p = rhs (Sec. 3.2, Eq. poisson), one step at a time or inside an
 *     adaptive Runge-Kutta integration.
 *
 * Conventions shared by every entry point:
 *   - Every call returns an mg_status.  Nothing throws across the ABI.  On failure
 *     mg_last_error() returns a message (thread-local, valid until the next failing call).
 *   - Vectors passed to operator and solver calls are DEVICE pointers to contiguous arrays
 *     of one value per vertex of the named level, in the natural vertex numbering: base mesh
 *     ids, then after each subdivision coarse ids are kept; a binary subdivision gives the
 *     midpoint of coarse edge e id V_coarse + e, a cubic one gives the points of edge e ids
 *     V_coarse + 2e (next to its lower endpoint) and V_coarse + 2e + 1, and the centroid of
 *     triangle t id V_coarse + 2 E_coarse + t; levels from given maps keep their meshes' own
 *     ids.  Edges are numbered by first appearance scanning triangles and their sides (v0v1,
 *     v1v2, v2v0) and are oriented from the smaller to the larger id.
 *     The caller owns these buffers; the library never frees or keeps them.
 *   - `stream` is a hipStream_t (NULL = the null stream).  All device work of a call is
 *     enqueued on it; calls that return host-side results (solver statistics) synchronise
 *     it before returning.
 *   - dtype is MG_F64 (double) or MG_F32 (float) for the calls that take `const void*`.
 *   - Handles are not thread-safe; distinct handles may be used from distinct threads.
 *   - Zero-Dirichlet hierarchies iterate on interior vertices only.  Boundary rows are
 *     identity rows: solvers return x = b there, operator calls return y = x there.
 */
#ifndef DECMG_H
#define DECMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MG_OK = 0,
  MG_EINVAL = 1,      /* bad argument or malformed mesh */
  MG_ENOMEM = 2,      /* host or device allocation failed */
  MG_EDEVICE = 3,     /* a HIP runtime call failed; the HIP error string is in the message */
  MG_ENOCONV = 4,     /* max_iter reached before rtol; result and x are still filled */
  MG_EBREAKDOWN = 5,  /* CG breakdown: p^T A p <= 0 or a non-positive preconditioned norm */
  MG_ENONFINITE = 6,  /* a non-finite value in the input or in a residual norm */
  MG_EINCOMPAT = 7    /* natural-boundary (singular) system whose right-hand side b is outside
                         the operator's range, |sum b| > 1e-8 sum |b| (mg_pcg and mg_solve
                         with mg_opts.compat_check set) */
} mg_status;

enum { MG_F64 = 0, MG_F32 = 1 };
enum { MG_BC_DIRICHLET0 = 0, MG_BC_NATURAL = 1 };
enum { MG_OUTER_CG = 0, MG_OUTER_FCG = 1, MG_OUTER_IR = 2 };
/* Internal (device) order of a level's unknowns.  Results do not depend on it beyond
 * summation order; it only changes memory locality.  STRIPES: strips one median edge length
 * wide across the axis of largest extent, sorted along the second axis (row-major on grids);
 * MORTON: Z-order of the coordinates. */
enum { MG_ORDER_STRIPES = 0, MG_ORDER_MORTON = 1 };

typedef struct dec_mesh dec_mesh;
typedef struct mg_hierarchy mg_hierarchy;

/* Message of the last failing call on this thread ("" if none). */
const char* mg_last_error(void);
/* ABI revision of this header. */
int32_t mg_abi_version(void);

/* ------------------------------------------------------------------ meshes (host)
 * Def. 1: a point cloud with triangles given by vertex triples.  Edges and face maps are
 * derived.  The mesh is copied; the caller keeps ownership of its arrays.  Rejected with
 * MG_EINVAL: nv < 3, nt < 1, an index out of range, a degenerate or duplicate triangle, an
 * edge shared by more than two triangles, a vertex in no triangle, a non-finite coordinate.
 */
mg_status dec_mesh_from_arrays(int64_t nv, const double* xyz /* nv x 3 */, int64_t nt,
                               const int32_t* tri /* nt x 3 */, dec_mesh** out);
/* Unit square, ncells x ncells cells; vertex (i,j) at (i/n, j/n, 0) has id j*(n+1)+i;
 * cell (i,j) (j outer) gives triangles (a,b,c), (a,c,d) with a=(i,j), b=(i+1,j),
 * c=(i+1,j+1), d=(i,j+1). */
mg_status dec_mesh_square_grid(int32_t ncells, dec_mesh** out);
/* Unit icosahedron: the cyclic permutations of (0, +-1, +-phi) in the order
 * (-1,phi,0) (1,phi,0) (-1,-phi,0) (1,-phi,0) (0,-1,phi) (0,1,phi) (0,-1,-phi) (0,1,-phi)
 * (phi,0,-1) (phi,0,1) (-phi,0,-1) (-phi,0,1), normalised; faces are the vertex triples at
 * mutual distance 2 in lexicographic order, oriented outward. */
mg_status dec_mesh_icosahedron(dec_mesh** out);
void dec_mesh_free(dec_mesh* m);

/* ------------------------------------------------------------------ hierarchy
 * n_subdiv subdivisions of the base (Sec. 2.2.1), each binary (1-to-4: edge midpoints) or
 * cubic (1-to-9: two points per edge at 1/3 and 2/3, one per triangle at the centroid; the
 * interpolation holds the barycentric weights 2/3, 1/3 and 1/3, 1/3, 1/3); project_sphere
 * pushes every new point radially onto the unit sphere.  All DEC operators are rebuilt on
 * every level (Sec. 3.1).  Device memory is allocated with hipMalloc and owned by the handle.
 * The fused single-workgroup bottom of the cycle covers binary levels only; batched solves
 * take hierarchies without cubic levels. */
typedef struct {
  int32_t n_subdiv;
  int32_t project_sphere;
  int32_t bc;      /* MG_BC_DIRICHLET0 (boundary vertices fixed at 0) or MG_BC_NATURAL */
  int32_t order;   /* internal order of the unknowns: MG_ORDER_STRIPES (0) or MG_ORDER_MORTON */
  int32_t cubic_mask;  /* bit k set: the (k+1)-th subdivision (producing level k+1) is cubic */
} mg_hier_opts;

mg_status mg_hierarchy_build(const dec_mesh* base, const mg_hier_opts* opts, void* stream,
                             mg_hierarchy** out);
void mg_hierarchy_free(mg_hierarchy* h);

typedef struct {
  int32_t n_levels;      /* levels 0 (base) .. n_levels-1 (finest) */
  int32_t level;
  int64_t nv, ne, nt;
  int64_t n_unknowns;    /* interior vertices (Dirichlet) or all vertices (natural) */
  int64_t nnz_operator;  /* stored off-diagonal entries of the device operator */
  int32_t index_bytes;   /* bytes per stored column index of the device operator (2 or 4) */
  int32_t scheme;        /* how the level was made: 0 base, 1 binary, 2 cubic subdivision,
                            3 a given geometric map (mg_hierarchy_build_maps) */
  int32_t fused_tiles;   /* workgroup tiles of the fused cycle legs (mg_opts.fuse_levels), or 0
                            when the level runs one launch per step */
  int32_t fused_tile_rows;  /* rows the tiles hold in total, own rows and overlap */
  int32_t weight_bytes32;   /* bytes per stored weight read by the FP32 row kernels (2 or 4):
                               2 when every weight is exactly an IEEE binary16 number */
  int32_t weight_bytes64;   /* the same for the FP64 row kernels (2, 4 or 8) */
  int32_t uniform_width;    /* entries of every operator slice when they are all equal, else -1 */
  int32_t rows_per_thread;  /* rows each thread of the sweep, residual and apply kernels takes */
  int32_t interp_packed16;  /* 1: the per-step interpolation onto this level reads its two
                               parents as int16 offsets from a per-64-row base (one 32-bit word
                               per row); 0: two int32 ids, or a weighted scheme, or level 0.
                               Packing is skipped when a DECMG_NO_PACKED_TRANSFERS environment
                               variable is set at build time. */
  int32_t restrict_offsets16;  /* 1: the per-step restriction onto level-1 reads int16 offsets
                                  from the kept vertex; 0: int32 ids (same condition) */
  int32_t row_patterns;  /* distinct row patterns (sequences of column offset and weight) the
                            two-row sweep, residual, apply and direction-update kernels read
                            through one byte per row, when a level of uniform width with 16-bit
                            offsets has at most 256 of them; 0: they read the SELL arrays.
                            Skipped when a DECMG_NO_ROW_PATTERNS environment variable is set
                            when the weights are built */
  int32_t restrict_width;  /* entries (midpoints) of every list of the binary restriction onto
                              level-1 when all its slices have one width, else -1 (also on the
                              base level and weighted levels) */
} mg_level_info;
mg_status mg_hierarchy_info(const mg_hierarchy* h, int32_t level, mg_level_info* out);

/* Host copies of one level, natural numbering.  Any pointer may be NULL to skip it.
 * Sizes: xyz nv*3, tri nt*3, edges ne*2 (lo,hi), tri_edges nt*3, tri_sign nt*3 (+1 where
 * the triangle's boundary cycle runs lo->hi), star0 nv, star1 ne, boundary nv (1 = on a
 * boundary edge), parents nv*2 (binary levels: coarse vertex ids (a,b) of each fine vertex,
 * a == b for kept vertices; row j of M(f)^T is 1/2 e_a + 1/2 e_b; MG_EINVAL on a cubic level,
 * see mg_hierarchy_export_interp). */
mg_status mg_hierarchy_export(const mg_hierarchy* h, int32_t level, double* xyz, int32_t* tri,
                              int32_t* edges, int32_t* tri_edges, int8_t* tri_sign,
                              double* star0, double* star1, uint8_t* boundary,
                              int32_t* parents);
/* ------------------------------------------------------------------ geometric maps
 * A geometric map f: X -> Y between triangle meshes, encoded as its matrix M(f) (Def. 4) in
 * compressed sparse column form: n_rows = vertices of Y, n_cols = vertices of X, and column j
 * holds the global barycentric coordinates of f(x_j) in Y.  Host arrays owned by the caller;
 * colptr has n_cols + 1 entries starting at 0, rowval and nzval colptr[n_cols] entries. */
typedef struct {
  int64_t n_rows;
  int64_t n_cols;
  const int64_t* colptr;
  const int32_t* rowval;
  const double* nzval;
} mg_geomap;

/* A hierarchy over given meshes related by given geometric maps (Sec. 2.2.1: interpolation by
 * M(f)^T, restriction by M(f); the meshes need not be nested, and each level's operators are
 * rediscretised on its own mesh, Sec. 3.1).  meshes[0] is the coarsest of n_levels >= 1;
 * maps[l] (n_levels - 1 of them) is f: mesh l+1 -> mesh l.  Every column of a map must hold
 * 1 to 3 entries on distinct rows that are the vertices of one simplex of the coarser mesh (a
 * vertex, an edge or a triangle), with finite nonnegative weights summing to 1 within 1e-12;
 * MG_EINVAL names the first column that does not.  opts->bc and opts->order apply as in
 * mg_hierarchy_build; opts->n_subdiv, project_sphere and cubic_mask must be 0.  The meshes are
 * copied; the caller keeps ownership of meshes and maps.  mg_hierarchy_set_vertex_coeff is
 * accepted only when every map keeps the coarse vertex ids (column j is e_j for every coarse
 * vertex j), as subdivisions do; batched solves refuse such hierarchies. */
mg_status mg_hierarchy_build_maps(int32_t n_levels, const dec_mesh* const* meshes,
                                  const mg_geomap* maps, const mg_hier_opts* opts, void* stream,
                                  mg_hierarchy** out);

/* Composition of geometric maps, M(g o f) = M(g) M(f) (Prop. 2), for f: X -> Y and g: Y -> Z
 * (f->n_rows == g->n_cols).  Host computation.  Column j of the result sums, over the entries
 * (k, a) of column j of f, a times column k of g; rows ascend and exact zeros are dropped.
 * Call with colptr, rowval and nzval null to get the entry count in *nnz; then call again with
 * colptr of f->n_cols + 1 entries and rowval / nzval of at least *nnz entries (*nnz is read as
 * their capacity: MG_EINVAL if too small).  Maps are checked only for index ranges here. */
mg_status mg_geomap_compose(const mg_geomap* g, const mg_geomap* f, int64_t* colptr,
                            int32_t* rowval, double* nzval, int64_t* nnz);

/* The interpolation M(f)^T into level >= 1 of any scheme (Def. 4, Def. 5): row j as three
 * (coarse vertex, weight) pairs, host arrays parents nv*3 and weights nv*3 (unused slots
 * repeat the first parent with weight 0). */
mg_status mg_hierarchy_export_interp(const mg_hierarchy* h, int32_t level, int32_t* parents,
                                     double* weights);

/* Darcy coefficient (Sec. 3.2, Eq. dec_darcy): k_vertex is a device array of nv_finest
 * positive values.  Every level takes the values at its own vertices (injection) and
 * uses edge weights star1_e * (k_lo + k_hi)/2.  Passing NULL restores k = 1.  MG_EINVAL on a
 * hierarchy from mg_hierarchy_build_maps whose maps do not keep the coarse vertex ids. */
mg_status mg_hierarchy_set_vertex_coeff(mg_hierarchy* h, const double* k_vertex, void* stream);

/* The same with the coefficient given by its logarithm (the permeability k = exp(g) of the
 * porous experiments, Sec. 3.2): the library forms k_v = exp(g_v) and sets it as above.
 * g_vertex: device array of nv_finest finite values.  MG_EINVAL as above. */
mg_status mg_hierarchy_set_log_coeff(mg_hierarchy* h, const double* g_vertex, void* stream);

/* Chain rule through k = exp(g): grad_g_v += k_v grad_k_v for the vertex coefficient the
 * hierarchy holds (k = 1 when none is set), so that a gradient with respect to k (the grad_k
 * of mg_pcg_adjoint and porous_step_adjoint) becomes one with respect to g.  Device arrays of
 * nv_finest doubles; grad_g ACCUMULATES.  MG_EINVAL when the hierarchy holds an edge
 * coefficient. */
mg_status mg_hierarchy_coeff_grad_log(mg_hierarchy* h, const double* grad_k, double* grad_g,
                                      void* stream);

/* Darcy coefficient as an edge field (Sec. 3.2, Eq. dec_darcy: K acts on the 1-form d0 p edge
 * by edge): k_edge is a device array of ne_finest positive values in the natural edge order of
 * the finest level, whose operator uses w_e = star1_e k_e.  Coarser levels take, for each of
 * their edges, the mean of the coefficients of the fine edges it was split into (its two
 * halves under a binary subdivision, its three thirds under a cubic one), recursively.  It
 * replaces a vertex coefficient (and the other way round); NULL restores k = 1.  The porous
 * step uses k_e as its Darcy coefficient.  The vertex-coefficient gradients (grad_k of
 * mg_pcg_adjoint and porous_step_adjoint) are refused while it is set; mg_pcg_adjoint's grad_w
 * gives the gradient for the finest edge weights.  MG_EINVAL for hierarchies from
 * mg_hierarchy_build_maps (no edge correspondence between levels) and for non-positive or
 * non-finite values. */
mg_status mg_hierarchy_set_edge_coeff(mg_hierarchy* h, const double* k_edge, void* stream);

/* Fault injection for tests of the failure handling (not part of the method): flags is 0 or
 * a combination of the MG_DEBUG_ bits, kept by the hierarchy until changed.
 * MG_DEBUG_ZERO_PRECOND32: every FP32 cycle of mg_pcg (and of the solves built on it) returns
 * zero, on which a preconditioned Krylov loop breaks down (p^T A p = 0) and iterative
 * refinement makes no progress, so that the FP64 fallback (mg_opts.stall_checks) must take
 * over.  Batched solves ignore it.  MG_EINVAL for unknown bits. */
#define MG_DEBUG_ZERO_PRECOND32 1
mg_status mg_hierarchy_set_debug(mg_hierarchy* h, int32_t flags);

/* ------------------------------------------------------------------ operators (device)
 * b = star0 f on `level` (Sec. 3.1 right-hand side of L u = star0 f); Dirichlet: b = 0 on
 * the boundary.  f, b: nv doubles. */
mg_status dec_star0_apply(mg_hierarchy* h, int32_t level, const double* f, double* b,
                          void* stream);
/* y = A x with A = L (natural) or the Dirichlet form M L M + (I - M). */
mg_status dec_laplacian_apply(mg_hierarchy* h, int32_t level, int32_t dtype, const void* x,
                              void* y, void* stream);
/* nsweeps of weighted Jacobi, x <- x + omega D^{-1} (b - A x), in place on x. */
mg_status mg_smooth(mg_hierarchy* h, int32_t level, int32_t dtype, int32_t nsweeps,
                    double omega, const void* b, void* x, void* stream);
/* r_coarse = R r_fine from `level` to level-1, R = M(f) (= P^T), zero at coarse Dirichlet
 * vertices.  r_fine has nv(level) entries, r_coarse nv(level-1).  Fine boundary entries
 * of r_fine are ignored on Dirichlet hierarchies. */
mg_status mg_restrict(mg_hierarchy* h, int32_t level, int32_t dtype, const void* r_fine,
                      void* r_coarse, void* stream);
/* x_fine += P e_coarse, P = M(f)^T (Def. 5), from level-1 to `level`.  Dirichlet: coarse
 * boundary entries of e_coarse are taken as 0 and fine boundary entries of x are kept. */
mg_status mg_prolong(mg_hierarchy* h, int32_t level, int32_t dtype, const void* e_coarse,
                     void* x_fine, void* stream);

/* ------------------------------------------------------------------ solvers */
/* Cycle shapes (Sec. 2 names V-, W- and F-cycles): the coarse-grid correction of a level is
 * one cycle of the same shape from zero (V), two (W: the second starts from the first's
 * result), or an F-cycle followed by a V-cycle (F).  The W-cycle is symmetric like the V-cycle;
 * the F-cycle is not, so pair it with MG_OUTER_FCG or MG_OUTER_IR. */
#define MG_CYCLE_V 0
#define MG_CYCLE_W 1
#define MG_CYCLE_F 2
/* Smoothers: weighted Jacobi (omega), or multicolour Gauss-Seidel (Sec. 3.1 and 3.2 smooth
 * with Gauss-Seidel): the unknowns of each level are coloured greedily in increasing vertex id
 * (smallest colour not used by a coupled, lower-numbered unknown); pre-smoothing sweeps the
 * colour classes in increasing order, post-smoothing in decreasing order, so the cycle stays
 * symmetric; omega is not used.  The batched solve supports Jacobi only. */
#define MG_SMOOTH_JACOBI 0
#define MG_SMOOTH_GS 1
/* CG smoothing (the smoother of the paper's V-cycle timings, Fig. time_per1vcycle): nu1 steps
 * of unpreconditioned CG on the level's unknowns before the coarse-grid correction and nu2
 * after it; a step with non-positive curvature leaves x unchanged.  The cycle is then a
 * nonlinear map, so mg_pcg requires MG_OUTER_FCG or MG_OUTER_IR with it. */
#define MG_SMOOTH_CG 2

typedef struct {
  int32_t nu1, nu2;      /* pre/post Jacobi sweeps (2, 2) */
  double omega;          /* Jacobi weight (0.8) */
  int32_t precision;     /* MG_F64 or MG_F32: arithmetic of the V-cycle preconditioner */
  int32_t outer;         /* MG_OUTER_CG, MG_OUTER_FCG or MG_OUTER_IR (mg_pcg only) */
  double rtol;           /* stop at ||b - A x||_2 <= rtol ||b||_2 (1e-10) */
  int32_t max_iter;      /* (200) */
  int32_t check_every;   /* iterations enqueued between host convergence checks (4) */
  int32_t use_graph;     /* replay the iteration as a hipGraph (1) */
  int32_t cycle;         /* MG_CYCLE_V, MG_CYCLE_W or MG_CYCLE_F (V) */
  int32_t smoother;      /* MG_SMOOTH_JACOBI, MG_SMOOTH_GS or MG_SMOOTH_CG (Jacobi) */
  int32_t fuse_levels;   /* 1: on binary levels of at most 2^19 unknowns, weighted-Jacobi
                            cycles run the smoothing, residual and transfers of each leg in one
                            launch over overlapping workgroup tiles (same results bit for bit);
                            0: one launch per step (1) */
  int32_t compat_check;  /* natural-boundary systems, mg_pcg and mg_solve: 1 refuses a
                            right-hand side outside the operator's range, |sum b| > 1e-8 sum |b|,
                            with MG_EINCOMPAT (x = 0); 0 projects it onto the range by removing
                            its vertex mean (0) */
  int32_t stall_checks;  /* mg_pcg with precision MG_F32: the FP32-preconditioned loop counts as
                            stagnating after this many host convergence checks in a row (after
                            the first) whose loop residual is not below the smallest seen
                            before; it then, or on a breakdown or a non-finite value of that
                            loop, continues from x with the FP64 cycle (mg_result.fp64_fallback).
                            0: no detection and no fallback.  0..1000 (3) */
} mg_opts;
void mg_opts_default(mg_opts* o);

typedef struct {
  int32_t iterations;          /* outer iterations (cycles for mg_solve) */
  int32_t status;              /* the mg_status of the call */
  double rel_residual;         /* true ||b - A x|| / ||b|| at exit, computed in FP64 */
  double rel_residual_loop;    /* the recursively updated value the loop stopped on */
  /* Residual history, filled when history is not null and history_cap > 0 (set both before
   * the call, or zero-initialise the struct to skip it): history[i] is the loop's relative
   * residual after iteration i + 1 (the recursively updated value for CG and FCG, the true one
   * for iterative refinement and mg_solve), for the first min(iterations, history_cap, 4096)
   * iterations, whose count is returned in history_len.  Host memory owned by the caller.
   * Batched solves leave it unused. */
  double* history;
  int32_t history_cap;
  int32_t history_len;
  int32_t fp64_fallback;       /* 1: the FP32-preconditioned loop stagnated, broke down or met a
                                  non-finite value, and the solve went on with the FP64 cycle */
} mg_result;

/* One V(nu1,nu2) cycle on `level` (normally the finest), in place: x <- V(b, x).  dtype
 * selects FP64 or FP32 arithmetic (b and x of that type); the coarsest solve is FP64. */
mg_status mg_vcycle(mg_hierarchy* h, const mg_opts* o, int32_t level, int32_t dtype,
                    const void* b, void* x, void* stream);
/* Stand-alone multigrid: V-cycles from x = 0 until rtol (FP64).  Natural-boundary systems
 * project b onto the range (its vertex mean removed), or with o->compat_check refuse one with
 * |sum b| > 1e-8 sum |b| (MG_EINCOMPAT, x = 0). */
mg_status mg_solve(mg_hierarchy* h, const mg_opts* o, const double* b, double* x,
                   mg_result* res, void* stream);
/* Krylov solve with one V-cycle as preconditioner, from x = 0: CG (symmetric FP64 cycle),
 * flexible CG FCG(1) (beta = -z^T q_prev / p_prev^T q_prev) or iterative refinement.  With
 * precision MG_F32 the cycle runs in FP32 on a scaled FP32 copy of the FP64 residual; the
 * residual, the solution update and the coarsest solve stay FP64.  Natural-BC hierarchies
 * remove the vertex mean of b, of every preconditioned vector and of x; with
 * o->compat_check a right-hand side with |sum b| > 1e-8 sum |b| is refused with MG_EINCOMPAT
 * (x = 0).
 * Stopping (Sec. 3.1): MG_OK only when the true relative residual ||b - A x|| / ||b||,
 * recomputed in FP64 from x, is <= rtol.  CG and FCG iterate on the recursively updated
 * residual; when that has met rtol but the true one has not, the iteration restarts from x
 * (r = b - A x, the next direction the preconditioned residual), within max_iter in total;
 * MG_ENOCONV when max_iter is reached first (x and the result are still filled).
 * FP32 fallback: with precision MG_F32 and o->stall_checks > 0, a loop that stagnates (see
 * stall_checks), breaks down or meets a non-finite value restarts from x in the same way with
 * the FP64 cycle, once, within the same max_iter; mg_result.fp64_fallback reports it, and the
 * status is that of the FP64 loop. */
mg_status mg_pcg(mg_hierarchy* h, const mg_opts* o, const double* b, double* x,
                 mg_result* res, void* stream);

/* Adjoint of mg_pcg (reverse-mode differentiation through the solve of Sec. 3.1; the paper
 * itself does not differentiate, this is an extension of its method).  For
 * u = A^-1 b (A^+ on natural-BC hierarchies) and an upstream gradient g_u = dJ/du, solves
 * A lambda = g_u with the same options and returns dJ/db = lambda in grad_b (nv doubles).
 * When grad_k is not null it ACCUMULATES dJ/dk_v for the vertex coefficient k
 * (k_e = (k_lo + k_hi)/2 on the finest level): grad_k_v += 1/2 sum over the edges e at v of
 * -star1_e (d0 lambda)_e (d0 u)_e, with u the solution the forward call returned (u_fine,
 * nv doubles; boundary vertices of a Dirichlet hierarchy count as zero).  When grad_w is not
 * null it ACCUMULATES dJ/dw_e for the finest operator's edge weights w_e = star1_e k_e (the
 * Hodge weights of L = d0^T diag(w) d0): grad_w_e += -(d0 lambda)_e (d0 u)_e, ne doubles in
 * the natural edge order; it also needs u_fine.  Vertex vectors are device pointers in
 * natural vertex order on the finest level. */
mg_status mg_pcg_adjoint(mg_hierarchy* h, const mg_opts* o, const double* u_fine,
                         const double* grad_u, double* grad_b, double* grad_k, double* grad_w,
                         mg_result* res, void* stream);

/* ------------------------------------------------------------------ batched solves
 * Many independent solves at once (not in the paper: a throughput mode for many small and
 * mid-size problems).  Instance i solves A_i x_i = b_i on hierarchy h[i] with the FCG(1)
 * recurrence of mg_pcg (outer must be MG_OUTER_FCG; precision MG_F32 or MG_F64 selects the
 * V-cycle arithmetic), with its own scalars and stopping test.  Instances that share a
 * hierarchy handle are packed into groups of up to max_cols right-hand sides solved together:
 * the operator is read once per group for all its columns.  Groups run concurrently on
 * `streams` internal streams; each group's iteration is replayed as a hipGraph when
 * o->use_graph is set.  The hierarchies must outlive the batch and must not be used by another
 * call while mg_batch_solve runs. */
typedef struct mg_batch mg_batch;
typedef struct {
  int32_t max_cols;     /* widest group: a power of two in 1..64 (default 32) */
  int32_t pad_groups;   /* 1: a hierarchy's last group is padded up to a power of two;
                           0: its instances are split exactly into power-of-two groups (1) */
  int32_t streams;      /* internal streams, 1..4 (4) */
  int32_t reserved;
} mg_batch_tuning;

/* h: n hierarchy handles (one per instance, repeated handles share a hierarchy).  tune
 * (nullable): explicit tuning; else tune_cache (nullable path of a text file written by
 * mg_batch_autotune) supplies the tuning recorded for this mix of instances, else defaults.
 * Allocates every device buffer of the batch. */
mg_status mg_batch_create(mg_hierarchy* const* h, int32_t n, const mg_opts* o,
                          const mg_batch_tuning* tune, const char* tune_cache, mg_batch** out);
/* b, x: host arrays of n device pointers; b[i] and x[i] hold nv doubles of instance i's finest
 * level in natural vertex order (x[i] is overwritten; Dirichlet vertices get b).  res
 * (nullable): n results.  Returns MG_OK when every instance converged, else the first failing
 * instance status (res tells which).  Synchronises `stream` with the batch's streams and the
 * host before returning. */
mg_status mg_batch_solve(mg_batch* bt, const double* const* b, double* const* x, mg_result* res,
                         void* stream);
/* Tries every tuning of max_cols in {8,16,32,64} x pad_groups in {1,0} x streams in {1,2,4} on
 * these inputs (one warm-up and `reps` timed solves each), keeps the fastest, and records it in
 * tune_cache (nullable) under this mix of instances.  chosen, best_ms (nullable) report it. */
mg_status mg_batch_autotune(mg_batch* bt, const double* const* b, double* const* x, int32_t reps,
                            const char* tune_cache, mg_batch_tuning* chosen, double* best_ms);
/* Current tuning and number of groups. */
mg_status mg_batch_info(const mg_batch* bt, mg_batch_tuning* tune, int32_t* n_groups);
void mg_batch_free(mg_batch* bt);

/* ------------------------------------------------------------------ porous convection
 * One forward-Euler step of the Darcy-Boussinesq model of Sec. 3.2 (advection factor 1/phi,
 * buoyancy alpha rho0 |g| = 1, permeability scale k/eta = 1, diffusivity
 * kappa = delta_T y_len / (phi Ra), the paper's product for lambda / (rho0 c_p); the scaled form
 * takes delta_T = y_len = 1) on the finest level of a natural-BC hierarchy of a mesh in the
 * plane, with permeability k = the hierarchy's vertex coefficient:
 *   b1_e = (y_hi - y_lo)(T_lo + T_hi)/2                 buoyancy 1-form
 *   L_K p = d0^T W b1,  W = star1 k_e                    pressure (zero-mean, MG-PCG)
 *   q = -k_e (d0 p - b1)                                 Darcy flux
 *   T' = T + dt mask/star0 ( -(1/phi) 1/2 |d0|^T (star1 q d0 T) - kappa L T )
 * where mask is 0 on the vertices with the smallest and the largest y (fixed temperature
 * walls) and 1 elsewhere. */
typedef struct {
  double Ra;        /* Rayleigh number (> 0) */
  double phi;       /* porosity (> 0) */
  double dt;        /* time step (> 0; not read by porous_rhs and porous_integrate) */
  mg_opts solve;    /* options of the pressure solves (mg_pcg) */
  double delta_T;   /* wall temperature difference in kappa (> 0; 1 in the scaled form) */
  double y_len;     /* extent of the domain in y in kappa (> 0; 1 in the scaled form) */
} porous_params;

/* T_out = step(T).  p (nullable) receives the pressure.  res (nullable) reports the pressure
 * solve.  T, T_out, p: nv doubles on the device, natural order; T_out must not alias T.
 * MG_EINVAL for a hierarchy with Dirichlet boundaries or a non-positive parameter. */
mg_status porous_step(mg_hierarchy* h, const porous_params* prm, const double* T, double* T_out,
                      double* p, mg_result* res, void* stream);
/* The right-hand side of the method of lines (Sec. 3.2): dTdt = mask/star0 ( ... ) of the step
 * above without the time step, so that porous_step is T + dt * dTdt.  Same arguments and
 * errors as porous_step; dTdt must not alias T. */
mg_status porous_rhs(mg_hierarchy* h, const porous_params* prm, const double* T, double* dTdt,
                     double* p, mg_result* res, void* stream);
/* Transpose of the step's Jacobian: lambda_out = (dT'/dT)^T lambda, with the pressure solve
 * differentiated through (one adjoint-pressure solve, zero-mean psi of
 * L_K psi = d0^T (k_e star1_e (mu_lo + mu_hi)/2 (d0 T)_e), mu = mask lambda / star0).  p
 * (nullable) is the pressure that porous_step returned for this T (recomputed when null).
 * grad_k (nullable) ACCUMULATES lambda^T dT'/dk_v (nv doubles).  psi (nullable) receives the
 * adjoint pressure (nv doubles).  lambda_out must not alias lambda. */
mg_status porous_step_adjoint(mg_hierarchy* h, const porous_params* prm, const double* T,
                              const double* p, const double* lambda, double* lambda_out,
                              double* grad_k, double* psi, void* stream);

/* Adaptive time integration of dT/dt = porous_rhs(T) from t = 0 to t_end (Sec. 3.2: method of
 * lines; the paper integrates with an explicit adaptive Runge-Kutta 5(4) pair).  The pair here
 * is Dormand-Prince 5(4): seven stages, the last equal to the next step's first, so six
 * right-hand sides per step.  The error of a step of size h is the weighted RMS norm
 *   err = sqrt(mean_i ((T5 - T4)_i / (atol + rtol max(|T_i|, |T5_i|)))^2)
 * of the difference between the 5th-order result T5 (which is kept) and the embedded
 * 4th-order one.  A step is accepted when err <= 1; the next step size is
 * h min(fmax, max(0.2, 0.9 err^(-1/5))), with fmax = 10, or 1 right after a rejection.  The
 * first step is h0 when h0 > 0, otherwise it is chosen from the first two right-hand sides by
 * Hairer, Norsett and Wanner's starting-step rule.  A step that would pass within 1% of a save
 * time or of t_end is cut to land on it.  fixed_step = 1 takes steps of h0 without error
 * control.  The first pressure solve starts from zero, the second from the first's result,
 * every later one from the linear extrapolation in time of the last two pressures (the
 * extrapolation factor clamped to [-2, 2]). */
typedef struct {
  porous_params model;  /* model.dt is not read */
  double t_end;         /* > 0 */
  double rtol, atol;    /* > 0 (adaptive mode) */
  double h0;            /* first step (> 0), or 0 for automatic (adaptive mode only) */
  int32_t max_steps;    /* limit on accepted + rejected steps (> 0) */
  int32_t fixed_step;
} porous_rk_opts;

typedef struct {
  int32_t accepted, rejected, rhs_evals, reserved;
  int64_t pressure_iterations;  /* summed over all pressure solves */
  double t;                     /* time reached */
  double h_min, h_max;          /* smallest and largest accepted step */
} porous_rk_stats;

/* T0: nv doubles (device, natural order).  t_save: n_save strictly increasing host times in
 * (0, t_end]; T_save (device, nullable when n_save == 0) receives T at each of them, row i at
 * T_save + i nv.  T_end (device) receives T(t_end).  stats (nullable).  MG_ENOCONV when
 * max_steps is reached or the step size falls below 1e-14 t_end (T_end then holds the last
 * accepted state); a failed pressure solve returns its status.  Allocates and frees its work
 * vectors (10 of nv + 1 doubles) on every call. */
mg_status porous_integrate(mg_hierarchy* h, const porous_rk_opts* o, const double* T0,
                           int32_t n_save, const double* t_save, double* T_save, double* T_end,
                           porous_rk_stats* stats, void* stream);

/* porous_integrate for callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid allocation): the same integration, arguments, results
 * and errors, bit for bit, but it calls no hipMalloc, hipFree or other allocating routine.
 * Its work vectors live in a static 8 MiB device work area, one per GPU, held until the
 * process ends: 12 (n + 1) doubles plus reduction partials, so a hierarchy of up to about
 * 87,000 finest-level unknowns (MG_EINVAL with the sizes beyond that; the 257 x 257 grid has
 * 66,049).  The pressure solves run eagerly whatever model.solve.use_graph says, since
 * capturing a graph allocates.  Set-up first: the hierarchy's porous data must exist, which
 * one porous_step, porous_rhs or porous_integrate call on it creates (MG_EINVAL otherwise);
 * a later change of the vertex coefficient is taken up with a host-to-device copy.  Calls
 * share their GPU's work area and each starts by clearing it, so calls that overlap on one
 * GPU (other streams, other threads, other hierarchies) race and must be serialised by the
 * caller. */
mg_status porous_integrate_noalloc(mg_hierarchy* h, const porous_rk_opts* o, const double* T0,
                                   int32_t n_save, const double* t_save, double* T_save,
                                   double* T_end, porous_rk_stats* stats, void* stream);

/* ------------------------------------------------------------------ measurement
 * Times `reps` back-to-back launches of one kernel of the path on `level` with hipEvents
 * recorded on `stream`, and returns the mean duration per launch in milliseconds.
 * kernel: 0 = Jacobi sweep, 1 = operator apply, 2 = residual, 3 = restriction,
 * 4 = interpolation.  Uses the hierarchy's own work vectors. */
mg_status mg_time_kernel(mg_hierarchy* h, int32_t kernel, int32_t level, int32_t dtype,
                         int32_t reps, void* stream, double* ms_per_launch);

/* In-solve timing of the smoother.  Between mg_probe_begin and mg_probe_end, every weighted-
 * Jacobi sweep kernel that an eager solve (use_graph = 0) launches on `level` in arithmetic
 * `dtype` is launched with start/stop hipEvents stamped by its dispatch on the solve's stream
 * (kernel execution time).  mg_probe_end synchronises that
 * stream and returns the mean duration per launch and the number of launches.  Sweeps replayed
 * from a captured graph are not probed. */
mg_status mg_probe_begin(mg_hierarchy* h, int32_t level, int32_t dtype);
mg_status mg_probe_end(mg_hierarchy* h, double* ms_per_launch, int32_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* DECMG_H */
