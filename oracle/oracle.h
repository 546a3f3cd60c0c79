/* FP64 CPU oracle for the layered-field method (Zayer, Mlakar, Steinberger,
 * Seidel, "Layered Fields for Natural Tessellations on Surfaces").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
 * reference used to check the HIP library.  Only the tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the library never does.
 * It shares no code, header or table with the HIP path.
 *
 * Field matrix convention: U = Phi^T, one CSR row per vertex, one column per
 * layer.  Columns 0..n_s-1 are the cells in seed order, column n_s is the base
 * layer (Section 3.2, Initialization paragraph).  Row pointers are int64,
 * column ids int32 ascending, values double.  Stored values are > 0.
 *
 * Memory: arrays returned through `T** out` arguments are malloc'd here and
 * must be released with orc_free().  Every function returns 0 on success,
 * a positive ORC_E* code otherwise.
 */
#ifndef LF_ORACLE_H
#define LF_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

/* Constants of the update.  base_mode 0 is the complete reading used
 * throughout (cells couple to the base only through the gradient term and an
 * antisymmetric band term); base_mode 1 treats the base as an ordinary layer. */
typedef struct {
  double w, a, e, mu, dt, theta;
  int32_t base_mode;
  /* Per-pair coefficients (equation (2) carries a, w, e per pair of layers;
   * the paper fixes one value each and foresees varying them, Section 3.1).
   * n_types = 0: the scalars above.  n_types > 0: layer l has type
   * types[l] (n_s + 1 entries, the base last) and a pair (j, l), j != l,
   * takes a, w, e from tab[3 * (types[j] * n_types + types[l]) + 0, 1, 2].
   * In base_mode 0 the pairs with the base keep the base reading: w = 0,
   * and e is negated for the base against a cell. */
  int32_t n_types;
  const int32_t* types;
  const double* tab;
} orc_params;

void orc_free(void* p);

/* Mesh Laplacian (Section 3.2, "Laplacian computation"): op 0 = graph
 * (L_ij = 1 per edge), op 1 = cotangent (L_ij = (cot a + cot b)/2); both
 * with L_ii = -sum_j L_ij.  Output CSR (n_v rows) includes the diagonal. */
int orc_operator(int32_t n_v, const double* V, int32_t n_f, const int32_t* F, int32_t op,
                 int64_t* ptr /* n_v+1, caller */, int32_t** col, double** val);

/* Initialisation (Algorithm 1, first line; Initialization paragraph): one
 * at each seed in its own layer, one in the base layer elsewhere. */
int orc_init(int32_t n_v, const int32_t* seeds, int32_t n_s,
             int64_t* ptr /* n_v+1 */, int32_t** col, double** val);

/* Seeds grown into regions of `rings` edge-rings (Algorithm 1, first line;
 * Initialization paragraph): each vertex within reach takes the layer of its
 * nearest seed, ties to the lowest seed index; every other vertex the base.
 * rings = 0 gives orc_init.  Output as orc_init. */
int orc_init_rings(int32_t n_v, int32_t n_f, const int32_t* F, const int32_t* seeds, int32_t n_s,
                   int32_t rings, int64_t* ptr, int32_t** col, double** val);

/* One explicit Euler step of Algorithm 1 (Jacobi form), followed by the
 * column normalisation, the theta prune and compaction.  L must include its
 * diagonal.  Optional outputs (may be NULL): margin[n_v] = smallest distance
 * of any discrete decision in the row from its threshold; skel[n_v] = size of
 * the row's active set; events = number of rows whose normalisation sum was
 * zero. */
int orc_step(int32_t n_v, int32_t n_s, const int64_t* Lp, const int32_t* Lc, const double* Lv,
             const int64_t* Up, const int32_t* Uc, const double* Uv, const orc_params* P,
             int64_t* Op /* n_v+1 */, int32_t** Oc, double** Ov,
             double* margin, int32_t* skel, int64_t* events);

/* orc_step over `threads` contiguous blocks of rows (OpenMP when built with
 * it; the blocks run one after the other otherwise).  Every row does the same
 * arithmetic as in orc_step, so the result is identical for any thread count.
 * smargin[n_v] (may be NULL) = smallest |L_t| over the row's zero entries,
 * the margin of its rows-of-interest decisions alone. */
int orc_step_threads(int32_t n_v, int32_t n_s, const int64_t* Lp, const int32_t* Lc,
                     const double* Lv, const int64_t* Up, const int32_t* Uc, const double* Uv,
                     const orc_params* P, int64_t* Op, int32_t** Oc, double** Ov, double* margin,
                     double* smargin, int32_t* skel, int64_t* events, int32_t threads);

/* n_steps free-running steps of orc_step_threads in one call (U_in is not
 * modified; the final fields go to Op[n_v+1], *Oc, *Ov).  skel_total and
 * events (may be NULL) sum the rows-of-interest sizes and empty-row events. */
int orc_run_threads(int32_t n_v, int32_t n_s, const int64_t* Lp, const int32_t* Lc,
                    const double* Lv, const int64_t* Up, const int32_t* Uc, const double* Uv,
                    const orc_params* P, int32_t n_steps, int32_t threads, int64_t* Op,
                    int32_t** Oc, double** Ov, int64_t* skel_total, int64_t* events);

/* Sharp labels (Section 5.2 and Figure 10): argmax over the cell columns of
 * a row, lowest column on ties, -1 when the row has no cell entry.
 * gap[n_v] (may be NULL) = best minus second-best cell value (second = 0 if
 * absent). */
int orc_labels(int32_t n_v, int32_t n_s, const int64_t* Up, const int32_t* Uc, const double* Uv,
               int32_t* labels, double* gap);

/* Lloyd-like re-seeding (Section 5): per cell, area-weighted centroid of the
 * barycentres of the faces having a vertex in the cell's support, line along
 * the area-weighted mean normal, closest hit, nearest vertex of the hit face.
 * status[c]: 0 moved or stayed on a hit, 1 ray miss, 2 reverted by a seed
 * collision.  margin[c]: smallest relative gap of the cell's floating-point
 * decisions (hit choice, barycentric edge tests, nearest vertex). */
int orc_lloyd(int32_t n_v, const double* V, int32_t n_f, const int32_t* F, int32_t n_s,
              const int64_t* Up, const int32_t* Uc, const double* Uv, const int32_t* seeds_in,
              int32_t* seeds_out, int32_t* status, double* margin);

/* Dual mesh (Sections 5.1 and 5.2). */
typedef struct {
  /* adjacency matrices over cells, CSR with n_s+1 pointers, no diagonal */
  int64_t* av_ptr;  int32_t* av_col;      /* vertex sharing  A_v */
  int64_t* at_ptr;  int32_t* at_col;      /* face sharing    A_t */
  int64_t* ad_ptr;  int32_t* ad_col;      /* curated adjacency   */
  /* candidate pairs (p<q) of A_t not in A_v, with their verdicts */
  int64_t n_cand;
  int32_t* cand;          /* 2*n_cand */
  int32_t* cand_state;    /* 0 rejected (no crossing), 1 kept, 2 dropped (manifold rule) */
  double* cand_margin;    /* smallest |orientation determinant| seen on the pair's faces */
  /* dual triangles, oriented */
  int64_t n_tri;
  int32_t* tri;           /* 3*n_tri */
  int64_t n_removed;      /* spurious triangles removed */
  int64_t n_conflict;     /* orientation conflicts met while propagating */
  int64_t n_nonmanifold;  /* dual edges with more than two triangles */
} orc_dual;

int orc_dual_mesh(int32_t n_v, const double* V, int32_t n_f, const int32_t* F, int32_t n_s,
                  const int64_t* Up, const int32_t* Uc, const double* Uv, const int32_t* seeds,
                  double tau, orc_dual* out);
void orc_dual_free(orc_dual* d);

#endif
