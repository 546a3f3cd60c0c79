/* FP64 CPU oracle for the layered-field method.  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU baseline, never
 * by the library.  See oracle.h for conventions.
 *
 * Written for readability against the paper, not for speed: every function
 * follows the passage it cites, in the paper's order and notation, with plain
 * loops.  Readings of points the paper leaves open are marked "Reading:".
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void orc_free(void* p) { free(p); }

/* ---- small growable arrays ------------------------------------------------ */

typedef struct { int32_t* a; int64_t n, cap; } vi32;
typedef struct { double* a; int64_t n, cap; } vf64;
typedef struct { int64_t* a; int64_t n, cap; } vi64;

static int vi32_push(vi32* v, int32_t x) {
  if (v->n == v->cap) {
    int64_t c = v->cap ? 2 * v->cap : 64;
    int32_t* p = (int32_t*)realloc(v->a, (size_t)c * sizeof(int32_t));
    if (!p) return ORC_ENOMEM;
    v->a = p; v->cap = c;
  }
  v->a[v->n++] = x;
  return ORC_OK;
}
static int vf64_push(vf64* v, double x) {
  if (v->n == v->cap) {
    int64_t c = v->cap ? 2 * v->cap : 64;
    double* p = (double*)realloc(v->a, (size_t)c * sizeof(double));
    if (!p) return ORC_ENOMEM;
    v->a = p; v->cap = c;
  }
  v->a[v->n++] = x;
  return ORC_OK;
}
static int vi64_push(vi64* v, int64_t x) {
  if (v->n == v->cap) {
    int64_t c = v->cap ? 2 * v->cap : 64;
    int64_t* p = (int64_t*)realloc(v->a, (size_t)c * sizeof(int64_t));
    if (!p) return ORC_ENOMEM;
    v->a = p; v->cap = c;
  }
  v->a[v->n++] = x;
  return ORC_OK;
}

static int cmp_i64(const void* x, const void* y) {
  int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
  return a < b ? -1 : (a > b ? 1 : 0);
}

/* sort + unique an int64 key array in place, returns the new length */
static int64_t sort_unique_i64(int64_t* a, int64_t n) {
  if (n == 0) return 0;
  qsort(a, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t m = 1;
  for (int64_t i = 1; i < n; ++i)
    if (a[i] != a[m - 1]) a[m++] = a[i];
  return m;
}

static void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

static int check_faces(int32_t n_v, int32_t n_f, const int32_t* F) {
  if (n_v <= 0 || n_f < 0 || (n_f > 0 && !F)) return ORC_EINVAL;
  for (int64_t f = 0; f < n_f; ++f) {
    int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n_v || b >= n_v || c >= n_v) return ORC_EINVAL;
    if (a == b || b == c || a == c) return ORC_EINVAL;
  }
  return ORC_OK;
}

/* ---- operator --------------------------------------------------------------
 * Section 3.2, "Laplacian computation": the mesh Laplacian is precomputed
 * once.  Reading: an unnormalised operator approximating +nabla^2 (positive
 * off-diagonals, zero row sums) so that the growth predicate of Algorithm 1
 * (field Laplacian > 0) fires ahead of a front.  op 0: graph weights 1 per
 * edge.  op 1: cotangent weights, half the sum of the cotangents of the two
 * angles opposite the edge. */

typedef struct { int32_t i, j, f; double w; } trip;

static int cmp_trip(const void* x, const void* y) {
  const trip* a = (const trip*)x;
  const trip* b = (const trip*)y;
  if (a->i != b->i) return a->i < b->i ? -1 : 1;
  if (a->j != b->j) return a->j < b->j ? -1 : 1;
  if (a->f != b->f) return a->f < b->f ? -1 : 1;
  return 0;
}

int orc_operator(int32_t n_v, const double* V, int32_t n_f, const int32_t* F, int32_t op,
                 int64_t* ptr, int32_t** col_out, double** val_out) {
  if (check_faces(n_v, n_f, F) || (op != 0 && op != 1) || (op == 1 && !V)) return ORC_EINVAL;
  int64_t nt = 6 * (int64_t)n_f;
  trip* t = (trip*)malloc((size_t)(nt ? nt : 1) * sizeof(trip));
  if (!t) return ORC_ENOMEM;
  int64_t k = 0;
  for (int32_t f = 0; f < n_f; ++f) {
    const int32_t* c = F + 3 * (int64_t)f;
    for (int corner = 0; corner < 3; ++corner) {
      /* the corner opposite edge (p, q) */
      int32_t o = c[corner], p = c[(corner + 1) % 3], q = c[(corner + 2) % 3];
      double w = 1.0;
      if (op == 1) {
        double u[3], v[3], x[3];
        sub3(V + 3 * (int64_t)p, V + 3 * (int64_t)o, u);
        sub3(V + 3 * (int64_t)q, V + 3 * (int64_t)o, v);
        cross3(u, v, x);
        double s = norm3(x);
        if (s == 0.0) { free(t); return ORC_EINVAL; }
        w = 0.5 * dot3(u, v) / s;
      }
      t[k].i = p; t[k].j = q; t[k].f = f; t[k].w = w; ++k;
      t[k].i = q; t[k].j = p; t[k].f = f; t[k].w = w; ++k;
    }
  }
  qsort(t, (size_t)nt, sizeof(trip), cmp_trip);

  /* merge duplicates: one entry per ordered vertex pair */
  int64_t m = 0;
  for (int64_t a = 0; a < nt;) {
    int64_t b = a;
    double s = 0.0;
    while (b < nt && t[b].i == t[a].i && t[b].j == t[a].j) { s += t[b].w; ++b; }
    t[m].i = t[a].i; t[m].j = t[a].j; t[m].w = (op == 0) ? 1.0 : s;
    ++m;
    a = b;
  }
  int64_t nnz = m + n_v;
  int32_t* col = (int32_t*)malloc((size_t)nnz * sizeof(int32_t));
  double* val = (double*)malloc((size_t)nnz * sizeof(double));
  if (!col || !val) { free(t); free(col); free(val); return ORC_ENOMEM; }
  int64_t e = 0, r = 0;
  for (int32_t i = 0; i < n_v; ++i) {
    ptr[i] = e;
    int64_t r0 = r;
    double diag = 0.0;
    while (r < m && t[r].i == i) { diag -= t[r].w; ++r; }
    int placed = 0;
    for (int64_t s = r0; s < r; ++s) {
      if (!placed && t[s].j > i) { col[e] = i; val[e] = diag; ++e; placed = 1; }
      col[e] = t[s].j; val[e] = t[s].w; ++e;
    }
    if (!placed) { col[e] = i; val[e] = diag; ++e; }
  }
  ptr[n_v] = e;
  free(t);
  *col_out = col;
  *val_out = val;
  return ORC_OK;
}

/* ---- initialisation -------------------------------------------------------
 * Algorithm 1, first line, and the Initialization paragraph of Section 3.2:
 * a seeded vertex holds 1 in its own layer; every other vertex holds 1 in
 * the base layer (column n_s). */
int orc_init(int32_t n_v, const int32_t* seeds, int32_t n_s, int64_t* ptr, int32_t** col_out,
             double** val_out) {
  if (n_v <= 0 || n_s < 0 || (n_s > 0 && !seeds)) return ORC_EINVAL;
  int32_t* owner = (int32_t*)malloc((size_t)n_v * sizeof(int32_t));
  int32_t* col = (int32_t*)malloc((size_t)n_v * sizeof(int32_t));
  double* val = (double*)malloc((size_t)n_v * sizeof(double));
  if (!owner || !col || !val) { free(owner); free(col); free(val); return ORC_ENOMEM; }
  for (int32_t i = 0; i < n_v; ++i) owner[i] = n_s;
  for (int32_t k = 0; k < n_s; ++k) {
    int32_t s = seeds[k];
    if (s < 0 || s >= n_v || owner[s] != n_s) { free(owner); free(col); free(val); return ORC_EINVAL; }
    owner[s] = k;
  }
  for (int32_t i = 0; i < n_v; ++i) { ptr[i] = i; col[i] = owner[i]; val[i] = 1.0; }
  ptr[n_v] = n_v;
  free(owner);
  *col_out = col;
  *val_out = val;
  return ORC_OK;
}

/* ---- coefficient matrices a, w, e ------------------------------------------
 * Equation (2) sums over pairs i<j, so a layer does not interact with itself:
 * the diagonals are zero.  Off the diagonal the paper uses one value per
 * matrix (w = 0.2 with a ratio of 5 to a).  Reading for the base layer b:
 * it diffuses like any layer (a), it carries no penalty w ("allow cells to
 * evolve freely"), and the band term is antisymmetric, +e for a cell against
 * the base and -e for the base against a cell.  base_mode 1 instead treats
 * the base as an ordinary layer. */

static double coef_tab(int32_t j, int32_t l, int q, const orc_params* P) {
  return P->tab[3 * ((int64_t)P->types[j] * P->n_types + P->types[l]) + q];
}
static double coef_a(int32_t j, int32_t l, int32_t b, const orc_params* P) {
  (void)b;
  if (j == l) return 0.0;
  return P->n_types > 0 ? coef_tab(j, l, 0, P) : P->a;
}
static double coef_w(int32_t j, int32_t l, int32_t b, const orc_params* P) {
  if (j == l) return 0.0;
  if (P->base_mode == 0 && (j == b || l == b)) return 0.0;
  return P->n_types > 0 ? coef_tab(j, l, 1, P) : P->w;
}
static double coef_e(int32_t j, int32_t k, int32_t b, const orc_params* P) {
  if (j == k) return 0.0;
  const double e = P->n_types > 0 ? coef_tab(j, k, 2, P) : P->e;
  if (P->base_mode == 1 || (j != b && k != b)) return e;
  return (j == b) ? -e : e;
}

static void isort_i32(int32_t* a, int32_t n) {
  for (int32_t i = 1; i < n; ++i) {
    int32_t x = a[i], j = i - 1;
    while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
    a[j + 1] = x;
  }
}

/* ---- seeds grown into rings ------------------------------------------------
 * Algorithm 1 starts from "seeds and/or initial regions"; the Initialization
 * paragraph of Section 3.2 suggests a vertex and its immediate neighbours.
 * Reading: the region of seed k holds the vertices within `rings` edges of
 * the mesh's triangles from s_k; a vertex within reach of several seeds
 * belongs to the nearest, ties to the lowest seed index (so a seed keeps
 * itself).  Plain definition: a breadth-first search from every seed, one
 * after the other, keeping for each vertex the lexicographically smallest
 * (distance, seed index). */
int orc_init_rings(int32_t n_v, int32_t n_f, const int32_t* F, const int32_t* seeds, int32_t n_s,
                   int32_t rings, int64_t* ptr, int32_t** col_out, double** val_out) {
  if (check_faces(n_v, n_f, F) || !seeds || n_s < 1 || rings < 0) return ORC_EINVAL;
  for (int32_t k = 0; k < n_s; ++k)
    if (seeds[k] < 0 || seeds[k] >= n_v) return ORC_EINVAL;
  /* vertex adjacency from the faces' edges (both directions, duplicates kept) */
  int64_t* ap = (int64_t*)calloc((size_t)n_v + 1, sizeof(int64_t));
  int32_t* aj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(6 * (int64_t)n_f + 1));
  int32_t* best_d = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
  int32_t* best_k = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
  int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
  double* val = (double*)malloc(sizeof(double) * (size_t)n_v);
  int rc = ORC_OK;
  if (!ap || !aj || !best_d || !best_k || !dist || !queue || !col || !val) { rc = ORC_ENOMEM; goto done; }
  for (int64_t f = 0; f < n_f; ++f)
    for (int e = 0; e < 3; ++e) {
      ap[F[3 * f + e] + 1]++;
      ap[F[3 * f + (e + 1) % 3] + 1]++;
    }
  for (int32_t v = 0; v < n_v; ++v) ap[v + 1] += ap[v];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_v);
    if (!fill) { rc = ORC_ENOMEM; goto done; }
    memcpy(fill, ap, sizeof(int64_t) * (size_t)n_v);
    for (int64_t f = 0; f < n_f; ++f)
      for (int e = 0; e < 3; ++e) {
        const int32_t a = F[3 * f + e], b = F[3 * f + (e + 1) % 3];
        aj[fill[a]++] = b;
        aj[fill[b]++] = a;
      }
    free(fill);
  }
  for (int32_t v = 0; v < n_v; ++v) { best_d[v] = INT32_MAX; best_k[v] = n_s; dist[v] = -1; }
  for (int32_t k = 0; k < n_s; ++k) {
    int32_t head = 0, tail = 0;
    queue[tail++] = seeds[k];
    dist[seeds[k]] = 0;
    while (head < tail) {
      const int32_t v = queue[head++];
      if (dist[v] < best_d[v] || (dist[v] == best_d[v] && k < best_k[v])) {
        best_d[v] = dist[v];
        best_k[v] = k;
      }
      if (dist[v] == rings) continue;
      for (int64_t q = ap[v]; q < ap[v + 1]; ++q)
        if (dist[aj[q]] < 0) {
          dist[aj[q]] = dist[v] + 1;
          queue[tail++] = aj[q];
        }
    }
    for (int32_t t = 0; t < tail; ++t) dist[queue[t]] = -1;
  }
  for (int32_t v = 0; v < n_v; ++v) {
    ptr[v] = v;
    col[v] = best_k[v]; /* n_s: the base layer */
    val[v] = 1.0;
  }
  ptr[n_v] = n_v;
  *col_out = col;
  *val_out = val;
  col = 0;
  val = 0;
done:
  free(ap); free(aj); free(best_d); free(best_k); free(dist); free(queue); free(col); free(val);
  return rc;
}

/* ---- one time step ----------------------------------------------------------
 * The explicit Euler step of Section 3 (equations (11)-(13)) restricted to
 * the rows of interest of Algorithm 1, row by row in U = Phi^T terms.
 *
 * For vertex i: the field Laplacian lambda_k = L_t(k, i) = sum_u L(i,u) U(u,k)
 * (the sparse product of Section 3.2), the current values phi_k = U(i, k),
 * and the rows of interest S: layers with phi_k > 0, or phi_k = 0 with
 * lambda_k > 0 (growth where the field Laplacian is positive).  n = |S|.
 * For every layer m of S (the paper's i in equation (11)):
 *   dphi_m/dt = - sum_{j in S} (mu/n) ( sum_{k in S} [ (w_mk - w_jk) phi_k
 *                   + (a_mk - a_jk) lambda_k / 2 ]  +  (dg_m - dg_j) ),
 * the g-difference of equation (12) being dg_m - dg_j = -e_mj sqrt(phi_m phi_j)
 * (the gradient coefficients enter linearly, see the readings); the Euler
 * step of equation (13) v_m = phi_m + dt dphi_m/dt, clamped to [0, 1]; and
 * the row is normalised by the sum of its clamped values (Section 4,
 * normalization).
 * Reading (Jacobi): every value of the step is computed from the fields of
 * the previous step (Section 4: the update produces an updated copy).
 * Reading (prune): after normalisation entries below theta are dropped
 * (theta = 0 keeps every positive entry); zeros are never stored. */

/* per-row work arrays (one set per thread), n_r = n_s + 1 long */
typedef struct {
  double *lam, *phi, *pre, *upd;
  char* touched;
  int32_t *list, *irows;
} row_ws;

static void ws_free(row_ws* w) {
  free(w->lam); free(w->phi); free(w->pre); free(w->upd);
  free(w->touched); free(w->list); free(w->irows);
}

static int ws_alloc(row_ws* w, int32_t n_r) {
  memset(w, 0, sizeof(*w));
  w->lam = (double*)calloc((size_t)n_r, sizeof(double));
  w->phi = (double*)calloc((size_t)n_r, sizeof(double));
  w->pre = (double*)calloc((size_t)n_r, sizeof(double));
  w->upd = (double*)calloc((size_t)n_r, sizeof(double));
  w->touched = (char*)calloc((size_t)n_r, 1);
  w->list = (int32_t*)calloc((size_t)n_r, sizeof(int32_t));
  w->irows = (int32_t*)calloc((size_t)n_r, sizeof(int32_t));
  if (!w->lam || !w->phi || !w->pre || !w->upd || !w->touched || !w->list || !w->irows) {
    ws_free(w);
    return ORC_ENOMEM;
  }
  return ORC_OK;
}

/* One row.  Appends the kept entries to (oc, ov); mg = smallest distance of
 * any discrete decision from its threshold, smg = the same over the
 * rows-of-interest decisions only; *ev counts a row whose clamped values
 * sum to zero (left empty). */
static int step_row(int32_t i, int32_t n_s, const int64_t* Lp, const int32_t* Lc,
                    const double* Lv, const int64_t* Up, const int32_t* Uc, const double* Uv,
                    const orc_params* P, row_ws* w, vi32* oc, vf64* ov, double* mg_out,
                    double* smg_out, int32_t* skel_out, int64_t* ev) {
  const int32_t n_r = n_s + 1, b = n_s;
  int32_t nt = 0;
  /* lambda: row i of L times U, over the layers met in the neighbourhood */
  for (int64_t q = Lp[i]; q < Lp[i + 1]; ++q) {
    const int32_t u = Lc[q];
    for (int64_t p = Up[u]; p < Up[u + 1]; ++p) {
      const int32_t l = Uc[p];
      if (l < 0 || l >= n_r) return ORC_EINVAL;
      if (!w->touched[l]) { w->touched[l] = 1; w->list[nt++] = l; w->lam[l] = 0.0; w->phi[l] = 0.0; }
      w->lam[l] += Lv[q] * Uv[p];
    }
  }
  for (int64_t p = Up[i]; p < Up[i + 1]; ++p) {
    const int32_t l = Uc[p];
    if (l < 0 || l >= n_r || Uv[p] < 0.0) return ORC_EINVAL;
    if (!w->touched[l]) { w->touched[l] = 1; w->list[nt++] = l; w->lam[l] = 0.0; w->phi[l] = 0.0; }
    w->phi[l] = Uv[p];
  }
  isort_i32(w->list, nt);
  const double* lam = w->lam;
  const double* phi = w->phi;

  /* rows of interest, and the margins of their decisions */
  double smg = INFINITY;
  int32_t n = 0;
  for (int32_t t = 0; t < nt; ++t) {
    const int32_t l = w->list[t];
    if (phi[l] > 0.0 || (phi[l] == 0.0 && lam[l] > 0.0)) w->irows[n++] = l;
    if (phi[l] == 0.0 && fabs(lam[l]) < smg) smg = fabs(lam[l]);
  }
  if (skel_out) *skel_out = n;
  const int32_t* S = w->irows;

  /* equation (11) for every layer m of S, then the Euler step (13) */
  for (int32_t mm = 0; mm < n; ++mm) {
    const int32_t m = S[mm];
    double rate = 0.0;
    for (int32_t jj = 0; jj < n; ++jj) {
      const int32_t j = S[jj];
      double inner = 0.0;
      for (int32_t kk = 0; kk < n; ++kk) {
        const int32_t k = S[kk];
        inner += (coef_w(m, k, b, P) - coef_w(j, k, b, P)) * phi[k] +
                 0.5 * (coef_a(m, k, b, P) - coef_a(j, k, b, P)) * lam[k];
      }
      const double dg = -coef_e(m, j, b, P) * sqrt(phi[m] * phi[j]);
      rate += -(P->mu / n) * (inner + dg);
    }
    const double v = phi[m] + rate * P->dt;
    w->pre[mm] = v;
    w->upd[mm] = v > 1.0 ? 1.0 : (v <= 0.0 ? 0.0 : v);
  }

  /* normalise by the sum of the clamped values, then prune */
  double mg = smg, sum = 0.0;
  for (int32_t jj = 0; jj < n; ++jj) sum += w->upd[jj];
  if (n > 0 && sum > 0.0) {
    for (int32_t jj = 0; jj < n; ++jj) {
      const double v = w->upd[jj] / sum;
      const double m = P->theta > 0.0 ? fabs(v - P->theta) : fabs(w->pre[jj]);
      if (m < mg) mg = m;
      if (v > 0.0 && v >= P->theta)
        if (vi32_push(oc, S[jj]) || vf64_push(ov, v)) return ORC_ENOMEM;
    }
  } else if (n > 0) {
    ++*ev; /* every value clamped to zero: the column is left empty */
  }
  if (mg_out) *mg_out = mg;
  if (smg_out) *smg_out = smg;
  for (int32_t t = 0; t < nt; ++t) w->touched[w->list[t]] = 0;
  return ORC_OK;
}

/* Rows in `nb` contiguous blocks, each with its own work arrays and output
 * lists; kept across the steps of a run so that long runs allocate nothing
 * per step. */
typedef struct {
  int32_t nb, n_r;
  row_ws* ws;
  vi32* oc;
  vf64* ov;
  int64_t* ev;
  int* rc;
} blocks;

static void blocks_free(blocks* B) {
  for (int32_t k = 0; k < B->nb; ++k) {
    if (B->ws) ws_free(&B->ws[k]);
    if (B->oc) free(B->oc[k].a);
    if (B->ov) free(B->ov[k].a);
  }
  free(B->ws); free(B->oc); free(B->ov); free(B->ev); free(B->rc);
  memset(B, 0, sizeof(*B));
}

static int blocks_alloc(blocks* B, int32_t nb, int32_t n_r) {
  memset(B, 0, sizeof(*B));
  B->nb = nb;
  B->n_r = n_r;
  B->ws = (row_ws*)calloc((size_t)nb, sizeof(row_ws));
  B->oc = (vi32*)calloc((size_t)nb, sizeof(vi32));
  B->ov = (vf64*)calloc((size_t)nb, sizeof(vf64));
  B->ev = (int64_t*)calloc((size_t)nb, sizeof(int64_t));
  B->rc = (int*)calloc((size_t)nb, sizeof(int));
  if (!B->ws || !B->oc || !B->ov || !B->ev || !B->rc) { blocks_free(B); return ORC_ENOMEM; }
  for (int32_t k = 0; k < nb; ++k)
    if (ws_alloc(&B->ws[k], n_r)) { blocks_free(B); return ORC_ENOMEM; }
  return ORC_OK;
}

/* One step of every row into the blocks' output lists; Op[i] is left
 * block-relative.  The blocks run in parallel. */
static int step_blocks(blocks* B, int32_t n_v, int32_t n_s, const int64_t* Lp, const int32_t* Lc,
                       const double* Lv, const int64_t* Up, const int32_t* Uc, const double* Uv,
                       const orc_params* P, int64_t* Op, double* margin, double* smargin,
                       int32_t* skel) {
  const int32_t nb = B->nb;
#pragma omp parallel for schedule(static, 1) num_threads(nb)
  for (int32_t k = 0; k < nb; ++k) {
    const int32_t i0 = (int32_t)((int64_t)n_v * k / nb), i1 = (int32_t)((int64_t)n_v * (k + 1) / nb);
    B->oc[k].n = 0;
    B->ov[k].n = 0;
    B->ev[k] = 0;
    B->rc[k] = ORC_OK;
    for (int32_t i = i0; i < i1 && !B->rc[k]; ++i) {
      Op[i] = B->oc[k].n;
      B->rc[k] = step_row(i, n_s, Lp, Lc, Lv, Up, Uc, Uv, P, &B->ws[k], &B->oc[k], &B->ov[k],
                          margin ? margin + i : 0, smargin ? smargin + i : 0, skel ? skel + i : 0,
                          &B->ev[k]);
    }
  }
  for (int32_t k = 0; k < nb; ++k)
    if (B->rc[k]) return B->rc[k];
  return ORC_OK;
}

/* joins the blocks' outputs in row order into oc / ov (room for the total),
 * makes Op absolute */
static int64_t join_blocks(const blocks* B, int32_t n_v, int64_t* Op, int32_t* oc, double* ov) {
  int64_t off = 0;
  for (int32_t k = 0; k < B->nb; ++k) {
    const int32_t i0 = (int32_t)((int64_t)n_v * k / B->nb);
    const int32_t i1 = (int32_t)((int64_t)n_v * (k + 1) / B->nb);
    for (int32_t i = i0; i < i1; ++i) Op[i] += off;
    if (B->oc[k].n) {
      memcpy(oc + off, B->oc[k].a, (size_t)B->oc[k].n * sizeof(int32_t));
      memcpy(ov + off, B->ov[k].a, (size_t)B->oc[k].n * sizeof(double));
    }
    off += B->oc[k].n;
  }
  Op[n_v] = off;
  return off;
}

static int64_t blocks_total(const blocks* B, int64_t* ev) {
  int64_t t = 0, e = 0;
  for (int32_t k = 0; k < B->nb; ++k) { t += B->oc[k].n; e += B->ev[k]; }
  if (ev) *ev = e;
  return t;
}

int orc_step_threads(int32_t n_v, int32_t n_s, const int64_t* Lp, const int32_t* Lc,
                     const double* Lv, const int64_t* Up, const int32_t* Uc, const double* Uv,
                     const orc_params* P, int64_t* Op, int32_t** Oc, double** Ov, double* margin,
                     double* smargin, int32_t* skel, int64_t* events, int32_t threads) {
  if (n_v <= 0 || n_s < 0 || !P || threads < 1) return ORC_EINVAL;
  const int32_t n_r = n_s + 1;
  if (P->n_types < 0 || (P->n_types > 0 && (!P->types || !P->tab))) return ORC_EINVAL;
  for (int32_t l = 0; P->n_types > 0 && l < n_r; ++l)
    if (P->types[l] < 0 || P->types[l] >= P->n_types) return ORC_EINVAL;
  blocks B;
  int rc = blocks_alloc(&B, threads < n_v ? threads : n_v, n_r);
  if (rc) return rc;
  rc = step_blocks(&B, n_v, n_s, Lp, Lc, Lv, Up, Uc, Uv, P, Op, margin, smargin, skel);
  if (!rc) {
    int64_t ev = 0;
    const int64_t total = blocks_total(&B, &ev);
    int32_t* oc = (int32_t*)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
    double* ov = (double*)malloc((size_t)(total ? total : 1) * sizeof(double));
    if (!oc || !ov) {
      free(oc); free(ov);
      rc = ORC_ENOMEM;
    } else {
      join_blocks(&B, n_v, Op, oc, ov);
      if (events) *events = ev;
      *Oc = oc;
      *Ov = ov;
    }
  }
  blocks_free(&B);
  return rc;
}

int orc_step(int32_t n_v, int32_t n_s, const int64_t* Lp, const int32_t* Lc, const double* Lv,
             const int64_t* Up, const int32_t* Uc, const double* Uv, const orc_params* P,
             int64_t* Op, int32_t** Oc, double** Ov, double* margin, int32_t* skel,
             int64_t* events) {
  return orc_step_threads(n_v, n_s, Lp, Lc, Lv, Up, Uc, Uv, P, Op, Oc, Ov, margin, 0, skel,
                          events, 1);
}

/* n_steps free-running steps (orc_step_threads repeated), in C so that long
 * trajectories need no round trip per step; the work arrays, block lists and
 * the two field buffers are kept across steps.  U_in is not modified; the
 * final fields are returned in (Op, Oc, Ov); *skel_total and *events sum the
 * rows-of-interest sizes and the empty-row events over the steps. */
int orc_run_threads(int32_t n_v, int32_t n_s, const int64_t* Lp, const int32_t* Lc,
                    const double* Lv, const int64_t* Up, const int32_t* Uc, const double* Uv,
                    const orc_params* P, int32_t n_steps, int32_t threads, int64_t* Op,
                    int32_t** Oc, double** Ov, int64_t* skel_total, int64_t* events) {
  if (n_v <= 0 || n_s < 0 || n_steps < 0 || !P || threads < 1) return ORC_EINVAL;
  const int32_t n_r = n_s + 1;
  if (P->n_types < 0 || (P->n_types > 0 && (!P->types || !P->tab))) return ORC_EINVAL;
  for (int32_t l = 0; P->n_types > 0 && l < n_r; ++l)
    if (P->types[l] < 0 || P->types[l] >= P->n_types) return ORC_EINVAL;
  blocks B;
  int rc = blocks_alloc(&B, threads < n_v ? threads : n_v, n_r);
  if (rc) return rc;
  int64_t *p[2] = {0, 0}, cap = Up[n_v] > 0 ? Up[n_v] : 1;
  int32_t *c[2] = {0, 0}, *skel = 0;
  double* v[2] = {0, 0};
  int64_t sk = 0, evs = 0;
  int cur = 0;
  for (int b = 0; b < 2; ++b) {
    p[b] = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_v + 1));
    c[b] = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    v[b] = (double*)malloc(sizeof(double) * (size_t)cap);
  }
  skel = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
  if (!p[0] || !p[1] || !c[0] || !c[1] || !v[0] || !v[1] || !skel) { rc = ORC_ENOMEM; goto done; }
  memcpy(p[0], Up, sizeof(int64_t) * ((size_t)n_v + 1));
  if (Up[n_v]) {
    memcpy(c[0], Uc, sizeof(int32_t) * (size_t)Up[n_v]);
    memcpy(v[0], Uv, sizeof(double) * (size_t)Up[n_v]);
  }
  for (int32_t t = 0; t < n_steps; ++t) {
    const int nx = 1 - cur;
    rc = step_blocks(&B, n_v, n_s, Lp, Lc, Lv, p[cur], c[cur], v[cur], P, p[nx], 0, 0, skel);
    if (rc) goto done;
    int64_t e = 0;
    const int64_t total = blocks_total(&B, &e);
    if (total > cap) { /* both buffers grow, the current one keeps its contents */
      const int64_t nc = total + total / 4 + 1024;
      int32_t* c0 = (int32_t*)realloc(c[cur], sizeof(int32_t) * (size_t)nc);
      if (c0) c[cur] = c0;
      double* v0 = (double*)realloc(v[cur], sizeof(double) * (size_t)nc);
      if (v0) v[cur] = v0;
      free(c[nx]);
      free(v[nx]);
      c[nx] = (int32_t*)malloc(sizeof(int32_t) * (size_t)nc);
      v[nx] = (double*)malloc(sizeof(double) * (size_t)nc);
      if (!c0 || !v0 || !c[nx] || !v[nx]) { rc = ORC_ENOMEM; goto done; }
      cap = nc;
    }
    join_blocks(&B, n_v, p[nx], c[nx], v[nx]);
    for (int32_t i = 0; i < n_v; ++i) sk += skel[i];
    evs += e;
    cur = nx;
  }
  {
    const int64_t nnz = p[cur][n_v];
    int32_t* oc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    double* ov = (double*)malloc(sizeof(double) * (size_t)(nnz ? nnz : 1));
    if (!oc || !ov) { free(oc); free(ov); rc = ORC_ENOMEM; goto done; }
    memcpy(Op, p[cur], sizeof(int64_t) * ((size_t)n_v + 1));
    if (nnz) {
      memcpy(oc, c[cur], sizeof(int32_t) * (size_t)nnz);
      memcpy(ov, v[cur], sizeof(double) * (size_t)nnz);
    }
    *Oc = oc;
    *Ov = ov;
    if (skel_total) *skel_total = sk;
    if (events) *events = evs;
  }
done:
  for (int b = 0; b < 2; ++b) { free(p[b]); free(c[b]); free(v[b]); }
  free(skel);
  blocks_free(&B);
  return rc;
}

/* ---- labels -------------------------------------------------------------------
 * The sharp visualisation (Figure 10, Section 7) shows, per vertex, the field
 * with the largest influence: the argmax over the cell layers. */
int orc_labels(int32_t n_v, int32_t n_s, const int64_t* Up, const int32_t* Uc, const double* Uv,
               int32_t* labels, double* gap) {
  if (n_v <= 0 || !labels) return ORC_EINVAL;
  for (int32_t i = 0; i < n_v; ++i) {
    /* columns are ascending, so a strict comparison keeps the lowest id */
    int32_t best = -1;
    double b1 = 0.0, b2 = 0.0;
    for (int64_t p = Up[i]; p < Up[i + 1]; ++p) {
      if (Uc[p] >= n_s) continue; /* the base layer is not a cell */
      if (best < 0 || Uv[p] > b1) { best = Uc[p]; b1 = Uv[p]; }
    }
    for (int64_t p = Up[i]; p < Up[i + 1]; ++p)
      if (Uc[p] < n_s && Uc[p] != best && Uv[p] > b2) b2 = Uv[p];
    labels[i] = best;
    if (gap) gap[i] = best < 0 ? INFINITY : b1 - b2;
  }
  return ORC_OK;
}

/* ---- Lloyd-like re-seeding ------------------------------------------------------
 * Section 5: the centre of mass of a cell is the area-weighted average of the
 * barycentres of all triangles having a vertex in the cell; it is projected
 * back onto the cell along the area-weighted average of the triangle normals;
 * among several intersections the one closest to the centre is taken; on a
 * miss the seed stays.  Readings: the cell is the support of its layer
 * (entries > 0); the projection line runs both ways from the centre and is
 * tested against the cell's own triangles with closed edges; equal distances
 * go to the lower face id; the new seed is the hit face's vertex nearest the
 * hit point (lower id on ties).  Seed collisions: when several cells pick the
 * same vertex the lowest cell id keeps it and the others stay; a mover that
 * lands on the seed of a cell that stays also stays; repeated until no two
 * seeds coincide. */

/* line orig + s*dir against triangle (p0,p1,p2); returns 1 on a hit */
static int line_tri(const double* orig, const double* dir, const double* p0, const double* p1,
                    const double* p2, double* s_out, double* edge_out) {
  double e1[3], e2[3], h[3], sv[3], q[3];
  sub3(p1, p0, e1);
  sub3(p2, p0, e2);
  cross3(dir, e2, h);
  double det = dot3(e1, h);
  if (det == 0.0) { *edge_out = 0.0; return 0; }
  double inv = 1.0 / det;
  sub3(orig, p0, sv);
  double u = inv * dot3(sv, h);
  cross3(sv, e1, q);
  double v = inv * dot3(dir, q);
  double s = inv * dot3(e2, q);
  double w = 1.0 - u - v;
  double m = fabs(u);
  if (fabs(v) < m) m = fabs(v);
  if (fabs(w) < m) m = fabs(w);
  *edge_out = m;
  *s_out = s;
  return (u >= 0.0 && v >= 0.0 && w >= 0.0) ? 1 : 0;
}

int orc_lloyd(int32_t n_v, const double* V, int32_t n_f, const int32_t* F, int32_t n_s,
              const int64_t* Up, const int32_t* Uc, const double* Uv, const int32_t* seeds_in,
              int32_t* seeds_out, int32_t* status, double* margin) {
  if (check_faces(n_v, n_f, F) || !V || n_s <= 0 || !seeds_in || !seeds_out) return ORC_EINVAL;
  /* faces of every cell, in increasing face id */
  vi32* fl = (vi32*)calloc((size_t)n_s, sizeof(vi32));
  int32_t* cand = (int32_t*)malloc((size_t)n_s * sizeof(int32_t));
  int32_t* st = (int32_t*)malloc((size_t)n_s * sizeof(int32_t));
  int32_t* owner = (int32_t*)malloc((size_t)n_v * sizeof(int32_t));
  int rc = ORC_OK;
  if (!fl || !cand || !st || !owner) { rc = ORC_ENOMEM; goto done; }
  for (int32_t f = 0; f < n_f; ++f) {
    int32_t cells[64];
    int nc = 0;
    for (int k = 0; k < 3; ++k) {
      int32_t v = F[3 * (int64_t)f + k];
      for (int64_t p = Up[v]; p < Up[v + 1]; ++p) {
        int32_t c = Uc[p];
        if (c >= n_s || !(Uv[p] > 0.0)) continue;
        int seen = 0;
        for (int t = 0; t < nc; ++t) seen |= (cells[t] == c);
        if (!seen) {
          if (nc == 64) { rc = ORC_EINVAL; goto done; }
          cells[nc++] = c;
        }
      }
    }
    for (int t = 0; t < nc; ++t)
      if (vi32_push(&fl[cells[t]], f)) { rc = ORC_ENOMEM; goto done; }
  }

  for (int32_t c = 0; c < n_s; ++c) {
    double sa = 0.0, sb[3] = {0, 0, 0}, sn[3] = {0, 0, 0};
    for (int64_t t = 0; t < fl[c].n; ++t) {
      const int32_t* fv = F + 3 * (int64_t)fl[c].a[t];
      const double *x0 = V + 3 * (int64_t)fv[0], *x1 = V + 3 * (int64_t)fv[1],
                   *x2 = V + 3 * (int64_t)fv[2];
      double e1[3], e2[3], cr[3];
      sub3(x1, x0, e1);
      sub3(x2, x0, e2);
      cross3(e1, e2, cr);
      double area = 0.5 * norm3(cr);
      sa += area;
      for (int d = 0; d < 3; ++d) {
        sb[d] += area * (x0[d] + x1[d] + x2[d]) / 3.0;
        sn[d] += 0.5 * cr[d]; /* area times unit normal */
      }
    }
    double mg = INFINITY;
    cand[c] = seeds_in[c];
    st[c] = 1;
    double nn = norm3(sn);
    if (fl[c].n > 0 && sa > 0.0 && nn > 0.0) {
      double ctr[3] = {sb[0] / sa, sb[1] / sa, sb[2] / sa};
      double dir[3] = {sn[0] / nn, sn[1] / nn, sn[2] / nn};
      int32_t bf = -1;
      double bs = INFINITY, second = INFINITY;
      double* es = (double*)malloc((size_t)fl[c].n * sizeof(double));
      double* ss = (double*)malloc((size_t)fl[c].n * sizeof(double));
      int* hit = (int*)malloc((size_t)fl[c].n * sizeof(int));
      if (!es || !ss || !hit) { free(es); free(ss); free(hit); rc = ORC_ENOMEM; goto done; }
      for (int64_t t = 0; t < fl[c].n; ++t) {
        int32_t f = fl[c].a[t];
        const int32_t* fv = F + 3 * (int64_t)f;
        double s = INFINITY, e = 0.0;
        hit[t] = line_tri(ctr, dir, V + 3 * (int64_t)fv[0], V + 3 * (int64_t)fv[1],
                          V + 3 * (int64_t)fv[2], &s, &e);
        es[t] = e;
        ss[t] = s;
        if (hit[t]) {
          double a = fabs(s);
          if (a < bs) { second = bs; bs = a; bf = f; }
          else if (a < second) second = a;
        }
      }
      /* margins: hit choice, and edge tests of faces that could win */
      if (bf >= 0) {
        double g = (second - bs) / (1.0 + bs);
        if (g < mg) mg = g;
      }
      for (int64_t t = 0; t < fl[c].n; ++t) {
        if (ss[t] == INFINITY || bf < 0 || fabs(ss[t]) <= bs * (1.0 + 1e-6) + 1e-12) {
          if (es[t] < mg) mg = es[t];
        }
      }
      free(es); free(ss); free(hit);
      if (bf >= 0) {
        const int32_t* fv = F + 3 * (int64_t)bf;
        double hp[3] = {ctr[0], ctr[1], ctr[2]};
        /* the hit point, recomputed from the chosen face's line parameter */
        double sbest = INFINITY, e = 0.0;
        line_tri(ctr, dir, V + 3 * (int64_t)fv[0], V + 3 * (int64_t)fv[1], V + 3 * (int64_t)fv[2],
                 &sbest, &e);
        for (int d = 0; d < 3; ++d) hp[d] += sbest * dir[d];
        int32_t bv = -1;
        double bd = INFINITY, bd2 = INFINITY;
        for (int k = 0; k < 3; ++k) {
          double dv[3];
          sub3(V + 3 * (int64_t)fv[k], hp, dv);
          double dd = dot3(dv, dv);
          if (dd < bd || (dd == bd && fv[k] < bv)) { bd2 = bd; bd = dd; bv = fv[k]; }
          else if (dd < bd2) bd2 = dd;
        }
        double g = (bd2 - bd) / (1.0 + bd);
        if (g < mg) mg = g;
        cand[c] = bv;
        st[c] = 0;
      }
    }
    if (margin) margin[c] = mg;
  }

  /* seed collisions, resolved to a fixed point */
  for (int32_t i = 0; i < n_v; ++i) owner[i] = -1;
  for (;;) {
    int changed = 0;
    for (int32_t i = 0; i < n_v; ++i) owner[i] = -1;
    /* a cell that stays holds its seed before any mover is considered */
    for (int32_t c = 0; c < n_s; ++c)
      if (cand[c] == seeds_in[c]) owner[cand[c]] = c;
    for (int32_t c = 0; c < n_s; ++c) {
      if (cand[c] == seeds_in[c]) continue;
      if (owner[cand[c]] == -1) owner[cand[c]] = c;
    }
    for (int32_t c = 0; c < n_s; ++c) {
      if (owner[cand[c]] != c) { cand[c] = seeds_in[c]; st[c] = 2; changed = 1; }
    }
    if (!changed) break;
  }
  for (int32_t c = 0; c < n_s; ++c) {
    seeds_out[c] = cand[c];
    if (status) status[c] = st[c];
  }
done:
  if (fl) for (int32_t c = 0; c < n_s; ++c) free(fl[c].a);
  free(fl); free(cand); free(st); free(owner);
  return rc;
}

/* ---- dual mesh -------------------------------------------------------------------
 * Section 5.1 (cell neighbourhoods) and 5.2 (mesh construction).
 *   Phibar = [U >= tau] on the cell layers (tau = 0.25)
 *   A_v = Phibar Phibar^T without diagonal     (cells sharing a vertex)
 *   B   = Phibar Mbar (logical)                 (cells touching a face)
 *   A_t = B B^T without diagonal                (cells sharing a face)
 *   candidates = A_t and not A_v; a candidate is confirmed when the two
 *   cells' tau-isolines cross on one of their common faces; a confirmed
 *   candidate whose cells already share two or more neighbours is dropped.
 *   Dual triangles are the 3-cliques of the curated adjacency; a triangle
 *   covering a cell of exactly three mutually adjacent neighbours is removed;
 *   triangles are then oriented consistently by edge-neighbour propagation.
 * Readings: the shared-neighbour count uses A_v (order-free); the isoline of
 * a cell on a face is the segment between the linearly interpolated tau
 * crossings on its edges (a vertex at exactly tau counts as inside); each
 * component's lowest triangle is oriented along the summed vertex normals at
 * its three seeds. */

static int cmp_pair(const void* x, const void* y) {
  const int32_t* a = (const int32_t*)x;
  const int32_t* b = (const int32_t*)y;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

/* symmetric CSR over n cells from a list of unordered pair keys p*n+q (p<q) */
static int pairs_to_csr(int64_t* keys, int64_t nk, int32_t n, int64_t** ptr_out,
                        int32_t** col_out) {
  nk = sort_unique_i64(keys, nk);
  int32_t* pr = (int32_t*)malloc((size_t)(2 * nk + 1) * 2 * sizeof(int32_t));
  int64_t* ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* col = (int32_t*)malloc((size_t)(2 * nk + 1) * sizeof(int32_t));
  if (!pr || !ptr || !col) { free(pr); free(ptr); free(col); return ORC_ENOMEM; }
  for (int64_t k = 0; k < nk; ++k) {
    int32_t p = (int32_t)(keys[k] / n), q = (int32_t)(keys[k] % n);
    pr[4 * k] = p; pr[4 * k + 1] = q;
    pr[4 * k + 2] = q; pr[4 * k + 3] = p;
  }
  qsort(pr, (size_t)(2 * nk), 2 * sizeof(int32_t), cmp_pair);
  for (int64_t k = 0; k < 2 * nk; ++k) { ptr[pr[2 * k] + 1]++; col[k] = pr[2 * k + 1]; }
  for (int32_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  free(pr);
  *ptr_out = ptr;
  *col_out = col;
  return ORC_OK;
}

static int csr_has(const int64_t* ptr, const int32_t* col, int32_t p, int32_t q) {
  for (int64_t t = ptr[p]; t < ptr[p + 1]; ++t)
    if (col[t] == q) return 1;
  return 0;
}

static int64_t csr_common(const int64_t* ptr, const int32_t* col, int32_t p, int32_t q) {
  int64_t a = ptr[p], b = ptr[q], n = 0;
  while (a < ptr[p + 1] && b < ptr[q + 1]) {
    if (col[a] == col[b]) { ++n; ++a; ++b; }
    else if (col[a] < col[b]) ++a;
    else ++b;
  }
  return n;
}

static double u_at(const int64_t* Up, const int32_t* Uc, const double* Uv, int32_t v, int32_t c) {
  for (int64_t p = Up[v]; p < Up[v + 1]; ++p)
    if (Uc[p] == c) return Uv[p];
  return 0.0;
}

/* tau-isoline of a field on one face, as a segment in barycentric
 * coordinates (weights of corners 1 and 2).  Returns 0 when the face is not
 * crossed. */
static int iso_segment(const double f[3], double tau, double seg[4]) {
  int in[3] = {f[0] >= tau, f[1] >= tau, f[2] >= tau};
  if (in[0] == in[1] && in[1] == in[2]) return 0;
  int m = 0;
  for (int e = 0; e < 3; ++e) {
    int a = e, b = (e + 1) % 3;
    if (in[a] == in[b]) continue;
    double t = (tau - f[a]) / (f[b] - f[a]);
    double bary[3] = {0, 0, 0};
    bary[a] = 1.0 - t;
    bary[b] = t;
    seg[2 * m] = bary[1];
    seg[2 * m + 1] = bary[2];
    ++m;
  }
  return m == 2;
}

static double orient2(const double* a, const double* b, const double* c) {
  return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}
static int on_seg(const double* a, const double* b, const double* c) {
  /* c collinear with a-b: is it within the bounding box? */
  return fmin(a[0], b[0]) <= c[0] && c[0] <= fmax(a[0], b[0]) && fmin(a[1], b[1]) <= c[1] &&
         c[1] <= fmax(a[1], b[1]);
}
/* closed segment intersection; *mg gets the smallest |determinant| used */
static int seg_cross(const double* P, const double* Q, double* mg) {
  const double *p0 = P, *p1 = P + 2, *q0 = Q, *q1 = Q + 2;
  double d1 = orient2(q0, q1, p0), d2 = orient2(q0, q1, p1);
  double d3 = orient2(p0, p1, q0), d4 = orient2(p0, p1, q1);
  double m = fabs(d1);
  if (fabs(d2) < m) m = fabs(d2);
  if (fabs(d3) < m) m = fabs(d3);
  if (fabs(d4) < m) m = fabs(d4);
  if (m < *mg) *mg = m;
  if (((d1 > 0 && d2 < 0) || (d1 < 0 && d2 > 0)) && ((d3 > 0 && d4 < 0) || (d3 < 0 && d4 > 0)))
    return 1;
  if (d1 == 0 && on_seg(q0, q1, p0)) return 1;
  if (d2 == 0 && on_seg(q0, q1, p1)) return 1;
  if (d3 == 0 && on_seg(p0, p1, q0)) return 1;
  if (d4 == 0 && on_seg(p0, p1, q1)) return 1;
  return 0;
}

void orc_dual_free(orc_dual* d) {
  if (!d) return;
  free(d->av_ptr); free(d->av_col); free(d->at_ptr); free(d->at_col);
  free(d->ad_ptr); free(d->ad_col); free(d->cand); free(d->cand_state);
  free(d->cand_margin); free(d->tri);
  memset(d, 0, sizeof(*d));
}

int orc_dual_mesh(int32_t n_v, const double* V, int32_t n_f, const int32_t* F, int32_t n_s,
                  const int64_t* Up, const int32_t* Uc, const double* Uv, const int32_t* seeds,
                  double tau, orc_dual* out) {
  if (check_faces(n_v, n_f, F) || !V || n_s <= 0 || !seeds || !out) return ORC_EINVAL;
  memset(out, 0, sizeof(*out));
  int rc = ORC_OK;
  vi64 kv = {0, 0, 0}, kt = {0, 0, 0}, kd = {0, 0, 0}, bf = {0, 0, 0}, ek = {0, 0, 0};
  vi32 cand = {0, 0, 0}, cst = {0, 0, 0}, tri = {0, 0, 0};
  vf64 cmg = {0, 0, 0};
  int64_t *bptr = 0, *tptr = 0;
  int32_t *bcol = 0, *orient = 0, *fq = 0, *eface = 0;
  char *removed = 0, *done_ = 0;
  double* vn = 0;
  const int64_t NS = n_s;

  /* Phibar rows: thresholded cells of each vertex */
#define THR(p) (Uc[p] < n_s && Uv[p] >= tau)
  /* A_v: pairs of cells above tau at one vertex */
  for (int32_t v = 0; v < n_v; ++v)
    for (int64_t a = Up[v]; a < Up[v + 1]; ++a)
      for (int64_t b = a + 1; b < Up[v + 1]; ++b)
        if (THR(a) && THR(b)) {
          int32_t p = Uc[a] < Uc[b] ? Uc[a] : Uc[b], q = Uc[a] < Uc[b] ? Uc[b] : Uc[a];
          if (p != q && vi64_push(&kv, p * NS + q)) { rc = ORC_ENOMEM; goto done; }
        }
  if ((rc = pairs_to_csr(kv.a, kv.n, n_s, &out->av_ptr, &out->av_col))) goto done;

  /* B = Phibar Mbar: cells touching each face; A_t = B B^T */
  for (int32_t f = 0; f < n_f; ++f) {
    int32_t cells[96];
    int nc = 0;
    for (int k = 0; k < 3; ++k) {
      int32_t v = F[3 * (int64_t)f + k];
      for (int64_t p = Up[v]; p < Up[v + 1]; ++p) {
        if (!THR(p)) continue;
        int seen = 0;
        for (int t = 0; t < nc; ++t) seen |= (cells[t] == Uc[p]);
        if (!seen) {
          if (nc == 96) { rc = ORC_EINVAL; goto done; }
          cells[nc++] = Uc[p];
        }
      }
    }
    isort_i32(cells, nc);
    for (int a = 0; a < nc; ++a) {
      if (vi64_push(&bf, cells[a] * (int64_t)n_f + f)) { rc = ORC_ENOMEM; goto done; }
      for (int b = a + 1; b < nc; ++b)
        if (vi64_push(&kt, cells[a] * NS + cells[b])) { rc = ORC_ENOMEM; goto done; }
    }
  }
  if ((rc = pairs_to_csr(kt.a, kt.n, n_s, &out->at_ptr, &out->at_col))) goto done;
  /* rows of B: faces of each cell, ascending */
  bf.n = sort_unique_i64(bf.a, bf.n);
  bptr = (int64_t*)calloc((size_t)n_s + 1, sizeof(int64_t));
  bcol = (int32_t*)malloc((size_t)(bf.n + 1) * sizeof(int32_t));
  if (!bptr || !bcol) { rc = ORC_ENOMEM; goto done; }
  for (int64_t k = 0; k < bf.n; ++k) {
    bptr[bf.a[k] / n_f + 1]++;
    bcol[k] = (int32_t)(bf.a[k] % n_f);
  }
  for (int32_t c = 0; c < n_s; ++c) bptr[c + 1] += bptr[c];

  /* candidates: A_t entries (p<q) absent from A_v */
  for (int32_t p = 0; p < n_s; ++p)
    for (int64_t t = out->at_ptr[p]; t < out->at_ptr[p + 1]; ++t) {
      int32_t q = out->at_col[t];
      if (q <= p || csr_has(out->av_ptr, out->av_col, p, q)) continue;
      /* isoline crossing on a common face */
      double mg = INFINITY;
      int crossed = 0;
      int64_t a = bptr[p], b = bptr[q];
      while (a < bptr[p + 1] && b < bptr[q + 1]) {
        if (bcol[a] < bcol[b]) { ++a; continue; }
        if (bcol[a] > bcol[b]) { ++b; continue; }
        int32_t f = bcol[a];
        double fp[3], fq3[3], sp[4], sq[4];
        for (int k = 0; k < 3; ++k) {
          int32_t v = F[3 * (int64_t)f + k];
          fp[k] = u_at(Up, Uc, Uv, v, p);
          fq3[k] = u_at(Up, Uc, Uv, v, q);
        }
        if (iso_segment(fp, tau, sp) && iso_segment(fq3, tau, sq))
          crossed |= seg_cross(sp, sq, &mg);
        ++a; ++b;
      }
      int state = 0;
      if (crossed) state = csr_common(out->av_ptr, out->av_col, p, q) >= 2 ? 2 : 1;
      if (vi32_push(&cand, p) || vi32_push(&cand, q) || vi32_push(&cst, state) ||
          vf64_push(&cmg, mg)) { rc = ORC_ENOMEM; goto done; }
      if (state == 1 && vi64_push(&kd, p * NS + q)) { rc = ORC_ENOMEM; goto done; }
    }
  out->n_cand = cst.n;
  out->cand = cand.a; cand.a = 0;
  out->cand_state = cst.a; cst.a = 0;
  out->cand_margin = cmg.a; cmg.a = 0;

  /* curated adjacency = A_v plus the kept candidates */
  for (int32_t p = 0; p < n_s; ++p)
    for (int64_t t = out->av_ptr[p]; t < out->av_ptr[p + 1]; ++t)
      if (out->av_col[t] > p && vi64_push(&kd, p * NS + out->av_col[t])) { rc = ORC_ENOMEM; goto done; }
  if ((rc = pairs_to_csr(kd.a, kd.n, n_s, &out->ad_ptr, &out->ad_col))) goto done;
  const int64_t* dp = out->ad_ptr;
  const int32_t* dc = out->ad_col;

  /* triangles: 3-cliques i<j<k, in lexicographic order */
  for (int32_t i = 0; i < n_s; ++i)
    for (int64_t a = dp[i]; a < dp[i + 1]; ++a) {
      int32_t j = dc[a];
      if (j <= i) continue;
      for (int64_t b = a + 1; b < dp[i + 1]; ++b) {
        int32_t k = dc[b];
        if (k > j && csr_has(dp, dc, j, k))
          if (vi32_push(&tri, i) || vi32_push(&tri, j) || vi32_push(&tri, k)) { rc = ORC_ENOMEM; goto done; }
      }
    }
  int64_t nt = tri.n / 3;

  /* spurious triangles: a cell with exactly three mutually adjacent
   * neighbours j<k<l; the triangle (j,k,l) covers it and is removed */
  removed = (char*)calloc((size_t)(nt + 1), 1);
  if (!removed) { rc = ORC_ENOMEM; goto done; }
  for (int32_t i = 0; i < n_s; ++i) {
    if (dp[i + 1] - dp[i] != 3) continue;
    int32_t j = dc[dp[i]], k = dc[dp[i] + 1], l = dc[dp[i] + 2];
    if (!(csr_has(dp, dc, j, k) && csr_has(dp, dc, k, l) && csr_has(dp, dc, j, l))) continue;
    for (int64_t t = 0; t < nt; ++t)
      if (tri.a[3 * t] == j && tri.a[3 * t + 1] == k && tri.a[3 * t + 2] == l) removed[t] = 1;
  }
  {
    int64_t m = 0;
    for (int64_t t = 0; t < nt; ++t) {
      if (removed[t]) { out->n_removed++; continue; }
      tri.a[3 * m] = tri.a[3 * t];
      tri.a[3 * m + 1] = tri.a[3 * t + 1];
      tri.a[3 * m + 2] = tri.a[3 * t + 2];
      ++m;
    }
    nt = m;
  }

  /* orientation.  Edge -> faces through sorted keys (edge key * nt + face). */
  for (int64_t t = 0; t < nt; ++t)
    for (int e = 0; e < 3; ++e) {
      int32_t x = tri.a[3 * t + e], y = tri.a[3 * t + (e + 1) % 3];
      int32_t lo = x < y ? x : y, hi = x < y ? y : x;
      if (vi64_push(&ek, (lo * NS + hi) * (nt + 1) + t)) { rc = ORC_ENOMEM; goto done; }
    }
  qsort(ek.a, (size_t)ek.n, sizeof(int64_t), cmp_i64);
  /* for every (face, local edge) the face across it, or -1 */
  eface = (int32_t*)malloc((size_t)(3 * nt + 1) * sizeof(int32_t));
  if (!eface) { rc = ORC_ENOMEM; goto done; }
  for (int64_t t = 0; t < 3 * nt; ++t) eface[t] = -1;
  for (int64_t a = 0; a < ek.n;) {
    int64_t b = a;
    int64_t key = ek.a[a] / (nt + 1);
    while (b < ek.n && ek.a[b] / (nt + 1) == key) ++b;
    if (b - a > 2) out->n_nonmanifold++;
    if (b - a == 2) {
      int64_t f0 = ek.a[a] % (nt + 1), f1 = ek.a[a + 1] % (nt + 1);
      int32_t lo = (int32_t)(key / NS), hi = (int32_t)(key % NS);
      for (int e = 0; e < 3; ++e) {
        int32_t x = tri.a[3 * f0 + e], y = tri.a[3 * f0 + (e + 1) % 3];
        if ((x == lo && y == hi) || (x == hi && y == lo)) eface[3 * f0 + e] = (int32_t)f1;
        x = tri.a[3 * f1 + e]; y = tri.a[3 * f1 + (e + 1) % 3];
        if ((x == lo && y == hi) || (x == hi && y == lo)) eface[3 * f1 + e] = (int32_t)f0;
      }
    }
    a = b;
  }
  /* primal vertex normals (area weighted) */
  vn = (double*)calloc((size_t)3 * n_v, sizeof(double));
  orient = (int32_t*)malloc((size_t)(3 * nt + 1) * sizeof(int32_t));
  done_ = (char*)calloc((size_t)(nt + 1), 1);
  fq = (int32_t*)malloc((size_t)(nt + 1) * sizeof(int32_t));
  if (!vn || !orient || !done_ || !fq) { rc = ORC_ENOMEM; goto done; }
  for (int32_t f = 0; f < n_f; ++f) {
    const int32_t* fv = F + 3 * (int64_t)f;
    double e1[3], e2[3], cr[3];
    sub3(V + 3 * (int64_t)fv[1], V + 3 * (int64_t)fv[0], e1);
    sub3(V + 3 * (int64_t)fv[2], V + 3 * (int64_t)fv[0], e2);
    cross3(e1, e2, cr);
    for (int k = 0; k < 3; ++k)
      for (int d = 0; d < 3; ++d) vn[3 * (int64_t)fv[k] + d] += cr[d];
  }
  for (int64_t r = 0; r < nt; ++r) {
    if (done_[r]) continue;
    /* orient the component's lowest triangle along the summed normals */
    int32_t* o = orient + 3 * r;
    o[0] = tri.a[3 * r]; o[1] = tri.a[3 * r + 1]; o[2] = tri.a[3 * r + 2];
    const double *x0 = V + 3 * (int64_t)seeds[o[0]], *x1 = V + 3 * (int64_t)seeds[o[1]],
                 *x2 = V + 3 * (int64_t)seeds[o[2]];
    double e1[3], e2[3], cr[3], ref[3];
    sub3(x1, x0, e1);
    sub3(x2, x0, e2);
    cross3(e1, e2, cr);
    for (int d = 0; d < 3; ++d)
      ref[d] = vn[3 * (int64_t)seeds[o[0]] + d] + vn[3 * (int64_t)seeds[o[1]] + d] +
               vn[3 * (int64_t)seeds[o[2]] + d];
    if (dot3(cr, ref) < 0.0) { int32_t s = o[1]; o[1] = o[2]; o[2] = s; }
    done_[r] = 1;
    int64_t head = 0, tail = 0;
    fq[tail++] = (int32_t)r;
    while (head < tail) {
      int32_t f = fq[head++];
      const int32_t* of = orient + 3 * (int64_t)f;
      for (int e = 0; e < 3; ++e) {
        int32_t x = of[e], y = of[(e + 1) % 3];
        /* the unoriented slot of the face across edge {x,y} */
        int32_t g = -1;
        for (int s = 0; s < 3; ++s) {
          int32_t a = tri.a[3 * (int64_t)f + s], b = tri.a[3 * (int64_t)f + (s + 1) % 3];
          if ((a == x && b == y) || (a == y && b == x)) g = eface[3 * (int64_t)f + s];
        }
        if (g < 0) continue;
        /* g must traverse the shared edge as y -> x */
        int32_t z = tri.a[3 * (int64_t)g] ^ tri.a[3 * (int64_t)g + 1] ^ tri.a[3 * (int64_t)g + 2] ^ x ^ y;
        if (!done_[g]) {
          orient[3 * (int64_t)g] = y;
          orient[3 * (int64_t)g + 1] = x;
          orient[3 * (int64_t)g + 2] = z;
          done_[g] = 1;
          fq[tail++] = g;
        } else {
          const int32_t* og = orient + 3 * (int64_t)g;
          int ok = 0;
          for (int s = 0; s < 3; ++s) ok |= (og[s] == y && og[(s + 1) % 3] == x);
          if (!ok) out->n_conflict++;
        }
      }
    }
  }
  /* each conflict is seen from both of its faces */
  out->n_conflict /= 2;
  out->n_tri = nt;
  out->tri = orient;
  orient = 0;
  if (!out->tri) out->tri = (int32_t*)malloc(sizeof(int32_t));
#undef THR
done:
  free(kv.a); free(kt.a); free(kd.a); free(bf.a); free(ek.a);
  free(cand.a); free(cst.a); free(cmg.a); free(tri.a);
  free(bptr); free(tptr); free(bcol); free(orient); free(fq); free(eface);
  free(removed); free(done_); free(vn);
  if (rc) orc_dual_free(out);
  return rc;
}
