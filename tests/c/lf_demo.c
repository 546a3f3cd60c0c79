/* A plain C caller of the library: reads a mesh and seeds from a binary
 * file, runs the whole path through the C ABI alone (no Python, no torch)
 * and writes the labels and the dual triangles.
 *
 *   lf_demo in.bin out.bin steps
 *
 * in.bin:  int32 n_v, n_f, n_s, op; float64 V[3 n_v]; int32 F[3 n_f];
 *          int32 seeds[n_s]
 * out.bin: int32 labels[n_v]; int64 n_tri; int32 tris[3 n_tri];
 *          int32 seeds[n_s] (after one Lloyd round of `steps` steps)
 * Prints one line of counters; exits non-zero with the library's message on
 * any error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "lf.h"

#define CHECK(call)                                                          \
  do {                                                                       \
    lf_status st_ = (call);                                                  \
    if (st_ != LF_OK) {                                                      \
      fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, lf_last_error()); \
      return 1;                                                              \
    }                                                                        \
  } while (0)

static int read_all(FILE* fp, void* p, size_t size, size_t n) {
  return fread(p, size, n, fp) == n ? 0 : -1;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: lf_demo in.bin out.bin steps\n");
    return 2;
  }
  const int32_t steps = atoi(argv[3]);
  FILE* fp = fopen(argv[1], "rb");
  if (!fp) return 2;
  int32_t hdr[4];
  if (read_all(fp, hdr, sizeof(int32_t), 4)) return 2;
  const int32_t n_v = hdr[0], n_f = hdr[1], n_s = hdr[2], op = hdr[3];
  double* V = malloc(sizeof(double) * 3 * (size_t)n_v);
  int32_t* F = malloc(sizeof(int32_t) * 3 * (size_t)n_f);
  int32_t* seeds = malloc(sizeof(int32_t) * (size_t)n_s);
  int32_t* labels = malloc(sizeof(int32_t) * (size_t)n_v);
  if (!V || !F || !seeds || !labels) return 2;
  if (read_all(fp, V, sizeof(double), 3 * (size_t)n_v) ||
      read_all(fp, F, sizeof(int32_t), 3 * (size_t)n_f) ||
      read_all(fp, seeds, sizeof(int32_t), (size_t)n_s))
    return 2;
  fclose(fp);

  lf_ctx* ctx = NULL;
  lf_mesh* mesh = NULL;
  lf_fields* f = NULL;
  lf_params P;
  lf_params_default(&P);
  CHECK(lf_ctx_create(0, NULL, &ctx));
  CHECK(lf_mesh_create(ctx, V, n_v, F, n_f, op, &mesh));
  CHECK(lf_fields_create(mesh, seeds, n_s, &P, &f));
  /* the steps run while the host goes on; lf_sync (or any later call on f)
     completes them */
  CHECK(lf_step_async(f, steps));
  CHECK(lf_sync(f));
  CHECK(lf_labels(f, labels, 0));

  int64_t n_tri = 0, adj_nnz = 0;
  CHECK(lf_dual_mesh(f, P.tau, &n_tri, NULL, &adj_nnz, NULL, NULL));
  int32_t* tris = malloc(sizeof(int32_t) * 3 * (size_t)(n_tri > 0 ? n_tri : 1));
  int32_t* adj_rp = malloc(sizeof(int32_t) * ((size_t)n_s + 1));
  int32_t* adj_col = malloc(sizeof(int32_t) * (size_t)(adj_nnz > 0 ? adj_nnz : 1));
  if (!tris || !adj_rp || !adj_col) return 2;
  CHECK(lf_dual_mesh(f, P.tau, &n_tri, tris, &adj_nnz, adj_rp, adj_col));
  CHECK(lf_lloyd(f, 1, steps, seeds));

  int64_t nnz = 0, skel = 0, done = 0, empty = 0, grows = 0;
  CHECK(lf_stats(f, &nnz, &skel, &done, &empty, &grows));
  printf("{\"n_v\": %d, \"steps\": %lld, \"nnz\": %lld, \"skeleton_total\": %lld, \"n_tri\": %lld}\n",
         n_v, (long long)done, (long long)nnz, (long long)skel, (long long)n_tri);

  fp = fopen(argv[2], "wb");
  if (!fp) return 2;
  fwrite(labels, sizeof(int32_t), (size_t)n_v, fp);
  fwrite(&n_tri, sizeof(int64_t), 1, fp);
  fwrite(tris, sizeof(int32_t), 3 * (size_t)n_tri, fp);
  fwrite(seeds, sizeof(int32_t), (size_t)n_s, fp);
  fclose(fp);

  CHECK(lf_fields_destroy(f));
  CHECK(lf_mesh_destroy(mesh));
  CHECK(lf_ctx_destroy(ctx));
  free(V);
  free(F);
  free(seeds);
  free(labels);
  free(tris);
  free(adj_rp);
  free(adj_col);
  return 0;
}
