/* Runs the oracle's whole chain (operator, init, steps with and without
 * per-pair coefficients, labels, re-seeding, dual mesh) on a small torus, for
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer.  Exits 0 when
 * every call succeeds; a sanitizer report aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

#define NX 16
#define NY 12

static int torus(double* V, int32_t* F) {
  int f = 0;
  for (int y = 0; y < NY; ++y)
    for (int x = 0; x < NX; ++x) {
      const double th = 2.0 * M_PI * x / NX, ph = 2.0 * M_PI * y / NY;
      const int v = x + NX * y;
      V[3 * v] = (3.0 + cos(ph)) * cos(th);
      V[3 * v + 1] = (3.0 + cos(ph)) * sin(th);
      V[3 * v + 2] = sin(ph);
      const int a = v, b = (x + 1) % NX + NX * y, c = (x + 1) % NX + NX * ((y + 1) % NY),
                d = x + NX * ((y + 1) % NY);
      F[3 * f] = a; F[3 * f + 1] = b; F[3 * f + 2] = c; ++f;
      F[3 * f] = a; F[3 * f + 1] = c; F[3 * f + 2] = d; ++f;
    }
  return f;
}

int main(void) {
  enum { NV = NX * NY, NS = 5 };
  static double V[3 * NV];
  static int32_t F[6 * NV];
  const int nf = torus(V, F);
  const int32_t seeds[NS] = {3, 40, 77, 120, 170};
  int64_t Lp[NV + 1], Up[NV + 1], Op[NV + 1];
  int32_t *Lc = NULL, *Uc = NULL;
  double *Lv = NULL, *Uv = NULL;
  int rc = 0;
  for (int op = 0; op < 2 && !rc; ++op) {
    rc |= orc_operator(NV, V, nf, F, op, Lp, &Lc, &Lv);
    rc |= orc_init(NV, seeds, NS, Up, &Uc, &Uv);
    if (rc) break;
    const int32_t types[NS + 1] = {0, 1, 0, 1, 1, 0};
    const double tab[2 * 2 * 3] = {0.04, 0.2, 1.0, 0.05, 0.3, 0.8, 0.05, 0.3, 0.8, 0.03, 0.1, 1.2};
    orc_params P = {0.2, 0.04, 1.0, 0.1, 5.0, 1e-3, 0, 0, NULL, NULL};
    for (int t = 0; t < 60 && !rc; ++t) {
      if (t == 30) {  // per-pair coefficients for the second half
        P.n_types = 2;
        P.types = types;
        P.tab = tab;
      }
      double margin[NV];
      int32_t skel[NV], *Oc = NULL;
      double* Ov = NULL;
      int64_t ev = 0;
      rc |= orc_step(NV, NS, Lp, Lc, Lv, Up, Uc, Uv, &P, Op, &Oc, &Ov, margin, skel, &ev);
      {  // the row-block variant gives the same step
        int64_t Op3[NV + 1];
        int32_t* Oc3 = NULL;
        double *Ov3 = NULL, sm[NV];
        rc |= orc_step_threads(NV, NS, Lp, Lc, Lv, Up, Uc, Uv, &P, Op3, &Oc3, &Ov3, NULL, sm,
                               NULL, NULL, 3);
        if (!rc) {
          for (int i = 0; i <= NV; ++i) rc |= Op3[i] != Op[i];
          for (int64_t q = 0; !rc && q < Op[NV]; ++q) rc |= Oc3[q] != Oc[q] || Ov3[q] != Ov[q];
        }
        orc_free(Oc3);
        orc_free(Ov3);
      }
      orc_free(Uc);
      orc_free(Uv);
      Uc = Oc;
      Uv = Ov;
      for (int i = 0; i <= NV; ++i) Up[i] = Op[i];
    }
    int32_t labels[NV], seeds2[NS], status[NS];
    double gap[NV], m2[NS];
    rc |= orc_labels(NV, NS, Up, Uc, Uv, labels, gap);
    rc |= orc_lloyd(NV, V, nf, F, NS, Up, Uc, Uv, seeds, seeds2, status, m2);
    orc_dual d;
    rc |= orc_dual_mesh(NV, V, nf, F, NS, Up, Uc, Uv, seeds, 0.25, &d);
    if (!rc) orc_dual_free(&d);
    orc_free(Lc);
    orc_free(Lv);
    orc_free(Uc);
    orc_free(Uv);
    Lc = NULL; Lv = NULL; Uc = NULL; Uv = NULL;
  }
  printf("oracle chain: %s\n", rc ? "error" : "ok");
  return rc ? 1 : 0;
}
