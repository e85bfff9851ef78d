/* Host-only driver for the AddressSanitizer / UndefinedBehaviorSanitizer
 * build of the seeded generators (graphgen/graphgen.c) and the CPU oracle
 * (oracle/oracle.c): it calls every exported function on small inputs,
 * including the degenerate ones (no vertices, no edges, one block, round
 * caps), and checks the results it can check cheaply.  Built and run by
 * tests/test_sanitize_cpu.py; exits non-zero on a failed check, and the
 * sanitizers abort on any memory or undefined-behaviour error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct gg_graph {
  int64_t n, nnz;
  int64_t *rowptr;
  int32_t *colidx;
} gg_graph;
typedef struct gg_batch {
  int64_t num_graphs;
  int64_t *voff, *eoff;
  int32_t *rowptr_local, *colidx_local;
} gg_batch;

gg_graph *gg_er(int64_t n, int64_t m, uint64_t seed);
gg_graph *gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed);
gg_graph *gg_stencil27(int64_t L, uint64_t seed);
gg_batch *gg_er_batch(int64_t G, uint64_t seed, int64_t nmin, int64_t nmax, double dmin,
                      double dmax);
int gg_batch_sizes(int64_t G, uint64_t seed, int64_t nmin, int64_t nmax, double dmin, double dmax,
                   int64_t *n_out, int64_t *m_out);
int gg_poisson_arrivals(int64_t count, double rate, uint64_t seed, double *t_out);
void gg_stream(uint64_t seed, uint64_t stream, int64_t count, uint64_t *out);
void gg_free(gg_graph *g);
void gg_batch_free(gg_batch *b);

int64_t oracle_rsc(int64_t n, const int64_t *rowptr, const int32_t *colidx, int32_t *color_out,
                   int32_t *round_out, int64_t *trace, int64_t cap);
int oracle_seq(int64_t n, const int64_t *rowptr, const int32_t *colidx, int32_t *color_out);
int64_t oracle_seq_rounds(int64_t n, const int64_t *rowptr, const int32_t *colidx,
                          int32_t *round_out);
int64_t oracle_blocks(int64_t n, const int64_t *rowptr, const int32_t *colidx, int64_t p,
                      int32_t *color_out, int32_t *recolours_out);
int64_t oracle_check_proper(int64_t n, const int64_t *rowptr, const int32_t *colidx,
                            const int32_t *color);
int64_t oracle_check_grundy(int64_t n, const int64_t *rowptr, const int32_t *colidx,
                            const int32_t *color);
int oracle_rsc_batch(int64_t G, const int64_t *voff, const int64_t *eoff,
                     const int32_t *rowptr_local, const int32_t *colidx_local,
                     int32_t *colors_out, int64_t *rounds_out);

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static void exercise(const gg_graph *g) {
  const int64_t n = g->n;
  int32_t *c = malloc((size_t)(n > 0 ? n : 1) * sizeof *c);
  int32_t *r = malloc((size_t)(n > 0 ? n : 1) * sizeof *r);
  int64_t trace[4 * 64];
  int64_t R = oracle_rsc(n, g->rowptr, g->colidx, c, r, trace, 64);
  CHECK(R >= 0);
  if (n > 0) {
    CHECK(oracle_check_proper(n, g->rowptr, g->colidx, c) == 0);
    CHECK(oracle_check_grundy(n, g->rowptr, g->colidx, c) == 0);
  }
  /* a trace shorter than the round count, and no per-vertex rounds */
  CHECK(oracle_rsc(n, g->rowptr, g->colidx, c, NULL, trace, 1) == R);
  CHECK(oracle_seq(n, g->rowptr, g->colidx, c) == 0);
  if (n > 0) CHECK(oracle_check_proper(n, g->rowptr, g->colidx, c) == 0);
  CHECK(oracle_seq_rounds(n, g->rowptr, g->colidx, r) >= 0);
  for (int64_t p = 1; p <= 64; p *= 4) {
    int64_t Rb = oracle_blocks(n, g->rowptr, g->colidx, p, c, r);
    CHECK(Rb >= 0 && Rb <= (p > n ? (n > 0 ? n : 0) : p) + 1);
    if (n > 0) CHECK(oracle_check_proper(n, g->rowptr, g->colidx, c) == 0);
  }
  free(c);
  free(r);
}

int main(void) {
  gg_graph *gs[] = {gg_er(0, 0, 1), gg_er(1, 0, 1), gg_er(50, 0, 2), gg_er(300, 2000, 3),
                    gg_er(40, 780, 4), /* complete */ gg_rmat(8, 8, 0.57, 0.19, 0.19, 5),
                    gg_stencil27(6, 6)};
  for (size_t i = 0; i < sizeof gs / sizeof gs[0]; ++i) {
    CHECK(gs[i] != NULL);
    if (gs[i]) exercise(gs[i]);
  }
  gg_batch *b = gg_er_batch(40, 7, 1, 2000, 0.0, 30.0);
  CHECK(b != NULL);
  if (b) {
    int32_t *c = malloc((size_t)(b->voff[b->num_graphs] + 1) * sizeof *c);
    int64_t *rr = malloc((size_t)b->num_graphs * sizeof *rr);
    CHECK(oracle_rsc_batch(b->num_graphs, b->voff, b->eoff, b->rowptr_local, b->colidx_local, c,
                           rr) == 0);
    free(c);
    free(rr);
    gg_batch_free(b);
  }
  int64_t ns[16], ms[16];
  CHECK(gg_batch_sizes(16, 3, 100, 50000, 4.0, 64.0, ns, ms) == 0);
  double t[100];
  CHECK(gg_poisson_arrivals(100, 1000.0, 1, t) == 0);
  for (int i = 1; i < 100; ++i) CHECK(t[i] >= t[i - 1]);
  uint64_t s[8];
  gg_stream(0, 0, 8, s);
  for (size_t i = 0; i < sizeof gs / sizeof gs[0]; ++i)
    if (gs[i]) gg_free(gs[i]);
  if (failures) return 1;
  printf("sanitized driver ok\n");
  return 0;
}
