/*
 * graphgen.c -- seeded synthetic graph generators (input construction only).
 *
 * This module builds the inputs that both the CPU oracle and the GPU path
 * colour.  It contains no colouring arithmetic.  Every generator is driven by
 * one portable counter-free PRNG, splitmix64 (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), so the same
 * (parameters, seed) give the same bytes on every machine.
 *
 * All outputs are simple undirected graphs (the problem statement of the
 * paper, Section 2.1, colours simple graphs): symmetric CSR, no self-loops,
 * no duplicate entries, every row sorted ascending.
 *
 * Memory: results are malloc'ed here and handed to the caller, who releases
 * them with gg_free().  Functions return NULL on bad parameters or when
 * memory runs out.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct gg_graph {
  int64_t n;        /* vertices                                     */
  int64_t nnz;      /* CSR entries = 2 * undirected edges           */
  int64_t *rowptr;  /* n + 1 entries                                */
  int32_t *colidx;  /* nnz entries, rows ascending                  */
} gg_graph;

typedef struct gg_batch {
  int64_t num_graphs;
  int64_t *voff;         /* G + 1: vertex offsets of each graph            */
  int64_t *eoff;         /* G + 1: CSR-entry offsets of each graph         */
  int32_t *rowptr_local; /* sum(n_g + 1): per-graph rowptr, local offsets  */
  int32_t *colidx_local; /* sum(nnz_g): per-graph local vertex ids         */
} gg_batch;

/* ---------------------------------------------------------------- PRNG -- */

static inline uint64_t sm64_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Independent stream `stream` of seed `seed`: the state starts at a
 * splitmix64 output of the seed, offset by a splitmix64 output of the
 * stream number, so streams (seed, 0), (seed, 1), ... do not overlap in
 * practice. */
static uint64_t stream_init(uint64_t seed, uint64_t stream) {
  uint64_t a = seed, b = stream ^ 0x5851F42D4C957F2DULL;
  uint64_t x = sm64_next(&a);
  uint64_t y = sm64_next(&b);
  return x ^ (y * 0xD1342543DE82EF95ULL);
}

/* Uniform integer in [0, n) by the multiply-high map (Lemire 2019). */
static inline uint64_t uniform_below(uint64_t *s, uint64_t n) {
  return (uint64_t)(((unsigned __int128)sm64_next(s) * n) >> 64);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double uniform01(uint64_t *s) {
  return (double)(sm64_next(s) >> 11) * (1.0 / 9007199254740992.0);
}

/* ----------------------------------------------------------- helpers -- */

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static void sort_row(int32_t *p, int64_t len) {
  if (len < 32) { /* insertion sort */
    for (int64_t i = 1; i < len; ++i) {
      int32_t x = p[i];
      int64_t j = i - 1;
      while (j >= 0 && p[j] > x) { p[j + 1] = p[j]; --j; }
      p[j + 1] = x;
    }
  } else {
    qsort(p, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

void gg_free(gg_graph *g) {
  if (!g) return;
  free(g->rowptr);
  free(g->colidx);
  free(g);
}

void gg_batch_free(gg_batch *b) {
  if (!b) return;
  free(b->voff);
  free(b->eoff);
  free(b->rowptr_local);
  free(b->colidx_local);
  free(b);
}

/* Build a symmetric CSR from an undirected edge list (a[i], b[i]).
 * Self-loops are dropped; duplicate entries are removed after sorting each
 * row.  The edge arrays are consumed read-only. */
static gg_graph *csr_from_edges(int64_t n, int64_t ne, const int32_t *ea,
                                const int32_t *eb) {
  gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
  if (!g) return NULL;
  g->n = n;
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) { free(g); return NULL; }
  for (int64_t i = 0; i < ne; ++i) {
    if (ea[i] == eb[i]) continue;
    cnt[ea[i] + 1]++;
    cnt[eb[i] + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  int64_t total = cnt[n];
  int32_t *col = (int32_t *)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
  int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!col || !fill) { free(cnt); free(col); free(fill); free(g); return NULL; }
  memcpy(fill, cnt, ((size_t)n + 1) * sizeof(int64_t));
  for (int64_t i = 0; i < ne; ++i) {
    int32_t a = ea[i], b = eb[i];
    if (a == b) continue;
    col[fill[a]++] = b;
    col[fill[b]++] = a;
  }
  free(fill);
  /* sort + dedup each row, compacting in place */
  int64_t w = 0;
  int64_t *rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!rp) { free(cnt); free(col); free(g); return NULL; }
  rp[0] = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t s = cnt[v], e = cnt[v + 1];
    sort_row(col + s, e - s);
    int64_t start = w;
    for (int64_t k = s; k < e; ++k) {
      if (k > s && col[k] == col[k - 1]) continue;
      col[w++] = col[k];
    }
    (void)start;
    rp[v + 1] = w;
  }
  free(cnt);
  g->rowptr = rp;
  g->nnz = w;
  int32_t *shrunk = (int32_t *)realloc(col, (size_t)(w ? w : 1) * sizeof(int32_t));
  g->colidx = shrunk ? shrunk : col;
  return g;
}

/* ---------------------------------------------------- Erdos-Renyi G(n,m) -- */

/* Open-addressing set of canonical pairs (a < b) packed as a * n + b + 1
 * (0 marks an empty slot). */
typedef struct {
  uint64_t *slot;
  uint64_t mask;
} pairset;

static int pairset_init(pairset *ps, int64_t m) {
  uint64_t cap = 16;
  while (cap < (uint64_t)m * 2 + 16) cap <<= 1;
  ps->slot = (uint64_t *)calloc(cap, sizeof(uint64_t));
  ps->mask = cap - 1;
  return ps->slot != NULL;
}

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 33)) * 0xFF51AFD7ED558CCDULL;
  z = (z ^ (z >> 33)) * 0xC4CEB9FE1A85EC53ULL;
  return z ^ (z >> 33);
}

/* returns 1 if inserted (was absent), 0 if present */
static inline int pairset_insert(pairset *ps, uint64_t key) {
  uint64_t h = mix64(key) & ps->mask;
  for (;;) {
    uint64_t k = ps->slot[h];
    if (k == 0) { ps->slot[h] = key; return 1; }
    if (k == key) return 0;
    h = (h + 1) & ps->mask;
  }
}

/* Draw unordered pairs uniformly from [0,n)^2 with stream state *s; drop
 * a == b and pairs already drawn; keep drawing until exactly m distinct
 * edges exist.  Writes the edges in draw order to ea/eb. */
static int er_edges(uint64_t *s, int64_t n, int64_t m, int32_t *ea, int32_t *eb) {
  pairset ps;
  if (!pairset_init(&ps, m)) return 0;
  int64_t k = 0;
  while (k < m) {
    uint64_t a = uniform_below(s, (uint64_t)n);
    uint64_t b = uniform_below(s, (uint64_t)n);
    if (a == b) continue;
    uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    if (pairset_insert(&ps, lo * (uint64_t)n + hi + 1)) {
      ea[k] = (int32_t)lo;
      eb[k] = (int32_t)hi;
      ++k;
    }
  }
  free(ps.slot);
  return 1;
}

gg_graph *gg_er(int64_t n, int64_t m, uint64_t seed) {
  if (n < 0 || m < 0 || n > INT32_MAX) return NULL;
  if (n < 2 && m > 0) return NULL;
  if (m > n * (n - 1) / 2) return NULL;
  int32_t *ea = (int32_t *)malloc((size_t)(m ? m : 1) * sizeof(int32_t));
  int32_t *eb = (int32_t *)malloc((size_t)(m ? m : 1) * sizeof(int32_t));
  if (!ea || !eb) { free(ea); free(eb); return NULL; }
  uint64_t s = stream_init(seed, 0);
  if (!er_edges(&s, n, m, ea, eb)) { free(ea); free(eb); return NULL; }
  gg_graph *g = csr_from_edges(n, m, ea, eb);
  free(ea);
  free(eb);
  return g;
}

/* ------------------------------------------------------------- R-MAT -- */

/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each of ef * 2^scale samples
 * descends `scale` levels; at each level one uniform draw picks quadrant
 * a (00), b (01: column bit), c (10: row bit) or d (11).  Bits are filled
 * from the most significant down.  No noise, no label permutation.  The
 * samples are then symmetrised, loops and duplicates dropped. */
gg_graph *gg_rmat(int scale, int64_t edge_factor, double a, double b, double c,
                  uint64_t seed) {
  if (scale < 1 || scale > 30 || edge_factor < 0) return NULL;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return NULL;
  int64_t n = (int64_t)1 << scale;
  int64_t ns = edge_factor * n;
  int32_t *ea = (int32_t *)malloc((size_t)(ns ? ns : 1) * sizeof(int32_t));
  int32_t *eb = (int32_t *)malloc((size_t)(ns ? ns : 1) * sizeof(int32_t));
  if (!ea || !eb) { free(ea); free(eb); return NULL; }
  const double ab = a + b, abc = a + b + c;
  /* Samples are split into fixed chunks with a stream per chunk, so the
   * result is the same for any thread count. */
  const int64_t chunk = 1 << 16;
  const int64_t nchunks = (ns + chunk - 1) / chunk;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    uint64_t s = stream_init(seed, (uint64_t)ch);
    int64_t lo = ch * chunk, hi = lo + chunk < ns ? lo + chunk : ns;
    for (int64_t i = lo; i < hi; ++i) {
      uint32_t u = 0, v = 0;
      for (int lev = scale - 1; lev >= 0; --lev) {
        double r = uniform01(&s);
        if (r < a) {
        } else if (r < ab) {
          v |= 1u << lev;
        } else if (r < abc) {
          u |= 1u << lev;
        } else {
          u |= 1u << lev;
          v |= 1u << lev;
        }
      }
      ea[i] = (int32_t)u;
      eb[i] = (int32_t)v;
    }
  }
  gg_graph *g = csr_from_edges(n, ns, ea, eb);
  free(ea);
  free(eb);
  return g;
}

/* ------------------------------------------------ 27-point stencil mesh -- */

/* L x L x L grid; (x, y, z) is adjacent to every other point at Chebyshev
 * distance 1.  Point (x, y, z) gets vertex id perm[(L*x + y)*L + z] where
 * perm is a Fisher-Yates shuffle of 0..L^3-1 drawn from stream (seed, 0). */
gg_graph *gg_stencil27(int64_t L, uint64_t seed) {
  if (L < 1 || L * L * L > INT32_MAX) return NULL;
  int64_t n = L * L * L;
  int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!perm) return NULL;
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  uint64_t s = stream_init(seed, 0);
  for (int64_t i = n - 1; i >= 1; --i) {
    int64_t j = (int64_t)uniform_below(&s, (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
  int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!g || !rp) { free(perm); free(g); free(rp); return NULL; }
  /* degree of each grid point, scattered to its id */
  for (int64_t x = 0; x < L; ++x)
    for (int64_t y = 0; y < L; ++y)
      for (int64_t z = 0; z < L; ++z) {
        int64_t ex = 1 + (x > 0) + (x < L - 1);
        int64_t ey = 1 + (y > 0) + (y < L - 1);
        int64_t ez = 1 + (z > 0) + (z < L - 1);
        rp[perm[(L * x + y) * L + z] + 1] = ex * ey * ez - 1;
      }
  for (int64_t v = 0; v < n; ++v) rp[v + 1] += rp[v];
  int64_t nnz = rp[n];
  int32_t *col = (int32_t *)malloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
  if (!col) { free(perm); free(g); free(rp); return NULL; }
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < L; ++x)
    for (int64_t y = 0; y < L; ++y)
      for (int64_t z = 0; z < L; ++z) {
        int32_t id = perm[(L * x + y) * L + z];
        int64_t w = rp[id];
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              if (!dx && !dy && !dz) continue;
              int64_t X = x + dx, Y = y + dy, Z = z + dz;
              if (X < 0 || Y < 0 || Z < 0 || X >= L || Y >= L || Z >= L) continue;
              col[w++] = perm[(L * X + Y) * L + Z];
            }
        sort_row(col + rp[id], w - rp[id]);
      }
  free(perm);
  g->n = n;
  g->nnz = nnz;
  g->rowptr = rp;
  g->colidx = col;
  return g;
}

/* --------------------------------------------------- batch of ER graphs -- */

/* Parameters of graph g of a batch, drawn from stream (seed, 2g):
 *   n_g = round(exp(U[ln nmin, ln nmax])),  d_g = U[dmin, dmax],
 *   m_g = min(round(n_g d_g / 2), n_g (n_g - 1) / 2).
 * Its edges come from stream (seed, 2g + 1) by the G(n, m) rule above. */
static void batch_params(uint64_t seed, int64_t g, int64_t nmin, int64_t nmax,
                         double dmin, double dmax, int64_t *n_out, int64_t *m_out) {
  uint64_t s = stream_init(seed, 2 * (uint64_t)g);
  double lo = log((double)nmin), hi = log((double)nmax);
  double u1 = uniform01(&s);
  double u2 = uniform01(&s);
  int64_t n = (int64_t)llround(exp(lo + u1 * (hi - lo)));
  if (n < 1) n = 1;
  double d = dmin + u2 * (dmax - dmin);
  int64_t m = (int64_t)llround((double)n * d / 2.0);
  int64_t mmax = n * (n - 1) / 2;
  if (m > mmax) m = mmax;
  *n_out = n;
  *m_out = m;
}

/* Sizes only (no edges): lets a caller plan memory before generating. */
int gg_batch_sizes(int64_t G, uint64_t seed, int64_t nmin, int64_t nmax,
                   double dmin, double dmax, int64_t *n_out, int64_t *m_out) {
  if (G < 0 || nmin < 1 || nmax < nmin || dmin < 0 || dmax < dmin) return -1;
  for (int64_t g = 0; g < G; ++g)
    batch_params(seed, g, nmin, nmax, dmin, dmax, &n_out[g], &m_out[g]);
  return 0;
}

gg_batch *gg_er_batch(int64_t G, uint64_t seed, int64_t nmin, int64_t nmax,
                      double dmin, double dmax) {
  if (G < 0 || nmin < 1 || nmax < nmin || nmax > INT32_MAX || dmin < 0 ||
      dmax < dmin)
    return NULL;
  gg_batch *B = (gg_batch *)calloc(1, sizeof(gg_batch));
  int64_t *ng = (int64_t *)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
  int64_t *mg = (int64_t *)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
  if (!B || !ng || !mg) { free(B); free(ng); free(mg); return NULL; }
  gg_batch_sizes(G, seed, nmin, nmax, dmin, dmax, ng, mg);
  B->num_graphs = G;
  B->voff = (int64_t *)malloc(((size_t)G + 1) * sizeof(int64_t));
  B->eoff = (int64_t *)malloc(((size_t)G + 1) * sizeof(int64_t));
  if (!B->voff || !B->eoff) { free(ng); free(mg); gg_batch_free(B); return NULL; }
  B->voff[0] = 0;
  B->eoff[0] = 0;
  for (int64_t g = 0; g < G; ++g) {
    B->voff[g + 1] = B->voff[g] + ng[g];
    B->eoff[g + 1] = B->eoff[g] + 2 * mg[g];
  }
  int64_t totv = B->voff[G], tote = B->eoff[G];
  B->rowptr_local = (int32_t *)malloc((size_t)(totv + G + 1) * sizeof(int32_t));
  B->colidx_local = (int32_t *)malloc((size_t)(tote ? tote : 1) * sizeof(int32_t));
  if (!B->rowptr_local || !B->colidx_local) {
    free(ng); free(mg); gg_batch_free(B); return NULL;
  }
  int failed = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
  for (int64_t g = 0; g < G; ++g) {
    int64_t n = ng[g], m = mg[g];
    int32_t *ea = (int32_t *)malloc((size_t)(m ? m : 1) * sizeof(int32_t));
    int32_t *eb = (int32_t *)malloc((size_t)(m ? m : 1) * sizeof(int32_t));
    gg_graph *sub = NULL;
    if (ea && eb) {
      uint64_t s = stream_init(seed, 2 * (uint64_t)g + 1);
      if (er_edges(&s, n, m, ea, eb)) sub = csr_from_edges(n, m, ea, eb);
    }
    free(ea);
    free(eb);
    if (!sub || sub->nnz != 2 * m) { failed |= 1; gg_free(sub); continue; }
    int32_t *rp = B->rowptr_local + B->voff[g] + g;
    for (int64_t v = 0; v <= n; ++v) rp[v] = (int32_t)sub->rowptr[v];
    memcpy(B->colidx_local + B->eoff[g], sub->colidx, (size_t)sub->nnz * sizeof(int32_t));
    gg_free(sub);
  }
  free(ng);
  free(mg);
  if (failed) { gg_batch_free(B); return NULL; }
  return B;
}

/* ------------------------------------------------- Poisson arrivals -- */

/* Arrival times of `count` requests of a Poisson process of rate `rate`
 * (per second): exponential gaps -ln(1 - U) / rate, stream (seed, 0). */
int gg_poisson_arrivals(int64_t count, double rate, uint64_t seed, double *t_out) {
  if (count < 0 || !(rate > 0)) return -1;
  uint64_t s = stream_init(seed, 0);
  double t = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    t += -log(1.0 - uniform01(&s)) / rate;
    t_out[i] = t;
  }
  return 0;
}

/* Raw stream access, for tests of the PRNG itself. */
void gg_stream(uint64_t seed, uint64_t stream, int64_t count, uint64_t *out) {
  uint64_t s = stream_init(seed, stream);
  for (int64_t i = 0; i < count; ++i) out[i] = sm64_next(&s);
}
