/*
 * oracle.c -- CPU oracle for round-synchronous speculative colouring.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code.  The GPU library
 * shares nothing with it: no headers, no helpers, no tables.
 *
 * It is deliberately plain, single-threaded and slow, and follows the
 * paper step by step:
 *
 *   oracle_rsc  -- Algorithm 1 (Section 3.1, "Using Barrier Synchronisation")
 *                  with every vertex its own block (p = n), so every
 *                  non-isolated vertex is a boundary vertex:
 *                    phase 1: each vertex still to be coloured takes the
 *                             least colour not used by a neighbour (First
 *                             Fit, Section 3); colours are 0-based, drawn
 *                             from {0, ..., max degree} (Algorithm 1's
 *                             TotalColors);
 *                    barrier;
 *                    phase 2: conflicts between two vertices coloured in the
 *                             same round are detected; one side is recoloured
 *                             in the next round;
 *                    barrier; repeat while some vertex must be recoloured.
 *                  Readings taken where the paper is silent or garbled:
 *                    - the HIGHER vertex id of a conflicting pair is
 *                      recoloured (the paper recolours the vertex in the
 *                      lower partition; with one vertex per partition that
 *                      is the same rule with partitions numbered by
 *                      decreasing id);
 *                    - the set of vertices to recolour collects the vertex
 *                      v under test (the pseudo-code's "R_i <- R_i U {u}"
 *                      names the foreign vertex; the text and both lemmas of
 *                      Section 4 recolour the vertex of the losing block);
 *                    - phase 1 sees only colours that are final (committed
 *                      in an earlier round); a neighbour that is itself
 *                      waiting to be recoloured forbids nothing;
 *                    - all vertices start uncoloured (ForbiddenColors
 *                      initialised to -1), so round 1 colours every vertex 0.
 *
 *   oracle_seq  -- the sequential First-Fit baseline of Section 5 (vertex
 *                  order 0, 1, ..., n-1; the paper does not state the order).
 *   oracle_seq_rounds -- the rounds in which an id-priority schedule gives
 *                  every vertex that same colour: the longest id-increasing
 *                  path ending at each vertex.
 *
 *   oracle_blocks -- Algorithm 1 with p blocks of consecutive ids, read
 *                  literally (per-edge ForbiddenColors slots, sequential
 *                  First Fit inside a block, the lower partition recoloured);
 *                  its own readings are listed at the function.
 *
 *   oracle_check_* -- what the problem statement (Section 2.1) and Lemma 1
 *                  (Section 4) fix: a proper colouring, and First-Fit's
 *                  Grundy property (each colour is the least one absent from
 *                  its neighbourhood).
 *
 * Graphs are CSR with int64 rowptr and int32 colidx; rows need not be
 * sorted.  Nothing here allocates more than O(n + max degree).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* least c >= 0 with used[c] == 0, where used has length len; len itself
 * when all of 0..len-1 are used */
static int32_t least_absent(const unsigned char *used, int64_t len) {
  int64_t c = 0;
  while (c < len && used[c]) ++c;
  return (int32_t)c;
}

/*
 * Round-synchronous speculative colouring (Algorithm 1, p = n).
 *
 * color_out[n]     final colours
 * round_out[n]     (may be NULL) the round in which each vertex's colour
 *                  became final, 1-based
 * trace[4*cap]     (may be NULL) per round r (0-based slot r-1):
 *                    trace[4(r-1)+0] = |U_r|       vertices coloured in round r
 *                    trace[4(r-1)+1] = sum of deg(v) over U_r
 *                    trace[4(r-1)+2] = sum over U_r of #neighbours u < v
 *                    trace[4(r-1)+3] = sum over U_r of the lower neighbours a
 *                      scan in row order examines until it meets the first
 *                      conflicting one (all of them when there is none): the
 *                      work of a conflict scan that stops early (a count for
 *                      byte accounting; it does not affect the colouring)
 * returns the number of rounds R (0 when n == 0), or -1 on bad arguments
 * or allocation failure.  Rounds beyond `cap` are not traced.
 */
int64_t oracle_rsc(int64_t n, const int64_t *rowptr, const int32_t *colidx,
                   int32_t *color_out, int32_t *round_out, int64_t *trace,
                   int64_t cap) {
  if (n < 0 || (n > 0 && (!rowptr || !color_out))) return -1;
  if (n == 0) return 0;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = rowptr[v + 1] - rowptr[v];
    if (d < 0) return -1;
    if (d > maxdeg) maxdeg = d;
  }
  int32_t *color = color_out;          /* -1 = not final yet            */
  int32_t *tent = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  unsigned char *inU = (unsigned char *)calloc((size_t)n, 1);
  unsigned char *lose = (unsigned char *)calloc((size_t)n, 1);
  int64_t *U = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  unsigned char *used = (unsigned char *)calloc((size_t)maxdeg + 1, 1);
  if (!tent || !inU || !lose || !U || !used) {
    free(tent); free(inU); free(lose); free(U); free(used);
    return -1;
  }
  /* Initialisation: nothing is coloured, U = V. */
  int64_t nU = n;
  for (int64_t v = 0; v < n; ++v) {
    color[v] = -1;
    U[v] = v;
    inU[v] = 1;
    if (round_out) round_out[v] = 0;
  }
  int64_t r = 0;
  while (nU > 0) {
    ++r;
    /* Phase 1 (tentative colouring): least colour not final on a neighbour.
     * Only colours 0..deg(v) can matter, since at most deg(v) are used. */
    for (int64_t i = 0; i < nU; ++i) {
      int64_t v = U[i];
      int64_t d = rowptr[v + 1] - rowptr[v];
      for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
        int32_t c = color[colidx[k]];
        if (c >= 0 && c <= d) used[c] = 1;
      }
      tent[v] = least_absent(used, d + 1);
      for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
        int32_t c = color[colidx[k]];
        if (c >= 0 && c <= d) used[c] = 0;
      }
    }
    /* (barrier) Phase 2 (conflict detection): v is recoloured when a
     * neighbour u of lower id, also coloured in this round, took the same
     * colour. */
    int64_t sdeg = 0, slow = 0, sscan = 0;
    for (int64_t i = 0; i < nU; ++i) {
      int64_t v = U[i];
      lose[v] = 0;
      sdeg += rowptr[v + 1] - rowptr[v];
      for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
        int64_t u = colidx[k];
        if (u < v) {
          ++slow;
          if (!lose[v]) ++sscan;
        }
        if (inU[u] && u < v && tent[u] == tent[v]) lose[v] = 1;
      }
    }
    if (trace && r <= cap) {
      trace[4 * (r - 1) + 0] = nU;
      trace[4 * (r - 1) + 1] = sdeg;
      trace[4 * (r - 1) + 2] = slow;
      trace[4 * (r - 1) + 3] = sscan;
    }
    /* Colours of the vertices that did not lose become final; the losers
     * form the next round's set (kept in ascending order). */
    for (int64_t i = 0; i < nU; ++i) {
      int64_t v = U[i];
      if (!lose[v]) {
        color[v] = tent[v];
        if (round_out) round_out[v] = (int32_t)r;
      }
    }
    int64_t w = 0;
    for (int64_t i = 0; i < nU; ++i) {
      int64_t v = U[i];
      if (lose[v]) U[w++] = v;
      else inU[v] = 0;
    }
    nU = w;
    /* (barrier) */
  }
  free(tent); free(inU); free(lose); free(U); free(used);
  return r;
}

/* Sequential First Fit in id order: color[v] = least colour not used by a
 * neighbour u < v.  Returns 0, or -1 on bad arguments. */
int oracle_seq(int64_t n, const int64_t *rowptr, const int32_t *colidx,
               int32_t *color) {
  if (n < 0 || (n > 0 && (!rowptr || !color))) return -1;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = rowptr[v + 1] - rowptr[v];
    if (d > maxdeg) maxdeg = d;
  }
  unsigned char *used = (unsigned char *)calloc((size_t)maxdeg + 1, 1);
  if (!used) return -1;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = rowptr[v + 1] - rowptr[v];
    for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
      int64_t u = colidx[k];
      if (u < v && color[u] <= d) used[color[u]] = 1;
    }
    color[v] = least_absent(used, d + 1);
    for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
      int64_t u = colidx[k];
      if (u < v && color[u] <= d) used[color[u]] = 0;
    }
  }
  free(used);
  return 0;
}

/* Rounds of the id-priority schedule that reproduces oracle_seq in parallel
 * (a vertex takes its First-Fit colour in the first round in which all of its
 * lower-id neighbours are coloured; the sequential baseline of Section 5 run
 * as a dependency schedule).  By definition, the round of v is
 *     depth(v) = 1 + max{ depth(u) : u in N(v), u < v }   (1 when there is none),
 * the number of vertices on the longest id-increasing path ending at v; it is
 * computed in id order, where every depth(u) needed is already known.
 * round_out[n] receives depth(v); returns R = max depth (0 when n == 0), or
 * -1 on bad arguments. */
int64_t oracle_seq_rounds(int64_t n, const int64_t *rowptr, const int32_t *colidx,
                          int32_t *round_out) {
  if (n < 0 || (n > 0 && (!rowptr || !round_out))) return -1;
  int64_t R = 0;
  for (int64_t v = 0; v < n; ++v) {
    int32_t d = 0;
    for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
      int64_t u = colidx[k];
      if (u < v && round_out[u] > d) d = round_out[u];
    }
    round_out[v] = d + 1;
    if (d + 1 > R) R = d + 1;
  }
  return R;
}

/*
 * Algorithm 1 of Section 3.1 read literally, with p blocks (the p-block
 * variant).  Readings taken where the paper is loose:
 *   - block(v) = floor(v * p / n): p blocks of consecutive ids, sizes
 *     differing by at most one (the paper's uniform partition with ids from 0);
 *   - every vertex keeps one ForbiddenColors slot per CSR entry, initialised
 *     to -1;
 *   - phase 1: each block takes its vertices still to colour in increasing id
 *     order; v gets the least colour in 0..(max degree) absent from its slots,
 *     then writes that colour into the slot for v of each neighbour in the
 *     same block (so a block colours sequentially, seeing its own colours at
 *     once);
 *   - phase 2: each vertex v still to colour that has a neighbour in another
 *     block refreshes its slot for every such neighbour u with u's colour
 *     after this round's phase 1, and is recoloured (the set to recolour
 *     collects v itself) when some such u has v's colour and lies in a
 *     higher-numbered block (the paper's "vertex in the lower partition is
 *     recoloured"); a slot for a foreign neighbour is therefore only as fresh
 *     as v's last phase 2 (stale colours stay visible);
 *   - rounds continue until no block has a vertex to recolour; R counts the
 *     phase-1 passes.
 * color_out[n] receives the colours, recolours_out[n] (may be NULL) the
 * number of rounds after the first in which each vertex was coloured again.
 * Returns R (0 when n == 0), or -1 on bad arguments or allocation failure.
 */
int64_t oracle_blocks(int64_t n, const int64_t *rowptr, const int32_t *colidx, int64_t p,
                      int32_t *color_out, int32_t *recolours_out) {
  if (n < 0 || p < 1 || (n > 0 && (!rowptr || !color_out))) return -1;
  if (n == 0) return 0;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = rowptr[v + 1] - rowptr[v];
    if (d > maxdeg) maxdeg = d;
  }
  const int64_t nnz = rowptr[n];
  int32_t *slot = (int32_t *)malloc(((size_t)nnz + 1) * sizeof(int32_t));
  int64_t *blk = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  unsigned char *todo = (unsigned char *)malloc((size_t)n);
  unsigned char *lose = (unsigned char *)malloc((size_t)n);
  unsigned char *used = (unsigned char *)calloc((size_t)maxdeg + 2, 1);
  if (!slot || !blk || !todo || !lose || !used) {
    free(slot); free(blk); free(todo); free(lose); free(used);
    return -1;
  }
  for (int64_t k = 0; k < nnz; ++k) slot[k] = -1;
  for (int64_t v = 0; v < n; ++v) {
    blk[v] = (int64_t)(((__int128)v * p) / n);
    todo[v] = 1;
    color_out[v] = -1;
    if (recolours_out) recolours_out[v] = 0;
  }
  int64_t rounds = 0, left = n;
  while (left > 0) {
    ++rounds;
    /* phase 1: blocks are independent (only same-block slots are written);
     * within a block, increasing id order */
    for (int64_t v = 0; v < n; ++v) {
      if (!todo[v]) continue;
      for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k)
        if (slot[k] >= 0 && slot[k] <= maxdeg) used[slot[k]] = 1;
      int32_t c = 0;
      while (used[c]) ++c;
      for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k)
        if (slot[k] >= 0 && slot[k] <= maxdeg) used[slot[k]] = 0;
      if (color_out[v] >= 0 && recolours_out) ++recolours_out[v];
      color_out[v] = c;
      /* the slot for v in each same-block neighbour's list */
      for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
        int64_t u = colidx[k];
        if (blk[u] != blk[v]) continue;
        for (int64_t q = rowptr[u]; q < rowptr[u + 1]; ++q)
          if (colidx[q] == v) slot[q] = c;
      }
    }
    /* (barrier) phase 2 */
    for (int64_t v = 0; v < n; ++v) {
      lose[v] = 0;
      if (!todo[v]) continue;
      for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
        int64_t u = colidx[k];
        if (blk[u] == blk[v]) continue;
        slot[k] = color_out[u];
        if (color_out[u] == color_out[v] && blk[v] < blk[u]) lose[v] = 1;
      }
    }
    left = 0;
    for (int64_t v = 0; v < n; ++v) {
      todo[v] = lose[v];
      left += lose[v];
    }
    /* (barrier) */
  }
  free(slot); free(blk); free(todo); free(lose); free(used);
  return rounds;
}

/* Number of CSR entries (v, u) with color[v] == color[u], plus the number of
 * vertices with a negative colour.  0 means a proper colouring
 * (Section 2.1; Lemma 1 of Section 4). */
int64_t oracle_check_proper(int64_t n, const int64_t *rowptr,
                            const int32_t *colidx, const int32_t *color) {
  int64_t bad = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (color[v] < 0) ++bad;
    for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k)
      if (color[colidx[k]] == color[v]) ++bad;
  }
  return bad;
}

/* Number of vertices whose colour is not the least colour absent from its
 * neighbourhood (First Fit, Section 3).  0 for every First-Fit colouring
 * whose vertices all see their final neighbourhood. */
int64_t oracle_check_grundy(int64_t n, const int64_t *rowptr,
                            const int32_t *colidx, const int32_t *color) {
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = rowptr[v + 1] - rowptr[v];
    if (d > maxdeg) maxdeg = d;
  }
  unsigned char *used = (unsigned char *)calloc((size_t)maxdeg + 1, 1);
  if (!used) return -1;
  int64_t bad = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = rowptr[v + 1] - rowptr[v];
    for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
      int32_t c = color[colidx[k]];
      if (c >= 0 && c <= d) used[c] = 1;
    }
    if (color[v] != least_absent(used, d + 1)) ++bad;
    for (int64_t k = rowptr[v]; k < rowptr[v + 1]; ++k) {
      int32_t c = color[colidx[k]];
      if (c >= 0 && c <= d) used[c] = 0;
    }
  }
  free(used);
  return bad;
}

/* Colour every graph of a packed batch independently with oracle_rsc.
 * voff/eoff are the per-graph vertex and CSR-entry offsets; graph g's local
 * rowptr (n_g + 1 int32 entries) starts at rowptr_local[voff[g] + g], its
 * local colidx at colidx_local[eoff[g]].  colors_out[voff[g] + v] receives
 * the colour of local vertex v; rounds_out[g] the round count.  Returns 0,
 * or -1 on failure. */
int oracle_rsc_batch(int64_t G, const int64_t *voff, const int64_t *eoff,
                     const int32_t *rowptr_local, const int32_t *colidx_local,
                     int32_t *colors_out, int64_t *rounds_out) {
  for (int64_t g = 0; g < G; ++g) {
    int64_t n = voff[g + 1] - voff[g];
    const int32_t *rp32 = rowptr_local + voff[g] + g;
    int64_t *rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!rp) return -1;
    for (int64_t v = 0; v <= n; ++v) rp[v] = rp32[v];
    int64_t R = oracle_rsc(n, rp, colidx_local + eoff[g], colors_out + voff[g],
                           NULL, NULL, 0);
    free(rp);
    if (R < 0) return -1;
    if (rounds_out) rounds_out[g] = R;
  }
  return 0;
}
