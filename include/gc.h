/*
 * gc.h -- C ABI of libgc: round-synchronous speculative graph colouring on
 * AMD Instinct MI355X (gfx950).
 *
 * The method is the barrier-synchronised parallel colouring of Singhal, Peri
 * and Kalyanasundaram, "Multi-threaded Graph Coloring Algorithm for Shared
 * Memory Architecture" (arXiv:1509.08267), Algorithm 1 (Section 3.1), run
 * with every vertex its own block:
 *
 *   round r = 1, 2, ...:
 *     speculate  every uncoloured vertex takes the least colour not yet final
 *                on any neighbour (First Fit, Section 3; colours 0-based as
 *                in Algorithm 1's TotalColors = {0, ..., max degree});
 *     barrier;
 *     detect     a vertex loses if a lower-id neighbour, also coloured this
 *                round, took the same colour (the paper recolours the lower
 *                partition; numbering partitions by decreasing id gives this
 *                rule); winners' colours become final;
 *     barrier;   losers form the next round's set; stop when it is empty.
 *
 * The result is a deterministic function of the graph (independent of launch
 * shape, row order, stream and batching): bit-identical to a plain
 * single-threaded simulation of the same rounds.  It is a proper colouring
 * (Lemma 1, Section 4) in which every colour is the least one absent from the
 * vertex's neighbourhood, so colour(v) <= deg(v) and at most Delta + 1
 * colours are used (Section 2.1).  Rounds never exceed n (Lemma 2 with
 * p = n blocks).
 *
 * Conventions for every entry point:
 *   - Graphs are simple and undirected (Section 2.1): CSR with each edge
 *     stored in both rows, no self-loops, no duplicate entries.  Vertex ids
 *     are 0-based int32.
 *   - Array arguments are DEVICE pointers unless stated otherwise, owned by
 *     the caller.  Calls are asynchronous on `stream` (a hipStream_t; NULL is
 *     the null stream); results are valid once that stream has synchronised.
 *   - A negative return value is an error (enum gc_status);
 *     gc_last_error() describes it.  Nothing throws across this boundary.
 *   - A GPU fault inside a call is reported as GC_EDEVICE by that call or by
 *     the next call that synchronises.
 */
#ifndef GC_H
#define GC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gc_ctx *gc_handle; /* opaque, library-owned */

enum gc_status {
  GC_OK = 0,
  GC_EINVAL = -1,  /* bad argument or (with GC_VALIDATE) malformed graph   */
  GC_ENOMEM = -2,  /* device or pinned-host allocation failed              */
  GC_EDEVICE = -3, /* HIP runtime error or GPU fault                       */
  GC_EROUNDS = -4, /* round cap (GC_OPT_MAX_ROUNDS) reached before the end */
  GC_EBUSY = -5,   /* reserved (calls on a handle are ordered instead)     */
  GC_ETOOBIG = -6  /* sizes exceed what the library supports               */
};

enum gc_flags {
  GC_ROWPTR_I64 = 1u << 0,  /* rowptr is int64 (default int32)              */
  GC_VALIDATE = 1u << 1,    /* check the CSR on the device in gc_create:
                               monotone rowptr, rowptr[0] = 0, rowptr[n] = m,
                               ids in range, no self-loops, no duplicates,
                               symmetric; rejects with GC_EINVAL           */
  GC_ROWS_SORTED = 1u << 2  /* caller promises strictly ascending rows;
                               enables the round-1 closed form, the early
                               stop of the conflict scan at the first higher
                               neighbour, a per-vertex resume point that
                               skips lower neighbours already final (also
                               where a winner's pushes start), and the
                               O(log deg) symmetry check of GC_VALIDATE,
                               which then rejects unsorted rows; without
                               GC_VALIDATE a broken promise gives an
                               unspecified (possibly improper) colouring    */
};

/*
 * gc_create -- bind a graph and allocate the colouring state.
 *
 *   out      receives the handle (set to NULL on failure)
 *   rowptr   device, n + 1 entries, int32 (or int64 with GC_ROWPTR_I64)
 *   colidx   device, m entries, int32 neighbour ids
 *   n        vertices, 0 <= n < 2^31
 *   m        CSR entries = rowptr[n] = 2 |E|
 *   flags    OR of enum gc_flags
 *   stream   stream for the set-up work (degree scan, validation)
 *
 * The graph arrays are BORROWED: they must stay allocated and unchanged
 * until gc_destroy.  The library allocates O(n) device scratch (the state
 * array of 1/2/4 bytes per vertex, a 4-byte resume offset per vertex,
 * worklists and counters; on the first push-algorithm call 32 flag bytes per
 * vertex plus 480 per vertex handled by a whole wave or workgroup, see
 * GC_OPT_MEDIUM_DEGREE, and, on sorted rows with such vertices, 4 bytes per
 * CSR entry and per vertex for their lower-neighbour lists) and a small
 * pinned host block; it synchronises
 * `stream` before returning.  The handle belongs to the device current at
 * this call.
 * Returns GC_OK, GC_EINVAL, GC_ENOMEM, GC_ETOOBIG or GC_EDEVICE.
 */
int gc_create(gc_handle *out, const void *rowptr, const int32_t *colidx,
              int64_t n, int64_t m, uint32_t flags, void *stream);

/*
 * gc_color -- colour the bound graph.
 *
 *   colors_out  device, n int32 entries; receives colour(v) in 0..deg(v)
 *               (its prior contents are ignored).  The working state is a
 *               library-owned array of 1, 2 or 4 bytes per vertex (by maximum
 *               degree), widened into colors_out at the end.
 *   stream      all work is queued here.  The first call on a handle reads a
 *               4-byte flag back every few rounds to find the round count R;
 *               later calls queue all R rounds and return at once (R depends
 *               on the graph only).  GC_MODE_HOST reads back every round.
 *
 * Calls on one handle are ordered: a call queued while the previous one is
 * still running (on any stream) first waits for it on the device, since both
 * use the handle's scratch; gc_get_stats then reports the later call.
 * Returns GC_OK, GC_EINVAL, GC_EROUNDS (GC_MODE_HOST only, when
 * GC_OPT_MAX_ROUNDS is reached) or GC_EDEVICE.
 */
int gc_color(gc_handle h, int32_t *colors_out, void *stream);

/*
 * gc_get_stats -- results of the last gc_color on this handle.
 * Waits for that call's stream.  `rounds` receives the number of rounds R
 * (0 when n = 0), `num_colors` max colour + 1 (0 when n = 0).  Either
 * pointer may be NULL.  Returns GC_EROUNDS if the call stopped at the round
 * cap (GC_OPT_MAX_ROUNDS) with vertices still uncoloured, GC_EINVAL if
 * vertices were left uncoloured otherwise (the graph arrays were changed
 * after gc_create, against the contract), GC_EDEVICE on a device error.
 */
int gc_get_stats(gc_handle h, int64_t *rounds, int32_t *num_colors);

/*
 * gc_get_round_sizes -- |U_r|, the number of vertices (re)coloured in round
 * r, for r = 1..min(R, cap) of the last gc_color (host array `sizes`).
 * `rounds` (may be NULL) receives R.  At most GC_TRACE_ROUNDS rounds are
 * recorded.  Waits for the last call's stream.
 */
#define GC_TRACE_ROUNDS 65536
int gc_get_round_sizes(gc_handle h, int64_t *sizes, int64_t cap, int64_t *rounds);

/* Tunables.  None changes the result (it is a function of the graph only).
 * Read-only values are marked (get only). */
enum gc_option {
  GC_OPT_MODE = 1,           /* enum gc_mode, default GC_MODE_AUTO                  */
  GC_OPT_LANES = 2,          /* lanes per light vertex, 1,2,4,..,64; 0 = auto (from
                                the average degree)                                */
  GC_OPT_HEAVY_DEGREE = 3,   /* deg >= this: a whole workgroup per vertex (4096)     */
  GC_OPT_BLOCKS_PER_CU = 4,  /* workgroups per compute unit of the round kernels (8) */
  GC_OPT_MAX_ROUNDS = 5,     /* stop after this many rounds (0 = no cap); leftover
                                vertices make gc_get_stats return GC_EROUNDS       */
  GC_OPT_CHUNK_ROUNDS = 6,   /* rounds queued per read-back in CHUNKED/GRAPH (8)     */
  GC_OPT_MEDIUM_DEGREE = 7,  /* deg > this: a wavefront per vertex; 0 = auto         */
  GC_OPT_MAX_DEGREE = 8,     /* (get only) maximum degree of the graph              */
  GC_OPT_MEDIUM_COUNT = 9,   /* (get only) vertices on the wavefront path           */
  GC_OPT_HEAVY_COUNT = 10,   /* (get only) vertices on the workgroup path           */
  GC_OPT_PERSISTENT_BLOCKS_PER_CU = 11, /* workgroups per CU of the persistent kernel,
                                1..4 (4); the library lowers it further to what
                                the kernel's register use lets a CU hold at once
                                (every workgroup of a grid barrier must be
                                resident): 3 with int64 row pointers          */
  GC_OPT_STATE_BYTES = 12,   /* (get only) bytes per vertex of the working state:
                                1 if max degree <= 126, 2 if <= 32766, else 4 */
  GC_OPT_PROFILE = 13,       /* 1: time the kernels of each call with HIP events
                                recorded on the call's stream; once R is known
                                the rounds are launched directly (not as a
                                captured graph) with an event around every
                                kernel; read with gc_get_profile           */
  GC_OPT_ALGORITHM = 14,     /* enum gc_algorithm (default GC_ALGO_AUTO)           */
  GC_OPT_PARTITIONS = 15,    /* p for GC_ALGO_BLOCKS; 0 = auto (64 per compute unit) */
  GC_OPT_ORDER = 16,         /* enum gc_order (default GC_ORDER_NATURAL)            */
  GC_OPT_ORDER_SEED = 17     /* seed of GC_ORDER_RANDOM (default 0)                 */
};
/* The vertex order the colouring follows (the paper's future work names
 * ordering schemes; its related work, Jones and Plassmann's random order).
 * Vertex sigma[i] of the order is renamed i, the relabelled graph is
 * coloured by the selected algorithm, and each vertex receives the colour of
 * its new name.  Any order but NATURAL builds a relabelled copy of the CSR on
 * the device at the next gc_color after the option changes (about 3x the
 * CSR's size while it is built, then one copy; GC_ETOOBIG when nnz exceeds
 * 2^31 - 1). */
enum gc_order {
  GC_ORDER_NATURAL = 0,        /* ids as given                                       */
  GC_ORDER_LARGEST_FIRST = 1,  /* degree descending, ties by id                     */
  GC_ORDER_RANDOM = 2          /* ascending by the splitmix64 generator's output at
                                  step v + 1 from state GC_OPT_ORDER_SEED          */
};
/* The colouring to compute.  AUTO, PULL and PUSH compute the same colouring
 * (round-synchronous speculation, Algorithm 1 of Section 3.1 with every vertex
 * its own block) and differ in how speculation learns the final colours of a
 * vertex's neighbours.  SEQ computes another one: the sequential First-Fit
 * colouring in id order (the baseline of Section 5). */
enum gc_algorithm {
  GC_ALGO_AUTO = 0,  /* currently PUSH                                             */
  GC_ALGO_PULL = 1,  /* each round, each uncoloured vertex gathers the state of all
                        its neighbours and builds its forbidden-colour mask        */
  GC_ALGO_PUSH = 2,  /* a vertex whose colour c < 32 becomes final marks colour c
                        as taken in a 32-byte flag block of each neighbour (one
                        plain byte store per CSR entry over the whole colouring,
                        no atomics); speculation reads its 32 flags and scans its
                        row only when colours 0..31 are all taken.  32 bytes per
                        vertex of device memory                                 */
  GC_ALGO_SEQ = 3,   /* sequential First Fit in id order, computed in rounds: a
                        vertex takes the least colour absent from its lower-id
                        neighbours in the first round in which all of them are
                        coloured.  The colours equal the sequential ones bit for
                        bit; R is the number of vertices on the longest path
                        whose ids increase                                      */
  GC_ALGO_BLOCKS = 4 /* Algorithm 1 of Section 3.1 read literally with p =
                        GC_OPT_PARTITIONS blocks of consecutive ids: every
                        vertex keeps a ForbiddenColors slot per neighbour; in
                        each round a block colours its pending vertices
                        sequentially (First Fit, increasing id), then each such
                        vertex refreshes its slots for neighbours in other
                        blocks and is recoloured if one in a higher block has
                        its colour.  The colouring depends on p by design;
                        R <= p.  4 bytes per CSR entry of device memory; the
                        rounds are driven from the host                       */
};
enum gc_mode {
  GC_MODE_AUTO = 0,       /* currently GRAPH                                      */
  GC_MODE_HOST = 1,       /* one round per host iteration, a flag read back       */
  GC_MODE_CHUNKED = 2,    /* rounds queued in chunks; empty rounds exit at once   */
  GC_MODE_PERSISTENT = 3, /* one cooperative kernel, device-side round loop      */
  GC_MODE_GRAPH = 4       /* a captured hipGraph of a chunk of rounds            */
};
int gc_set_option(gc_handle h, int option, int64_t value);
int gc_get_option(gc_handle h, int option, int64_t *value);

/*
 * gc_get_profile -- kernel times accumulated over profiled calls
 * (GC_OPT_PROFILE = 1), per kernel kind: [0] round 1, [1] speculate,
 * [2] detect/commit, [3] finish (colour count and widening).  `ms` (4
 * doubles) receives total milliseconds, `launches` (4 int64) the launch
 * counts; either may be NULL.  Speculate and detect are timed once the round
 * count is known (calls still discovering R, and persistent calls, add only
 * round 1 and finish).  Waits for the handle's last call.  reset != 0 zeroes
 * the totals after reading.
 */
int gc_get_profile(gc_handle h, double *ms, int64_t *launches, int reset);

/* gc_destroy -- wait for outstanding work, free the handle's scratch.
 * The borrowed graph arrays are not touched.  NULL is accepted. */
int gc_destroy(gc_handle h);

/* gc_last_error -- message of the last failure on `h`, or of the calling
 * thread's last failure when h is NULL (e.g. a failed gc_create).  The
 * string is owned by the library and valid until the next call. */
const char *gc_last_error(gc_handle h);

/* ------------------------------------------------------------------ batch --
 * Many independent graphs coloured in one persistent launch.  Graph g has
 * n_g = voff[g+1] - voff[g] vertices and nnz_g = eoff[g+1] - eoff[g] CSR
 * entries; its local rowptr (n_g + 1 int32 entries, starting at 0) begins at
 * rowptr_local[voff[g] + g] and its local colidx (ids 0..n_g-1) at
 * colidx_local[eoff[g]].  Each graph is coloured exactly as gc_color would
 * colour it alone (same bits; the batching never changes a result).
 */

/*
 * gc_batch_workspace_bytes -- device workspace needed by gc_color_batch.
 * voff and eoff are HOST arrays of num_graphs + 1 entries (only sizes are
 * read).  Returns 0 on bad arguments.
 */
size_t gc_batch_workspace_bytes(int64_t num_graphs, const int64_t *voff,
                                const int64_t *eoff);

/*
 * gc_color_batch -- colour every graph of a packed batch.  A graph whose work
 * (entries + vertices) is at least 1/(2 x CUs) of the batch's is coloured by
 * a team of workgroups (up to one per 65,536 units of its work), the others
 * by one workgroup each; the colours are the same either way.
 *
 *   voff, eoff      device, int64[num_graphs + 1], non-decreasing, from 0
 *   rowptr_local    device, int32, sum(n_g + 1) entries (layout above)
 *   colidx_local    device, int32, sum(nnz_g) entries
 *   colors_out      device, int32, sum(n_g): colour of local vertex v of
 *                   graph g at colors_out[voff[g] + v]; also working state
 *   rounds_out      device, int32[num_graphs] rounds per graph, or NULL
 *   workspace       device scratch of at least gc_batch_workspace_bytes
 *                   (caller-owned; contents on entry are ignored)
 *
 * Each graph must satisfy the gc_create preconditions with sorted rows.
 * Returns GC_OK, GC_EINVAL (bad sizes or too small a workspace) or
 * GC_EDEVICE.  Asynchronous on `stream`.
 */
int gc_color_batch(int64_t num_graphs, const int64_t *voff, const int64_t *eoff,
                   const int32_t *rowptr_local, const int32_t *colidx_local,
                   int32_t *colors_out, int32_t *rounds_out, void *workspace,
                   size_t workspace_bytes, void *stream);

/*
 * gc_color_batch_noalloc -- gc_color_batch without a workspace argument and
 * without any allocation, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).
 *
 * The arguments and the result are those of gc_color_batch.  The workspace
 * is a fixed device array inside the library (about 3.5 MB, one per GPU the
 * library runs on, held until the process ends), so:
 *   - num_graphs may not exceed GC_STATIC_BATCH_MAX_GRAPHS (GC_ETOOBIG);
 *   - calls that overlap in time on one GPU (on different streams, or from
 *     different threads) share that array and race: order them on one
 *     stream.  Nothing in it needs to survive between calls; each call
 *     rewrites what it reads.
 * No hipMalloc, hipFree or allocating library routine is called.  Returns
 * GC_OK, GC_EINVAL, GC_ETOOBIG or GC_EDEVICE.  Asynchronous on `stream`.
 */
#define GC_STATIC_BATCH_MAX_GRAPHS 65536
int gc_color_batch_noalloc(int64_t num_graphs, const int64_t *voff, const int64_t *eoff,
                           const int32_t *rowptr_local, const int32_t *colidx_local,
                           int32_t *colors_out, int32_t *rounds_out, void *stream);

/*
 * Resumable batch steps for continuous batching.  A graph's whole state
 * between rounds is its colour array (final colours >= 0; a negative entry
 * marks a vertex still to be coloured) plus the count of rounds done, so a
 * colouring can be advanced a few rounds at a time, with graphs joining and
 * leaving between steps, and still give the same bits as one gc_color call.
 *
 * gc_graph_desc (device array, one per graph in the step):
 *   rowptr_off   index into rowptr_base of the graph's local rowptr
 *   colidx_off   index into colidx_base of its local colidx
 *   color_off    index into colors_base of its colour/state array
 *   n            vertices of the graph
 *   rounds       in: rounds already done (0 = fresh: the state is
 *                initialised); out: rounds done after the step
 *   active       out: vertices still uncoloured after the step (0 = done);
 *                in (rounds > 0): the value the previous step left, used
 *                only to order the step's graphs and size their teams of
 *                workgroups by the work left (any value gives the same
 *                colours)
 */
typedef struct gc_graph_desc {
  int64_t rowptr_off;
  int64_t colidx_off;
  int64_t color_off;
  int32_t n;
  int32_t rounds;
  int32_t active;
  int32_t max_degree; /* in: max degree of the graph (sizes state encodings) */
} gc_graph_desc;

/*
 * gc_batch_step -- advance each listed graph by at most `max_rounds` rounds
 * (0 = until done).  `descs` is a device array of num_graphs entries;
 * `workspace` at least gc_batch_step_workspace_bytes(num_graphs,
 * max_vertices) bytes, where max_vertices bounds every n.  Asynchronous on
 * `stream`.
 */
size_t gc_batch_step_workspace_bytes(int64_t num_graphs, int64_t total_vertices);
int gc_batch_step(int64_t num_graphs, gc_graph_desc *descs,
                  const int32_t *rowptr_base, const int32_t *colidx_base,
                  int32_t *colors_base, int32_t max_rounds, void *workspace,
                  size_t workspace_bytes, void *stream);

/*
 * gc_copy_segments -- copy many int32 arrays in one launch (staging of many
 * small requests, e.g. a server admitting graphs whose CSR is already on the
 * device; not part of the colouring itself).
 *
 *   segs     device array of `count` descriptors:
 *              src          device address of the source words
 *              dst          device address of the destination words
 *              words        int32 words to copy (>= 0)
 *              first_piece  exclusive prefix sum over the descriptors of
 *                           ceil(words / GC_COPY_PIECE_WORDS)
 *   pieces   total pieces (the sum of all ceil(words / GC_COPY_PIECE_WORDS))
 *
 * Sources and destinations must not overlap.  A workgroup copies one piece
 * at a time; a piece that lies past its segment's length copies nothing,
 * so inconsistent prefix sums never write outside [dst, dst + words).
 * Asynchronous on `stream`; the descriptors must stay valid until it has
 * run.  Returns GC_OK or GC_EINVAL.
 */
#define GC_COPY_PIECE_WORDS 4096
typedef struct gc_segment {
  int64_t src;
  int64_t dst;
  int64_t words;
  int64_t first_piece;
} gc_segment;
int gc_copy_segments(int64_t count, const gc_segment *segs, int64_t pieces, void *stream);

/* Library version, "major.minor.patch". */
const char *gc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GC_H */
