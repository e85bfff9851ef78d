// gc_internal.h -- shared between the C-ABI engine and the gfx950 kernels.
//
// State encoding (one signed integer per vertex, of width S = int8, int16 or
// int32 chosen from the maximum degree):
//   s >= 0   the vertex's colour is final (= s)
//   s <  0   the vertex is still being coloured; its tentative colour of the
//            current round is ~s (so the initial -1 means "tentative 0")
// Every colour and tentative colour is at most deg(v) (First Fit picks the
// least of deg(v) + 1 candidates), so S = int8 holds any graph with maximum
// degree <= 126 and int16 any with maximum degree <= 32766 (the type's least
// value stays spare: it marks a vertex that waits under the id-priority
// schedule).
// A round's speculate phase rewrites only negative entries (negative stays
// negative), and its detect phase turns a winner's ~t into t.  A reader that
// decodes (s < 0 ? ~s : s) therefore sees the same tentative colour before and
// after a concurrent commit, which is what lets detect and commit share one
// pass.
#pragma once
#include <cstdint>

namespace gc {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kBlock = 256;         // threads per workgroup of the round kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kTraceRounds = 65536; // rounds whose |U_r| is recorded
constexpr int kHeavyWindow = 4096;  // LDS colour window of the block-per-vertex path (bits)
constexpr int kPushColors = 32;     // colours tracked per vertex by pushed flags
constexpr int kWideColors = 480;    // further colours (32..511) tracked for medium/heavy vertices
constexpr int kSparseChunk = 32;    // detect: at most this many uncoloured vertices in a chunk
                                    // -> a group of lanes each (at least 2)
constexpr int kMaxBlocksPerCu = 64; // workgroups per CU of any round kernel (option limit)
constexpr int kFinishBlocks = 512;  // most workgroups of the finishing pass (one stats pair each)
constexpr int kDeferRow = 512;      // a wavefront- or workgroup-class winner with more row entries
                                    // than this left to push queues them for the grid-wide push pass
constexpr int kPieceEntries = 1024; // row entries of one piece of that pass: one workgroup,
                                    // four entries per thread in flight, one step
constexpr int kFinishHeader = 4;   // its leading output words (see launch_finish)
constexpr int kFinishWords = kFinishHeader + 2 * kFinishBlocks;

// One 128-byte line per field that different blocks write, so that flags and
// counters never share a line.
struct alignas(128) Line {
  int32_t v;
  int32_t pad[31];
};

// Which degree classes still have uncoloured vertices in a round (1 = yes or
// not known to be none): a pass skips a class with none.
struct alignas(128) ClassLine {
  int32_t light, medium, heavy;
  int32_t pad[29];
};

struct Ctrl {
  Line more[3];          // slot r % 3 == 1 when round r has uncoloured vertices
  ClassLine cls[3];      // slot r % 3: the classes with uncoloured vertices in round r
  Line last_round;       // last round that had uncoloured vertices
  Line round_base;       // first round of the next captured chunk
  Line bar;              // grid barrier arrivals (monotonic within a launch)
  Line abort;            // set when a barrier wait exceeded its spin limit
  Line left;             // vertices still uncoloured after the last round
  Line epoch;            // value marking this call's pushed colour flags (1..255)
  Line pend;             // round whose per-workgroup counts in KArgs::part are not yet in
                         // trace (0: none)
  Line pend_grid;        // workgroups of that round's detect pass
  Line tasks;            // 64-bit: push tasks (high half) and their pieces (low half)
                         // queued by this round's detect pass (KArgs::tasks)
  int32_t trace[kTraceRounds];  // |U_r| at slot r - 1
};

// A winner's pushes handed to the grid-wide push pass: colour t to the row
// entries [b, e) (to the list entries lst[b, e) when t carries kFromList),
// cut into pieces first .. first + ceil((e - b) / kPieceEntries) - 1 of the
// pass's piece numbering.
constexpr int32_t kFromList = 1 << 30;

struct PushTask {
  int64_t b;
  int64_t e;
  int32_t t;
  int32_t first;
};

// Arguments of every round kernel.
struct KArgs {
  const void* rowptr;     // int32 or int64, n + 1
  const int32_t* colidx;  // nnz
  void* st;               // n entries of the state type
  int32_t* colors;        // n, the caller's output (the widened state)
  int32_t n;
  int32_t light_max;      // deg <= light_max: a group of L lanes per vertex
  const int32_t* mlist;   // medium vertices (light_max < deg < heavy): a wavefront each
  int32_t mcount;
  const int32_t* hlist;   // heavy vertices: a whole workgroup each
  int32_t hcount;
  int32_t sorted;         // rows ascending: the conflict scan may stop early
  int32_t push;           // forbidden colours pushed by committing neighbours
  int32_t seq;            // id-priority First Fit: speculate picks the vertices whose lower
                          // neighbours are all final, detect commits them (no conflicts)
  uint8_t* seen;          // ceil(n / 64) * 64 * kPushColors: byte c of v == epoch when a
                          // neighbour of v has final colour c (plain byte stores, no atomics);
                          // at flag_index(v, c) (gc_device.h)
  int32_t flags_by_chunk; // flag layout: 1 = colour-major within each 64-vertex chunk (only
                          // when there are no medium or heavy vertices), 0 = 32 bytes per vertex
  int32_t epoch;          // epoch of this call (written to ctrl by the init kernel)
  int32_t clear_seen;     // the init kernel zeroes `seen` and `wide` (first call, epoch wrap)
  int32_t clear_trace;    // the init kernel zeroes ctrl->trace (p-block passes add into it)
  uint8_t* wide;          // (mcount + hcount) * kWideColors flags for colours 32..511
  int32_t wide_clear;     // wide blocks allocated: the init kernel's clear covers all of them,
                          // so a block left over from a larger degree-class split of an
                          // earlier call cannot keep a byte equal to a later epoch
  const int32_t* widx;    // n: index of v's wide flag block, -1 for light vertices
  int32_t* skip;          // n: lower neighbours before this offset of v's row are final
                          // (sorted rows); zeroed by round 1
  int32_t* lst;           // nnz, parallel to colidx: each medium or heavy vertex's list of lower
                          // neighbours not yet seen final (detect_wave_list, detect_block_list),
                          // at its row's offset; null unless the push algorithm runs on sorted
                          // rows with such vertices
  int32_t* llen;          // n: length of that list; zeroed by round 1 with skip
  int32_t* part;          // cus * kMaxBlocksPerCu: active vertices of each workgroup of the
                          // last detect pass; the next pass folds them into ctrl->trace
  PushTask* tasks;        // 2 * (mcount + hcount): pushes of long rows or lists queued by a
                          // detect pass for the grid-wide push pass that follows it (push
                          // algorithm with medium or heavy vertices, not in the persistent
                          // kernel; null otherwise)
  Ctrl* ctrl;
};

// Arguments of the p-block kernels (GC_ALGO_BLOCKS, gc_blocks.hip).
struct BArgs {
  const void* rowptr;     // int32 or int64, n + 1
  const int32_t* colidx;  // nnz
  int32_t* color;         // n: current colours (-1 before a vertex's first), the caller's output
  int32_t* slot;          // nnz: ForbiddenColors slot of each entry whose neighbour is in
                          // another block (entries within a block are not used)
  uint8_t* todo;          // n: 1 while the vertex is to be (re)coloured
  int32_t n;
  int64_t p;              // blocks
  int32_t round;          // round being run (1-based), for the trace
  Ctrl* ctrl;
};

int launch_blocks_init(const BArgs& a, bool rp64, int grid, void* stream);
// Phase 1 (phase = 1) or phase 2 (phase = 2) of one round; after phase 2,
// ctrl->left holds the vertices to recolour and ctrl->trace / last_round the
// round's size.
int launch_blocks_phase(const BArgs& a, bool rp64, int phase, int grid, void* stream);
// ctrl->left = value (vertices still to recolour when a round cap stops the loop)
int launch_blocks_set_left(Ctrl* c, int value, void* stream);

// Relabelling by a vertex order (gc_order.hip).  Writes the relabelled CSR
// (rows ascending) into rowptr2 (n + 1 entries of the input's width) and
// colidx2 (nnz), and newid[v] = the new id of v.  Synchronises `stream`.
int build_order(const void* rowptr, bool rp64, const int32_t* colidx, int32_t n, int64_t nnz,
                int kind, uint64_t seed, void* rowptr2, int32_t* colidx2, int32_t* newid, int grid,
                void* stream);
// out[v] = coloured[newid[v]]
int launch_permute_back(const int32_t* newid, const int32_t* coloured, int32_t n, int32_t* out,
                        int grid, void* stream);

// Records `msg` as the calling thread's last error (gc_last_error(NULL)).
void set_thread_error(const char* msg);

// Launch helpers implemented in gc_kernels.hip.  All return a hipError_t
// cast to int.  `sbytes` is the state width in bytes (1, 2 or 4).
int launch_init(const KArgs& a, void* stream);
int launch_round1(const KArgs& a, bool rp64, int sbytes, int lanes, int grid, void* stream);
int launch_round(const KArgs& a, bool rp64, int sbytes, int lanes, int phase /*0 spec, 1 detect*/,
                 int round, bool round_from_base, int grid, void* stream);
int launch_advance_base(const KArgs& a, int by, void* stream);
// The state becomes the caller's int32 colours.  `out` (kFinishWords words of
// device-visible pinned host memory) receives, by system-scope stores:
//   out[0] last round, out[1] abort flag, out[2] uncoloured count recorded by
//   earlier passes (ctrl->left), out[3] workgroups G of this pass, and for
//   each workgroup b < G: out[4 + 2b] = its largest colour + 1 (0 if none),
//   out[5 + 2b] = its uncoloured vertices.
// The host folds them once the stream has passed this kernel.
int launch_finish(const KArgs& a, int sbytes, int32_t* out, void* stream);
int launch_persistent(const KArgs& a, bool rp64, int sbytes, int lanes, int max_rounds, int grid,
                      void* stream);
int persistent_max_grid(bool rp64, int sbytes, int lanes, int* grid_out);
int launch_classify(const void* rowptr, bool rp64, int32_t n, int32_t light_max, int32_t heavy_min,
                    int32_t* mlist, int32_t* hlist, int32_t* counts /*[3]: medium, heavy, maxdeg*/,
                    int32_t* widx, int grid, void* stream);
int launch_wide_index(const int32_t* hlist, int32_t hcount, int32_t mcount, int32_t* widx,
                      void* stream);
int launch_validate(const void* rowptr, bool rp64, const int32_t* colidx, int32_t n, int64_t m,
                    bool sorted, int32_t* err /*[2]: code, where*/, int grid, void* stream);

}  // namespace gc
