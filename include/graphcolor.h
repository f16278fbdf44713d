/*
 * graphcolor.h — C-ABI of the MI355X (gfx950) speculative graph-coloring
 * library (libgraphcolor.so).
 *
 * The library computes the on-node step of the distributed speculative
 * coloring of Bogle et al., "Parallel Graph Coloring Algorithms for
 * Distributed GPU Environments": distance-1 (D1), distance-2 (D2) and partial
 * distance-2 (PD2) colorings (Section 2.1), by speculate-and-iterate rounds
 * (Section 2.3; Section 3, Algorithm 2): every uncolored vertex takes the
 * smallest color its neighbourhood does not use (first-fit, Section 2.2,
 * Algorithm 1), conflicts are detected (Section 3.2, Algorithms 3 and 4;
 * Section 3.5, Algorithm 5) and one endpoint of each conflict is uncolored and
 * recolored in the next round.
 *
 * Result contract.  Rounds are synchronous: in each round every worklist
 * vertex reads only the colors committed before the round, and all conflicts
 * are judged at once on the round's tentative colors.  In a conflict the
 * vertex with the LOWER key loses, key(v) = (p(v), gid(v)) compared
 * lexicographically, p(v) = fmix32(gid(v) ^ fmix32(seed ^ 0x9E3779B9)) with
 * fmix32 the MurmurHash3 32-bit finalizer (a bijection, so keys never tie);
 * with COLOR_FLAG_RECOLOR_DEGREES the key is (deg(v), p(v), gid(v)).
 * The coloring is therefore a deterministic function of (graph, keys) and is
 * identical for every launch geometry, degree-bin setting, stream and
 * batching mode.  Colors are 1-based; 0 means "uncolored" (Section 3.2) and
 * never appears in a successful result.
 *
 * Memory.  Unless stated otherwise every array argument is a DEVICE pointer
 * (memory from hipMalloc / a torch CUDA tensor) owned by the caller; the
 * library never frees or retains it.  `stream` is a hipStream_t (NULL = the
 * default stream).  Calls are blocking: they return after all work they
 * enqueued on `stream` has finished.  Each call runs on a workspace that no
 * other call holds at the same time, taken from a per-device pool (up to 8
 * workspaces per device, each growing to the largest call it served, kept
 * until color_release_workspace; a 9th concurrent call waits for one), so
 * calls made at the same time from different host threads on different
 * streams are independent: they neither wait for nor share memory with each
 * other.  Only color_d1_noalloc (one static array per device) serializes
 * its calls.
 *
 * Graph layout.  A graph with n vertices is CSR: row_ptr int32[n+1]
 * (row_ptr[0] = 0, non-decreasing), col_idx int32[row_ptr[n]] with
 * 0 <= col_idx < n.  D1/D2 need a symmetric adjacency without self-loops
 * (the paper removes self-loops and multi-edges before coloring, Section 4).
 * With COLOR_FLAG_VALIDATE the library checks the contract on the device
 * (rows must then be strictly increasing) and returns COLOR_EGRAPH on a
 * violation; without it the input is trusted.
 *
 * Errors.  Every entry point returns COLOR_OK (0) or a negative code; no
 * entry point aborts the process.  On an error the output arrays are
 * unspecified except for COLOR_ENOCONVERGE, where they hold the committed
 * partial coloring (0 = not yet colored) from which a later call can resume
 * via init_colors.
 */
#ifndef GRAPHCOLOR_H
#define GRAPHCOLOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COLOR_OK            0
#define COLOR_EINVAL       -1   /* bad size, null pointer, bad parameter */
#define COLOR_EGRAPH       -2   /* COLOR_FLAG_VALIDATE: graph violates the input contract */
#define COLOR_EOVERFLOW    -3   /* a size does not fit the int32 indexing */
#define COLOR_ENOMEM       -4   /* device or host allocation failed */
#define COLOR_EHIP         -5   /* a HIP runtime call failed */
#define COLOR_ENOCONVERGE  -6   /* params->max_rounds reached: outputs hold the partial state */
#define COLOR_E2BIG        -7   /* server: the job can never fit the HBM budget */
#define COLOR_EMISMATCH    -8   /* autotune: two mappings gave different colorings (a library defect) */
#define COLOR_ESCRATCH     -9   /* color_d1_noalloc: n above COLOR_NOALLOC_MAX_N */
#define COLOR_EQUEUED       1   /* server: job accepted, waiting for memory/slots */
#define COLOR_EPENDING      2   /* server: job not finished yet */

#define COLOR_FLAG_VALIDATE 0x1u  /* check the input contract on the device first */
#define COLOR_FLAG_NO_TAIL  0x2u  /* incremental engine: run every round as its own pair of
                                     launches, never finish with the cooperative tail kernel */
#define COLOR_FLAG_KERNEL_TIMING 0x4u  /* time every round kernel with HIP events on `stream` */
/* recolorDegrees (Section 3.3; Algorithm 4 with recolorDegrees set): the one
 * flag that CHANGES the coloring.  The key becomes key(v) = (deg(v), p(v),
 * gid(v)), compared lexicographically, so that of two conflicting vertices the
 * one of LOWER degree is uncolored and p, then gid, only decide between equal
 * degrees.  deg(v) is computed once, before the rounds: the length of v's row
 * in row_ptr (color_d1, color_d2), the number of rows of column v in col_ptr
 * (color_pd2), and for the ghost step an owned vertex's row and a ghost's
 * ghost_degree entry.  Honoured by color_d1, color_d2, color_pd2 and
 * color_d1_ghost_step (color_d1_ghost has no ghost degrees and returns
 * COLOR_EINVAL with it when n_ghost > 0); color_batch and the server return
 * COLOR_EINVAL.  The library sorts the vertices by this key once per call
 * (about 36 bytes of workspace per vertex). */
#define COLOR_FLAG_RECOLOR_DEGREES 0x8u
/* Tentative ghost recoloring (Section 3.2: a rank may temporarily recolor
 * ghosts in its recoloring step and restores their colors afterwards;
 * Section 3.4: with two ghost layers that recoloring sees the ghosts' whole
 * neighbourhoods).  Also changes the coloring.  Honoured by color_d1_ghost,
 * color_d1_ghost_step and color_d1_distributed (ignored elsewhere): phase 2
 * uncolors the losing end of every conflicting owned-ghost pair, ghost or
 * owned; phase 3 recolors the owned losers and the losing ghosts together,
 * in the same synchronous rounds, on the local graph: a ghost's neighbours
 * are its row with two layers (layer-1 rows), and with one layer the owned
 * vertices adjacent to it; ghosts whose colors are not known (0) stay out of
 * it.  Only the owned colors are returned: the ghosts' tentative colors are
 * dropped (restored).  With one layer the call builds the ghosts' rows (about
 * 4 bytes per owned-ghost entry plus 12 per ghost of workspace). */
#define COLOR_FLAG_GHOST_RECOLOR 0x10u

/* Per-call statistics (HOST struct, every pointer argument of this type is
 * nullable). */
typedef struct color_stats {
    int32_t num_colors;          /* largest color in the output */
    int32_t rounds;              /* rounds with a non-empty worklist */
    int64_t vertex_visits;       /* sum over rounds of |W_r| */
    int64_t edge_visits;         /* sum over rounds of the adjacency entries of W_r
                                    (D2/PD2: entries of the two-hop walk) */
    int64_t boundary_conflicts;  /* ghost variant: equal-colored owned-ghost pairs after phase 1 */
    int64_t remote_losers;       /* ghost variant: ghosts that lost a boundary conflict */
    int64_t* worklist_trace;     /* in: HOST array or NULL; out: |W_r| for r = 1..min(rounds, trace_cap) */
    int32_t trace_cap;           /* in: capacity of worklist_trace */
    int32_t kernel_launches;     /* kernels the call enqueued */
    /* COLOR_FLAG_KERNEL_TIMING only (else 0): summed HIP-event durations of
       the color and the detect round kernels, and their launch counts */
    int64_t color_kernel_ns;
    int64_t detect_kernel_ns;
    int32_t color_launches;
    int32_t detect_launches;
    int32_t engine;              /* COLOR_ENGINE_* that ran */
    int32_t tail_rounds;         /* INCREMENTAL: rounds run by the cooperative tail kernel */
    int64_t list_visits;         /* INCREMENTAL: active-list entries scanned by the detect kernels */
    int64_t pushes;              /* INCREMENTAL: forbidden-color bits pushed */
    int64_t color_bytes;         /* algorithmic bytes of the per-round color kernels (INCREMENTAL; PULL: 0) */
    int64_t detect_bytes;        /* algorithmic bytes of the per-round detect kernels (INCREMENTAL; PULL: 0) */
    int64_t tail_kernel_ns;      /* COLOR_FLAG_KERNEL_TIMING: HIP-event duration of the tail kernel */
    int64_t tail_bytes;          /* algorithmic bytes of the tail kernel's rounds (color + detect) */
    int32_t tail_fallbacks;      /* INCREMENTAL: tail launches whose workgroups were not all resident
                                    (they ran nothing; the rounds went on as per-round launches) */
} color_stats;

/* Tuning knobs (HOST struct, nullable = library defaults / autotuned).  None
 * of them changes a coloring, except the COLOR_FLAG_RECOLOR_DEGREES flag, which
 * selects the recolorDegrees key; the rest only change how the work is mapped
 * onto the GPU.  A zero field means "default". */
typedef struct color_params {
    int32_t bin_hi[4];      /* work bounds of degree bins 0..3 (bin 4 = above bin_hi[3]) */
    int32_t lanes[3];       /* lanes per vertex of bins 0..2: 1,2,4,8,16,32 or 64 */
    int32_t split_chunks;   /* workgroups per vertex in bin 4 */
    int32_t max_rounds;     /* stop after this many rounds: COLOR_ENOCONVERGE (0: n + 1, which
                               no run reaches: each round commits at least one vertex) */
    int32_t rounds_per_poll;/* rounds enqueued between host checks of the worklist size */
    int32_t tail_threshold; /* INCREMENTAL: worklist size at or below which one cooperative launch
                               runs all remaining rounds (grid barriers between the steps;
                               default 32768).  Its workgroups wait on each other, so they
                               must all be resident: before writing anything they check in
                               and wait up to tail_checkin_us for each other; if they are not
                               all resident by then (other streams keep the device full), the
                               launch does nothing and the rounds continue as per-round
                               launches (stats->tail_fallbacks counts this).  The same happens
                               if the runtime refuses the cooperative launch.  A grid barrier
                               that still stalls for 30 s makes the call start over with
                               per-round launches only (COLOR_FLAG_NO_TAIL), which gives the
                               same coloring. */
    int32_t max_workgroups; /* cap on the grid of the round kernels */
    uint32_t flags;         /* COLOR_FLAG_* */
    int32_t engine;         /* COLOR_ENGINE_*: 0 = library choice */
    int32_t tail_checkin_us;/* INCREMENTAL: how long the tail kernel's workgroups wait for each other
                               at entry (0: 2000 us; -1: no wait, so every tail launch falls back
                               to per-round launches) */
} color_params;

/* Engines (identical colorings).  PULL re-reads every worklist vertex's full
 * neighbourhood in both kernels of a round.  INCREMENTAL keeps per-vertex
 * forbidden-color bitsets that committing neighbours push into, and per-vertex
 * active-neighbour lists compacted as neighbours commit; it needs extra
 * device memory of about 8 bytes per list entry (D1: per adjacency entry;
 * D2/PD2: per two-hop walk entry) plus worklists of up to 4n entries, falls
 * back to PULL when the lists do not fit int32 offsets, and returns
 * COLOR_EOVERFLOW when its worklists would not.  Unless the caller sets
 * bin_hi, it uses its own bin bounds (D1 16/96/1024, D2 and PD2
 * 64/256/1024). */
#define COLOR_ENGINE_AUTO        0
#define COLOR_ENGINE_PULL        1
#define COLOR_ENGINE_INCREMENTAL 2
#define COLOR_ENGINE_BATCH       3   /* stats only: the batched persistent engine ran the job */

/* Distance-1 coloring (Section 2.1; Section 3.2).
 *   n            vertices (>= 0)
 *   row_ptr      int32[n+1], col_idx int32[row_ptr[n]]: symmetric CSR
 *   seed         selects the priority hash p(v) (gid(v) = v)
 *   prio         nullable uint32[n]: explicit p(v) replacing the hash
 *   init_colors  nullable int32[n]: non-zero entries are committed colors
 *                that stay fixed (a proper partial coloring, e.g. the
 *                partial state returned with COLOR_ENOCONVERGE); zero
 *                entries are colored (Section 3.2: the coloring functions
 *                accept a partial coloring)
 *   colors       out int32[n]
 * Returns COLOR_OK, COLOR_EINVAL, COLOR_EGRAPH, COLOR_EOVERFLOW,
 * COLOR_ENOMEM, COLOR_EHIP or COLOR_ENOCONVERGE. */
int color_d1(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
             const uint32_t* prio, const int32_t* init_colors, int32_t* colors,
             color_stats* stats, const color_params* params, void* stream);

/* Distance-2 coloring (Section 2.1; Section 3.5, Algorithm 5 without
 * doPartialColoring): vertices within two hops get different colors;
 * the two-hop neighbourhood of v is N(v) u N(N(v)) minus v.  Same arguments
 * and errors as color_d1. */
int color_d2(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
             const uint32_t* prio, const int32_t* init_colors, int32_t* colors,
             color_stats* stats, const color_params* params, void* stream);

/* Partial distance-2 coloring of the columns of an n_rows x n_cols sparse
 * pattern (Section 2.1; Section 3.6, doPartialColoring): two columns that
 * share a row get different colors; rows are not colored.
 *   row_ptr int32[n_rows+1], col_idx int32[nnz]  pattern in CSR
 *   col_ptr int32[n_cols+1], row_idx int32[nnz]  the same pattern in CSC
 *   prio, init_colors: nullable, indexed by column; col_colors out int32[n_cols]
 * gid(column) = column index.  Same errors as color_d1. */
int color_pd2(int32_t n_rows, int32_t n_cols, const int32_t* row_ptr, const int32_t* col_idx,
              const int32_t* col_ptr, const int32_t* row_idx, uint32_t seed,
              const uint32_t* prio, const int32_t* init_colors, int32_t* col_colors,
              color_stats* stats, const color_params* params, void* stream);

/* One rank's step of the distributed D1 method (Section 3, Algorithm 2 with
 * Algorithms 3 and 4; Section 3.4 for the second ghost layer) on its local
 * graph G_l = {V_l + V_g, E_l + E_g} (Section 2.4).
 *   Local ids: owned vertices [0, n_owned), then ghosts
 *   [n_owned, n_owned + n_ghost); with layers == 2 the first n_g1 ghosts are
 *   the first ghost layer and carry rows.
 *   row_ptr int32[n_rows+1], n_rows = n_owned (layers 1) or n_owned + n_g1
 *   (layers 2); col_idx local ids in [0, n_owned + n_ghost).
 *   gid          int32[n_owned + n_ghost]: global ids (keys use gid)
 *   ghost_colors int32[n_ghost]: the ghosts' fixed colors (>= 1), read only
 *   owned_colors out int32[n_owned]
 *   remote_loser out uint8[n_ghost], nullable: 1 where a ghost lost a
 *                boundary conflict to an owned vertex (its owner recolors it)
 * Phase 1 colors the owned vertices ignoring ghosts (Section 3.2: the
 * initial coloring needs no ghost information); phase 2 compares every
 * owned-ghost edge with the key rule on the ghosts' colors; phase 3 recolors
 * the owned losers with the ghost colors as constraints.  Ghost colors are
 * never written (the save/restore of gc in Algorithm 2).  The second layer's
 * rows are accepted; with fixed ghost colors they do not change the result
 * (with COLOR_FLAG_GHOST_RECOLOR the ghosts are recolored tentatively on
 * them, which does).
 * Same errors as color_d1 (COLOR_EINVAL also for layers not 1 or 2). */
int color_d1_ghost(int32_t n_owned, int32_t n_ghost, int32_t layers, int32_t n_g1,
                   const int32_t* row_ptr, const int32_t* col_idx, const int32_t* gid,
                   const int32_t* ghost_colors, uint32_t seed, int32_t* owned_colors,
                   uint8_t* remote_loser, color_stats* stats, const color_params* params,
                   void* stream);

/* The ghost step of color_d1_ghost for every iteration of Algorithm 2's loop
 * (Section 3, Algorithm 2; Sections 3.2 and 3.3), with two more inputs:
 *   ghost_colors int32[n_ghost], each >= 0: the ghosts' current colors as
 *                their owners last communicated them; 0 = not known yet (the
 *                ghost constrains nothing and conflicts with nothing, as color
 *                zero means uncolored in Section 3.2)
 *   ghost_degree nullable int32[n_ghost]: the ghosts' degrees in the global
 *                graph, as their owners report them; required with
 *                COLOR_FLAG_RECOLOR_DEGREES when n_ghost > 0 (else
 *                COLOR_EINVAL)
 *   init_owned   nullable int32[n_owned]: committed owned colors to start from
 *                (the previous iteration's output); phase 1 then colors only
 *                the owned vertices it leaves at 0, ghost-blind, and phases 2
 *                and 3 judge and repair the boundary against ghost_colors
 * With init_owned NULL and ghost_degree NULL this is color_d1_ghost.  One
 * iteration of Algorithm 2's while loop is one call per rank with
 * init_owned = that rank's colors and ghost_colors = what its neighbours
 * sent; the loop ends when the calls' boundary_conflicts sum to 0.  Same
 * errors as color_d1_ghost. */
int color_d1_ghost_step(int32_t n_owned, int32_t n_ghost, int32_t layers, int32_t n_g1,
                        const int32_t* row_ptr, const int32_t* col_idx, const int32_t* gid,
                        const int32_t* ghost_colors, const int32_t* ghost_degree, uint32_t seed,
                        const int32_t* init_owned, int32_t* owned_colors, uint8_t* remote_loser,
                        color_stats* stats, const color_params* params, void* stream);

/* color_d1 for callers that cannot allocate memory (serving loops and
 * harnesses that forbid hipMalloc between requests): same arguments, same
 * coloring and statistics as color_d1, and the call allocates no device or
 * host memory.  Its workspace is a static device array of about 17 MiB that
 * each GPU the library runs on holds until the process ends; its address is
 * taken once per device on the device's first call.  It always runs the pull
 * engine with workgroup-wide heavy vertices (the layouts that fit that array),
 * which gives the same coloring as every other engine.  Limits and errors:
 * n above COLOR_NOALLOC_MAX_N returns COLOR_ESCRATCH; COLOR_FLAG_KERNEL_TIMING,
 * COLOR_FLAG_RECOLOR_DEGREES, engine = COLOR_ENGINE_INCREMENTAL and a
 * stats->trace_cap above 4096 return COLOR_EINVAL; otherwise as color_d1.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents; calls on one device are serialized by an internal lock
 * (calls that overlapped on one device would race on the array).  Blocking
 * like color_d1 (it synchronizes `stream` to read the worklist sizes), so it
 * cannot be recorded into a graph. */
#define COLOR_NOALLOC_MAX_N (1 << 20)
int color_d1_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t seed,
                     const uint32_t* prio, const int32_t* init_colors, int32_t* colors,
                     color_stats* stats, const color_params* params, void* stream);

/* One rank's step of the distributed distance-2 method (Section 3,
 * Algorithm 2, with the distance-2 conflict detection of Section 3.5,
 * Algorithm 5, over the rank's owned vertices) on a local graph with two
 * ghost layers, which carries the full two-hop neighbourhood of every owned
 * vertex:
 *   local ids: owned [0, n_owned), then ghosts [n_owned, n_owned + n_ghost),
 *   the first n_g1 of them the first layer;
 *   row_ptr int32[n_owned + n_g1 + 1], col_idx local ids: the rows of the
 *   owned vertices, then of the first-layer ghosts (complete rows)
 *   gid int32[n_owned + n_ghost]; ghost_colors int32[n_ghost] (>= 0; 0 = not
 *   known yet); owned_colors out int32[n_owned]; remote_loser out
 *   uint8[n_ghost], nullable.
 * Phase 1 colors the owned vertices at distance 2 with every ghost
 * uncolored (walks pass through ghosts, the ghosts' colors are not used);
 * phase 2 compares every owned vertex with every distinct ghost within two
 * hops against the ghosts' colors (the lower key loses; boundary_conflicts
 * counts each such pair once); phase 3 recolors the owned losers with the
 * ghosts' colors as constraints.  Both phases run on the engine `params`
 * names or the library's choice (the incremental engine's lists then hold
 * only the owned members of each walk; in phase 3 the ghosts' colors enter
 * the losers' forbidden sets once, before its first round).  Errors as
 * color_d2. */
int color_d2_ghost(int32_t n_owned, int32_t n_ghost, int32_t n_g1, const int32_t* row_ptr,
                   const int32_t* col_idx, const int32_t* gid, const int32_t* ghost_colors, uint32_t seed,
                   int32_t* owned_colors, uint8_t* remote_loser, color_stats* stats,
                   const color_params* params, void* stream);

/* The same step for partial distance-2 coloring of columns (Section 3.6): a
 * rank owns columns; its local pattern holds the rows that touch an owned
 * column and all of those rows' columns:
 *   col_ptr int32[n_owned + 1], row_idx: the owned columns' rows (local row
 *   ids in [0, n_rows)); row_ptr int32[n_rows + 1], col_idx: the local rows'
 *   columns (local column ids: owned [0, n_owned), then ghost columns).
 * Other arguments, phases and errors as color_d2_ghost. */
int color_pd2_ghost(int32_t n_owned, int32_t n_ghost, int32_t n_rows, const int32_t* col_ptr,
                    const int32_t* row_idx, const int32_t* row_ptr, const int32_t* col_idx,
                    const int32_t* gid, const int32_t* ghost_colors, uint32_t seed, int32_t* owned_colors,
                    uint8_t* remote_loser, color_stats* stats, const color_params* params, void* stream);

/* ----------------------------------------------------------------------- */
/* Algorithm 2 over several ranks, emulated on one GPU.                      */
/* ----------------------------------------------------------------------- */

/* One rank's local graph (DEVICE arrays, as color_d1_ghost_step takes them)
 * and where each of its ghosts is owned. */
typedef struct color_part {
    int32_t n_owned, n_ghost, layers, n_g1;
    const int32_t* row_ptr;       /* rows of the owned (and, layers == 2, layer-1) vertices */
    const int32_t* col_idx;       /* local ids */
    const int32_t* gid;           /* int32[n_owned + n_ghost]: global ids */
    const int32_t* ghost_owner;   /* int32[n_ghost]: the rank owning ghost j, in [0, num_parts) */
    const int32_t* ghost_index;   /* int32[n_ghost]: ghost j's index among that rank's owned vertices */
    const int32_t* ghost_degree;  /* nullable int32[n_ghost]: global degrees (COLOR_FLAG_RECOLOR_DEGREES) */
    int32_t* owned_colors;        /* out: int32[n_owned] */
} color_part;

typedef struct color_dist_stats {
    int32_t detects;              /* conflict detections run (the last one found none) */
    int32_t iterations;           /* recolorings: Algorithm 2's while-loop iterations (detects - 1) */
    int32_t num_colors;           /* largest color over all ranks */
    int32_t trace_cap;            /* in: capacity of the two trace arrays */
    int64_t* conflicts_trace;     /* in: HOST array or NULL; out: per detection, conflicts summed over
                                     the ranks (each owned-ghost pair counted by the rank that owns its
                                     owned end) */
    int64_t* exchanged_trace;     /* in: HOST array or NULL; out: per exchange, ghost copies sent */
    int64_t exchanged_total;      /* ghost copies sent over all exchanges: the messages of an MPI run
                                     would carry this many (index, color) pairs */
    int64_t rounds_total;         /* on-node rounds summed over ranks and steps */
} color_dist_stats;

/* Algorithm 2 (Section 3; Sections 3.2 and 3.3) on num_parts ranks whose
 * local graphs are all on this GPU.  Every rank first colors its owned
 * vertices without ghost information.  Then, until the conflicts summed
 * over the ranks (the Allreduce) are zero: each rank receives its ghosts'
 * current colors from their owners (the first time every ghost copy, later
 * only the copies whose owner recolored them; here a gather kernel stands in
 * for the messages), and each rank runs color_d1_ghost_step from its
 * committed colors: detect against the received colors (the lower key
 * loses, Algorithm 4), recolor its losers with the ghosts' colors as fixed
 * constraints.  Ranks read only the colors of the last exchange, so the
 * result does not depend on the order the ranks run in.
 *   parts        HOST array of num_parts descriptors (device arrays inside;
 *                ghost_owner / ghost_index are trusted unless
 *                COLOR_FLAG_VALIDATE is set)
 *   max_detects  stop after this many detections (0: no limit):
 *                COLOR_ENOCONVERGE, owned_colors hold the last step's colors
 *   stats        nullable HOST struct
 * params as for color_d1_ghost_step (COLOR_FLAG_RECOLOR_DEGREES needs every
 * part's ghost_degree).  The call allocates and frees its own exchange
 * buffers (8 bytes per ghost copy); the steps use the single-graph
 * workspace.  Returns COLOR_OK, COLOR_EINVAL (also for a ghost_owner /
 * ghost_index out of range with COLOR_FLAG_VALIDATE), COLOR_EOVERFLOW,
 * COLOR_ENOMEM, COLOR_EHIP, COLOR_EGRAPH or COLOR_ENOCONVERGE. */
int color_d1_distributed(int32_t num_parts, const color_part* parts, uint32_t seed, int32_t max_detects,
                         color_dist_stats* stats, const color_params* params, void* stream);

/* The priority p of Algorithm 4's rand(GID) as the kernels compute it:
 * out[i] = p(gid ? gid[i] : i) for i < n.  gid nullable (identity).
 * Returns COLOR_OK, COLOR_EINVAL or COLOR_EHIP. */
int color_priority(int32_t n, const int32_t* gid, uint32_t seed, uint32_t* out, void* stream);

/* ----------------------------------------------------------------------- */
/* Batched form: many graphs in one persistent, worklist-driven launch.     */
/* ----------------------------------------------------------------------- */

#define COLOR_KIND_D1  1
#define COLOR_KIND_D2  2
#define COLOR_KIND_PD2 3

/* One coloring job.  D1/D2: n = vertices, row_ptr/col_idx = adjacency,
 * col_ptr/row_idx unused.  PD2: n = columns, n_rows = rows, row_ptr/col_idx
 * = CSR, col_ptr/row_idx = CSC.  Device pointers; colors = output. */
typedef struct color_job {
    int32_t kind;
    int32_t n;
    int32_t n_rows;
    uint32_t seed;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* col_ptr;
    const int32_t* row_idx;
    int32_t* colors;
} color_job;

/* Colors num_jobs independent graphs in one persistent launch (no grid-wide
 * barrier): every job advances through its own synchronous rounds, phase by
 * phase, and the launch's workgroups take (job, phase, chunk) units of any
 * open phase from per-job phase words; the workgroup that completes a
 * phase's last unit opens the job's next phase.  Each job's coloring,
 * rounds, vertex_visits, edge_visits and num_colors equal those of the
 * single-graph call of its kind (color_d1 / color_d2 / color_pd2 with the
 * job's seed, prio and init_colors NULL).
 *   jobs     HOST array of num_jobs descriptors (device pointers inside);
 *            n <= 2^23 per job (larger graphs: the single-graph calls)
 *   per_job  nullable HOST array of num_jobs stats (engine =
 *            COLOR_ENGINE_BATCH, kernel_launches = 1)
 *   params   nullable; honoured: max_rounds (capped at 32000),
 *            max_workgroups, flags & COLOR_FLAG_VALIDATE (every job is
 *            validated first).  Bins and lanes come from the autotuner's
 *            per-device record for the job's kind and average degree class
 *            (library defaults until color_autotune has run).
 * D2/PD2 jobs whose two-hop walk per visit is long (>= 128 entries,
 * estimated from nnz/n) are colored after the persistent launch by the
 * single-graph call of their kind, whose incremental engine serves them
 * better than the launch's pull-style steps (their stats say so in
 * `engine`); every other job shares the one persistent launch.
 * The library allocates 16 bytes per vertex of workspace (grow-only, per
 * device).  Returns COLOR_OK, COLOR_EINVAL, COLOR_EOVERFLOW, COLOR_EGRAPH,
 * COLOR_ENOMEM, COLOR_EHIP or the first job's COLOR_ENOCONVERGE. */
int color_batch(int32_t num_jobs, const color_job* jobs, color_stats* per_job,
                const color_params* params, void* stream);

/* Autotuner of the batched and served forms.  Runs `job` alone through the
 * batched engine once per candidate mapping (lanes per vertex of bins 0..2
 * and bin bounds scaled around the library defaults), `reps` times each
 * (>= 1), keeps the fastest by wall time, and records it for the job's kind
 * and average-degree class floor(log2(nnz / n)) on the current device; later
 * color_batch calls and servers created afterwards use the record.  Every
 * candidate's colors are compared with the first's: a difference returns
 * COLOR_EMISMATCH (no mapping may change a coloring).  best (nullable, HOST)
 * receives the chosen bin_hi[0..2] and lanes.  Returns COLOR_OK, COLOR_EINVAL,
 * COLOR_EOVERFLOW, COLOR_ENOMEM, COLOR_EHIP or COLOR_EMISMATCH. */
int color_autotune(const color_job* job, int32_t reps, color_params* best, void* stream);

/* Forgets every autotuner record of the current device. */
int color_autotune_reset(void);

/* ----------------------------------------------------------------------- */
/* Served form: continuous batching with HBM-footprint admission.          */
/* ----------------------------------------------------------------------- */

typedef struct color_server color_server;

/* A served job carries HOST arrays (the server copies them to the device
 * while other jobs run).  Same field meaning as color_job. */
typedef struct color_host_job {
    int32_t kind;
    int32_t n;
    int32_t n_rows;
    uint32_t seed;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* col_ptr;
    const int32_t* row_idx;
} color_host_job;

/* Creates a server on the current device with an HBM budget (bytes) for
 * resident job state and at most max_slots jobs on the device at once.
 * *err receives COLOR_OK or an error; returns NULL on error. */
color_server* color_server_create(size_t hbm_budget_bytes, int32_t max_slots, int* err);

/* Queues a job (arrays are copied before return).  Returns COLOR_OK (job
 * admitted to the device), COLOR_EQUEUED (waiting for memory or a slot),
 * COLOR_E2BIG (can never fit the budget) or COLOR_EINVAL.  *job_id is set
 * when the job was accepted. */
int color_server_submit(color_server* s, const color_host_job* job, uint64_t* job_id);

/* Advances the server (admits queued jobs, runs rounds of the resident
 * jobs).  Returns COLOR_OK when job_id has finished (host_colors receives
 * its n colors, stats is filled; the job's slot and memory are freed), the
 * job's own error code when its coloring failed (COLOR_ENOCONVERGE at the
 * round cap, the colors then holding the committed partial state; other
 * jobs go on), COLOR_EPENDING when it has not finished, COLOR_EINVAL for an
 * unknown id.  A failed launch, copy or event on the server's streams is
 * the server's error: this call and every later one return COLOR_EHIP. */
int color_server_poll(color_server* s, uint64_t job_id, int32_t* host_colors, color_stats* stats);

/* Runs the server until every accepted job has finished. */
int color_server_drain(color_server* s);

int color_server_destroy(color_server* s);

/* Frees the per-device workspace cache of the single-graph entry points. */
int color_release_workspace(void);

/* Static description of an error code. */
const char* color_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* GRAPHCOLOR_H */
