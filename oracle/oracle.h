/* CPU oracle for synchronous speculative graph coloring: test infrastructure
 * only (tests, smoke check, benchmark CPU baseline).  Shares nothing with the
 * GPU library. */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#define ORC_TRACE_ROUNDS 4096
#define ORC_RECOLOR_DEGREES 1   /* key(v) = (deg(v), p(v), gid(v)): recolorDegrees */
#define ORC_GHOST_RECOLOR   2   /* ghost step: losing ghosts are recolored tentatively, then restored */

typedef struct {
    int32_t num_colors;          /* largest color used */
    int32_t rounds;              /* rounds with a non-empty worklist */
    int64_t vertex_visits;       /* sum over rounds of |W_r| */
    int64_t edge_visits;         /* adjacency entries read by the color steps */
    int64_t boundary_conflicts;  /* ghost variant: equal-colored owned-ghost pairs after phase 1 */
    int64_t remote_losers;       /* ghost variant: ghosts that lost a boundary conflict */
    int64_t worklist_trace[ORC_TRACE_ROUNDS];  /* |W_r| per round */
} orc_stats;

int orc_threads(void);   /* threads of the per-vertex loops (1 unless built with -fopenmp) */
uint32_t orc_fmix32(uint32_t h);
uint32_t orc_priority(uint32_t gid, uint32_t seed);
void orc_priorities(int32_t n, uint32_t seed, uint32_t *out);  /* out[i] = p(i) */

/* Return 0 when every vertex is colored, 1 when max_rounds (>0) stopped the
 * loop first (colors then hold the committed partial state, 0 = uncolored). */
int orc_color_d1(int32_t n, const int32_t *row_ptr, const int32_t *col, uint32_t seed,
                 const uint32_t *prio, const int32_t *init, int32_t max_rounds,
                 int32_t *colors, orc_stats *st, int flags);
int orc_color_d2(int32_t n, const int32_t *row_ptr, const int32_t *col, uint32_t seed,
                 const uint32_t *prio, const int32_t *init, int32_t max_rounds,
                 int32_t *colors, orc_stats *st, int flags);
int orc_color_pd2(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                  const int32_t *col_ptr, const int32_t *row_idx, uint32_t seed,
                  const uint32_t *prio, const int32_t *init, int32_t max_rounds,
                  int32_t *col_colors, orc_stats *st, int flags);
int orc_color_d1_ghost(int32_t n_owned, int32_t n_ghost, int32_t layers, int32_t n_g1,
                       const int32_t *row_ptr, const int32_t *col, const int32_t *gid,
                       const int32_t *ghost_colors, uint32_t seed, const int32_t *init_owned,
                       const int32_t *ghost_degree, int32_t *owned_colors,
                       unsigned char *remote_loser, orc_stats *st, int flags);
int orc_color_d2_ghost(int kind, int32_t n_owned, int32_t n_ghost, const int32_t *hop1_ptr,
                       const int32_t *hop1_idx, const int32_t *hop2_ptr, const int32_t *hop2_idx,
                       const int32_t *gid, const int32_t *ghost_colors, uint32_t seed,
                       int32_t *owned_colors, unsigned char *remote_loser, orc_stats *st, int flags);
void orc_serial_greedy(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const int32_t *order, int32_t *colors);
#endif
