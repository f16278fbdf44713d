/*
 * CPU oracle for synchronous speculative graph coloring.  TEST INFRASTRUCTURE
 * ONLY: it is called by the test suite, by the smoke check and by the
 * benchmark's CPU-baseline leg, never by the library's product path.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * Plain, slow C: every per-round loop below is written the way the method is
 * defined, with no bitmasks, no blocking and no fusion, so that a reader can
 * check it against the paper by eye.  Built plainly (as the tests build it)
 * it is single-threaded.  Built with -fopenmp (the benchmark's all-core CPU
 * baseline only) the per-vertex loops of the color and detect steps run on
 * several threads: each vertex of those loops reads only the previous step's
 * arrays and writes only its own entry, so the result is the same.
 *
 * The method (Bogle et al., "Parallel Graph Coloring Algorithms for
 * Distributed GPU Environments"):
 *   - colors are integers, 0 means "uncolored" (Section 2.2, Algorithm 1;
 *     Section 3.2, the coloring functions treat color zero as uncolored);
 *   - a vertex takes the smallest color not used by its neighbours
 *     (first-fit, Section 2.2, Algorithm 1);
 *   - speculate and iterate (Section 2.3, Section 3, Algorithm 2): color every
 *     uncolored vertex, detect conflicts, uncolor one endpoint of each
 *     conflict, repeat until no conflict remains;
 *   - the endpoint to recolor is chosen by a random number derived from the
 *     global id, ties broken by the id (Section 3.2, Algorithm 4).
 *
 * Readings taken where the paper leaves freedom (each is listed with its
 * reason in the design notes):
 *   R1  rounds are synchronous: every vertex of the round's worklist picks its
 *       tentative color from the colors committed before the round, and all
 *       conflicts of the round are judged at once on the tentative colors;
 *   R2  key(v) = (p(v), gid(v)) compared lexicographically; in a conflict the
 *       LOWER key is uncolored (the mirror of Algorithm 4's direction, which
 *       is statistically equivalent);
 *   R3  p(v) = fmix32(gid ^ S), S = fmix32(seed ^ 0x9E3779B9), fmix32 being
 *       the MurmurHash3 32-bit finalizer (public domain, A. Appleby); a
 *       bijection of uint32, so keys never tie;
 *   R4  distance-2 neighbourhood N2(v) = (N(v) u N(N(v))) \ {v}
 *       (Section 2.1: all vertices within two hops differ);
 *   R5  partial distance-2 colors the columns of a pattern only; two columns
 *       conflict when they share a row (Section 2.1; Section 3.6, the
 *       doPartialColoring mode of Algorithm 5 checks two-hop pairs only);
 *   R6  ghost variant (Algorithm 2, one rank's step): phase 1 colors the
 *       owned vertices ghost-blind (Section 3.2: the initial coloring does not
 *       need ghost information); phase 2 compares every owned-ghost edge
 *       against the ghosts' fixed colors with the key rule (Algorithm 3/4);
 *       phase 3 recolors the owned losers with the ghost colors as
 *       constraints; ghost colors are never written (save/restore of gc);
 *   R8  tentative ghost recoloring (Section 3.2, save/restore of the ghosts'
 *       colors gc in Algorithm 2; Section 3.4 for two layers), when asked
 *       for: phase 2 uncolors the losing end of every conflicting owned-ghost
 *       pair, ghost or owned; phase 3 recolors every uncolored owned vertex
 *       and losing ghost together, in the same synchronous rounds, on the
 *       local graph (a ghost's neighbourhood is its row with two layers, and
 *       with one layer the owned vertices adjacent to it); then the ghosts'
 *       colors are restored: only the owned colors are kept;
 *   R9  distance-2 and partial distance-2 ghost step (Section 3.5,
 *       Algorithm 5 over the rank's owned vertices; Section 3.6): the local
 *       graph carries the full two-hop neighbourhood of every owned vertex
 *       (D2: rows of the owned vertices and of the first ghost layer; PD2:
 *       the owned columns' rows and those rows' columns).  Phase 1 colors the
 *       owned vertices with every ghost uncolored (ghost colors are not
 *       used, the adjacency through ghosts is); phase 2 compares every owned
 *       vertex with every distinct ghost of its two-hop neighbourhood
 *       against the ghosts' fixed colors (key rule; each pair counted once);
 *       phase 3 recolors the owned losers with the ghosts' colors as
 *       constraints;
 *   R7  recolorDegrees (Section 3.3; Algorithm 4 with recolorDegrees true):
 *       when asked for, key(v) = (deg(v), p(v), gid(v)), so that of two
 *       conflicting vertices the one of lower degree is uncolored and the
 *       random key only decides between equal degrees.  deg(v) is the number
 *       of stored neighbours of v in the graph being colored (D1, D2: its
 *       adjacency row; PD2: the rows of column v; a ghost: the degree its
 *       owner reports), computed once before the rounds.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the per-vertex loops may use: 1 in the plain build. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Priority: rand(GID) of Algorithm 4                                      */
/* ---------------------------------------------------------------------- */

/* MurmurHash3 32-bit finalizer: xor-shift 16, multiply, xor-shift 13,
 * multiply, xor-shift 16, all modulo 2^32. */
uint32_t orc_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

uint32_t orc_priority(uint32_t gid, uint32_t seed)
{
    uint32_t s = orc_fmix32(seed ^ 0x9E3779B9u);
    return orc_fmix32(gid ^ s);
}

void orc_priorities(int32_t n, uint32_t seed, uint32_t *out)
{
    for (int32_t i = 0; i < n; i++) out[i] = orc_priority((uint32_t)i, seed);
}

/* Keys of the vertices the rules may compare: p(v), gid(v) and, with
 * recolorDegrees (reading R7), deg(v). */
typedef struct {
    const uint32_t *p;
    const uint32_t *gid;
    const int64_t *deg;       /* nullable: keys without degrees (reading R2) */
} keys_t;

/* 1 if key(a) > key(b): (deg, p, gid) or (p, gid), lexicographic. */
static int key_greater(const keys_t *k, int32_t a, int32_t b)
{
    if (k->deg && k->deg[a] != k->deg[b]) return k->deg[a] > k->deg[b];
    if (k->p[a] != k->p[b]) return k->p[a] > k->p[b];
    return k->gid[a] > k->gid[b];
}

/* ---------------------------------------------------------------------- */
/* A neighbourhood is a plain list of vertex ids (duplicates allowed: the  */
/* rules below only ask "does some member satisfy ...", which duplicates   */
/* do not change).                                                         */
/* ---------------------------------------------------------------------- */

typedef struct {
    int kind;                 /* 1 = distance-1, 2 = distance-2, 3 = partial distance-2 */
    int32_t n;                /* vertices being colored */
    const int32_t *row_ptr;   /* D1/D2: adjacency CSR; PD2: pattern CSR (rows -> cols) */
    const int32_t *col;
    const int32_t *col_ptr;   /* PD2 only: pattern CSC (cols -> rows) */
    const int32_t *row_idx;
} graph_t;

typedef struct {
    int32_t *ids;
    int64_t len, cap;
} list_t;

static void list_push(list_t *l, int32_t x)
{
    if (l->len == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 64;
        l->ids = (int32_t *)realloc(l->ids, (size_t)l->cap * sizeof(int32_t));
    }
    l->ids[l->len++] = x;
}

/* Fills l with the neighbourhood of v used by the coloring problem:
 * D1: N(v); D2: N(v) and N(u) for u in N(v), minus v (reading R4);
 * PD2: every column sharing a row with column v, minus v (reading R5).
 * Returns the number of adjacency entries read (for the work counters). */
static int64_t neighbourhood(const graph_t *g, int32_t v, list_t *l)
{
    int64_t visits = 0;
    l->len = 0;
    if (g->kind == 1) {
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; e++) {
            list_push(l, g->col[e]);
            visits++;
        }
    } else if (g->kind == 2) {
        for (int32_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; e++) {
            int32_t u = g->col[e];
            list_push(l, u);
            visits++;
            for (int32_t f = g->row_ptr[u]; f < g->row_ptr[u + 1]; f++) {
                int32_t x = g->col[f];
                visits++;
                if (x != v) list_push(l, x);
            }
        }
    } else {
        for (int32_t e = g->col_ptr[v]; e < g->col_ptr[v + 1]; e++) {
            int32_t r = g->row_idx[e];
            visits++;
            for (int32_t f = g->row_ptr[r]; f < g->row_ptr[r + 1]; f++) {
                int32_t c = g->col[f];
                visits++;
                if (c != v) list_push(l, c);
            }
        }
    }
    return visits;
}

/* Smallest color c >= 1 that no member of nb carries in colors[] (first-fit,
 * Algorithm 1).  'extra' (nullable) supplies the colors of ids >= n_base
 * (ghosts), which are read as extra[id - n_base]. */
static int32_t first_fit(const list_t *nb, const int32_t *colors, int32_t n_base,
                         const int32_t *extra, int32_t ignore_from)
{
    /* used[c] for c in [0, len+1]: a color above len+1 can never be the answer */
    int64_t m = nb->len + 2;
    unsigned char *used = (unsigned char *)calloc((size_t)m, 1);
    for (int64_t i = 0; i < nb->len; i++) {
        int32_t u = nb->ids[i];
        int32_t c;
        if (u >= ignore_from) continue;
        c = (u < n_base) ? colors[u] : extra[u - n_base];
        if (c > 0 && c < m) used[c] = 1;
    }
    int32_t c = 1;
    while (used[c]) c++;
    free(used);
    return c;
}

/* ---------------------------------------------------------------------- */
/* The synchronous round loop (readings R1, R2)                            */
/* ---------------------------------------------------------------------- */

typedef struct {
    const graph_t *g;
    int32_t n;                /* colorable vertices: ids [0, n) */
    int32_t n_base;           /* ids >= n_base are fixed-color ghosts */
    const int32_t *ghost_col; /* colors of ids >= n_base */
    int32_t ignore_from;      /* neighbours with id >= ignore_from are ignored */
    keys_t keys;              /* keys of every id the rules may read */
    int32_t max_rounds;
    const unsigned char *eligible;  /* nullable: only these uncolored ids form the worklist */
} rounds_t;

/* Runs rounds until the worklist is empty or max_rounds is reached.
 * colors[] holds the committed colors C on entry (0 = in the worklist) and
 * on exit.  Returns the number of rounds; accumulates work counters. */
static int32_t run_rounds(const rounds_t *rc, int32_t *colors, orc_stats *st,
                          int32_t round0)
{
    int32_t n = rc->n;
    int32_t *T = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    unsigned char *in_w = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    unsigned char *lost = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    list_t W = {0};
    int32_t r = 0;

    for (int32_t v = 0; v < n; v++)
        if (colors[v] == 0 && (!rc->eligible || rc->eligible[v])) { list_push(&W, v); in_w[v] = 1; }

    while (W.len > 0 && r < rc->max_rounds) {
        r++;
        if (st) {
            st->vertex_visits += W.len;
            if (round0 + r - 1 < ORC_TRACE_ROUNDS) st->worklist_trace[round0 + r - 1] = W.len;
        }
        /* color step: reads the committed snapshot only */
        {
            int64_t vis = 0;
#pragma omp parallel if (W.len > 4096) reduction(+ : vis)
            {
                list_t nbt = {0};
#pragma omp for schedule(dynamic, 256)
                for (int64_t i = 0; i < W.len; i++) {
                    int32_t v = W.ids[i];
                    vis += neighbourhood(rc->g, v, &nbt);
                    T[v] = first_fit(&nbt, colors, rc->n_base, rc->ghost_col, rc->ignore_from);
                }
                free(nbt.ids);
            }
            if (st) st->edge_visits += vis;
        }
        /* detect step: v loses when a worklist neighbour holds the same
         * tentative color with a greater key; judged all at once */
#pragma omp parallel if (W.len > 4096)
        {
            list_t nbt = {0};
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < W.len; i++) {
                int32_t v = W.ids[i];
                lost[v] = 0;
                neighbourhood(rc->g, v, &nbt);
                for (int64_t k = 0; k < nbt.len; k++) {
                    int32_t u = nbt.ids[k];
                    if (u >= rc->ignore_from || u >= n) continue;  /* ghosts are never in the worklist */
                    if (!in_w[u]) continue;
                    if (T[u] == T[v] && key_greater(&rc->keys, u, v)) {
                        lost[v] = 1;
                        break;
                    }
                }
            }
            free(nbt.ids);
        }
        /* commit winners, losers form the next worklist */
        {
            list_t next = {0};
            for (int64_t i = 0; i < W.len; i++) {
                int32_t v = W.ids[i];
                if (lost[v]) {
                    list_push(&next, v);
                } else {
                    colors[v] = T[v];
                    in_w[v] = 0;
                }
            }
            free(W.ids);
            W = next;
        }
    }
    free(T);
    free(in_w);
    free(lost);
    free(W.ids);
    return r;
}

/* Fills the keys of ids [0, m): gid (identity when gid is NULL), p from the
 * hash or from prio, and with recolorDegrees (reading R7) the degrees: for
 * ids below n_rows the length of their row in (deg_ptr), for the others
 * extra_deg[id - n_rows].  Returns the arrays to free through *owned. */
static keys_t make_keys(int32_t m, const int32_t *gid, uint32_t seed, const uint32_t *prio,
                        int degrees, const int32_t *deg_ptr, int32_t n_rows, const int32_t *extra_deg)
{
    keys_t k;
    size_t cnt = (size_t)(m > 0 ? m : 1);
    uint32_t *p = (uint32_t *)malloc(cnt * sizeof(uint32_t));
    uint32_t *g = (uint32_t *)malloc(cnt * sizeof(uint32_t));
    int64_t *d = NULL;
    for (int32_t v = 0; v < m; v++) {
        g[v] = gid ? (uint32_t)gid[v] : (uint32_t)v;
        p[v] = prio ? prio[v] : orc_priority(g[v], seed);
    }
    if (degrees) {
        d = (int64_t *)malloc(cnt * sizeof(int64_t));
        for (int32_t v = 0; v < m; v++)
            d[v] = v < n_rows ? (int64_t)deg_ptr[v + 1] - deg_ptr[v] : (int64_t)extra_deg[v - n_rows];
    }
    k.p = p;
    k.gid = g;
    k.deg = d;
    return k;
}

static void free_keys(keys_t *k)
{
    free((void *)k->p);
    free((void *)k->gid);
    free((void *)k->deg);
}

static void finish_stats(orc_stats *st, const int32_t *colors, int32_t n, int32_t rounds)
{
    if (!st) return;
    int32_t mx = 0;
    for (int32_t v = 0; v < n; v++)
        if (colors[v] > mx) mx = colors[v];
    st->num_colors = mx;
    st->rounds = rounds;
}

static int color_common(const graph_t *g, uint32_t seed, const uint32_t *prio,
                        const int32_t *init, int32_t max_rounds, int32_t *colors, orc_stats *st,
                        int flags)
{
    int32_t n = g->n;
    /* the degree of a vertex being colored: its adjacency row (D1, D2) or
     * its column's rows (PD2) */
    const int32_t *deg_ptr = g->kind == 3 ? g->col_ptr : g->row_ptr;
    rounds_t rc;
    int32_t rounds;
    if (st) memset(st, 0, sizeof(*st));
    rc.keys = make_keys(n, NULL, seed, prio, flags & ORC_RECOLOR_DEGREES, deg_ptr, n, NULL);
    for (int32_t v = 0; v < n; v++) colors[v] = init ? init[v] : 0;
    rc.g = g;
    rc.n = n;
    rc.n_base = n;
    rc.ghost_col = NULL;
    rc.ignore_from = n;
    rc.max_rounds = max_rounds > 0 ? max_rounds : INT32_MAX;
    rc.eligible = NULL;
    rounds = run_rounds(&rc, colors, st, 0);
    finish_stats(st, colors, n, rounds);
    free_keys(&rc.keys);
    for (int32_t v = 0; v < n; v++)
        if (colors[v] == 0) return 1;   /* round cap reached: partial state */
    return 0;
}

int orc_color_d1(int32_t n, const int32_t *row_ptr, const int32_t *col, uint32_t seed,
                 const uint32_t *prio, const int32_t *init, int32_t max_rounds,
                 int32_t *colors, orc_stats *st, int flags)
{
    graph_t g = {1, n, row_ptr, col, NULL, NULL};
    return color_common(&g, seed, prio, init, max_rounds, colors, st, flags);
}

int orc_color_d2(int32_t n, const int32_t *row_ptr, const int32_t *col, uint32_t seed,
                 const uint32_t *prio, const int32_t *init, int32_t max_rounds,
                 int32_t *colors, orc_stats *st, int flags)
{
    graph_t g = {2, n, row_ptr, col, NULL, NULL};
    return color_common(&g, seed, prio, init, max_rounds, colors, st, flags);
}

int orc_color_pd2(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                  const int32_t *col_ptr, const int32_t *row_idx, uint32_t seed,
                  const uint32_t *prio, const int32_t *init, int32_t max_rounds,
                  int32_t *col_colors, orc_stats *st, int flags)
{
    (void)n_rows;
    graph_t g = {3, n_cols, row_ptr, col_idx, col_ptr, row_idx};
    return color_common(&g, seed, prio, init, max_rounds, col_colors, st, flags);
}

/* One rank's step of Algorithm 2 for distance-1 (reading R6).  init_owned
 * (nullable) holds committed owned colors to start from (a later iteration
 * of Algorithm 2's loop: phase 1 then only colors the owned vertices init
 * leaves at 0). */
int orc_color_d1_ghost(int32_t n_owned, int32_t n_ghost, int32_t layers, int32_t n_g1,
                       const int32_t *row_ptr, const int32_t *col, const int32_t *gid,
                       const int32_t *ghost_colors, uint32_t seed, const int32_t *init_owned,
                       const int32_t *ghost_degree, int32_t *owned_colors,
                       unsigned char *remote_loser, orc_stats *st, int flags)
{
    int32_t m = n_owned + n_ghost;
    unsigned char *loser = (unsigned char *)calloc((size_t)(n_owned > 0 ? n_owned : 1), 1);
    unsigned char *glose = (unsigned char *)calloc((size_t)(n_ghost > 0 ? n_ghost : 1), 1);
    graph_t g = {1, n_owned, row_ptr, col, NULL, NULL};
    rounds_t rc;
    int32_t r1, r3;
    /* second-layer rows are read only with tentative ghost recoloring
     * (reading R8); with fixed ghost colors they cannot change the result */
    if (st) memset(st, 0, sizeof(*st));
    /* an owned vertex's row holds all its edges; a ghost's degree comes from
     * its owner */
    rc.keys = make_keys(m, gid, seed, NULL, flags & ORC_RECOLOR_DEGREES, row_ptr, n_owned, ghost_degree);
    for (int32_t v = 0; v < n_owned; v++) owned_colors[v] = init_owned ? init_owned[v] : 0;
    if (remote_loser)
        for (int32_t j = 0; j < n_ghost; j++) remote_loser[j] = 0;

    /* phase 1: ghost-blind rounds on the owned-induced subgraph: the owned
     * rows without their ghost entries (a vertex's visit reads only its
     * owned neighbours) */
    {
        int32_t *rp1 = (int32_t *)calloc((size_t)n_owned + 1, sizeof(int32_t));
        int32_t *col1;
        int32_t k1 = 0;
        graph_t g1;
        for (int32_t v = 0; v < n_owned; v++)
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                if (col[e] < n_owned) rp1[v + 1]++;
        for (int32_t v = 0; v < n_owned; v++) rp1[v + 1] += rp1[v];
        col1 = (int32_t *)malloc((size_t)(rp1[n_owned] > 0 ? rp1[n_owned] : 1) * sizeof(int32_t));
        for (int32_t v = 0; v < n_owned; v++)
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                if (col[e] < n_owned) col1[k1++] = col[e];
        g1.kind = 1;
        g1.n = n_owned;
        g1.row_ptr = rp1;
        g1.col = col1;
        g1.col_ptr = NULL;
        g1.row_idx = NULL;
        rc.g = &g1;
        rc.n = n_owned;
        rc.n_base = n_owned;
        rc.ghost_col = ghost_colors;
        rc.ignore_from = n_owned;
        rc.max_rounds = INT32_MAX;
        rc.eligible = NULL;
        r1 = run_rounds(&rc, owned_colors, st, 0);
        free(rp1);
        free(col1);
    }
    rc.g = &g;

    /* phase 2: every owned-ghost edge against the fixed ghost colors, all
     * pairs judged on the phase-1 colors (Algorithm 3 with Algorithm 4) */
    for (int32_t v = 0; v < n_owned; v++) {
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            int32_t u = col[e];
            if (u < n_owned) continue;
            if (owned_colors[v] != ghost_colors[u - n_owned]) continue;
            if (st) st->boundary_conflicts++;
            if (key_greater(&rc.keys, u, v))
                loser[v] = 1;
            else
                glose[u - n_owned] = 1;
        }
    }
    for (int32_t v = 0; v < n_owned; v++)
        if (loser[v]) owned_colors[v] = 0;
    if (remote_loser)
        for (int32_t j = 0; j < n_ghost; j++) remote_loser[j] = glose[j];

    if (!(flags & ORC_GHOST_RECOLOR)) {
        /* phase 3: recolor the losers; ghosts are constraints with fixed colors */
        rc.ignore_from = m;
        r3 = run_rounds(&rc, owned_colors, st, r1);
    } else {
        /* phase 3 with tentative ghost recoloring (reading R8): the local
         * graph over all m ids; rows of owned vertices (and with two layers
         * of layer-1 ghosts) as given, with one layer a ghost's row lists the
         * owned vertices adjacent to it */
        int32_t rows = layers == 2 ? n_owned + n_g1 : n_owned;
        int32_t *rp3 = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
        int32_t *col3;
        int32_t *local = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
        unsigned char *elig = (unsigned char *)calloc((size_t)(m > 0 ? m : 1), 1);
        graph_t g3;
        rounds_t rc3;
        int64_t nnz3 = row_ptr[rows];
        for (int32_t v = 0; v < rows; v++) rp3[v + 1] = row_ptr[v + 1] - row_ptr[v];
        if (layers == 1) {
            for (int32_t v = 0; v < n_owned; v++)
                for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                    if (col[e] >= n_owned) { rp3[col[e] + 1]++; nnz3++; }
        }
        for (int32_t v = 0; v < m; v++) rp3[v + 1] += rp3[v];
        col3 = (int32_t *)malloc((size_t)(nnz3 > 0 ? nnz3 : 1) * sizeof(int32_t));
        {
            int32_t *fill = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
            for (int32_t v = 0; v < m; v++) fill[v] = rp3[v];
            for (int32_t v = 0; v < rows; v++)
                for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) col3[fill[v]++] = col[e];
            if (layers == 1)
                for (int32_t v = 0; v < n_owned; v++)
                    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; e++)
                        if (col[e] >= n_owned) col3[fill[col[e]]++] = v;
            free(fill);
        }
        /* colors of the local graph: owned as committed (losers 0), ghosts
         * as received, except the ghosts that lost phase 2 (0); the worklist
         * is the owned losers and the losing ghosts */
        for (int32_t v = 0; v < n_owned; v++) {
            local[v] = owned_colors[v];
            elig[v] = loser[v];
        }
        for (int32_t j = 0; j < n_ghost; j++) {
            local[n_owned + j] = glose[j] ? 0 : ghost_colors[j];
            elig[n_owned + j] = glose[j];
        }
        g3.kind = 1;
        g3.n = m;
        g3.row_ptr = rp3;
        g3.col = col3;
        g3.col_ptr = NULL;
        g3.row_idx = NULL;
        rc3 = rc;
        rc3.g = &g3;
        rc3.n = m;
        rc3.n_base = m;
        rc3.ghost_col = NULL;
        rc3.ignore_from = m;
        rc3.eligible = elig;
        r3 = run_rounds(&rc3, local, st, r1);
        for (int32_t v = 0; v < n_owned; v++) owned_colors[v] = local[v];   /* ghosts restored: dropped */
        free(rp3);
        free(col3);
        free(local);
        free(elig);
    }

    finish_stats(st, owned_colors, n_owned, r1 + r3);
    if (st && remote_loser) {
        for (int32_t j = 0; j < n_ghost; j++) st->remote_losers += remote_loser[j];
    }
    free_keys(&rc.keys);
    free(loser);
    free(glose);
    return 0;
}

/* One rank's step for distance-2 (kind 2) or partial distance-2 (kind 3)
 * coloring (reading R9).  D2: hop-1 and hop-2 arrays are one local CSR whose
 * rows are the owned vertices then the first ghost layer; PD2: hop 1 is the
 * owned columns' rows (col_ptr, row_idx: local row ids), hop 2 the local
 * rows' columns (row_ptr, col_idx: local column ids, owned first, then
 * ghosts).  The first n_owned local ids are owned, the next n_ghost ghosts. */
int orc_color_d2_ghost(int kind, int32_t n_owned, int32_t n_ghost, const int32_t *hop1_ptr,
                       const int32_t *hop1_idx, const int32_t *hop2_ptr, const int32_t *hop2_idx,
                       const int32_t *gid, const int32_t *ghost_colors, uint32_t seed,
                       int32_t *owned_colors, unsigned char *remote_loser, orc_stats *st, int flags)
{
    int32_t m = n_owned + n_ghost;
    unsigned char *loser = (unsigned char *)calloc((size_t)(n_owned > 0 ? n_owned : 1), 1);
    unsigned char *glose = (unsigned char *)calloc((size_t)(n_ghost > 0 ? n_ghost : 1), 1);
    int32_t *none = (int32_t *)calloc((size_t)(n_ghost > 0 ? n_ghost : 1), sizeof(int32_t));
    int32_t *seen = (int32_t *)malloc((size_t)(n_ghost > 0 ? n_ghost : 1) * sizeof(int32_t));
    graph_t g;
    rounds_t rc;
    list_t nb = {0};
    int32_t r1, r3;
    if (kind == 2) {
        g.kind = 2;
        g.row_ptr = hop1_ptr;
        g.col = hop1_idx;
        g.col_ptr = NULL;
        g.row_idx = NULL;
    } else {
        g.kind = 3;
        g.row_ptr = hop2_ptr;
        g.col = hop2_idx;
        g.col_ptr = hop1_ptr;
        g.row_idx = hop1_idx;
    }
    g.n = n_owned;
    if (st) memset(st, 0, sizeof(*st));
    /* an owned vertex's degree: its hop-1 row; degrees of ghosts are not
     * used by this step */
    rc.keys = make_keys(m, gid, seed, NULL, 0, hop1_ptr, n_owned, NULL);
    for (int32_t v = 0; v < n_owned; v++) owned_colors[v] = 0;
    (void)flags;

    /* phase 1: owned vertices only; ghosts are walked through but
     * uncolored (color 0 constrains nothing; ghosts never join a worklist) */
    rc.g = &g;
    rc.n = n_owned;
    rc.n_base = n_owned;
    rc.ghost_col = none;
    rc.ignore_from = m;
    rc.max_rounds = INT32_MAX;
    rc.eligible = NULL;
    r1 = run_rounds(&rc, owned_colors, st, 0);

    /* phase 2: every distinct ghost of every owned vertex's two-hop
     * neighbourhood against the ghosts' fixed colors, judged all at once */
    for (int32_t j = 0; j < n_ghost; j++) seen[j] = -1;
    for (int32_t v = 0; v < n_owned; v++) {
        neighbourhood(&g, v, &nb);
        for (int64_t i = 0; i < nb.len; i++) {
            int32_t x = nb.ids[i];
            if (x < n_owned || seen[x - n_owned] == v) continue;
            seen[x - n_owned] = v;
            if (owned_colors[v] != ghost_colors[x - n_owned]) continue;
            if (st) st->boundary_conflicts++;
            if (key_greater(&rc.keys, x, v))
                loser[v] = 1;
            else
                glose[x - n_owned] = 1;
        }
    }
    for (int32_t v = 0; v < n_owned; v++)
        if (loser[v]) owned_colors[v] = 0;
    if (remote_loser)
        for (int32_t j = 0; j < n_ghost; j++) remote_loser[j] = glose[j];

    /* phase 3: recolor the losers; ghosts are constraints with fixed colors */
    rc.ghost_col = ghost_colors;
    r3 = run_rounds(&rc, owned_colors, st, r1);

    finish_stats(st, owned_colors, n_owned, r1 + r3);
    if (st && remote_loser)
        for (int32_t j = 0; j < n_ghost; j++) st->remote_losers += remote_loser[j];
    free_keys(&rc.keys);
    free(loser);
    free(glose);
    free(none);
    free(seen);
    free(nb.ids);
    return 0;
}

/* Algorithm 1: serial greedy in the given order. */
void orc_serial_greedy(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const int32_t *order, int32_t *colors)
{
    graph_t g = {1, n, row_ptr, col, NULL, NULL};
    list_t nb = {0};
    for (int32_t v = 0; v < n; v++) colors[v] = 0;
    for (int32_t i = 0; i < n; i++) {
        int32_t v = order[i];
        neighbourhood(&g, v, &nb);
        colors[v] = first_fit(&nb, colors, n, NULL, n);
    }
    free(nb.ids);
}
