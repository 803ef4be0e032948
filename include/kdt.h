/*
 * kdt.h -- C-ABI of the kinetic Delaunay library (libkdt.so) for MI355X.
 *
 * The method (Hadiniya & Ghodsi, "A parallel algorithm for Delaunay
 * triangulation of moving points on the plane"): the point set is split into
 * blocks (Sec. III, "Data structure"; Sec. IV), every block keeps the Delaunay
 * triangulation of its points, and at every time step a chosen point of every
 * block moves in one of four directions (Lemma 1, Sec. V); each block then
 * deletes the point from its triangulation and inserts it at its new place
 * (Fig. 4; Sec. IV, "Insertion and Deletion"), all blocks in parallel.
 *
 * The triangulation kept is DT*: the Delaunay triangulation made unique on
 * cocircular input by lifting every point by an infinitesimal that grows
 * with its global id (Sec. I states uniqueness, which lattice input needs
 * this rule for).  Collinear points on the hull are vertices.
 *
 * Conventions for every call:
 *  - Coordinates are int32 lattice points in [0, 2^24).
 *  - A point's global id is its row in the xy array given to kdt_init.
 *    Block b owns the ids block_off[b] .. block_off[b+1]-1 (points grouped
 *    by block), and its frame is the half-open rectangle
 *    [x0, x1) x [y0, y1) from frames[4b .. 4b+3] = (x0, y0, x1, y1).
 *  - Directions: 0 = +x (right), 1 = -x (left), 2 = +y (up), 3 = -y (down).
 *  - Move rule: within a block the moves of one step apply one after the
 *    other in the order given; a move jumps the point `dist` >= 1 lattice
 *    units; it is BLOCKED (a no-op, counted apart) if the target lies
 *    outside the block's frame or on a cell held by a point of the block.
 *  - "dev" marks a device pointer, "host" a host pointer.  The caller owns
 *    every buffer it passes; the library never allocates or frees device
 *    memory: all device state lives in the caller's workspace.
 *  - One context = one stream = one host thread.  Calls that launch work
 *    are asynchronous on that stream; errors raised by kernels are sticky
 *    and surface at kdt_sync, kdt_query* and kdt_stats.
 *  - Status: 0 KDT_OK, negative KDT_E_* on error.  Nothing aborts and no
 *    C++ exception crosses this interface.
 */
#ifndef KDT_H
#define KDT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KDT_OK 0
#define KDT_BLOCKED 1       /* per-move status: the move rule blocked the move (a no-op, not an error) */
#define KDT_E_ARG (-1)      /* bad argument (null pointer, size, index, dir, dist) */
#define KDT_E_RANGE (-2)    /* coordinate outside [0, 2^24) or outside its frame */
#define KDT_E_DUP (-3)      /* two points of a block on one lattice cell */
#define KDT_E_DEGEN (-4)    /* a block with fewer than 4 points, or all collinear */
#define KDT_E_CAPACITY (-5) /* workspace too small, or a local limit exceeded */
#define KDT_E_DEVICE (-6)   /* HIP runtime error */
#define KDT_E_STATE (-7)    /* call out of order (e.g. use after an error) */
#define KDT_E_INTERNAL (-8) /* a device-side invariant check failed */

/* One move (Sec. III, "movepoint"; Lemma 1 of Sec. V: one of four
 * directions): `point` is the LOCAL index of the point in its block
 * (global id - block_off[block]) -- the same convention for every per-block
 * call (kdt_move, kdt_moves, kdt_run); the block is implied by where the
 * record sits in a step's per-block offsets (kdt_run) or given beside it
 * (kdt_move, kdt_moves).  The global mode (kdt_run_global) takes global ids,
 * since it has one block.  16 bytes. */
typedef struct kdt_move_s {
    int32_t point;
    int32_t dir;
    int32_t dist;
    int32_t pad;
} kdt_move_t;

/* Counters accumulated on the device since kdt_init (read by kdt_stats). */
typedef struct kdt_stats_t {
    int64_t applied;      /* moves applied (delete + reinsert done) */
    int64_t blocked;      /* moves blocked by the move rule */
    int64_t star_sum;     /* sum over applied moves of the moved point's degree */
    int64_t cavity_sum;   /* sum of Bowyer-Watson cavity sizes (triangles) */
    int64_t walk_sum;     /* sum of visibility-walk steps */
    int64_t tri_touched;  /* triangle records read or written */
    int64_t alg_bytes;    /* algorithmic HBM bytes of the repair (see DESIGN) */
    int64_t errors;       /* blocks stopped by an error */
    /* time the blocks' wavefronts spent per phase of applied moves, in
     * ticks of the device wall clock (clock_khz ticks per millisecond):
     * gathering the star, locating the target, retriangulating the hole,
     * inserting (cavity and fan) */
    int64_t t_star, t_locate, t_hole, t_insert;
    int64_t clock_khz;
    /* applied moves by the time one move took: bucket b counts moves of
     * [2^b, 2^(b+1)) wall-clock ticks */
    int64_t hist[16];
    /* applied moves whose target lay inside the moved point's star and
     * destroyed no triangle around it (the star polygon alone changed) */
    int64_t fast;
    int64_t rebuilt;  /* block steps done by the rebuild branch */
    int64_t flipped;  /* moves done by move-and-flip (kdt_set_repair) */
    int64_t flips;    /* edge flips of those moves */
} kdt_stats_t;

typedef struct kdt_ctx kdt_ctx;

/* Library-side partition (Sec. III, "Data structure"; Sec. IV,
 * Quad-treeDvision): the smallest square covering the points -- lower-left
 * corner at the coordinate minima, side rounded up to a power of two so
 * that halving keeps lattice cells whole -- is cut into four equal squares,
 * recursively.
 *   KDT_PART_GRID      param = partition count P, a power of four (1 .. 4^12):
 *                      every square cut log4(P) times; blocks = the cells
 *                      that hold a point, row by row (y, then x)
 *   KDT_PART_QUADTREE  param = threshold (>= 4): a square holding more than
 *                      `param` points is cut into its four quarters, quarters
 *                      holding no point are dropped; a square whose cut would
 *                      leave a quarter with fewer than 4 points or all of
 *                      them on one line stays whole (a block needs a
 *                      triangulation); blocks = the leaves, depth first,
 *                      quarters in the order (low x, low y), (high x, low y),
 *                      (low x, high y), (high x, high y)
 * Input: xy host int32 [n][2] in [0, 2^24), distinct.  Output (host):
 *   perm       int64 [n]: row i of the partitioned set is input point
 *              perm[i]; a block's points keep their input order
 *   block_off  int64 [cap_blocks + 1], frames int32 [cap_blocks][4]: the
 *              arguments kdt_init takes (a frame is the block's square,
 *              half-open, clipped to [0, 2^24))
 *   n_blocks   the number of blocks (written even when it exceeds
 *              cap_blocks: then KDT_E_CAPACITY and nothing else is written)
 * KDT_E_RANGE / KDT_E_DUP for bad points, KDT_E_ARG for a bad scheme or
 * param.  Pure host computation; no context needed. */
#define KDT_PART_GRID 0
#define KDT_PART_QUADTREE 1
int kdt_partition(const int32_t* xy, int64_t n, int32_t scheme, int64_t param, int64_t* perm,
                  int64_t* block_off, int32_t* frames, int32_t cap_blocks, int32_t* n_blocks);

/* Size in bytes of the device workspace kdt_init needs for n points in
 * n_blocks blocks with the given host block offsets (n_blocks + 1 entries,
 * block_off[0] = 0, block_off[n_blocks] = n) and room to stage up to
 * max_staged moves per step through kdt_move.  Pure host computation. */
int kdt_workspace_size(int64_t n, int32_t n_blocks, const int64_t* block_off,
                       int32_t max_staged, size_t* dev_bytes);

/* Create a context and build every block's DT* on the device (paper's
 * starting state: a dataset that satisfies the Delaunay constraints, Fig. 4).
 *   xy         host int32 [n][2]
 *   block_off  host int64 [n_blocks + 1]
 *   frames     host int32 [n_blocks][4], or NULL for [0, 2^24)^2 everywhere
 *   dev_ws     dev workspace of ws_bytes >= kdt_workspace_size(...) bytes,
 *              256-byte aligned, owned by the caller, must outlive the ctx
 *   stream     hipStream_t to run on (NULL: the null stream)
 * Validation is done on the host first: RANGE, DUP, DEGEN, ARG, CAPACITY. */
int kdt_init(kdt_ctx** out, const int32_t* xy, int64_t n, int32_t n_blocks,
             const int64_t* block_off, const int32_t* frames, int32_t max_staged,
             void* dev_ws, size_t ws_bytes, void* stream);

/* Stage one move of the current step (host call; nothing runs yet): block
 * i's chosen point (Sec. III, "movepoint_i") jumps `dist` >= 1 lattice units
 * in direction `dir` (Lemma 1, Sec. V).  `point` is the point's LOCAL index
 * in `block` (0 .. size - 1), as in kdt_move_t.  KDT_E_ARG for a bad block,
 * point, dir or dist; KDT_E_CAPACITY when max_staged moves are staged. */
int kdt_move(kdt_ctx* ctx, int32_t block, int64_t point, int32_t dir, int32_t dist);

/* Stage `count` moves at once (host arrays): moves[i] for block blocks[i],
 * staged in array order.  status (host int32 [count] or NULL) receives
 * KDT_OK, KDT_E_ARG or KDT_E_CAPACITY per move as kdt_move would return
 * it; moves with an error are not staged.  Returns KDT_OK when all were
 * staged, else the first error. */
int kdt_moves(kdt_ctx* ctx, const int32_t* blocks, const kdt_move_t* moves, int64_t count,
              int32_t* status);

/* Apply the staged moves as one time step (one kernel launch) and clear the
 * stage.  Fig. 4: every block deletes its moved point (Delete) and inserts
 * it at its new place (Insert), all blocks in parallel.  Asynchronous. */
int kdt_step(kdt_ctx* ctx);

/* kdt_step, then wait for it and report what happened to every staged move,
 * in staging order (host int32 [number staged]): KDT_OK if the move was
 * applied, KDT_BLOCKED if the move rule blocked it (target outside the
 * block's frame, or held by a point of the block at that moment).  A
 * device error is returned (and is sticky) instead. */
int kdt_step_status(kdt_ctx* ctx, int32_t* status);

/* The main loop of Fig. 4 for n_steps time steps (every block deletes and
 * reinserts its moved points, Sec. IV), from a move stream already in
 * device memory:
 *   moves     dev kdt_move_t [M]
 *   step_off  dev int32 [n_steps][n_blocks + 1]: the moves of step t for
 *             block b are moves[step_off[t][b] .. step_off[t][b+1]-1]
 *   applied   dev int8 [M] or NULL: 1 if the move was applied, 0 if blocked
 *   flags     KDT_RUN_* below
 * KDT_RUN_PER_STEP (0) launches one kernel per step.  KDT_RUN_FUSED runs
 * all steps of a block in one persistent launch; blocks are independent, so
 * the result is the same.  A move beyond the repair path's fixed capacities
 * (a point of degree above 64, or a cavity or write-back table larger than
 * its on-chip arrays) changes nothing and sends its block through the
 * rebuild branch for the rest of the step (same result, slower); only a
 * block with more than 256 moves left in that step then fails with
 * KDT_E_CAPACITY. */
#define KDT_RUN_PER_STEP 0
#define KDT_RUN_FUSED 1
#define KDT_RUN_PERSISTENT 2
/* KDT_RUN_PERSISTENT launches, per step, a fixed grid of workgroups (a few
 * per compute unit, see kdt_set_launch) that share the blocks sorted by
 * size, largest first, each workgroup taking ranks alternately from the
 * large and the small end of every round, so blocks of uneven size share the
 * machine evenly.  All three forms give identical results. */
int kdt_run(kdt_ctx* ctx, const kdt_move_t* moves, const int32_t* step_off,
            int32_t n_steps, int8_t* applied, int32_t flags);

/* Workgroups per compute unit of the persistent launch (1..64, default 4;
 * the LDS of an MI355X compute unit holds 5 step workgroups). */
int kdt_set_launch(kdt_ctx* ctx, int32_t persist_per_cu);

/* Repair variant of the per-block modes.
 *   KDT_REPAIR_DELINS (default)  every move deletes the point and inserts it
 *              at its new place (Fig. 4; Sec. IV, "Insertion and Deletion")
 *   KDT_REPAIR_FLIP  move-and-flip, the other update De Berg et al. give for
 *              points moving in discrete steps (Sec. II): when the new place
 *              lies strictly inside the kernel of the point's star (the point
 *              not on the hull, every triangle of its star still
 *              counter-clockwise with the point there), the point moves in
 *              place and Lawson flips with the perturbed incircle test make
 *              the triangulation Delaunay again; other moves delete and
 *              insert.  Same DT*, different work (kdt_stats: flipped,
 *              flips).
 * KDT_E_ARG for another value, KDT_E_STATE in global mode. */
#define KDT_REPAIR_DELINS 0
#define KDT_REPAIR_FLIP 1
int kdt_set_repair(kdt_ctx* ctx, int32_t variant);

/* Staging depth of the star prefetch (a tuning knob, not a semantic one):
 * before a block's moves of a step run one after another, its wavefront
 * walks the stars of all the step's movers at once, reading and dropping
 * the records, so that the moves find them in cache: depth 0 off, 1 (the
 * default) the star and the triangle beyond each link edge, 2 also the
 * triangles beyond those; the positions and move records are touched too.
 * Same results at every depth.  KDT_E_ARG for a depth outside 0..2. */
int kdt_set_prefetch(kdt_ctx* ctx, int32_t depth);

/* Wavefronts per block of the per-step launch (KDT_RUN_PER_STEP): 1
 * (default: one wavefront applies the block's moves one after another), 2
 * or 4.  With more than one, the wavefronts of a block's workgroup share
 * its moves (Fig. 4, Update/Delete/Insert per block; several moves per
 * block at once, as many moves per step allow): the moves whose source and
 * target cells no other move of the block's step names commute with every
 * move, and run in reservation rounds -- each wavefront plans one without
 * writing, claims every triangle its plan read, and the plans whose claims
 * no lower move index contests are written; the others plan again -- and
 * the remaining moves (sharing a cell with another, beyond the rounds'
 * capacities -- a plan keeps at most 50 records in its wavefront's table,
 * a quarter of the sequential path's, so that more workgroups share a
 * compute unit -- or of a block taking the rebuild branch, or all of a
 * block with more than 64 moves in the step or whose step moves some point
 * more than once) follow one after another in list order, in a second
 * launch.  Same triangulations and
 * applied flags as one wavefront.  The per-step log then records, for a
 * block, the rounds' ticks; the rest launch logs blocks all of whose moves
 * it ran.  KDT_E_ARG for another count, KDT_E_STATE in global mode. */
int kdt_set_block_waves(kdt_ctx* ctx, int32_t waves);

/* Schedule of the per-step launch (KDT_RUN_PER_STEP; tuning only, the
 * results are the same).  order = 1: every step, a small kernel sorts the
 * blocks by their number of moves in the step, most first, and the step's
 * workgroups take them in that order, so that the blocks that set the
 * step's length start first (a step lasts as long as its slowest block).
 * heavy_cut > 0 (needs order = 1, and matters with kdt_set_block_waves
 * above 1): size classes -- only the blocks with at least heavy_cut moves
 * in the step get the several-wavefront workgroups, on a second stream of
 * the context, while the one-wavefront kernel takes the others at the same
 * time on the context's stream; the rest launch follows both.  mid_cut in
 * 1 .. heavy_cut - 1 (with four wavefronts per block): a middle class --
 * the blocks with mid_cut .. heavy_cut - 1 moves get two-wavefront
 * workgroups on a third stream, at the same time.  Default order 0,
 * heavy_cut 0, mid_cut 0.  KDT_E_ARG for order outside {0, 1}, a negative
 * cut, heavy_cut > 0 with order 0, or mid_cut > 0 without
 * 0 < mid_cut < heavy_cut; KDT_E_STATE in global mode. */
int kdt_set_block_order(kdt_ctx* ctx, int32_t order, int32_t heavy_cut, int32_t mid_cut);

/* The same n_steps steps captured once as a HIP graph and replayed by
 * kdt_graph_launch (each replay applies the same move stream again, from the
 * state it finds).  The context's stream must not be the null stream.  The
 * graph records the given pointers: the move stream and `applied` must stay
 * valid while the graph lives.  It also records the policy, the log and the
 * launch shape of the moment: after kdt_set_policy, kdt_set_log or
 * kdt_set_launch, kdt_graph_launch returns KDT_E_STATE (build the graph
 * again); a replay writes the log rows of the steps it captured again.
 * kdt_graph_destroy releases it. */
typedef struct kdt_graph kdt_graph;
int kdt_graph_build(kdt_ctx* ctx, const kdt_move_t* moves, const int32_t* step_off,
                    int32_t n_steps, int8_t* applied, int32_t flags, kdt_graph** out);
int kdt_graph_launch(kdt_ctx* ctx, kdt_graph* graph);
void kdt_graph_destroy(kdt_graph* graph);

/* Query the current triangulation -- "return dataset(t)" of Fig. 4, the DT
 * after the time step (Sec. III: only the triangulation after a step is
 * valid) -- (synchronises the stream).
 *   tris      dev int32 [cap][3]: real triangles as global ids,
 *             counter-clockwise, each rotated to start at its smallest id,
 *             grouped by block
 *   adj       dev int32 [cap][3] or NULL: adj[t][j] is the index (in this
 *             output) of the triangle across the edge opposite vertex j,
 *             -1 on the convex hull of the block
 *   blk_off   host int64 [n_blocks + 1] or NULL: block b's triangles are
 *             rows blk_off[b] .. blk_off[b+1]-1
 *   n_tri     host: number of triangles (written even if > cap, then
 *             KDT_E_CAPACITY is returned and nothing else is written) */
int kdt_query(kdt_ctx* ctx, int32_t* tris, int32_t* adj, int64_t* blk_off,
              int64_t cap, int64_t* n_tri);

/* Same triangles in canonical order (rows sorted lexicographically) written
 * to a HOST buffer int32 [cap][3]; used to compare with a reference. */
int kdt_query_canonical(kdt_ctx* ctx, int32_t* host_tris, int64_t cap, int64_t* n_tri);

/* Triangles of the listed blocks only (Fig. 4, "return dataset(t)", per
 * block), canonical, written to HOST buffers; synchronises.
 *   blocks     host int32 [count], distinct block indices (global mode: {0})
 *   host_tris  host int32 [cap][3]: block blocks[i]'s real triangles in rows
 *              host_off[i] .. host_off[i+1]-1, global ids, counter-clockwise,
 *              each rotated to start at its smallest id, rows of a block
 *              sorted lexicographically
 *   host_adj   host int32 [cap][3] or NULL: the row (in host_tris) of the
 *              triangle across the edge opposite column j's vertex, -1 on
 *              the block's convex hull
 *   host_off   host int64 [count + 1] (written even when the triangles do
 *              not fit: then KDT_E_CAPACITY and nothing else is written)
 * KDT_E_ARG for an empty list, an index out of range or a repeated block.
 * Blocks are independent: after a block failed (its error is sticky for the
 * context), the others can still be queried; listing the failed block
 * returns its error. */
int kdt_query_blocks(kdt_ctx* ctx, const int32_t* blocks, int32_t count, int32_t* host_tris,
                     int32_t* host_adj, int64_t cap, int64_t* host_off);

/* Order-independent 64-bit digest of every block's triangulation (host
 * uint64 [n_blocks]; synchronises): the wrapping sum over its real triangles,
 * each rotated to start at its smallest global id (a, b, c), of
 * M(a ^ M(b ^ M(c))) with M the splitmix64 finaliser
 * (z += 0x9E3779B97F4A7C15; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
 *  z = (z ^ z>>27) * 0x94D049BB133111EB; z ^ z>>31).  Equal triangulations
 * give equal digests; used to compare runs cheaply. */
int kdt_digest(kdt_ctx* ctx, uint64_t* host_per_block);

/* d-calculation (Sec. III, "Notation and definitions"; Sec. IV; Sec. V):
 * for the current positions and a constant N (1 .. 8), the squared distance
 * of every point to its N-th nearest neighbour among the points of its
 * block (the blocks are independent), and its minimum over the block --
 * mindistance(P_i)^2 -- written to host_mind2 (host int64 [n_blocks] or
 * NULL; INT64_MAX for a block of at most N points); the block's squared
 * diameter to host_diam2 (host int64 [n_blocks] or NULL); the minimum over
 * all blocks, mindistance(P_t)^2, to *d2_now (taken on the device, one
 * atomic minimum per block: the paper's tree minimum); d^2, the minimum of
 * mindistance(P_t)^2 over the calls made with this N, to *d2_min; and every
 * block's N-spread diam(P_i) / mindistance(P_t), kept at its largest over
 * those calls, to host_spread (host double [n_blocks] or NULL).  A new N
 * starts a new history.  Every comparison is of exact integer squared
 * distances.  Synchronises.  KDT_E_ARG for N outside 1 .. 8; KDT_E_CAPACITY
 * when a point's search needs more than 64 candidates (a vertex of very
 * high degree). */
int kdt_dcalc(kdt_ctx* ctx, int32_t N, int64_t* host_mind2, int64_t* host_diam2, int64_t* d2_now,
              int64_t* d2_min, double* host_spread);

/* Current positions: host int32 [n][2] (synchronises). */
int kdt_positions(kdt_ctx* ctx, int32_t* host_xy);

/* Sum of the per-block counters (synchronises). */
int kdt_stats(kdt_ctx* ctx, kdt_stats_t* out);

/* Per-block status (synchronises): host int32 [n_blocks], 0 or KDT_E_*. */
int kdt_block_status(kdt_ctx* ctx, int32_t* host_status);

/* Kernel timing.  With enable = P > 0, kdt_run and kdt_step record HIP
 * event pairs on the context's stream, each spanning a run of P consecutive
 * time-step launches (P = 1: one pair around every launch; a pair costs the
 * stream a few microseconds, so a larger P disturbs the steps less and
 * measures the stream's time per launch, gaps between launches included);
 * kdt_timing_read closes a run cut short, waits for the pairs and returns
 * their summed time (ms) and the number of launches they span since timing
 * was last enabled.  Recording stops (and the pairs are released) when
 * enable == 0; enable < 0 is KDT_E_ARG. */
int kdt_timing(kdt_ctx* ctx, int32_t enable);
int kdt_timing_read(kdt_ctx* ctx, double* total_ms, int64_t* launches);

/* Repair or rebuild.  The paper's trade-off (Sec. I): points that move far
 * are better served by rebuilding the triangulation than by updating it.
 * Per block and time step the policy picks one branch; both end in the same
 * DT* (it is unique), so the policy changes only the time taken.
 *   REPAIR     delete + insert every move (default)
 *   REBUILD    apply the moves to the positions (same move rule), then
 *              rebuild the block's DT* from scratch (Bowyer-Watson)
 *   THRESHOLD  rebuild iff sum over the block's moves of dist / spacing > tau,
 *              spacing = sqrt(frame area / points)
 *   MLP        rebuild iff the network's predicted log2 cost of rebuilding is
 *              below that of repairing; mlp_w: dev float [KDT_MLP_PARAMS],
 *              must stay valid while used
 *   DLIMIT     rebuild iff some move of the block goes farther than tau * d,
 *              d the paper's limited distance (Sec. III: points are assumed
 *              to move at most d per step, else rebuilding is better) as the
 *              latest kdt_dcalc left it; repair while no kdt_dcalc was made
 * A block with more than 256 moves in one step is repaired whatever the
 * policy (the rebuild branch checks at most 256 moves per block and step).
 * The network: 16 features -> 32 ReLU -> 32 ReLU -> 2, parameters laid out
 * as W1[32][16], b1[32], W2[32][32], b2[32], W3[2][32], b3[2]. */
#define KDT_POLICY_REPAIR 0
#define KDT_POLICY_REBUILD 1
#define KDT_POLICY_THRESHOLD 2
#define KDT_POLICY_MLP 3
#define KDT_POLICY_DLIMIT 4
#define KDT_MLP_PARAMS 1666
int kdt_set_policy(kdt_ctx* ctx, int32_t policy, float tau, const float* mlp_w);

/* Per step and block log (dev float [cap_steps][n_blocks][KDT_LOG_FIELDS],
 * a ring over the steps launched since this call; NULL / 0 turns it off):
 * fields 0..15 the block's features for the step (log2 n, k, log2(1+k),
 * sum d/s, log2(1+sum d/s), max d/s, log2(1+max d/s), mean d/s, #(d>s),
 * #(d>4s), 100k/n, sum (d/s)^2/k, log2(1+sum d/s)*log2(1+k), log2 s,
 * log2(1+k)/log2 n, max d / d of the latest kdt_dcalc (0 if none)), 16 branch taken (0 repair, 1 rebuild, 2 repair that
 * hit the repair path's capacity and finished the step by rebuilding: no
 * clean cost of either branch), 17 device clock ticks the branch took,
 * 18 k, 19 1 if the block's rebuild would run after the step's kernel (the
 * launch forms that defer, and a build that does not fit the step kernel's
 * LDS), else 0.  Steps without moves
 * are not logged. */
#define KDT_LOG_FIELDS 20
int kdt_set_log(kdt_ctx* ctx, float* log, int64_t cap_steps);

/* MLP kernels (FP32, hand-written; stream = hipStream_t or NULL).
 *   forward: out[n][2] = f(x[n][16])
 *   grad:    grad[0..1665] = sum over samples of d/dw 0.5*|f(x)-y|^2,
 *            grad[1666] = the summed loss (grad: dev float [1667])
 *   train:   epochs of mini-batch gradient descent on the mean gradient,
 *            w updated in place; scratch: dev float [1667] (the batch's
 *            gradient)
 * Sums over samples are taken in a fixed order -- chunks of 64 samples in
 * sample order, the chunks' sums added in chunk order -- with no atomics,
 * so the results are the same floats on every run. */
int kdt_mlp_forward(const float* w, const float* x, int64_t n, float* out, void* stream);
int kdt_mlp_grad(const float* w, const float* x, const float* y, int64_t n, float* grad, void* stream);
int kdt_mlp_train(float* w, const float* x, const float* y, int64_t n, int32_t epochs, int32_t batch,
                  float lr, float* scratch, void* stream);

/* kdt_mlp_train for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same training with no scratch argument and no allocation
 * of any kind.  Its working memory is a fixed array inside the library,
 * ~449 KB per GPU, held by each GPU it runs on until the process ends: the
 * sums of every chunk of 64 samples of a batch (one workgroup per chunk, so
 * a batch spreads over the GPU) and the batch's gradient.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (two streams,
 * two threads) race.  Nothing in it needs clearing: every call writes what
 * it reads.  The weights are the same floats kdt_mlp_train gives (the sums
 * are added in the same order).  Arguments as for kdt_mlp_train; the stream
 * must belong to the current device.  KDT_E_CAPACITY when batch exceeds
 * KDT_MLP_NOALLOC_BATCH, KDT_E_ARG for a bad argument. */
#define KDT_MLP_NOALLOC_BATCH 4096
int kdt_mlp_train_noalloc(float* w, const float* x, const float* y, int64_t n, int32_t epochs, int32_t batch,
                          float lr, void* stream);

/* ---- Global mode: one DT* over every point ------------------------------
 * The paper lets a moved point leave its block and be sent to the
 * neighbouring block that now holds it (Sec. IV, Fig. 4), with at most one
 * such hand-over per block and step (Theorem 1, Sec. V).  Here the blocks
 * are the 2^depth cells of a kd partition of the initial points (median
 * splits, x first: a node's first half by (x, y) at even levels, (y, x) at
 * odd levels goes left, and a position goes right iff its key is not below
 * the key of the first right point), and every point belongs to the cell
 * that holds its current position.  The triangulation is one DT* of all
 * points in the domain, with ghosts on the global hull.
 *
 * Move rule: the moves of a step apply one after the other in list order; a
 * move is blocked when its target lies outside the domain or on a cell held
 * by any point at that moment.  Moves with no cell in common with another
 * move of the step run concurrently (reservation rounds on the triangles
 * their plans read); the others, and moves still contended after the
 * rounds, run afterwards in list order; a step that moves some point more
 * than once runs wholly in list order.  The triangulation after each step
 * is DT* of the positions the sequential rule gives.
 *
 * Query, digest, positions, stats and sync work as for one block holding
 * every point (kdt_stats: n_blocks = 1); the per-block move calls return
 * KDT_E_STATE on a global context. */

/* Workspace of a global context: n points (4 .. 2^22), 2^depth kd cells
 * (0 <= depth <= 20, 2^depth <= n), at most max_moves moves per step. */
int kdt_workspace_size_global(int64_t n, int32_t depth, int32_t max_moves, size_t* dev_bytes);

/* Build the global DT* on the device (all threads of the GPU insert points
 * at once; Sec. IV, "Insertion").  xy: host int32 [n][2], distinct, not all
 * collinear, inside domain = host int32 [4] (x0, y0, x1, y1), a half-open
 * rectangle in [0, 2^24).  Errors as for kdt_init. */
int kdt_init_global(kdt_ctx** out, const int32_t* xy, int64_t n, int32_t depth, const int32_t* domain,
                    int32_t max_moves, void* dev_ws, size_t ws_bytes, void* stream);

/* The global mode with the paper's own partition (Sec. III, "Data
 * structure"; Fig. 2, 3): the cells are the leaves of a quad-tree of the
 * initial points -- the root is the smallest power-of-two square at the
 * domain's lower-left corner covering the domain; a square holding more than
 * `threshold` points is cut into its four quarters (empty ones kept, so the
 * leaves tile the root) -- and every leaf is linked to the node across each
 * of its four sides (equal or larger).  A moved point that leaves its cell
 * is handed to the block holding its new place ("new-block", Fig. 4): found
 * through the direct link on the side it moved across when the neighbour
 * holds it (O(1), Sec. V after Theorem 1), else down from the root
 * (O(log4 B), Theorem 1); kdt_global_stats counts both (KDT_GSTAT_LINK,
 * KDT_GSTAT_TREE).  The tree is the initial points' unless re-partitioned
 * (kdt_repartition, kdt_set_repartition).
 * Arguments and errors as for kdt_workspace_size_global / kdt_init_global,
 * with threshold >= 1 in place of depth; the workspace size needs the
 * points (the tree's size depends on them).  kdt_owner returns the leaf's
 * node index (kdt_quadtree). */
int kdt_workspace_size_global_qt(const int32_t* xy, int64_t n, const int32_t* domain, int64_t threshold,
                                 int32_t max_moves, size_t* dev_bytes);
int kdt_init_global_qt(kdt_ctx** out, const int32_t* xy, int64_t n, const int32_t* domain, int64_t threshold,
                       int32_t max_moves, void* dev_ws, size_t ws_bytes, void* stream);

/* The quad-tree of a context made by kdt_init_global_qt (host; KDT_E_STATE
 * otherwise): host_nodes int32 [cap][8], node k = (x0, y0, side, first of
 * its four children or -1 for a leaf, then for a leaf the node across its
 * +x, -x, +y and -y sides or -1 at the root's border, -1 for inner nodes);
 * node 0 is the root; the children of a node are its quarters (low x low y,
 * high x low y, low x high y, high x high y).  *n_nodes is written even
 * when it exceeds cap (then KDT_E_CAPACITY and nothing else). */
int kdt_quadtree(kdt_ctx* ctx, int32_t* host_nodes, int32_t cap, int32_t* n_nodes);

/* Quad-treeDvision of the current positions (Fig. 4, step 5: the partition
 * is made again for the dataset of every time step): the quad-tree is
 * computed from scratch on the device -- the same definition as at init,
 * with the nodes numbered breadth first -- with its links, and every
 * point's cell is its new leaf.  Synchronises (the host waits for each
 * level's count of cut cells).  KDT_E_STATE unless made by
 * kdt_init_global_qt; KDT_E_CAPACITY if the tree outgrows its arrays
 * (cannot happen for points in the domain).
 * kdt_set_repartition(ctx, 1) makes kdt_run_global re-partition after
 * every step, 0 stops it. */
int kdt_repartition(kdt_ctx* ctx);
int kdt_set_repartition(kdt_ctx* ctx, int32_t every_step);

/* Run n_steps steps.  moves: dev kdt_move_t [*] with point = global id;
 * step_off: HOST int64 [n_steps + 1], step t = moves step_off[t] ..
 * step_off[t+1]-1 (at most max_moves).  applied: dev int8 indexed like
 * moves (1 applied, 0 blocked) or NULL.  Asynchronous. */
int kdt_run_global(kdt_ctx* ctx, const kdt_move_t* moves, const int64_t* step_off, int32_t n_steps,
                   int8_t* applied);

/* The same n_steps global steps captured once as a HIP graph (replayed by
 * kdt_graph_launch, released by kdt_graph_destroy, as for kdt_graph_build):
 * the step's nine launches without the host between them.  Arguments as for
 * kdt_run_global; the move stream's pointers and step sizes are recorded.
 * KDT_E_STATE for the null stream, a context not in global mode, or one
 * that re-partitions after every step (kdt_set_repartition: that
 * synchronises); a graph captured before a later kdt_set_repartition is
 * refused by kdt_graph_launch (KDT_E_STATE). */
int kdt_graph_build_global(kdt_ctx* ctx, const kdt_move_t* moves, const int64_t* step_off, int32_t n_steps,
                           int8_t* applied, kdt_graph** out);

/* Rebuild the whole DT* from scratch from the current positions with the
 * device builder (the full-rebuild alternative the paper weighs against
 * updating, Sec. I).  Synchronises. */
int kdt_rebuild_global(kdt_ctx* ctx);

/* kd cell of every point's current position: host int32 [n]. */
int kdt_owner(kdt_ctx* ctx, int32_t* host_owner);

/* Counters of the global mode: host uint64 [KDT_GSTAT_N]. */
#define KDT_GSTAT_INTERACTING 0  /* moves sharing a cell with another move of their step */
#define KDT_GSTAT_SERIAL 1       /* moves run by the ordered pass */
#define KDT_GSTAT_LOST 2         /* plans that lost a claim (retried or passed on) */
#define KDT_GSTAT_TRANSFERS 3    /* applied moves that changed the point's kd cell */
#define KDT_GSTAT_OVERFLOW 4     /* plans too large for a reservation (ordered pass) */
#define KDT_GSTAT_BUILD_ROUNDS 5 /* reservation rounds of the builds so far */
#define KDT_GSTAT_LINK 6         /* quad-tree cells: transfers whose new cell came through a direct link */
#define KDT_GSTAT_TREE 7         /* quad-tree cells: transfers whose new cell came down from the root */
#define KDT_GSTAT_N 8
int kdt_global_stats(kdt_ctx* ctx, uint64_t* host_counters);

/* Wait for the stream; return the first sticky error, or KDT_OK. */
int kdt_sync(kdt_ctx* ctx);

/* Release the context (not the workspace, which the caller owns). */
void kdt_destroy(kdt_ctx* ctx);

/* Text for a status code. */
const char* kdt_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* KDT_H */
