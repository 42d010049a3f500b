/*
 * sfmm.h -- C ABI of libsfmm.so, the MI355X (gfx950) symmetric fast multipole
 * (SFMM) gravity solve with adaptive cubic-spline softening.
 *
 * Method: Bernard, David-Cleris, Price & Lau, "Momentum-conserving
 * self-gravity in the Phantom SPH code" (arXiv 2602.05804).  One solve
 * computes, for every particle i,
 *   acc_i = -G sum_j m_j g_ij (x_i - x_j),   pot_i = -G sum_j m_j psi_ij
 * (Sect. 2, Eqs. directsum/softdirectsum) approximated as the paper's SFMM:
 *   - a tree over the particles (here a Morton binary radix tree);
 *   - node mass moments (Sect. 2.1 Eq. massmom; Appendix A.1 Eq. massmomtrans);
 *   - for every leaf, the dual tree walk of Sect. 3 (Algorithms 1 and 2): the
 *     multipole acceptance criterion on the opening angle plus the softening
 *     criterion on R_kern * max(h_max); accepted node pairs become Cartesian
 *     M2L interactions (Sect. 2.2, Eq. dmkdeffmm) on the leaf's ancestors,
 *     rejected leaf pairs become direct softened particle pairs (P2P);
 *   - the ancestors' field moments are carried down the leaf's branch with
 *     the translation of Appendix A.2 (Eq. gravmtranslat) and evaluated at
 *     the particles (L2P).
 * Every node-node interaction is pairwise, so linear momentum is conserved
 * to rounding (Newton's third law).
 *
 * Conventions shared by every entry point:
 *   - Particle arrays are DEVICE pointers in the caller's order:
 *       x   [n][3] row-major FP64 positions,
 *       m   [n]    FP64 masses (> 0),
 *       h   [n]    FP64 softening lengths (> 0; kernel support R_kern * h),
 *       acc [n][3] FP64 accelerations (written),
 *       pot [n]    FP64 potentials (written).
 *     The caller owns them; the library never frees or keeps them past a call.
 *   - The context owns its workspace (tree, lists, expansions).  The
 *     workspace only grows, is reused by later solves and is released by
 *     sfmm_destroy.
 *   - Work is enqueued on the context's HIP stream.  sfmm_solve synchronises
 *     that stream at a few points (to size the tree, the interaction lists
 *     and the P2P work items) and returns once the results are enqueued; they
 *     are valid after the next synchronisation of the stream.
 *   - Errors are returned as negative sfmm_status values; no C++ exception
 *     crosses this boundary.  After an error the outputs are undefined.
 *   - A context may be used by one host thread at a time.
 */
#ifndef SFMM_H
#define SFMM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfmm_ctx sfmm_ctx;

typedef enum {
  SFMM_OK = 0,
  SFMM_EINVAL = -1,       /* bad argument (sizes, pointers, theta, config)          */
  SFMM_ENOMEM = -2,       /* device allocation failed                               */
  SFMM_EDEVICE = -3,      /* a HIP call failed                                      */
  SFMM_EUNSUPPORTED = -4, /* expansion order or precision not built in              */
  SFMM_ENONFINITE = -5    /* a position is not finite, or m <= 0, or h <= 0         */
} sfmm_status;

/* SFMM_FP64   every step in FP64.
 * SFMM_FP32C  tree geometry, moments, the L2L chain, L2P and all sums in
 *             FP64; the M2L contractions of targets at depth >= fp64_top_depth
 *             and the P2P pair terms in FP32 (pair separations formed from
 *             FP32 leaf-relative offsets plus the FP32-rounded FP64 difference
 *             of the two leaf centres, so each pair stays antisymmetric), each
 *             term added into an FP64 accumulator. */
typedef enum { SFMM_FP64 = 0, SFMM_FP32C = 1 } sfmm_precision;

/* How the interaction lists are found (both give every leaf the same pairs):
 * SFMM_WALK_LEVEL  each (ancestor, source) test is made once, level by level
 *                  from the root, and every leaf's list is the union of its
 *                  ancestors' lists (default);
 * SFMM_WALK_LEAF   Algorithm 1 literally: every leaf walks from (root, root)
 *                  with its own stack. */
typedef enum { SFMM_WALK_LEVEL = 0, SFMM_WALK_LEAF = 1 } sfmm_walk_mode;

/* How the far field is evaluated (the same interaction set either way):
 * SFMM_FAR_LEAF    Sect. 3: every leaf evaluates the M2L lists of all its
 *                  ancestors itself while it carries the field moments down
 *                  its branch, so an ancestor's interactions are recomputed
 *                  once per leaf below it;
 * SFMM_FAR_SHARED  the caching of shared long-range interactions proposed in
 *                  Sect. 5 (Discussion): each node's M2L list is evaluated
 *                  once into the node's own field moments, and every leaf
 *                  then only translates and sums them down its branch
 *                  (L2L) before L2P.  Results agree with SFMM_FAR_LEAF to
 *                  rounding (the per-node sums are formed before they are
 *                  added to the translated parent moments).  Needs
 *                  SFMM_WALK_LEVEL.  Default; with SFMM_WALK_LEAF the
 *                  context falls back to SFMM_FAR_LEAF.
 * SFMM_FAR_MUTUAL  as SFMM_FAR_SHARED, with each unordered node pair of the
 *                  interaction set evaluated once: one derivative tensor
 *                  D(r) for both nodes, the contraction for the second node
 *                  using D(-r) = (-1)^|k| D(r) (the symmetric one-sided M2L
 *                  the paper's Sect. 5 points to, after Dehnen 2002) and
 *                  added to that node's coefficients with atomic adds, so
 *                  the summation order is not fixed (results agree with
 *                  SFMM_FAR_SHARED to rounding).  FP64 only
 *                  (SFMM_EUNSUPPORTED with SFMM_FP32C); needs
 *                  SFMM_WALK_LEVEL (falls back to SFMM_FAR_LEAF otherwise). */
typedef enum { SFMM_FAR_LEAF = 0, SFMM_FAR_SHARED = 1, SFMM_FAR_MUTUAL = 2 } sfmm_far_mode;

typedef struct {
  double G;                   /* gravitational constant (default 1)                   */
  int leaf_size;              /* a node with <= leaf_size particles is a leaf (10)    */
  double r_kern;              /* kernel support radius in units of h (2, cubic spline) */
  int include_self_potential; /* add -G m_i psi(0, h_i) to pot_i (1)                  */
  int check_inputs;           /* validate m, h and positions on the device (1)        */
  int walk_mode;              /* sfmm_walk_mode (SFMM_WALK_LEVEL)                     */
  int fp64_top_depth;         /* SFMM_FP32C: M2L on targets above this depth in FP64 (8) */
  int far_mode;               /* sfmm_far_mode (SFMM_FAR_SHARED)                      */
  int far_kernel;             /* far-field kernel shape: 0 is the only one            */
  int near_kernel;            /* P2P kernel shape: 0, 1, 6, 7 or 13 (0)               */
} sfmm_config;
/* P2P kernel shapes (same results up to summation order; sfmm_create returns
 * SFMM_EINVAL for any other value, and for far_kernel != 0):
 *   0  a wave per work item, the targets in scalar registers, wave-uniform
 *      loop control, the pairs inside a kernel queued per target and
 *      evaluated 64 at a time; passes of 5 targets at four waves per SIMD
 *      (leaf_size <= 10), of 6 at four (leaf_size <= 16) or of 8 at three
 *      (leaf_size <= 32);
 *   13 the targets of a leaf in lanes, in stripes over sources staged through
 *      LDS, source leaves split into near and far by the target leaf's sphere
 *      (leaf_size <= 32; faster on the polytrope, slower on a Plummer halo);
 *   6  a wave per work item with the targets in LDS, passes of 5 (8 for
 *      leaf_size > 10), the queue shared by the pass; in SFMM_FP32C the same
 *      layout with the softened branch taken in the pass;
 *   7  SFMM_FP32C only: shape 0 with each sum kept as a TwoSum pair of FP32
 *      words instead of an FP64 accumulator (in FP64, shape 0);
 *   1  one thread per particle (also every leaf_size > 32; SFMM_FP32C needs
 *      leaf_size <= 16).
 * The far field has one shape per mode: 8 lanes per node (SFMM_FAR_SHARED,
 * two waves per SIMD in FP64, one in FP32C), 4 lanes per leaf (SFMM_FAR_LEAF). */

/* Solve statistics of the last sfmm_solve on a context (host copy). */
typedef struct {
  int64_t n;                /* particles                                            */
  int64_t num_nodes;        /* tree nodes (internal + leaves)                       */
  int64_t num_leaves;
  int32_t max_depth;        /* depth of the deepest leaf (root = 0)                 */
  int64_t n_m2l;            /* M2L evaluations, replication over leaves included    */
  int64_t n_l2l;            /* L2L translations carried out down the branches       */
  int64_t n_p2p_leaf_pairs; /* P2P list entries: (target leaf, source) with the source
                               a leaf, or (level walk) a whole subtree that lies
                               inside the target's kernel reach                     */
  int64_t n_p2p_pairs;      /* ordered particle pairs summed directly               */
  double momentum[3];       /* sum_i m_i acc_i (FP64), valid after a stream sync    */
  double momentum_abs;      /* sum_i |m_i acc_i|                                    */
  int64_t n_m2l_unique;     /* distinct (target node, source node) M2L pairs (level
                               walk; 0 with SFMM_WALK_LEAF)                         */
  int64_t n_p2p_soft_pairs; /* ordered particle pairs inside a softening kernel
                               (counted by the default P2P kernel shape of either
                               precision; 0 for the other shapes)                  */
  int32_t walk_attempts;    /* level walks the solve made: 1, plus one more each
                               time the list pools had to grow                     */
  int32_t leaf_slot_m2l;    /* level walk: per-leaf M2L and P2P list slots of the   */
  int32_t leaf_slot_p2p;    /* last walk (entries)                                  */
  int64_t n_leaf_overflow;  /* leaves whose lists did not fit those slots (walked a
                               second time)                                         */
  int64_t max_leaf_m2l;     /* longest M2L list and longest P2P list of a leaf      */
  int64_t max_leaf_p2p;
} sfmm_stats;

/* Fill *cfg with the defaults listed above.  Returns SFMM_EINVAL if cfg is NULL. */
int sfmm_config_default(sfmm_config* cfg);

/* Create a context on HIP device `device` that enqueues its work on
 * `hip_stream` (a hipStream_t; NULL = the default stream).  cfg may be NULL
 * (defaults).  On success *out owns nothing yet; the first build allocates.
 * Environment read here (measurement and tests; SFMM_EINVAL for a bad value):
 *   SFMM_NEAR_VARIANT=v  P2P kernel shape v instead of cfg->near_kernel;
 *   SFMM_OVERLAP=0|1|2   run the P2P kernel on a second stream of the
 *                        context beside the far field (1: P2P queued first,
 *                        2: far field first; 0, the default: one stream);
 *   SFMM_LEAF_SLOTS=m,p[,i]  first per-leaf M2L / P2P list slots of the
 *                        level walk (1..1024 / 1..512) and, optionally, the
 *                        internal nodes' region slots (1..4096); later walks
 *                        adapt them to the lists they meet;
 *   SFMM_CHECK_POOLS=1   clear the list pools before each walk and check
 *                        every list entry after it;
 *   SFMM_POOL_INIT=k     start the list pools at k entries. */
int sfmm_create(sfmm_ctx** out, int device, void* hip_stream, const sfmm_config* cfg);

/* Release every device buffer of the context; ctx may be NULL. */
int sfmm_destroy(sfmm_ctx* ctx);

/* Change the stream later calls enqueue on.  Work enqueued afterwards waits
 * (on the device, through an event) for the work already queued on the
 * previous stream, since both use the context's workspace. */
int sfmm_set_stream(sfmm_ctx* ctx, void* hip_stream);

/* Build the tree of (x, m, h): Morton keys, radix sort, binary radix tree,
 * node geometry (centre of mass, size, h_max) and mass moments up to
 * `order` (Sect. 2.1 Eq. massmom via Appendix A.1 Eq. massmomtrans).
 * n == 0 is a no-op.  Errors: SFMM_EINVAL (n < 0, NULL pointer with n > 0,
 * n >= 2^30, order outside 0..4), SFMM_ENONFINITE (check_inputs set and an
 * input is invalid), SFMM_ENOMEM, SFMM_EDEVICE. */
int sfmm_build(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
               int order);

/* Build, walk and evaluate: acc and pot for every particle (see the header
 * comment).  theta is the critical opening angle (0 < theta < 1), order the
 * expansion order p (0..4; p = 3 is the tuned one), precision SFMM_FP64 or
 * SFMM_FP32C (sfmm_precision).
 * n == 0: OK, nothing written.  n == 1: acc = 0, pot = self term only.
 * Errors: as sfmm_build, plus SFMM_EINVAL for theta outside (0, 1) or a
 * NULL acc/pot with n > 0, SFMM_EUNSUPPORTED for an unknown precision. */
int sfmm_solve(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
               double theta, int order, int precision, double* acc, double* pot);

/* Solve k independent systems together (the packed launch of the serving
 * loop).  System s owns particles [offsets[s], offsets[s+1]) of the
 * concatenated device arrays x, m, h, acc, pot; offsets is a HOST array of
 * k+1 non-decreasing values starting at 0.  Every phase runs once for the
 * whole set: the keys are sorted by (system, key, position), no tree node over
 * two systems becomes a leaf or is walked, and each system's walk starts at
 * its own root.  Each system therefore gets the tree, interaction lists and
 * results it would get alone: bit for bit in SFMM_FP64; in SFMM_FP32C the
 * fp64_top_depth levels count from the root of the whole set, so a packed
 * system may run a few more of its top levels in FP64 than alone (results
 * within the FP32C bound).  Momentum is conserved per system.  Needs
 * SFMM_WALK_LEVEL.  Errors: as sfmm_solve, plus SFMM_EINVAL
 * for k < 1 or bad offsets, SFMM_EUNSUPPORTED with SFMM_WALK_LEAF. */
int sfmm_solve_batch(sfmm_ctx* ctx, int k, const int64_t* offsets, const double* x,
                     const double* m, const double* h, double theta, int order, int precision,
                     double* acc, double* pot);

/* Copy the statistics of the last solve (synchronises the stream). */
int sfmm_get_stats(sfmm_ctx* ctx, sfmm_stats* out);

/* ---- introspection (parity tests): HOST output buffers ----------------
 * Valid after sfmm_build/sfmm_solve; each call synchronises the stream.
 * sfmm_get_tree: perm [n] (sorted position -> caller index), keys [n],
 *   per node lo/cnt (particle range in sorted order), child (index of the
 *   left child, the right one follows it; -1 for a leaf), parent (-1 for the
 *   root), geometry s [nn][3], mass, l (size), hmax, and the moments
 *   Q [nn][ncoef] (ncoef = (p+1)(p+2)(p+3)/6, graded order: degree, then
 *   the x exponent descending, then the y exponent descending).  Any output
 *   pointer may be NULL.  Node 0 is the root. */
int sfmm_get_tree(sfmm_ctx* ctx, int64_t* num_nodes, int64_t* num_leaves, int32_t* perm,
                  uint64_t* keys, int32_t* lo, int32_t* cnt, int32_t* child, int32_t* parent,
                  double* s, double* mass, double* l, double* hmax, double* Q);
/* Leaf node ids in Morton order and their depths (arrays of num_leaves). */
int sfmm_get_leaves(sfmm_ctx* ctx, int32_t* leaf_node, int32_t* leaf_depth);
/* Interaction lists of the last solve for leaf index `leaf` (0..num_leaves-1):
 * M2L entries as (depth of the target ancestor, source node), grouped by
 * depth, and P2P source leaves.  Returns the counts in *n_m2l / *n_p2p and
 * copies at most cap_m2l / cap_p2p entries. */
int sfmm_get_leaf_lists(sfmm_ctx* ctx, int64_t leaf, int32_t* m2l_depth, int32_t* m2l_src,
                        int64_t cap_m2l, int64_t* n_m2l, int32_t* p2p_src, int64_t cap_p2p,
                        int64_t* n_p2p);

/* ---- phase timing --------------------------------------------------------
 * Phases of one solve, in order: 0 tree (keys, sort, tree, geometry,
 * moments), 1 walk (SFMM_WALK_LEVEL: all of it; SFMM_WALK_LEAF: the count
 * pass), 2 walk fill pass (SFMM_WALK_LEAF only), 3 far field (M2L + L2L +
 * L2P), 4 near field (P2P + output), 5 momentum reduction; 6 is the main
 * P2P kernel alone (inside phase 4, without the work-item set-up and the
 * reduction of the partial sums).  Between
 * sfmm_timing_start and sfmm_timing_stop each solve records a pair of HIP
 * events around every phase on the context's stream (no extra
 * synchronisation).  sfmm_timing_stop synchronises, writes the durations in
 * milliseconds to ms[k * SFMM_NUM_PHASES + phase] for the first
 * min(recorded, cap) solves, stores the number recorded in *nsolves and
 * frees the events.  Solves beyond max_solves are not timed. */
#define SFMM_NUM_PHASES 7
int sfmm_timing_start(sfmm_ctx* ctx, int max_solves);
int sfmm_timing_stop(sfmm_ctx* ctx, double* ms, int cap, int* nsolves);
const char* sfmm_phase_name(int phase);

/* Device bytes the context holds (its workspace), for footprint models. */
int sfmm_workspace_bytes(const sfmm_ctx* ctx, uint64_t* out);

/* One leapfrog update of a system on `hip_stream` (device arrays [n][3]):
 * v += kick * acc, then x += drift * v.  A kick-drift-kick step of length dt
 * is (dt/2, dt) before the solve and (dt/2, 0) after it; consecutive steps
 * merge the two half kicks into (dt, dt).  Used by the serving loop, which
 * evolves each request for a few steps. */
int sfmm_leapfrog(void* hip_stream, int64_t n, double* x, double* v, const double* acc,
                  double kick, double drift);

/* The softened direct sum of Sect. 2, Eq. softdirectsum, over all n sources
 * (x, m, h as in sfmm_solve; the context's G, include_self_potential and
 * stream), for nt targets: targets is a DEVICE array of nt particle indices
 * in [0, n), or NULL for 0..nt-1.  acc [nt][3] and pot [nt] are written in
 * target order.  O(n nt) work: the reference the SFMM approximates, for
 * accuracy studies.  Errors: SFMM_EINVAL (sizes, NULL arrays, a target index
 * outside [0, n), found on the device; the call then synchronises). */
int sfmm_direct(sfmm_ctx* ctx, int64_t n, const double* x, const double* m, const double* h,
                int64_t nt, const int64_t* targets, double* acc, double* pot);

/* sfmm_direct without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same kernels and arguments as sfmm_direct; the
 * status word and the partial sums of the source chunks live in a fixed
 * 32 MiB device array of the library, one per GPU, held until the process
 * ends.  Limit: nt <= 1048568 targets per call (SFMM_EINVAL beyond; every
 * other error as sfmm_direct).  Every call on a GPU uses that GPU's array and
 * clears what must start at zero: calls that overlap on one GPU (two host
 * threads, or two streams) race and must be ordered by the caller.  The call
 * synchronises the context's stream to read the status word back. */
int sfmm_direct_noalloc(sfmm_ctx* ctx, int64_t n, const double* x, const double* m,
                        const double* h, int64_t nt, const int64_t* targets, double* acc,
                        double* pot);

/* Human-readable text of a status code (static storage). */
const char* sfmm_strerror(int status);

/* Text of the last error on this context (empty when none). */
const char* sfmm_last_error(const sfmm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
