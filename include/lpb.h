/*
 * lpb.h -- C ABI of the MI355X layered-media linearized Poisson-Boltzmann
 * (screened Coulomb) fast multipole library.
 *
 * Problem (Wang, Zhang, Cai, "Fast Multipole Method for 3-D Linearized
 * Poisson-Boltzmann Equation in Layered Media", Sec. 2): layers l = 0..L
 * stacked top to bottom, interfaces z = d_0 > d_1 > ... > d_{L-1}; layer l
 * has dielectric constant eps_l > 0 and inverse Debye length lambda_l > 0.
 * For charges Q_j at r_j strictly inside the layers, the library returns
 *
 *   Phi(r_i) = sum_{j != i, same layer} Q_j e^{-lambda_l |r_i-r_j|} / (4 pi eps_l |r_i-r_j|)
 *            + sum_{all j} Q_j u^react_{l l'}(r_i, r_j)                       (eq. potential1)
 *
 * where u^react is the reaction part of the layered Green's function
 * (eqs. layeredGreensfun, reactioncomponent).  The free-space part is a
 * Yukawa FMM per layer; every reaction component (l, l', a, b) is an FMM over
 * equivalent polarization sources (Sec. 3.3-3.5, Algorithms 1 and 2).
 *
 * Conventions
 *  - Every function returns lpb_status (0 = LPB_OK, < 0 = error) except
 *    lpb_last_error / lpb_destroy / lpb_default_options.  No exception or
 *    abort crosses the ABI; on error the message is available from
 *    lpb_last_error(ctx) until the next call on that context.
 *  - Pointers marked "host or device" may be either; the flag `on_device`
 *    tells which (1 = device memory of the context's GPU, 0 = host memory).
 *    The caller owns every array it passes and the library never frees it.
 *  - A context belongs to one GPU and one HIP stream (lpb_options.stream,
 *    NULL = the null stream).  An evaluation forks two internal streams of
 *    the context (default priority) from it, for the untiled V-list
 *    translations and the free-space near field, and joins them back on it
 *    before its last kernel, so all of its work is ordered on the caller's
 *    stream.  Calls on one context are not thread-safe.
 *  - Call order: lpb_set_layers, then lpb_build_tree, then lpb_evaluate
 *    (repeatable with new charges).  Calling lpb_set_layers again rebuilds
 *    the plan for the stored charge positions; lpb_build_tree again replaces
 *    them.  Anything else returns LPB_ESTATE.
 *  - Precision: LPB_FP64 runs every stage in double precision.  LPB_MIXED
 *    runs P2M/M2M/M2L/L2L/L2P/P2P in single precision with double-precision
 *    Bessel ratios and double-precision operator generation (quadrature,
 *    recurrence, translation coefficients); the output is double in both.
 */
#ifndef LPB_H
#define LPB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lpb_ctx lpb_ctx;

typedef enum {
    LPB_OK = 0,
    LPB_EINVAL = -1,   /* bad argument (null pointer, size, non-monotone interfaces, eps/lambda <= 0) */
    LPB_ERANGE = -2,   /* charge on or too close to an interface, p or leaf_cap out of range */
    LPB_ENOMEM = -3,   /* device or host allocation failed */
    LPB_EDEVICE = -4,  /* HIP runtime error */
    LPB_ESTATE = -5,   /* wrong call order */
    LPB_ENUMERIC = -6  /* NaN/Inf input, quadrature budget exceeded, recurrence stability bound violated */
} lpb_status;

typedef enum { LPB_FP64 = 0, LPB_MIXED = 1 } lpb_precision;

#define LPB_MAX_P 20        /* largest order in mixed precision */
#define LPB_MAX_P_FP64 15   /* largest order in FP64: the matrix-core translation kernels stage a
                               64-column FP64 operand slab per block in LDS, (p+1)^2 rows padded to
                               16, and above p = 15 that exceeds the 160 KiB of one workgroup */
#define LPB_MAX_LAYERS 9

typedef struct {
    int p;                  /* expansion order: degrees n = 0..p (1 <= p <= LPB_MAX_P in mixed precision,
                               1 <= p <= LPB_MAX_P_FP64 in FP64); default 10 */
    int leaf_cap;           /* target mean charges per leaf (tree depth rule, see lpb_build_tree); default 50 */
    int precision;          /* lpb_precision; default LPB_FP64 */
    double quad_tol;        /* relative cut of the Sommerfeld quadrature envelope; default 1e-16 */
    double iface_tol;       /* minimum distance of a charge from an interface; default 1e-9 */
    int device;             /* HIP device ordinal; default 0 */
    void* stream;           /* hipStream_t for all work; NULL = null stream */
    int stages;             /* diagnostics: bit 0 far field (P2M..L2P), bit 1 near field; default 3 (both) */
    int timing;             /* 1 = record stream events between stages (lpb_stats.t_stage_ms); default 0 */
    int graph;              /* 1 = capture the evaluation passes in a HIP graph on the first evaluate after
                               a tree or operator change and replay it; ignored while timing = 1 (the
                               per-stage events need the passes launched one by one); default 1 */
    int autotune;           /* 1 = time the candidate block-to-work schedules of the matrix-core M2L
                               kernels on the first evaluate after a change and keep the fastest
                               (results do not depend on the choice); 2 = also time the per-offset form
                               of the tiled M2L against the reflection-orbit form (mixed precision,
                               5 <= p <= 15: the two round differently, so results then depend on the
                               choice, within the mixed-precision error); default 1 */
    int schedule;           /* with autotune = 0, the schedules to use: tile | batch << 4, with the codes of
                               lpb_stats.tile_schedule (0..15) and batch_schedule (0..7); default 0 */
    /* Device-memory hook (e.g. a framework's caching allocator).  When alloc is
     * not NULL, every device buffer the context holds (tables, tree, lists,
     * expansions, operators, partial potentials) comes from
     * alloc(bytes, alloc_user), which must return memory of the context's GPU
     * aligned to at least 256 bytes, or NULL when it cannot (the call then
     * fails with LPB_ENOMEM and the context keeps no partial state); each
     * buffer goes back through free(ptr, alloc_user) when the context drops
     * it (a rebuild of the plan or operators, lpb_destroy, or a failed
     * lpb_create).  free must be set with alloc.  Both are called on the
     * thread that calls the library, between kernels of the context's
     * stream, which is synchronized before a buffer is returned.  NULL
     * (default): hipMalloc / hipFree. */
    void* (*alloc)(size_t bytes, void* alloc_user);
    void (*free)(void* ptr, void* alloc_user);
    void* alloc_user;
    /* Tree form (Sec. 3.5, closing remarks on adaptive trees).  0 (default):
     * uniform trees, every leaf of an FMM at its depth (see lpb_build_tree).
     * 1: adaptive trees: each point set (a layer's charges; a layer side's
     * targets or equivalent polarization sources) divides a box while it holds
     * more than leaf_cap points, down to level 12, and the sets of the
     * reaction components also divide a box while it is wider than the
     * distance of its nearest point from the interface (fine cells), up to 3
     * levels below the occupancy rule (the per-box form of the uniform trees'
     * separation depth, which keeps most reaction near-field pairs away); the
     * lists add W-list pairs (a finer source box's multipole expansion
     * evaluated at a coarser leaf's targets, M2P) and X-list pairs (a coarser
     * leaf's sources formed into a finer target box's local expansion, P2L).
     * 2: adaptive trees by occupancy alone (more reaction near-field, W- and
     * X-list pairs).  Reaction M2P / P2L use point operators from the F~ and
     * L rows of eq. coefintable, whose Sommerfeld tables combine the forward
     * (eq. recurrence1) and backward (eq. backwardrecurrence1) recurrences;
     * they are generated with the translation operators (FP64) and kept, K
     * doubles per (point, box) pair.  All forms converge to the same
     * potential. */
    int adaptive;
} lpb_options;

typedef struct {
    int n_fmm;              /* free-space + reaction FMMs in the plan */
    int max_depth;          /* deepest tree level over all FMMs */
    int64_t n_m2l_pairs;    /* V-list pairs */
    int64_t n_m2l_tile_pairs; /* V-list pairs evaluated by the tiled matrix-core M2L (free space) */
    int64_t n_p2p_pairs;    /* near-field charge pairs (free + reaction) */
    int64_t n_react_p2p_pairs; /* near-field reaction pairs (each a Sommerfeld quadrature) */
    int64_t n_operators;    /* translation operators generated */
    int64_t operator_bytes; /* device bytes held by operators */
    double t_build_ms;      /* last lpb_build_tree (host tree + upload) */
    double t_opgen_ms;      /* last operator generation (GPU, FP64) */
    double t_eval_ms;       /* last lpb_evaluate, stream time between its first and last kernel */
    /* per-stage stream time of the last evaluate when options.timing = 1:
     * [0] charge gather + clears, [1] P2M, [2] M2M, [3] tiled M2L (free space),
     * [4] list M2L (reaction, deep levels) and X-list P2L, [5] L2L, [6] L2P and W-list M2P,
     * [7] free-space near field, [8] reaction near field, [9] component sum */
    double t_stage_ms[10];
    int tile_schedule;      /* schedule and form chosen for the tiled M2L: bit 0 = 0 linear, 1 blocks of one
                               XCD take a contiguous run of tiles (tiles sharing operators share that XCD's
                               L2); bit 1 = blocks of one wave per 16-row block instead of four waves
                               (per-offset form); bit 2 = the per-offset form (one product per V-list offset)
                               where the reflection-orbit form exists (mixed precision, 5 <= p <= 15; FP64
                               and other orders always use the per-offset form); bit 3 = orbit form with its
                               operator slabs in registers instead of LDS */
    int batch_schedule;     /* the choice for the batched translations (M2M, L2L, untiled M2L): bit 0 as
                               above; bits 1-2 = 0 one block per work item, k = 1..3 a grid of 256 x 2^k
                               resident blocks that loop over the items, each gathering the next item's
                               sources during the current product */
    double t_tune_ms;       /* time spent by the last schedule autotuning */
    int64_t n_m2l_tiles;    /* tiles (64 target boxes, one child octant) of the tiled M2L */
    /* units of work of each stage (the plan's counts, for work models):
     * P2M charge expansions (every source point of every source tree), L2P
     * charge evaluations (every target point of every target tree), M2M and
     * L2L child links, distinct operators of the V-list pairs outside the
     * tiled levels (their products run in the batched kernel) */
    int64_t n_p2m_points, n_l2p_points, n_m2m_links, n_l2l_links, n_m2l_list_ops;
    /* adaptive trees (options.adaptive = 1): W-list and X-list box pairs, the
     * target evaluations of the W-list pairs (M2P) and source formations of
     * the X-list pairs (P2L), and the reaction point operators among them */
    int64_t n_w_pairs, n_x_pairs, n_w_points, n_x_points, n_point_ops;
} lpb_stats;

/* Fill *opt with the defaults listed above.  Never fails. */
void lpb_default_options(lpb_options* opt);

/* Create a context on opt->device.  opt may be NULL (defaults).
 * Errors: LPB_EINVAL (out == NULL, alloc without free, schedule codes out of range), LPB_ERANGE (p outside
 * 1..LPB_MAX_P, or above LPB_MAX_P_FP64 with precision LPB_FP64; leaf_cap < 1),
 * LPB_EDEVICE, LPB_ENOMEM (the allocator refused the context's tables).  On
 * error *out is NULL and everything allocated so far has been released. */
lpb_status lpb_create(const lpb_options* opt, lpb_ctx** out);

/* Set the layered medium (Sec. 2.1): n_layers = L+1 layers (1..LPB_MAX_LAYERS),
 * eps[n_layers] > 0, lambda[n_layers] > 0, interfaces[L] strictly decreasing
 * (d_0 > d_1 > ...); all host pointers.  The reaction densities sigma^{ab}_{l l'}
 * are obtained on the GPU by solving the transmission conditions.
 * Invalidates operators (regenerated by the next evaluate). */
lpb_status lpb_set_layers(lpb_ctx* ctx, int n_layers, const double* eps, const double* lambda,
                          const double* interfaces);

/* Set the charge positions of one system (host or device, n doubles each)
 * and build the plan: the layer of every charge, the equivalent polarization
 * coordinates (eq. equivpolarcoord) of every reaction component, and uniform
 * octrees.  Free space: one tree per layer, root cube = bounding cube of the
 * layer's charges, depth = smallest level at which the layer averages at
 * most leaf_cap charges per non-empty box.  Reaction components: in the
 * frame of a component (its interface at z = 0, targets above, mirrored in z
 * when the interface is the upper one of the target layer) targets sit at
 * height +tau and equivalent sources at -tau', tau being the distance of a
 * charge to an interface of its own layer; all components of the medium
 * share one root cube (x, y centre of all charges, z centre on the
 * interface, half side = the largest tau or half x, y extent) and one depth
 * (largest per-set occupancy depth, raised by at most 3 levels until the box
 * side is no larger than the smallest tau), so each (layer, side) point set
 * has one source and one target tree shared by the components using it.
 * V-lists and U-lists as in the classic FMM.  Requires lpb_set_layers first
 * (the layer of a charge depends on the interfaces).  Errors: LPB_ERANGE if a
 * charge lies within iface_tol of an interface, LPB_ENUMERIC for NaN/Inf. */
lpb_status lpb_build_tree(lpb_ctx* ctx, int64_t n, const double* x, const double* y, const double* z, int on_device);

/* Evaluate Phi at every charge (input order) for charges q[n]; q and phi are
 * host or device memory as on_device says.  Runs Algorithm 2 on the
 * context's stream and waits for it.  Generates the translation operators
 * first if the layers or the tree changed.  phi may not alias q. */
lpb_status lpb_evaluate(lpb_ctx* ctx, const double* q, double* phi, int on_device);

/* Batched form: one context holding n_sys independent layered systems, all
 * evaluated by the same stage launches (each stage covers every FMM of every
 * system).  Set up with lpb_set_systems + lpb_build_trees (arrays of
 * per-system pointers); evaluate with lpb_evaluate_batch.  A context is
 * either single-system (set_layers/build_tree/evaluate) or batched. */
lpb_status lpb_set_systems(lpb_ctx* ctx, int n_sys, const int* n_layers, const double* const* eps,
                           const double* const* lambda, const double* const* interfaces);
lpb_status lpb_build_trees(lpb_ctx* ctx, int n_sys, const int64_t* n, const double* const* x,
                           const double* const* y, const double* const* z, int on_device);
lpb_status lpb_evaluate_batch(lpb_ctx* ctx, int n_sys, const double* const* q, double* const* phi, int on_device);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lpb_evaluate with
 * device pointers that calls no allocating routine.  q[n] and phi[n] are
 * device memory of the context's GPU, in input order; phi may not alias q.
 * The partial potentials of the output slots (n_slots * n doubles: the
 * component slots, 1 for a single layer, 3 otherwise, and one for the
 * free-space near field, so n_slots = 2 or 4) live in a
 * library-wide device array of LPB_NOALLOC_MAX_PARTS doubles (96 MiB) that
 * each GPU the library runs on holds until the process ends; every call on a
 * GPU shares that GPU's array (cleared at the start of each call), so calls
 * that overlap on one GPU (several contexts, streams or threads) race and
 * must be serialized by the caller.  The passes are launched one by one on
 * the context's stream (and its two internal streams, joined back) with the
 * schedules the context already chose (no graph instantiation, no
 * autotuning), then the call waits for the stream.
 * The context must be prepared: a single-system context on which
 * lpb_evaluate has run since the last lpb_set_layers / lpb_build_tree (that
 * call generates the operators and picks the schedules).  Results are bit
 * for bit those of lpb_evaluate.  Errors: LPB_EINVAL (null pointers, phi ==
 * q), LPB_ESTATE (not prepared, or a batched context), LPB_ERANGE (n_slots *
 * n > LPB_NOALLOC_MAX_PARTS), LPB_EDEVICE. */
#define LPB_NOALLOC_MAX_PARTS (12u << 20)
lpb_status lpb_evaluate_noalloc(lpb_ctx* ctx, const double* q, double* phi);

/* Counters and timings of the last calls.  Errors: LPB_EINVAL. */
lpb_status lpb_get_stats(const lpb_ctx* ctx, lpb_stats* stats);

/* Description of FMM number `fmm` of system `sys` in the plan (0 <= fmm < n_fmm):
 * desc[0] = kind (0 free space, 1 reaction), desc[1] = target layer l,
 * desc[2] = source layer l', desc[3] = a, desc[4] = b (0 for free space),
 * desc[5] = depth H; root[4] = centre x, y, z and half side R;
 * if tkeys/skeys are not NULL they receive, for the targets / sources of
 * that FMM in increasing charge-index order, the Morton key of their leaf at
 * level H (cell index per axis = floor((w + R) / (2R) * 2^16) clamped to
 * [0, 65535], shifted right by 16 - H, with w = x - cx, y - cy and, for free
 * space, z - cz; for a reaction component w_z = +tau (targets) or -tau'
 * (sources), and the z cell is mirrored (2^H - 1 - c) when a = 2; bits
 * interleaved x, y, z from the most significant level down); on adaptive
 * trees the key is at the leaf's own level L (in place of H) and carries L in
 * bits 58-61; *nt, *ns receive the counts.  Host memory. */
lpb_status lpb_fmm_info(const lpb_ctx* ctx, int sys, int fmm, int* desc, double* root, int64_t* nt, int64_t* ns,
                        uint64_t* tkeys, uint64_t* skeys);

/* Diagnostic: copy the partial potentials of the last evaluate to host
 * memory out[nslots * n_total] (slot k of charge i at out[k * n_total + i],
 * charges of all systems concatenated in system order; slot 0 is the
 * free-space part, slot 1 the sum of the reaction components through the
 * lower interface of the charge's layer (a = 1), slot 2 through the upper
 * one (a = 2); nslots = 1 for single-layer media).  *nslots receives the
 * slot count; out may be NULL to query it. */
lpb_status lpb_debug_parts(const lpb_ctx* ctx, double* out, int* nslots);

/* Message of the last failed call on ctx (owned by ctx).  ctx == NULL gives
 * the message of the last failed lpb_create in this thread. */
const char* lpb_last_error(const lpb_ctx* ctx);

/* Free the context and all device memory it holds.  NULL is a no-op. */
void lpb_destroy(lpb_ctx* ctx);

/* Host-side diagnostic: the Gaunt integral int Y_{n1}^{m1} Y_{n2}^{m2} Y_{n3}^{m3} dOmega
 * (harmonics Y_n^m = P^_n^m(cos t) e^{i m p}, no Condon-Shortley phase) the
 * library tabulates for its translation operators (Theorems 3.2, 3.3).
 * Runs on the host only. */
double lpb_host_gaunt(int n1, int m1, int n2, int m2, int n3, int m3);

#ifdef __cplusplus
}
#endif
#endif /* LPB_H */
