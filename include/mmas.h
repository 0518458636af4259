/*
 * mmas.h -- C ABI of the MI355X (gfx950) MAX-MIN Ant System hot path.
 *
 * The method is the GPU MAX-MIN Ant System of Skinderowicz, "Implementing a
 * GPU-based parallel MAX-MIN Ant System" (FGCS 2020): every ant builds a TSP
 * tour (Alg. 1) by repeated node selection with weighted reservoir sampling
 * (Alg. 4, Sec. 4.2.2) over the candidate list of its current node (Sec. 4.3),
 * falling back to every unvisited node when the list is exhausted, with its
 * visited set in a bitmask tabu or the compact tabu (Sec. 4.1); then the
 * iteration best deposits pheromone after evaporation, within the trail limits
 * [tau_min, tau_max] (Sec. 2.1).
 *
 * Conventions shared by every call:
 *  - Device memory: the caller owns one device buffer (the workspace, at
 *    least mmas_workspace_bytes() bytes, 256-byte aligned) and lends it to the
 *    context from mmas_create until mmas_destroy. The library allocates no
 *    device memory of its own (its one static device array serves
 *    mmas_mlp_features_noalloc).
 *  - Streams: every call enqueues on the hipStream_t given to mmas_create and
 *    returns without waiting, except where a call says it synchronises.
 *  - Errors: every call returns a status and never aborts. Kernel faults show
 *    up as MMAS_EHIP at the next synchronising call.
 *  - Determinism: one (distance matrix, parameters, seed, iteration) has
 *    exactly one result. Every random number is drawn from Philox4x32-10
 *    keyed on (seed, iteration, ant, step, slot); keys are ln(u) * (1/w) in
 *    FP32 (the reciprocal by IEEE division, computed ahead as Sec. 4.2.2
 *    suggests, then one product); equal keys go to the lowest node index. The tabu
 *    variant and the launch shape never change a result.
 *  - Threading: a context is not thread-safe; separate contexts are
 *    independent.
 */
#ifndef MMAS_H
#define MMAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mmas_status {
    MMAS_OK = 0,
    MMAS_EINVAL = -1,      /* an argument or the distance matrix is invalid */
    MMAS_EUNSUPPORTED = -2,/* valid, but outside what this library implements */
    MMAS_ENOSPACE = -3,    /* workspace smaller than mmas_workspace_bytes() */
    MMAS_EHIP = -4,        /* a HIP runtime call or a kernel failed */
    MMAS_ESTATE = -5       /* call out of order (e.g. update before construct) */
} mmas_status;

/* Tabu (visited set) of an ant in LDS, Sec. 4.1: a bitmask (n/8 bytes), the
 * compact tabu (2n bytes) or the list tabu (4n bytes); tours never depend on it. */
enum { MMAS_TABU_BITMASK = 0, MMAS_TABU_COMPACT = 1, MMAS_TABU_LIST = 2 };
enum { MMAS_PHER_DENSE = 0, MMAS_PHER_CANDIDATES = 1 };
/* Whose tour deposits in the update (Sec. 2.1): the iteration best, or the
 * global best, which the paper allows instead. */
enum { MMAS_DEPOSIT_ITERATION_BEST = 0, MMAS_DEPOSIT_GLOBAL_BEST = 1 };
/* Node selection: weighted reservoir sampling (Alg. 4, the default) or the
 * parallel roulette wheel of Sec. 4.2.1 (the paper's baseline). */
enum { MMAS_SELECT_WRS = 0, MMAS_SELECT_PRWM = 1 };
/* The problem (Sec. 2.1): the symmetric TSP, or the asymmetric TSP, whose
 * d_ij may differ from d_ji. An ATSP edge (i,j) is directed: its trail is
 * tau_ij alone, a tour's length sums d along its direction, and the deposit
 * goes to (i,j) only. */
enum { MMAS_PROBLEM_TSP = 0, MMAS_PROBLEM_ATSP = 1 };

/* Run parameters. Sec. 5 lists the paper's settings (m = n ants, alpha = 1,
 * beta = 2, p_best = 0.01); Sec. 4.3 the candidate lists. */
typedef struct mmas_params {
    int32_t n;         /* cities, 3 <= n <= 65535 (node ids fit in 16 bits, Table 1) */
    int32_t ants;      /* m >= 1 */
    int32_t cand_len;  /* candidate-list length cl, 0..64; cl >= n-1 means all other
                          cities (used as n-1); 0 means no list (every step is the
                          all-node fallback) */
    int32_t alpha;     /* pheromone exponent, integer 0..8 */
    int32_t beta;      /* heuristic exponent, integer 0..8 */
    float rho;         /* evaporation rate in (0,1): tau <- max((1-rho) tau, tau_min) */
    double p_best;     /* (0,1): probability of rebuilding the best tour once converged */
    uint64_t seed;     /* Philox key */
    int32_t tabu;      /* MMAS_TABU_BITMASK, MMAS_TABU_COMPACT or MMAS_TABU_LIST */
    int32_t pher_mode; /* MMAS_PHER_DENSE: n*n trails; MMAS_PHER_CANDIDATES: trails
                          stored only on the (i, cand[i][r]) edges, every other edge
                          held at tau_min (needs cand_len >= 1) */
    int32_t ls_nn;     /* 2-opt neighbour-list length 0..32 (the paper uses 32),
                          0 = no local search */
    int32_t deposit;   /* MMAS_DEPOSIT_ITERATION_BEST (0) or MMAS_DEPOSIT_GLOBAL_BEST */
    int32_t problem;   /* MMAS_PROBLEM_TSP (0) or MMAS_PROBLEM_ATSP; ATSP needs
                          ls_nn == 0 (2-opt reverses paths, which changes the
                          length of an asymmetric tour) */
} mmas_params;

typedef struct mmas_ctx mmas_ctx;

/* Per-context scalars kept in device memory (layout fixed; read it with
 * mmas_read(MMAS_BUF_STATE)). */
typedef struct mmas_device_state {
    float tau_min;     /* current trail limits */
    float tau_max;
    float delta;       /* deposit of the last update, 1/C_ib */
    int32_t ib_ant;    /* iteration-best ant of the last update, -1 before */
    int64_t ib_len;    /* its length, -1 before */
    int64_t gb_len;    /* global-best length, -1 while there is none */
    int64_t nn_len;    /* nearest-neighbour tour length (set-up) */
    uint32_t flags;    /* 1/2/4: distance matrix asymmetric (TSP only) / non-zero diagonal /
                          non-positive off the diagonal (set-up); 8: a
                          construction step found no city (never expected);
                          16: a 2-opt search hit its round limit (never
                          expected; that ant's tour is left as it was);
                          32: a construction wave gave up waiting for its
                          draw helper wave (never expected; that tour is
                          void) */
    uint32_t updates;  /* number of completed updates */
} mmas_device_state;

/* Views into the workspace, for mmas_buffer and mmas_read. */
enum {
    MMAS_BUF_DIST = 0,      /* int32 n*n, row-major */
    MMAS_BUF_PHEROMONE = 1, /* float n*n (dense) or n*cl (candidates; row i, rank r) */
    MMAS_BUF_CHOICE = 2,    /* float n*n, tau^alpha * eta^beta (dense only) */
    MMAS_BUF_CHC = 3,       /* float n*cl, choice_info along the candidate lists */
    MMAS_BUF_CAND = 4,      /* uint16 n*cl, candidate lists sorted by (d, index) */
    MMAS_BUF_HEUR = 5,      /* float n*n eta^beta (dense) or n*cl (candidates) */
    MMAS_BUF_TOURS = 6,     /* uint16 ants*n, tour of ant a at row a */
    MMAS_BUF_LENGTHS = 7,   /* int64 ants, closing edge included */
    MMAS_BUF_GB_TOUR = 8,   /* uint16 n */
    MMAS_BUF_NN_TOUR = 9,   /* uint16 n */
    MMAS_BUF_FALLBACK = 10, /* int64 2*ants: fallback steps, then nodes enumerated */
    MMAS_BUF_STATE = 11,    /* mmas_device_state */
    MMAS_BUF_LSNN = 12,     /* uint16 n*ls_nn, 2-opt neighbour lists */
    MMAS_BUF_COUNT = 13
};

/* Bytes the workspace must have for these parameters; 0 if they are invalid. */
size_t mmas_workspace_bytes(const mmas_params* p);

/* Set-up (Alg. 1 before its loop). Copies `dist_host` (n*n int32, row-major,
 * host memory; the caller may free it on return) into the workspace, checks it
 * (zero diagonal, positive elsewhere: Sec. 2.1 requires positive distances;
 * for MMAS_PROBLEM_TSP also symmetric, since its deposit treats (i,j) and
 * (j,i) as one edge),
 * and then on the GPU: eta = 1/d and eta^beta (Sec. 2.1), the candidate lists of
 * the cl nearest cities by (distance, index) (Sec. 4.3), the 2-opt neighbour
 * lists, the nearest-neighbour tour from city 0 (ties to the lowest index),
 * the trail limits from its length (tau_max = 1/(rho C), tau_min =
 * tau_max (1 - p_best^(1/n)) / ((n/2 - 1) p_best^(1/n)) in FP64, rounded to
 * FP32, tau_min capped at tau_max), and tau <- tau_max.
 * `dev_ws`/`ws_bytes`: the workspace; `hip_stream`: a hipStream_t (NULL = the
 * null stream). Synchronises once (to report a bad matrix).
 * Errors: EINVAL (parameters or matrix), ENOSPACE, EHIP. */
mmas_status mmas_create(const int32_t* dist_host, const mmas_params* p, void* dev_ws,
                        size_t ws_bytes, void* hip_stream, mmas_ctx** out);

/* choice_info = tau^alpha * eta^beta in FP32 (Sec. 2.1), dense and along the
 * candidate lists, with its reciprocal 1/choice_info beside both (the keys'
 * factor, Sec. 4.2.2; internal to the workspace). The pheromone update
 * refreshes both as it writes tau, so this launches only when tau changed in
 * another way (set-up, mmas_set_pheromone). */
mmas_status mmas_prepare_choice_info(mmas_ctx* ctx);

/* Tour construction for iteration `iteration` (the inner loops of Alg. 1):
 * every ant starts at a uniformly drawn city and takes n-1 steps; each step
 * selects, among the unvisited cities of the current city's candidate list,
 * the one with the largest key ln(u)/choice_info (Alg. 4 with logarithmic
 * keys, Sec. 4.2.2), or, when none is left, among all unvisited cities with
 * the same rule. Writes MMAS_BUF_TOURS, MMAS_BUF_LENGTHS, MMAS_BUF_FALLBACK. */
mmas_status mmas_construct(mmas_ctx* ctx, uint32_t iteration);

/* Launch shape of the construction kernel; results never depend on it.
 * `ants_per_block`: ants per workgroup, 1, 2, 4, 8 or 16 (0 = default 4;
 * fewer are used if their LDS does not fit). `table_rows`: how many rows of
 * the candidate table (ids and choice_info) each workgroup stages in LDS:
 * -1 = as many as fit (default; when the grid needs several workgroups per
 * CU, as many as fit in one workgroup's share of the CU's LDS), 0 = none,
 * k = at most k. `lanes_per_ant`:
 * 64 (one ant per wave64, default, also for 0) or 32 (two ants per wave64,
 * each on a half; applies when 1 <= cand_len <= 32, with an even number of
 * ants per workgroup, else 64 is used). `waves_per_ant`: 1, 2, 4, 8 or 16
 * waves serve each ant (one workgroup per ant: the first wave takes the
 * steps, all of them share every all-city fallback; ignored with 32 lanes
 * per ant); 0 (default): several only where the all-city fallback dominates
 * (n >= 8192: the largest power of two up to 16 such that ants x waves fit
 * the GPU's SIMDs once; no candidate list and n >= 512: 4), else 1; and
 * where that is one wave with 9 <= cand_len <= 32 and at most as many ants
 * as the GPU has SIMDs, a second wave per ant computes the steps' draws
 * ahead into LDS (a draw helper; at most 8 ants per workgroup then).
 * 1 = the ant's wave alone. Without a candidate list, with the bitmask
 * tabu and n <= 1024, four waves per ant (by default or asked for) form a
 * team that splits every step's keys (one barrier a step). EINVAL for other
 * values. */
mmas_status mmas_set_launch(mmas_ctx* ctx, int32_t ants_per_block, int32_t table_rows, int32_t lanes_per_ant,
                            int32_t waves_per_ant);

/* Node selection of the construction. MMAS_SELECT_PRWM: the parallel
 * roulette wheel of Sec. 4.2.1 with p = 64 (one wave per ant): one draw per
 * step (slot 0); over the unvisited candidates by rank, or over every
 * unvisited city in index order; 64 chunks a stage, chunk sums left to
 * right, their prefix sums by a wave scan (log steps within rows of 16, then
 * the earlier rows' totals: an FP32 summation order of its own, so the wheel
 * is defined by its selection probabilities, w_j / sum of w, not by the bits
 * of a sequential sum), target u times the total, the first chunk whose
 * prefix exceeds the target (else the last with a positive sum), repeated
 * inside it with the target less the prefix before it; every weight 0 gives
 * the lowest entry. Bitmask tabu only (EUNSUPPORTED otherwise), the
 * launch options do not apply, and a batch's constructions ignore it.
 * MMAS_SELECT_WRS (default): Alg. 4. */
mmas_status mmas_set_selection(mmas_ctx* ctx, int32_t select);

/* 2-opt on every ant's tour with ls_nn-nearest-neighbour lists and don't-look
 * bits (Sec. 5.7), as a sequential first-improvement search (cities in index
 * order, successor direction before predecessor, neighbours by rank while the
 * first partial gain is positive; the shorter path is reversed). Updates
 * tours and lengths. EUNSUPPORTED if ls_nn == 0; ESTATE before a construct. */
mmas_status mmas_two_opt(mmas_ctx* ctx);

/* Launch shape of the 2-opt kernel; results never depend on it.
 * `waves_per_ant`: wave64s of the workgroup that runs one ant's search, 1, 2,
 * 4, 8 or 16 (0 = by the instance: 4 below 1024 cities, 8 below 8192, 16
 * from there); each round examines min(64, threads / (2*ls_nn rounded up to
 * a power of two)) cities. EINVAL for other values. */
mmas_status mmas_set_two_opt_launch(mmas_ctx* ctx, int32_t waves_per_ant);

/* The end of an iteration of Alg. 1: the iteration best (shortest tour,
 * lowest ant on ties); if it beats the global best (or there is none) it
 * becomes the global best and the limits are recomputed from its length;
 * then tau <- max(fl((1-rho) tau), tau_min), plus 1/C_ib on both directions
 * of the iteration best's edges (MMAS_PROBLEM_ATSP: on (i, succ(i)) only;
 * with MMAS_DEPOSIT_GLOBAL_BEST: 1/C_gb on the global best's), then
 * min(., tau_max) on every stored trail;
 * choice_info is refreshed in the same pass. ESTATE unless a construct came
 * after the previous update (Alg. 1 deposits each iteration's tours once). */
mmas_status mmas_update_pheromone(mmas_ctx* ctx);

/* Global best so far: the shortest tour of all iterations, which Alg. 1
 * keeps beside the trails and uses for the limits (Sec. 2.1). Synchronises.
 * `tour_host` (n int32) may be NULL.
 * *len_host = -1 while there is no global best. */
mmas_status mmas_best(mmas_ctx* ctx, int32_t* tour_host, int64_t* len_host);

/* Device address and size of a workspace view (MMAS_BUF_*). No copy. */
mmas_status mmas_buffer(mmas_ctx* ctx, int which, void** dev_ptr, size_t* bytes);

/* Copies a view to host memory (`bytes` must equal the view's size).
 * Synchronises. */
mmas_status mmas_read(mmas_ctx* ctx, int which, void* host_dst, size_t bytes);

/* Replaces the stored trails (n*n or n*cl floats, host memory; finite,
 * positive). Synchronises. Marks choice_info stale. */
mmas_status mmas_set_pheromone(mmas_ctx* ctx, const float* host_src);

/* Resume (Alg. 1 carries the trails, the trail limits and the global best
 * from one iteration to the next; draws are keyed by the iteration number).
 * Restores what mmas_read returns for MMAS_BUF_PHEROMONE (`tau_host`, as
 * mmas_set_pheromone), MMAS_BUF_STATE (`state_host`: tau_min, tau_max, delta,
 * ib_ant, ib_len, gb_len and updates are taken; nn_len and flags stay the
 * context's own) and MMAS_BUF_GB_TOUR (`gb_tour_host`, n entries, read only
 * when gb_len >= 0), all host memory. A context created with the same
 * distances and parameters, restored from a run stopped after iteration t-1
 * and driven from iteration t, repeats that run bit for bit (a learned
 * heuristic has to be installed again). Synchronises. EINVAL for trails that
 * are not finite and >= 0, limits that are not finite with
 * 0 < tau_min <= tau_max, gb_len < -1, or a global-best tour that is not a
 * permutation of 0..n-1. */
mmas_status mmas_restore(mmas_ctx* ctx, const float* tau_host, const mmas_device_state* state_host,
                         const uint16_t* gb_tour_host);

/* Per-call GPU timing: with `on` != 0 every later call that enqueues GPU work
 * (choice_info, construct, 2-opt, update) is bracketed by two hipEvents on
 * the context's stream; off by default, and turning it off keeps what was
 * gathered. */
enum { MMAS_TIMING_CHOICE = 0, MMAS_TIMING_CONSTRUCT = 1, MMAS_TIMING_TWO_OPT = 2, MMAS_TIMING_UPDATE = 3,
       MMAS_TIMING_KINDS = 4 };
mmas_status mmas_set_timing(mmas_ctx* ctx, int32_t on);

/* Milliseconds and launch counts gathered per kind (host arrays of
 * MMAS_TIMING_KINDS entries; either may be NULL); `reset` != 0 clears them
 * afterwards. Synchronises. */
mmas_status mmas_read_timing(mmas_ctx* ctx, double* ms_host, int64_t* calls_host, int32_t reset);

/* Waits for all work the context has enqueued. */
mmas_status mmas_synchronize(mmas_ctx* ctx);

/* Frees the context (not the workspace). NULL is a no-op. */
void mmas_destroy(mmas_ctx* ctx);

/* ---- batches ------------------------------------------------------------
 * Many instances (uneven n) advance one iteration of Alg. 1 per step for all
 * of them at once: one persistent construction launch pulling (instance,
 * group of ants) tiles from a queue ordered by decreasing n, one launch for
 * every instance's iteration best / global best / limits, one launch for the
 * fused update of every row. The iteration number lives in device memory, so
 * a step can be captured once into a hipGraph and replayed. Instance i gets
 * exactly the tours and trails of a single context with params[i] driven with
 * iterations 0, 1, 2, ... */
typedef struct mmas_batch mmas_batch;

/* Workspace bytes for `count` instances (params[i].n gives the size of the
 * i-th distance matrix). EINVAL if any parameters are invalid. */
mmas_status mmas_batch_workspace_bytes(int32_t count, const mmas_params* params, size_t* bytes);

/* Set-up of every instance (as mmas_create) inside one workspace.
 * `dists_host[i]` is instance i's n_i*n_i int32 matrix (host, copied). All
 * instances must share `tabu` and `pher_mode`; ls_nn must be 0
 * (EUNSUPPORTED otherwise). `hip_stream` should not be the null stream if the
 * step is to be captured. Synchronises. */
mmas_status mmas_batch_create(int32_t count, const int32_t* const* dists_host, const mmas_params* params,
                              void* dev_ws, size_t ws_bytes, void* hip_stream, mmas_batch** out);

/* Launch shape of the batched construction (results never depend on it):
 * `ants_per_block` 1, 2, 4, 8 or 16 ants per workgroup, `table_bytes` of LDS
 * per workgroup for the candidate table (-1 = all that is left after the
 * ants' regions) and `lanes_per_ant` 64 (one ant per wave64; also 0) or 32
 * (two ants per wave64: EUNSUPPORTED unless every instance has
 * 1 <= cand_len <= 32 and ants_per_block >= 2). Drops a captured graph. */
mmas_status mmas_batch_set_launch(mmas_batch* b, int32_t ants_per_block, int32_t table_bytes,
                                  int32_t lanes_per_ant);

/* Tabu of the batch's constructions, MMAS_TABU_BITMASK, _COMPACT or _LIST
 * (tours never depend on it); keeps the launch shape, EUNSUPPORTED if that
 * shape's LDS no longer fits. Drops a captured graph. */
mmas_status mmas_batch_set_tabu(mmas_batch* b, int32_t tabu);

/* Autotuner: times one construction launch for each ants_per_block in
 * {4, 8, 16}, the LDS table on and off, 64 or 32 lanes per ant (32 where
 * allowed) and the bitmask, compact or list tabu (where its LDS fits), keeps
 * the fastest and reports
 * it (any pointer may be NULL). Trails are not touched. Synchronises; drops
 * a captured graph. */
mmas_status mmas_batch_tune(mmas_batch* b, int32_t* ants_per_block, int32_t* table_bytes, int32_t* lanes_per_ant,
                            int32_t* tabu);

/* Captures one step into a hipGraph; later steps replay it. */
mmas_status mmas_batch_capture(mmas_batch* b);

/* One iteration for every instance (graph replay if captured). */
mmas_status mmas_batch_step(mmas_batch* b);

/* Per-launch timing of the batched construction: with `on` != 0 every later
 * step runs its launches directly (a captured graph is kept but not replayed
 * meanwhile; the kernels and their launch shape are the graph's) and a
 * hipEvent pair brackets the construction launch on the batch's stream. Off
 * by default; turning it off keeps what was gathered. */
mmas_status mmas_batch_set_timing(mmas_batch* b, int32_t on);

/* Milliseconds and launch count of the timed constructions (either pointer
 * may be NULL); `reset` != 0 clears them afterwards. Synchronises. */
mmas_status mmas_batch_read_timing(mmas_batch* b, double* construct_ms, int64_t* calls, int32_t reset);

/* Number of completed steps (synchronises). */
mmas_status mmas_batch_iteration(mmas_batch* b, uint32_t* iteration);

/* The context of instance `index` (owned by the batch), for mmas_read,
 * mmas_best and mmas_buffer. Do not drive it with the per-iteration calls. */
mmas_status mmas_batch_context(mmas_batch* b, int32_t index, mmas_ctx** ctx);

/* Waits for the batch's enqueued steps, then frees it and its contexts (not
 * the workspace). NULL is a no-op. */
void mmas_batch_destroy(mmas_batch* b);

/* ---- learned heuristic -----------------------------------------------------
 * A project addition beside the paper's eta = 1/d (Sec. 2.1): an edge-scoring
 * MLP (8 features -> 128 -> 128 -> 1, GELU, bfloat16 on MFMA with FP32
 * accumulation) over the 16 nearest cities of each city, and
 * eta_ij = (1/d_ij) * 2 sigmoid(s_ij) on those edges (1/d elsewhere), so that
 * s = 0 is exactly the plain heuristic. Parameters are one FP32 array of
 * mmas_mlp_param_count() floats: W1 [16][128] (rows 8..15 multiply zero
 * inputs), b1 [128], W2 [128][128] (row = input unit), b2 [128], w3 [128],
 * b3. Kernels read bfloat16 copies (mmas_mlp_packed_count() uint16) made by
 * mmas_mlp_pack. All pointers are device memory; every call enqueues on
 * `hip_stream` and returns. */
int32_t mmas_mlp_param_count(void);
int32_t mmas_mlp_packed_count(void);

/* Features of the directed edges i -> knn[i][r] (e = 16 i + r, E = 16 n):
 * the 16 nearest cities by (distance, index) into knn_dev (n*16 uint16), the
 * 8 FP32 features into feat_dev (E*8, may be NULL) and the bfloat16 MLP input
 * into x_dev (E*16, features then 8 zeros). Features, with dbar_i the mean
 * distance of i to its 16 nearest: d_ij/dbar_i, r/15, (rank of i among the 16
 * nearest of j, or 16)/16, (x_j-x_i)/dbar_i, (y_j-y_i)/dbar_i, indeg(j)/16,
 * indeg(i)/16, dbar_j/dbar_i (indeg = how many cities list it). xy_dev: n*2
 * FP32 coordinates; scratch_dev: 8n bytes. n >= 17. */
mmas_status mmas_mlp_features(const int32_t* dist_dev, const float* xy_dev, int32_t n, void* scratch_dev,
                              uint16_t* knn_dev, float* feat_dev, uint16_t* x_dev, void* hip_stream);

/* mmas_mlp_features without a scratch argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops, harnesses
 * that forbid hipMalloc): the per-city scratch (8n bytes) is the library's
 * static device array of 8 * 65535 bytes, which every GPU the library runs
 * on holds until the process ends. It allocates nothing; its first call on a
 * device looks up that device's copy (hipGetSymbolAddress). All calls on one
 * GPU share the array (it keeps the last call's contents; the pass clears
 * what must start at zero), so calls that overlap on one GPU race. Same
 * outputs and limits as mmas_mlp_features; EINVAL for n outside 17..65535. */
mmas_status mmas_mlp_features_noalloc(const int32_t* dist_dev, const float* xy_dev, int32_t n, uint16_t* knn_dev,
                                      float* feat_dev, uint16_t* x_dev, void* hip_stream);

/* bfloat16 working copies of the parameters. */
mmas_status mmas_mlp_pack(const float* params_dev, uint16_t* packed_dev, void* hip_stream);

/* Scores s (E floats) of E input rows. */
mmas_status mmas_mlp_forward(const uint16_t* x_dev, int64_t edges, const float* params_dev,
                             const uint16_t* packed_dev, float* s_dev, void* hip_stream);

/* Gradient of the mean binary cross-entropy with logits against targets in
 * [0,1] (E floats): grad_dev receives param_count floats and then the loss
 * sum. `groups` workgroups (1..4096) each write a partial sum into
 * partial_dev (groups * (param_count + 1) floats); they are added in a fixed
 * order, so the result is deterministic. */
mmas_status mmas_mlp_grad(const uint16_t* x_dev, const float* target_dev, int64_t edges, const float* params_dev,
                          const uint16_t* packed_dev, float* partial_dev, int32_t groups, float* grad_dev,
                          void* hip_stream);

/* One Adam step (step >= 1) in FP32 on all parameters:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
mmas_status mmas_mlp_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, float lr, float beta1,
                          float beta2, float eps, int32_t step, void* hip_stream);

/* Training targets: for each kNN edge (16 i + r), the share of the `tours`
 * tours (tours x n uint16, device) that contain the edge {i, knn[i][r]}. */
mmas_status mmas_mlp_labels(const uint16_t* tours_dev, int32_t tours, int32_t n, const uint16_t* knn_dev,
                            float* target_dev, void* hip_stream);

/* Installs the learned heuristic in a context: eta^beta with
 * eta_ij = fl(fl(1/d_ij) * fl(2 sigmoid(s_ij))) on the kNN edges (score_dev:
 * n*16 floats by edge 16 i + r, knn_dev: n*16); every other edge of i takes
 * the multiplier of i's lowest score, fl(2 sigmoid(min_r s_ir)), so all-zero
 * scores give the plain eta = 1/d; sigmoid uses the library's FP32 exp.
 * Marks choice_info stale. n >= 17. EUNSUPPORTED for MMAS_PROBLEM_ATSP (the
 * features and labels treat edges as undirected). */
mmas_status mmas_set_learned_heuristic(mmas_ctx* ctx, const uint16_t* knn_dev, const float* score_dev);

/* Diagnostics, for checking the device arithmetic against an independent
 * implementation: the device FP32 logarithm of `count` values in (0,1)
 * (`dev_u` -> `dev_out`, device arrays), and the Philox draw words for
 * (seed, it[i], ant[i], step[i], slot[i]) (device arrays of `count`). Both
 * enqueue on `hip_stream` and return without waiting. */
mmas_status mmas_eval_log(const float* dev_u, float* dev_out, size_t count, void* hip_stream);
mmas_status mmas_eval_draws(uint64_t seed, const uint32_t* dev_it, const uint32_t* dev_ant,
                            const uint32_t* dev_step, const uint32_t* dev_slot, uint32_t* dev_out,
                            size_t count, void* hip_stream);

/* The construction's tabu (Sec. 4.1) on its own: one wave marks the cities
 * dev_marks[0 .. count) in order in a fresh tabu of type `tabu` for n cities
 * (1 <= n <= 8192, count <= n) and writes dev_visited[v] (n bytes, 0/1), the
 * tabu's cells to dev_state (bitmask: ceil(n/32) words as pairs of 16-bit
 * halves, low half first; compact: entries, n values; list: unv then idx, 2n
 * values) and to *dev_left the number of unvisited cities, or -1 if a mark
 * was out of range or already marked (marking stops there). Device arrays;
 * enqueues on `hip_stream`. EINVAL for other arguments. */
mmas_status mmas_eval_tabu(int32_t tabu, int32_t n, const int32_t* dev_marks, int32_t count,
                           uint8_t* dev_visited, uint16_t* dev_state, int32_t* dev_left, void* hip_stream);

/* Text of the HIP error behind the calling thread's last MMAS_EHIP (which
 * step failed and HIP's message); "" if none. */
const char* mmas_last_error(void);

/* Static text for a status. */
const char* mmas_status_str(mmas_status s);

#ifdef __cplusplus
}
#endif
#endif
