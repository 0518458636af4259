/*
 * CPU oracle for the MAX-MIN Ant System hot path (Skinderowicz, "Implementing
 * a GPU-based parallel MAX-MIN Ant System", FGCS 2020).
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow reference that the HIP
 * library is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does. It shares
 * no source with the HIP library.
 *
 * Everything follows the paper's method in its own order (Alg. 1 for the main
 * loop, Eq. (1) for the selection distribution, Alg. 4 / Sec. 4.2.2 for the
 * weighted-reservoir-sampling selection with logarithmic keys, Sec. 4.3 for
 * candidate lists, Sec. 2.1 for evaporation, deposit and the trail limits),
 * with every random draw taken from a counter-based generator so that one
 * (instance, parameters, seed) has exactly one correct result.
 *
 * Arithmetic: FP32 with IEEE round-to-nearest on every operation, no
 * contraction into fused multiply-add, no flush of denormals; the trail limits
 * are computed in FP64 and rounded to FP32. Build with -ffp-contract=off and
 * without -ffast-math.
 */
#ifndef MMAS_ORACLE_H
#define MMAS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- random numbers ---------------------------------------------------- */

/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): 10 rounds of the
 * Philox S-box on a 128-bit counter with a 64-bit key bumped by the Weyl
 * constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The 32-bit word a draw uses. key = (seed low, seed high); counter =
 * ((slot >> 2) | (step << 16), ant, iteration, 0); the word is slot & 3.
 * Slots 0..cl-1 are the candidate ranks, slot cl+v is node v in the
 * all-node fallback, step 0 slot 0 picks the start node. */
uint32_t orc_draw_word(uint64_t seed, uint32_t it, uint32_t ant, uint32_t step, uint32_t slot);

/* u = (2*(x >> 9) + 1) * 2^-24: exact in FP32, strictly inside (0, 1). */
float orc_u01(uint32_t x);

/* Natural logarithm in FP32 for the random(0,1) draws of Sec. 4.2.2:
 * u = m * 2^e with m in (sqrt(2)/2, sqrt(2)], f = m - 1,
 * ln(1+f) = f + f^2 Q(f) with a fitted degree-10 polynomial Q evaluated by
 * fused multiply-adds, and ln(u) = e*ln2 + ln(1+f) (ln 2 split into a head
 * that e multiplies exactly and a tail). */
float orc_logf(float u);

/* Array forms of the three above, for exhaustive tests. */
void orc_logf_n(int64_t count, const float* u, float* out);
void orc_u01_n(int64_t count, const uint32_t* x, float* out);
void orc_draw_words_n(int64_t count, uint64_t seed, const uint32_t* it, const uint32_t* ant,
                      const uint32_t* step, const uint32_t* slot, uint32_t* out);

/* Start node of an ant: floor(x * n / 2^32) of draw (step 0, slot 0). */
uint32_t orc_start_node(uint64_t seed, uint32_t it, uint32_t ant, uint32_t n);

/* ---- one colony ---------------------------------------------------------- */

enum { ORC_PHER_DENSE = 0, ORC_PHER_CANDIDATES = 1 };

typedef struct orc_colony orc_colony;

/* Builds the colony state for one instance and runs the set-up steps of
 * Alg. 1 before its main loop: eta = 1/d (Sec. 2.1), the candidate lists
 * (Sec. 4.3), the nearest-neighbour tour, the trail limits from its length
 * and tau <- tau_max. `dist` (n*n, row-major, int32) is copied.
 * alpha and beta are small non-negative integers. rho is the evaporation
 * rate: tau <- (1 - rho) * tau. pdec = p_best^(1/n), computed by the caller.
 * pher_mode: dense n*n trails, or trails stored only for the (i, cand[i][r])
 * edges with every other edge held at tau_min.
 * ls_nn > 0 enables 2-opt on ls_nn-nearest-neighbour lists.
 * Returns NULL on invalid arguments. */
orc_colony* orc_create(int n, const int32_t* dist, int ants, int cand_len,
                       int alpha, int beta, float rho, double pdec,
                       uint64_t seed, int pher_mode, int ls_nn);
void orc_destroy(orc_colony* c);

/* Whose tour deposits (Sec. 2.1): the iteration best (default) or the global
 * best, which may replace it. Returns -1 for another mode. */
enum { ORC_DEPOSIT_ITERATION_BEST = 0, ORC_DEPOSIT_GLOBAL_BEST = 1 };
int orc_set_deposit(orc_colony* c, int mode);

/* Node selection: weighted reservoir sampling (Alg. 4, default) or the
 * parallel roulette wheel of Sec. 4.2.1 (64 chunks a stage, chunk sums and
 * their prefix sums left to right, one draw per step). Returns -1 for
 * another mode. */
enum { ORC_SELECT_WRS = 0, ORC_SELECT_PRWM = 1 };
int orc_set_select(orc_colony* c, int mode);

/* The problem (Sec. 2.1): the symmetric TSP (default), or the asymmetric TSP,
 * where d_ij and d_ji may differ, an edge (i,j) is directed and the deposit
 * reaches (i,j) only. Returns -1 for another mode, and for the ATSP when 2-opt
 * is on (reversing a path changes an asymmetric tour's length). */
enum { ORC_PROBLEM_TSP = 0, ORC_PROBLEM_ATSP = 1 };
int orc_set_problem(orc_colony* c, int mode);

/* The per-iteration calls, in Alg. 1 order. */
void orc_prepare_choice(orc_colony* c);              /* choice_info = tau^alpha * eta^beta */
void orc_construct(orc_colony* c, uint32_t it, int nthreads); /* every ant builds a tour */
void orc_two_opt(orc_colony* c, int nthreads);       /* optional local search on every tour */
void orc_update(orc_colony* c);                      /* best, limits, evaporate, deposit, clamp */
/* All four in order. */
void orc_iterate(orc_colony* c, uint32_t it, int nthreads);

/* One selection step for ant `ant` at node `cur` with the visited flags
 * `visited[n]` (non-zero = visited); uses the colony's current choice_info.
 * Sets *fallback to 1 if the all-node fallback ran. Returns the node. */
int orc_select_next(const orc_colony* c, int cur, const uint8_t* visited,
                    uint32_t it, uint32_t ant, uint32_t step, int* fallback);

/* Accessors (copies out). Sizes: tours ants*n, lengths ants, pheromone
 * n*n (dense) or n*cl (candidates), choice n*n (dense only), chc n*cl,
 * cand n*cl, fallback counters ants each. */
int  orc_n(const orc_colony* c);
int  orc_cl(const orc_colony* c);
void orc_get_tours(const orc_colony* c, uint16_t* out);
void orc_get_lengths(const orc_colony* c, int64_t* out);
void orc_get_pheromone(const orc_colony* c, float* out);
void orc_set_pheromone(orc_colony* c, const float* in);
void orc_get_choice(const orc_colony* c, float* out);
void orc_get_chc(const orc_colony* c, float* out);
void orc_get_cand(const orc_colony* c, uint16_t* out);
void orc_get_heuristic(const orc_colony* c, float* out); /* dense eta^beta, n*n */
int orc_set_heuristic(orc_colony* c, const float* heur); /* dense mode: replace eta^beta (n*n); -1 otherwise */
void orc_get_fallback(const orc_colony* c, int64_t* steps, int64_t* nodes);
/* limits[0] = tau_min, limits[1] = tau_max */
void orc_get_limits(const orc_colony* c, float* limits);
/* gb_len = -1 while there is no global best. */
int64_t orc_get_best(const orc_colony* c, uint16_t* gb_tour);
int64_t orc_get_nn_tour(const orc_colony* c, uint16_t* tour);
/* ib[0] = iteration-best ant, ib[1] = its length (after orc_update). */
void orc_get_iteration_best(const orc_colony* c, int64_t* ib);
/* Resume: the state Alg. 1 carries from one iteration to the next besides
 * the trails (set them with orc_set_pheromone): the limits, and the global
 * best (gb_len = -1 for none; gb_tour n entries, ignored then). Draws are
 * keyed by the iteration number, so a colony restored after iteration t and
 * run from t on repeats the uninterrupted run. */
void orc_restore(orc_colony* c, const float* limits, int64_t gb_len, const uint16_t* gb_tour);

/* ---- stand-alone pieces ----------------------------------------------- */

/* Trail limits (Stuetzle and Hoos, p_best): tau_max = 1/(rho*C),
 * tau_min = tau_max*(1-pdec) / ((n/2 - 1)*pdec), in FP64, rounded to FP32;
 * if tau_min > tau_max then tau_min = tau_max. */
void orc_limits(float rho, int64_t C, int n, double pdec, float* tmin, float* tmax);

/* The k nearest other nodes of every node, by (distance, index). out n*k. */
void orc_nearest(int n, const int32_t* dist, int k, uint16_t* out);

/* Nearest-neighbour tour from node 0, ties to the lowest index. Returns its
 * length, closing edge included. */
int64_t orc_nn_tour(int n, const int32_t* dist, uint16_t* tour);

/* 2-opt with neighbour lists and don't-look bits on one tour (in place);
 * returns the new length. nn is n*k. */
int64_t orc_two_opt_tour(int n, const int32_t* dist, const uint16_t* nn, int k, uint16_t* tour);

/* Tour length, closing edge included. */
int64_t orc_tour_length(int n, const int32_t* dist, const uint16_t* tour);

/* ---- learned heuristic (learned_oracle.c) -------------------------------- */

float orc_bf16_round(float x);
float orc_expf(float x);
void orc_knn_features(int n, const int32_t* dist, const float* xy, uint16_t* knn, float* feat);
void orc_mlp_forward(int64_t E, const float* X, const float* W1, const float* b1, const float* W2, const float* b2,
                     const float* w3, float b3, int quantize, float* s_out);
double orc_mlp_backward(int64_t E, const float* X, const float* f, const float* W1, const float* b1, const float* W2,
                        const float* b2, const float* w3, float b3, int quantize, float* gW1, float* gb1, float* gW2,
                        float* gb2, float* gw3, float* gb3);
void orc_adam(int64_t count, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
              float c1, float c2);
void orc_install_eta(int n, const int32_t* dist, const uint16_t* knn, const float* s, int beta, float* heur);

#ifdef __cplusplus
}
#endif
#endif
