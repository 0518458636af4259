// Host-side declarations shared by the translation units of libmmas: the
// workspace views of one context and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mmas.h"

namespace mmas {

// Device views of one context's workspace (all inside the caller's buffer).
struct Views {
    int32_t* dist;      // n*n
    float* heur;        // n*n (dense) or n*cl (candidates): eta^beta
    float* tau;         // n*n (dense) or n*cl (candidates)
    float* choice;      // n*n (dense) or nullptr
    float* choice_inv;  // n*n (dense) or nullptr: 1 / choice (IEEE division), the fallback keys' factor
    float* chc;         // n*cl
    float* chc_inv;     // n*cl: 1 / chc (IEEE division), the key's factor
    uint16_t* cand;     // n*cl
    uint16_t* lsnn;     // n*ls_nn or nullptr
    uint16_t* tours;    // ants*n
    int64_t* lengths;   // ants
    int64_t* fallback;  // 2*ants
    uint16_t* gb_tour;  // n
    uint16_t* nn_tour;  // n
    uint16_t* succ;     // n: successor of each city in the iteration best
    uint16_t* pred;     // n
    mmas_device_state* state;
};

// Problem constants every kernel needs.
struct Shape {
    int n;
    int ants;
    int cl;      // effective candidate-list length, min(cand_len, n-1)
    int alpha;
    int beta;
    int ls_nn;
    int pher;    // MMAS_PHER_*
    int tabu;    // MMAS_TABU_*
    int deposit; // MMAS_DEPOSIT_*
    int select;  // MMAS_SELECT_* (node selection)
    int directed; // 1 for MMAS_PROBLEM_ATSP: deposit on (i, succ(i)) only
    float rho;
    double pdec; // p_best^(1/n)
    uint64_t seed;
    int ants_per_block;  // construction launch: ants per workgroup
    int lanes_per_ant;   // construction launch: 64 (one ant per wave) or 32 (two)
    int construct_waves; // construction launch: waves per ant (0 = from the ant count)
    int table_rows;      // rows of the candidate table staged in LDS (-1: all that fit)
    int list_cap;        // construction: entries of a bitmask fallback's city list
                         // (0: min(n, kListCap); the launcher may raise it to n)
    int two_opt_waves;   // 2-opt launch: waves per ant (1..16; 0: by the instance size)
};

// One instance of a batch (device array, one entry per instance).
struct BatchItem {
    Views v;
    Shape s;
};

// One construction tile of a batch: ants ant0 .. ant0 + ants_per_block - 1
// of instance `inst`.
struct BatchTile {
    int inst;
    int ant0;
};

// Records the HIP error behind an MMAS_EHIP (per thread) and returns
// MMAS_EHIP; mmas_last_error() reads it back.
mmas_status hip_fail(hipError_t e, const char* where);

// ---- set-up (prep.hip) ----
hipError_t launch_validate(const Views& v, const Shape& s, hipStream_t st);
hipError_t launch_heuristic(const Views& v, const Shape& s, hipStream_t st);
hipError_t launch_nearest(const int32_t* dist, int n, int k, uint16_t* out, hipStream_t st);
hipError_t launch_nn_tour(const Views& v, const Shape& s, hipStream_t st);
hipError_t launch_init_trails(const Views& v, const Shape& s, hipStream_t st);

// ---- per iteration ----
hipError_t launch_choice(const Views& v, const Shape& s, hipStream_t st);             // update.hip
hipError_t launch_construct(const Views& v, const Shape& s, uint32_t it, hipStream_t st); // construct.hip
// construct.hip: the tabu of one ant after some marks (diagnostics)
hipError_t launch_eval_tabu(int tabu, int n, const int32_t* marks, int count, uint8_t* visited, uint16_t* state,
                            int32_t* left, hipStream_t st);
hipError_t launch_two_opt_prepare(const Views& v, const Shape& s, int32_t* nnd, hipStream_t st);  // two_opt.hip
hipError_t launch_two_opt(const Views& v, const Shape& s, const int32_t* nnd, hipStream_t st);
hipError_t launch_update(const Views& v, const Shape& s, hipStream_t st);            // update.hip

// ---- batches (one launch per step for all instances) ----
// construct.hip: persistent construction over `ntiles` tiles; `queue` must be
// 0 at launch (the batched best kernel re-arms it).
// lanes_per_ant 32 (two ants per wave, ants_per_block even) needs 1 <= cl <= 32
// in every instance.
hipError_t launch_batch_construct(const BatchItem* items, const BatchTile* tiles, int ntiles, uint32_t* queue,
                                  const uint32_t* it_dev, int tabu, int pher, int ants_per_block, int lanes_per_ant,
                                  int table_bytes, int per_ant, int grid, hipStream_t st);
// Persistent-grid size for this LDS footprint (workgroups that fit at once).
int batch_construct_grid(int tabu, int pher, int ants_per_block, int lanes_per_ant, int lds_bytes);
// update.hip: best/limits for every instance (one workgroup each), then the
// fused update of every row of every instance (`row_start` = prefix sums of
// the instances' row counts, count + 1 entries); increments *it_dev and
// re-arms *queue.
hipError_t launch_batch_update(const BatchItem* items, int count, const int* row_start, int total_rows,
                               uint32_t* it_dev, uint32_t* queue, hipStream_t st);
int max_lds_per_block();

// ---- learned heuristic (learned.hip) ----
int mlp_param_count();
int mlp_packed_count();
hipError_t launch_features(const int32_t* dist, const float* xy, const uint16_t* knn, int n, float* dbar, int* indeg,
                           float* feat, uint16_t* X, hipStream_t st);
hipError_t launch_pack(const float* p, uint16_t* pk, hipStream_t st);
hipError_t launch_mlp_forward(const uint16_t* X, const float* p, const uint16_t* pk, int64_t E, float* s,
                              hipStream_t st);
hipError_t launch_mlp_train(const uint16_t* X, const float* f, const float* p, const uint16_t* pk, int64_t E,
                            float* partial, int groups, float* grad, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, float c1,
                       float c2, hipStream_t st);
hipError_t launch_install(const int32_t* dist, const uint16_t* knn, const float* s, const uint16_t* cand, int n, int cl,
                          int beta, int dense, float* heur, hipStream_t st);
hipError_t launch_labels(const uint16_t* tours, int R, int n, const uint16_t* knn, float* label, hipStream_t st);

// LDS bytes one ant needs in the construction kernels with one wave (or half
// a wave) per ant, and with several waves per ant.
size_t construct_lds_per_ant(const Shape& s);
size_t wide_lds_per_ant(const Shape& s);
// LDS bytes of the 2-opt kernel (one tour per workgroup).
size_t two_opt_lds_bytes(const Shape& s, bool with_len);
// LDS the 2-opt kernel declares statically (city list, per-wave records)
constexpr size_t kTwoOptStaticLds = 4096;

}  // namespace mmas
