/* Drives every entry point of the oracle over its option combinations on
 * small synthetic instances, so that the oracle can be built and run under
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure, like
 * the rest of this directory). Exit status 0 when every run completed and
 * every consistency check held. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mmas_oracle.h"

static uint32_t lcg(uint32_t* s) {
    *s = *s * 1664525u + 1013904223u;
    return *s >> 8;
}

/* integer Euclidean distances of random points; asym adds a one-way surcharge */
static void make_dist(int n, int asym, uint32_t seed, int32_t* d, float* xy) {
    uint32_t s = seed;
    for (int i = 0; i < n; ++i) {
        xy[2 * i] = (float)(lcg(&s) % 1000u);
        xy[2 * i + 1] = (float)(lcg(&s) % 1000u);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const double dx = (double)xy[2 * i] - xy[2 * j], dy = (double)xy[2 * i + 1] - xy[2 * j + 1];
            int32_t v = (int32_t)floor(sqrt(dx * dx + dy * dy) + 0.5);
            if (i != j && v < 1) v = 1;
            if (i != j && asym) v += (int32_t)(lcg(&s) % 17u);
            d[(size_t)i * n + j] = i == j ? 0 : v;
        }
}

static int fail(const char* what, int n, int cl) {
    fprintf(stderr, "check failed: %s (n=%d cl=%d)\n", what, n, cl);
    return 1;
}

static int colony_runs(void) {
    const int sizes[] = {5, 37, 130};
    int bad = 0;
    for (int si = 0; si < 3; ++si) {
        const int n = sizes[si];
        int32_t* d = malloc(sizeof(int32_t) * (size_t)n * n);
        float* xy = malloc(sizeof(float) * 2 * (size_t)n);
        const int cls[] = {0, 1, 8, n - 1};
        for (int asym = 0; asym < 2; ++asym) {
            make_dist(n, asym, 7u + (uint32_t)n, d, xy);
            for (int ci = 0; ci < 4; ++ci)
                for (int pher = 0; pher < 2; ++pher)
                    for (int sel = 0; sel < 2; ++sel)
                        for (int dep = 0; dep < 2; ++dep) {
                            const int cl = cls[ci];
                            if (pher == ORC_PHER_CANDIDATES && cl == 0) continue;
                            const int ls = asym ? 0 : (n > 4 ? 4 : 0);
                            const double pdec = pow(0.01, 1.0 / n);
                            orc_colony* c = orc_create(n, d, 9, cl, 1, 2, 0.1f, pdec, 5u, pher, ls);
                            orc_colony* r = orc_create(n, d, 9, cl, 1, 2, 0.1f, pdec, 5u, pher, ls);
                            if (!c || !r) return fail("create", n, cl);
                            orc_colony* both[2] = {c, r};
                            for (int k = 0; k < 2; ++k) {
                                if (orc_set_select(both[k], sel) || orc_set_deposit(both[k], dep) ||
                                    orc_set_problem(both[k], asym ? ORC_PROBLEM_ATSP : ORC_PROBLEM_TSP))
                                    return fail("options", n, cl);
                            }
                            for (uint32_t it = 0; it < 3; ++it) orc_iterate(c, it, 2);
                            /* checkpoint c, restore into r, run one more iteration on both */
                            const size_t nt = pher == ORC_PHER_DENSE ? (size_t)n * n : (size_t)n * orc_cl(c);
                            float* tau = malloc(sizeof(float) * nt);
                            uint16_t* gb = malloc(sizeof(uint16_t) * (size_t)n);
                            float lim[2];
                            orc_get_pheromone(c, tau);
                            orc_get_limits(c, lim);
                            const int64_t gl = orc_get_best(c, gb);
                            orc_set_pheromone(r, tau);
                            orc_restore(r, lim, gl, gb);
                            orc_iterate(c, 3, 2);
                            orc_iterate(r, 3, 1);
                            uint16_t* t1 = malloc(sizeof(uint16_t) * 9 * (size_t)n);
                            uint16_t* t2 = malloc(sizeof(uint16_t) * 9 * (size_t)n);
                            orc_get_tours(c, t1);
                            orc_get_tours(r, t2);
                            if (memcmp(t1, t2, sizeof(uint16_t) * 9 * (size_t)n)) bad |= fail("resume", n, cl);
                            int64_t len[9], fs[9], fn[9], ib[2];
                            orc_get_lengths(c, len);
                            orc_get_fallback(c, fs, fn);
                            orc_get_iteration_best(c, ib);
                            for (int a = 0; a < 9; ++a)
                                if (len[a] != orc_tour_length(n, d, t1 + (size_t)a * n)) bad |= fail("length", n, cl);
                            if (orc_cl(c) > 0) {
                                uint16_t* cand = malloc(sizeof(uint16_t) * (size_t)n * orc_cl(c));
                                float* chc = malloc(sizeof(float) * (size_t)n * orc_cl(c));
                                orc_get_cand(c, cand);
                                orc_get_chc(c, chc);
                                free(cand);
                                free(chc);
                            }
                            if (pher == ORC_PHER_DENSE) {
                                float* m = malloc(sizeof(float) * (size_t)n * n);
                                orc_get_choice(c, m);
                                orc_get_heuristic(c, m);
                                if (orc_set_heuristic(c, m)) bad |= fail("set_heuristic", n, cl);
                                free(m);
                            }
                            uint8_t* vis = calloc((size_t)n, 1);
                            vis[0] = 1;
                            int fb = 0;
                            const int v = orc_select_next(c, 0, vis, 1u, 2u, 3u, &fb);
                            if (v <= 0 || v >= n) bad |= fail("select_next", n, cl);
                            uint16_t* nn = malloc(sizeof(uint16_t) * (size_t)n);
                            orc_get_nn_tour(c, nn);
                            free(nn);
                            free(vis);
                            free(t1);
                            free(t2);
                            free(tau);
                            free(gb);
                            orc_destroy(c);
                            orc_destroy(r);
                        }
        }
        free(d);
        free(xy);
    }
    return bad;
}

static int pieces(void) {
    int bad = 0;
    const int n = 40, K = 16, IN = 16, H = 128;
    int32_t* d = malloc(sizeof(int32_t) * n * n);
    float* xy = malloc(sizeof(float) * 2 * n);
    make_dist(n, 0, 3u, d, xy);
    uint16_t* knn = malloc(sizeof(uint16_t) * n * K);
    float* feat = malloc(sizeof(float) * n * K * 8);
    orc_knn_features(n, d, xy, knn, feat);
    const int64_t E = (int64_t)n * K;
    float* X = calloc((size_t)E * IN, sizeof(float));
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 8; ++f) X[e * IN + f] = feat[e * 8 + f];
    float* W1 = malloc(sizeof(float) * IN * H);
    float* W2 = malloc(sizeof(float) * H * H);
    float *b1 = calloc(H, sizeof(float)), *b2 = calloc(H, sizeof(float)), *w3 = malloc(sizeof(float) * H);
    uint32_t s = 11u;
    for (int i = 0; i < IN * H; ++i) W1[i] = (float)((int)(lcg(&s) % 200u) - 100) / 400.0f;
    for (int i = 0; i < H * H; ++i) W2[i] = (float)((int)(lcg(&s) % 200u) - 100) / 1000.0f;
    for (int i = 0; i < H; ++i) w3[i] = (float)((int)(lcg(&s) % 200u) - 100) / 1000.0f;
    float* sc = malloc(sizeof(float) * E);
    float* tgt = malloc(sizeof(float) * E);
    for (int64_t e = 0; e < E; ++e) tgt[e] = (float)(e % 3 == 0);
    orc_mlp_forward(E, X, W1, b1, W2, b2, w3, 0.0f, 1, sc);
    float* g1 = malloc(sizeof(float) * IN * H);
    float* g2 = malloc(sizeof(float) * H * H);
    float *gb1 = malloc(sizeof(float) * H), *gb2 = malloc(sizeof(float) * H), *g3 = malloc(sizeof(float) * H), gb3;
    const double loss = orc_mlp_backward(E, X, tgt, W1, b1, W2, b2, w3, 0.0f, 0, g1, gb1, g2, gb2, g3, &gb3);
    if (!(loss > 0.0)) bad |= fail("loss", n, K);
    float* m = calloc(IN * H, sizeof(float));
    float* v = calloc(IN * H, sizeof(float));
    orc_adam(IN * H, W1, g1, m, v, 1e-3f, 0.9f, 0.999f, 1e-8f, 0.1f, 0.001f);
    float* heur = malloc(sizeof(float) * n * n);
    orc_install_eta(n, d, knn, sc, 2, heur);
    uint16_t* tour = malloc(sizeof(uint16_t) * n);
    uint16_t* lsnn = malloc(sizeof(uint16_t) * n * 8);
    orc_nearest(n, d, 8, lsnn);
    const int64_t L0 = orc_nn_tour(n, d, tour);
    const int64_t L1 = orc_two_opt_tour(n, d, lsnn, 8, tour);
    if (L1 > L0 || L1 != orc_tour_length(n, d, tour)) bad |= fail("two_opt", n, 8);
    float lo, hi;
    orc_limits(0.1f, L1, n, pow(0.01, 1.0 / n), &lo, &hi);
    if (!(lo > 0.0f && lo <= hi)) bad |= fail("limits", n, 0);
    const float u = orc_u01(orc_draw_word(1u, 2u, 3u, 4u, 5u));
    if (!(u > 0.0f && u < 1.0f) || !(orc_logf(u) < 0.0f)) bad |= fail("draw", n, 0);
    if (orc_start_node(1u, 2u, 3u, (uint32_t)n) >= (uint32_t)n) bad |= fail("start", n, 0);
    (void)orc_expf(1.0f);
    (void)orc_bf16_round(1.3f);
    free(d), free(xy), free(knn), free(feat), free(X), free(W1), free(W2), free(b1), free(b2), free(w3);
    free(sc), free(tgt), free(g1), free(g2), free(gb1), free(gb2), free(g3), free(m), free(v), free(heur);
    free(tour), free(lsnn);
    return bad;
}

int main(void) {
    const int bad = colony_runs() | pieces();
    if (!bad) printf("oracle exercise: all runs completed\n");
    return bad;
}
