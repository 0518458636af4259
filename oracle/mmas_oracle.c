/*
 * CPU oracle for the MAX-MIN Ant System hot path. TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg,
 * never by the product. Plain loops, one node at a time, in the order the
 * paper states the method. See mmas_oracle.h for the conventions.
 */
#include "mmas_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Philox4x32-10, from its published definition (Salmon et al., SC'11):
 * each round multiplies counter words 0 and 2 by two fixed 32-bit constants,
 * and the new counter is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
 * lo(M0*c0)); the key is bumped by the two Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

uint32_t orc_draw_word(uint64_t seed, uint32_t it, uint32_t ant, uint32_t step, uint32_t slot) {
    uint32_t ctr[4] = {(slot >> 2) | (step << 16), ant, it, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[slot & 3u];
}

float orc_u01(uint32_t x) {
    /* an odd multiple of 2^-24 below 2^24: exact, never 0 or 1 */
    return (float)(2u * (x >> 9) + 1u) * 0x1p-24f;
}

/* ------------------------------------------------------------------------
 * Natural logarithm (Sec. 4.2.2 replaces r^(1/w) by a logarithm divided by
 * w). u = m 2^e with m in (sqrt(2)/2, sqrt(2)], f = m - 1 (exact), and
 * ln(1+f) = f + f^2 Q(f), where Q(f) = (ln(1+f) - f) / f^2 is replaced by a
 * degree-10 polynomial fitted by this project (iteratively reweighted least
 * squares towards the minimax of f^2 |error| on the reduced interval,
 * coefficients rounded to FP32; Q(0) = -1/2 exactly), evaluated by Horner's
 * rule with single-rounding fused multiply-adds (fmaf). ln 2 is split into
 * LN2_HI (15 significant bits: e*LN2_HI + f is exact for e = 0 and e = -1)
 * and LN2_LO = ln 2 - LN2_HI rounded to FP32, and
 * ln(u) = (e*LN2_HI + f) + (f^2 Q(f) + e*LN2_LO).
 * Over all 2^23 draws u the result is within 0.83 ulp of ln(u) and
 * monotone in u.
 * ---------------------------------------------------------------------- */
static float f32_from_bits(uint32_t b) {
    float f;
    memcpy(&f, &b, 4);
    return f;
}
static uint32_t bits_from_f32(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

float orc_logf(float u) {
    const float LN2_HI = f32_from_bits(0x3F317200u); /* 0.693145751953125 */
    const float LN2_LO = f32_from_bits(0x35BFBE8Eu); /* ln2 - LN2_HI, nearest FP32 */
    const float SQRT2 = f32_from_bits(0x3FB504F3u);  /* sqrt(2) rounded */
    /* Q(f) ~ q0 + q1 f + ... + q10 f^10 */
    static const uint32_t QBITS[11] = {0xBF000000u, 0x3EAAAAAAu, 0xBE7FFFD3u, 0x3E4CCCE5u,
                                       0xBE2AB49Fu, 0x3E124E2Fu, 0xBDFE32BFu, 0x3DE13229u,
                                       0xBDDE3E43u, 0x3DDE0BBCu, 0xBD7C39FAu};
    uint32_t b = bits_from_f32(u);
    int e = (int)(b >> 23) - 127;
    float m = f32_from_bits((b & 0x007FFFFFu) | 0x3F800000u); /* [1, 2) */
    if (m > SQRT2) {
        m = m * 0.5f;
        e = e + 1;
    }
    float f = m - 1.0f;
    float q = f32_from_bits(QBITS[10]);
    for (int k = 9; k >= 0; --k) q = fmaf(q, f, f32_from_bits(QBITS[k]));
    float ef = (float)e;
    float small = fmaf(f * f, q, ef * LN2_LO);
    return (ef * LN2_HI + f) + small;
}

void orc_logf_n(int64_t count, const float* u, float* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = orc_logf(u[i]);
}
void orc_u01_n(int64_t count, const uint32_t* x, float* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = orc_u01(x[i]);
}
void orc_draw_words_n(int64_t count, uint64_t seed, const uint32_t* it, const uint32_t* ant,
                      const uint32_t* step, const uint32_t* slot, uint32_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = orc_draw_word(seed, it[i], ant[i], step[i], slot[i]);
}

uint32_t orc_start_node(uint64_t seed, uint32_t it, uint32_t ant, uint32_t n) {
    uint32_t x = orc_draw_word(seed, it, ant, 0u, 0u);
    return (uint32_t)(((uint64_t)x * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------------
 * Small helpers
 * ---------------------------------------------------------------------- */
static float powi_f32(float x, int k) {
    /* left-to-right repeated multiplication; x^0 = 1 */
    float r = 1.0f;
    for (int i = 0; i < k; ++i) r = r * x;
    return r;
}

/* eta_ij^beta with eta = 1/d (Sec. 2.1) */
static float heur_of(int32_t d, int beta) {
    float eta = 1.0f / (float)d;
    return powi_f32(eta, beta);
}

int64_t orc_tour_length(int n, const int32_t* dist, const uint16_t* tour) {
    int64_t len = 0;
    for (int k = 0; k < n; ++k) {
        int a = tour[k], b = tour[(k + 1) % n];
        len += dist[(size_t)a * n + b];
    }
    return len;
}

void orc_limits(float rho, int64_t C, int n, double pdec, float* tmin, float* tmax) {
    double tmax_d = 1.0 / ((double)rho * (double)C);
    double tmin_d = (tmax_d * (1.0 - pdec)) / (((double)n / 2.0 - 1.0) * pdec);
    float hi = (float)tmax_d;
    float lo = (float)tmin_d;
    if (lo > hi) lo = hi;
    *tmin = lo;
    *tmax = hi;
}

/* first k of the other nodes sorted by (d, index): insertion into a sorted
 * window of length k while scanning the row once */
void orc_nearest(int n, const int32_t* dist, int k, uint16_t* out) {
    int32_t* wd = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k + 1));
    int* wj = (int*)malloc(sizeof(int) * (size_t)(k + 1));
    for (int i = 0; i < n; ++i) {
        int cnt = 0;
        const int32_t* row = dist + (size_t)i * n;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            int32_t d = row[j];
            /* (d, j) sorts after the window's last entry: skip */
            if (cnt == k && !(d < wd[k - 1])) continue; /* j is larger than all kept */
            int p = (cnt < k) ? cnt : k - 1;
            while (p > 0 && (wd[p - 1] > d)) {
                wd[p] = wd[p - 1];
                wj[p] = wj[p - 1];
                --p;
            }
            wd[p] = d;
            wj[p] = j;
            if (cnt < k) ++cnt;
        }
        for (int r = 0; r < k; ++r) out[(size_t)i * k + r] = (uint16_t)wj[r];
    }
    free(wd);
    free(wj);
}

int64_t orc_nn_tour(int n, const int32_t* dist, uint16_t* tour) {
    uint8_t* vis = (uint8_t*)calloc((size_t)n, 1);
    int cur = 0;
    tour[0] = 0;
    vis[0] = 1;
    for (int k = 1; k < n; ++k) {
        int best = -1;
        int32_t bd = 0;
        for (int j = 0; j < n; ++j) {
            if (vis[j]) continue;
            int32_t d = dist[(size_t)cur * n + j];
            if (best < 0 || d < bd) {
                best = j;
                bd = d;
            }
        }
        tour[k] = (uint16_t)best;
        vis[best] = 1;
        cur = best;
    }
    free(vis);
    return orc_tour_length(n, dist, tour);
}

/* ------------------------------------------------------------------------
 * 2-opt with neighbour lists and don't-look bits (Sec. 5.7, after Bentley),
 * as a sequential first-improvement search:
 *  - cities are examined in index order, cyclically, skipping those whose
 *    don't-look bit is set; the search ends when every bit is set;
 *  - for city a the successor direction is tried first, then the
 *    predecessor direction; in each, the neighbours c of a are taken by rank
 *    while g1 = d(a, a') - d(a, c) > 0 (a' is a's successor, resp.
 *    predecessor);
 *  - the first move whose gain is positive is applied, the bits of its four
 *    end points are cleared and a is examined again; a city with no such
 *    move gets its bit set;
 *  - the move reverses the shorter of the two paths it may reverse (the one
 *    starting next to a on a tie).
 * ---------------------------------------------------------------------- */
static void reverse_path(int n, uint16_t* tour, int* pos, int i, int j) {
    int len = ((j - i + n) % n) + 1;
    for (int s = 0; s < len / 2; ++s) {
        int p = (i + s) % n, q = (j - s + n) % n;
        uint16_t tp = tour[p], tq = tour[q];
        tour[p] = tq;
        tour[q] = tp;
        pos[tq] = p;
        pos[tp] = q;
    }
}

int64_t orc_two_opt_tour(int n, const int32_t* dist, const uint16_t* nn, int k, uint16_t* tour) {
    int* pos = (int*)malloc(sizeof(int) * (size_t)n);
    uint8_t* dlb = (uint8_t*)calloc((size_t)n, 1);
    for (int i = 0; i < n; ++i) pos[tour[i]] = i;
#define D(x, y) ((int64_t)dist[(size_t)(x) * n + (y)])
    int active = n; /* cities whose bit is clear */
    int a = 0;
    while (active > 0) {
        if (dlb[a]) {
            a = (a + 1) % n;
            continue;
        }
        int moved = 0;
        for (int dir = 0; dir < 2 && !moved; ++dir) {
            int pa = pos[a];
            int a1 = dir == 0 ? tour[(pa + 1) % n] : tour[(pa - 1 + n) % n];
            int64_t d_aa1 = D(a, a1);
            for (int r = 0; r < k; ++r) {
                int c = nn[(size_t)a * k + r];
                int64_t g1 = d_aa1 - D(a, c);
                if (g1 <= 0) break;
                int pc = pos[c];
                int c1 = dir == 0 ? tour[(pc + 1) % n] : tour[(pc - 1 + n) % n];
                if (c == a1 || c1 == a) continue;
                int64_t gain = g1 + D(c, c1) - D(a1, c1);
                if (gain <= 0) continue;
                /* apply: the two paths the move may reverse */
                int i1, j1, i2, j2;
                if (dir == 0) { /* a -> a1 ... c -> c1: reverse a1..c or c1..a */
                    i1 = pos[a1]; j1 = pos[c];
                    i2 = pos[c1]; j2 = pos[a];
                } else {        /* a1 -> a ... c1 -> c: reverse a..c1 or c..a1 */
                    i1 = pos[a]; j1 = pos[c1];
                    i2 = pos[c]; j2 = pos[a1];
                }
                int len1 = ((j1 - i1 + n) % n) + 1;
                if (len1 <= n - len1)
                    reverse_path(n, tour, pos, i1, j1);
                else
                    reverse_path(n, tour, pos, i2, j2);
                int ends[4] = {a, a1, c, c1};
                for (int e = 0; e < 4; ++e) {
                    if (dlb[ends[e]]) {
                        dlb[ends[e]] = 0;
                        ++active;
                    }
                }
                moved = 1;
                break;
            }
        }
        if (!moved) {
            dlb[a] = 1;
            --active;
            a = (a + 1) % n;
        }
    }
#undef D
    free(pos);
    free(dlb);
    return orc_tour_length(n, dist, tour);
}

/* ------------------------------------------------------------------------
 * Colony
 * ---------------------------------------------------------------------- */
struct orc_colony {
    int n, ants, cl, alpha, beta, pher_mode, ls_nn;
    float rho;
    double pdec;
    uint64_t seed;
    int32_t* dist;    /* n*n */
    float* heur;      /* n*n eta^beta (dense mode) */
    uint16_t* cand;   /* n*cl */
    float* tau;       /* n*n (dense) or n*cl (candidates) */
    float* choice;    /* n*n (dense) */
    float* chc;       /* n*cl: choice_info along the candidate lists */
    uint16_t* lsnn;   /* n*ls_nn */
    uint16_t* tours;  /* ants*n */
    int64_t* lengths; /* ants */
    int64_t* fb_steps;
    int64_t* fb_nodes;
    uint16_t* nn_tour;
    int64_t nn_len;
    int has_gb;
    int deposit;      /* ORC_DEPOSIT_ITERATION_BEST or ORC_DEPOSIT_GLOBAL_BEST */
    int select;       /* ORC_SELECT_WRS or ORC_SELECT_PRWM */
    int directed;     /* ORC_PROBLEM_ATSP: edges (i,j) are directed */
    int64_t gb_len;
    uint16_t* gb_tour;
    float tmin, tmax;
    int64_t ib_ant, ib_len;
};

orc_colony* orc_create(int n, const int32_t* dist, int ants, int cand_len, int alpha, int beta,
                       float rho, double pdec, uint64_t seed, int pher_mode, int ls_nn) {
    if (n < 3 || n > 65535 || ants < 1 || cand_len < 0 || alpha < 0 || beta < 0 || alpha > 8 ||
        beta > 8 || !(rho > 0.0f && rho < 1.0f) || !(pdec > 0.0 && pdec < 1.0) || ls_nn < 0 ||
        ls_nn > n - 1 || (pher_mode != ORC_PHER_DENSE && pher_mode != ORC_PHER_CANDIDATES))
        return NULL;
    int cl = cand_len < n - 1 ? cand_len : n - 1;
    if (pher_mode == ORC_PHER_CANDIDATES && cl == 0) return NULL;
    orc_colony* c = (orc_colony*)calloc(1, sizeof(orc_colony));
    size_t nn2 = (size_t)n * n;
    c->n = n;
    c->ants = ants;
    c->cl = cl;
    c->alpha = alpha;
    c->beta = beta;
    c->rho = rho;
    c->pdec = pdec;
    c->seed = seed;
    c->pher_mode = pher_mode;
    c->ls_nn = ls_nn;
    c->dist = (int32_t*)malloc(sizeof(int32_t) * nn2);
    memcpy(c->dist, dist, sizeof(int32_t) * nn2);
    c->cand = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n * (cl ? cl : 1));
    c->chc = (float*)calloc((size_t)n * (cl ? cl : 1), sizeof(float));
    if (cl) orc_nearest(n, dist, cl, c->cand);
    if (ls_nn) {
        c->lsnn = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n * ls_nn);
        orc_nearest(n, dist, ls_nn, c->lsnn);
    }
    if (pher_mode == ORC_PHER_DENSE) {
        c->heur = (float*)malloc(sizeof(float) * nn2);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                c->heur[(size_t)i * n + j] = (i == j) ? 0.0f : heur_of(dist[(size_t)i * n + j], beta);
        c->tau = (float*)malloc(sizeof(float) * nn2);
        c->choice = (float*)malloc(sizeof(float) * nn2);
    } else {
        c->tau = (float*)malloc(sizeof(float) * (size_t)n * cl);
    }
    c->tours = (uint16_t*)calloc((size_t)ants * n, sizeof(uint16_t));
    c->lengths = (int64_t*)calloc((size_t)ants, sizeof(int64_t));
    c->fb_steps = (int64_t*)calloc((size_t)ants, sizeof(int64_t));
    c->fb_nodes = (int64_t*)calloc((size_t)ants, sizeof(int64_t));
    c->gb_tour = (uint16_t*)calloc((size_t)n, sizeof(uint16_t));
    c->nn_tour = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n);
    /* Alg. 1 set-up: limits from the nearest-neighbour tour, tau <- tau_max */
    c->nn_len = orc_nn_tour(n, dist, c->nn_tour);
    orc_limits(rho, c->nn_len, n, pdec, &c->tmin, &c->tmax);
    size_t ntau = pher_mode == ORC_PHER_DENSE ? nn2 : (size_t)n * cl;
    for (size_t e = 0; e < ntau; ++e) c->tau[e] = c->tmax;
    c->has_gb = 0;
    c->gb_len = -1;
    c->ib_ant = -1;
    c->ib_len = -1;
    return c;
}

void orc_destroy(orc_colony* c) {
    if (!c) return;
    free(c->dist);
    free(c->heur);
    free(c->cand);
    free(c->tau);
    free(c->choice);
    free(c->chc);
    free(c->lsnn);
    free(c->tours);
    free(c->lengths);
    free(c->fb_steps);
    free(c->fb_nodes);
    free(c->nn_tour);
    free(c->gb_tour);
    free(c);
}

/* choice_info = tau^alpha * eta^beta (Sec. 2.1), along the candidate lists too */
void orc_prepare_choice(orc_colony* c) {
    int n = c->n, cl = c->cl;
    if (c->pher_mode == ORC_PHER_DENSE) {
        for (size_t e = 0; e < (size_t)n * n; ++e)
            c->choice[e] = powi_f32(c->tau[e], c->alpha) * c->heur[e];
        for (int i = 0; i < n; ++i)
            for (int r = 0; r < cl; ++r)
                c->chc[(size_t)i * cl + r] = c->choice[(size_t)i * n + c->cand[(size_t)i * cl + r]];
    } else {
        for (int i = 0; i < n; ++i)
            for (int r = 0; r < cl; ++r) {
                int j = c->cand[(size_t)i * cl + r];
                c->chc[(size_t)i * cl + r] =
                    powi_f32(c->tau[(size_t)i * cl + r], c->alpha) * heur_of(c->dist[(size_t)i * n + j], c->beta);
            }
    }
}

/* weight of the edge (cur, v) in the all-node fallback */
static float fallback_weight(const orc_colony* c, int cur, int v) {
    if (c->pher_mode == ORC_PHER_DENSE) return c->choice[(size_t)cur * c->n + v];
    return powi_f32(c->tmin, c->alpha) * heur_of(c->dist[(size_t)cur * c->n + v], c->beta);
}

/* The parallel roulette wheel of Sec. 4.2.1 with p = 64 workers: the m
 * weights are cut into 64 chunks of ceil(m/64) consecutive entries (the last
 * chunks may be short or empty); each chunk's weights are summed left to
 * right, and the chunk sums' inclusive prefix sums are formed left to right,
 * P[l] = P[l-1] + s[l]. The draw u times the total P[63] is the target; the
 * winning chunk is the first with a positive sum whose prefix exceeds the
 * target (the last chunk with a positive sum if rounding leaves none). Inside
 * it the same is done again, with the target less the prefix before the
 * chunk, until a chunk holds one weight. Returns the winning index; m >= 1
 * and some weight > 0. */
static int prwm_pick(const float* w, int m, float u) {
    int lo = 0, len = m;
    float target = 0.0f;
    int first = 1;
    for (;;) {
        const int c = (len + 63) / 64;
        float s[64], P[64];
        for (int l = 0; l < 64; ++l) {
            float a = 0.0f;
            for (int q = l * c; q < (l + 1) * c && q < len; ++q) a = a + w[lo + q];
            s[l] = a;
            P[l] = l == 0 ? a : P[l - 1] + a;
        }
        if (first) {
            target = u * P[63];
            first = 0;
        }
        int win = -1;
        for (int l = 0; l < 64 && win < 0; ++l)
            if (s[l] > 0.0f && P[l] > target) win = l;
        for (int l = 63; l >= 0 && win < 0; --l)
            if (s[l] > 0.0f) win = l;
        if (win < 0) win = 0;
        if (win > 0) target = target - P[win - 1];
        lo += win * c;
        if (c == 1) return lo;
        len = len - win * c < c ? len - win * c : c;
    }
}

/* Node selection by the parallel roulette wheel (Sec. 4.2.1), the paper's
 * baseline: one draw per step (slot 0); the wheel over the unvisited
 * candidates by rank (visited ones weigh 0), or, when none is left, over
 * every unvisited node in index order. */
static int select_prwm(const orc_colony* c, int cur, const uint8_t* visited, uint32_t it, uint32_t ant,
                       uint32_t step, int* fallback) {
    int cl = c->cl, n = c->n;
    float u = orc_u01(orc_draw_word(c->seed, it, ant, step, 0u));
    float* w = (float*)malloc(sizeof(float) * (size_t)(cl > 0 ? cl : 1)); /* cl may exceed 64 */
    int any = 0;
    for (int r = 0; r < cl; ++r) {
        int v = c->cand[(size_t)cur * cl + r];
        w[r] = visited[v] ? 0.0f : c->chc[(size_t)cur * cl + r];
        any |= w[r] > 0.0f;
    }
    *fallback = 0;
    if (any) {
        const int pick = c->cand[(size_t)cur * cl + prwm_pick(w, cl, u)];
        free(w);
        return pick;
    }
    free(w);
    *fallback = 1;
    int* list = (int*)malloc(sizeof(int) * (size_t)n);
    float* wl = (float*)malloc(sizeof(float) * (size_t)n);
    int L = 0, pos = 0;
    for (int v = 0; v < n; ++v)
        if (!visited[v]) {
            list[L] = v;
            wl[L] = fallback_weight(c, cur, v);
            pos |= wl[L] > 0.0f;
            ++L;
        }
    /* (every weight 0: the lowest unvisited node, as WRS's equal keys give) */
    int v = L == 0 ? -1 : pos ? list[prwm_pick(wl, L, u)] : list[0];
    free(list);
    free(wl);
    return v;
}

/* Node selection by weighted reservoir sampling (Alg. 4, Sec. 4.2.2): every
 * eligible node v draws u and gets the key ln(u) * (1/w_v), the logarithm of
 * Sec. 4.2.2 times the weight's reciprocal, which that section suggests
 * computing in advance (here: one IEEE division, then one product); the
 * largest key wins (a reservoir of size one); equal keys go to the lowest
 * node index. The eligible set is the unvisited part of the candidate list
 * of `cur` (Sec. 4.3); when it is empty, every unvisited node. */
int orc_select_next(const orc_colony* c, int cur, const uint8_t* visited, uint32_t it, uint32_t ant,
                    uint32_t step, int* fallback) {
    if (c->select == ORC_SELECT_PRWM) return select_prwm(c, cur, visited, it, ant, step, fallback);
    int cl = c->cl;
    int best = -1;
    float best_key = 0.0f;
    for (int r = 0; r < cl; ++r) {
        int v = c->cand[(size_t)cur * cl + r];
        if (visited[v]) continue;
        float u = orc_u01(orc_draw_word(c->seed, it, ant, step, (uint32_t)r));
        float recip = 1.0f / c->chc[(size_t)cur * cl + r];
        float key = orc_logf(u) * recip;
        if (best < 0 || key > best_key || (key == best_key && v < best)) {
            best = v;
            best_key = key;
        }
    }
    *fallback = 0;
    if (best >= 0) return best;
    *fallback = 1;
    for (int v = 0; v < c->n; ++v) {
        if (visited[v]) continue;
        float u = orc_u01(orc_draw_word(c->seed, it, ant, step, (uint32_t)(cl + v)));
        float recip = 1.0f / fallback_weight(c, cur, v);
        float key = orc_logf(u) * recip;
        if (best < 0 || key > best_key || (key == best_key && v < best)) {
            best = v;
            best_key = key;
        }
    }
    return best;
}

static void construct_ant(orc_colony* c, uint32_t it, int a, uint8_t* visited) {
    int n = c->n;
    uint16_t* tour = c->tours + (size_t)a * n;
    memset(visited, 0, (size_t)n);
    int cur = (int)orc_start_node(c->seed, it, (uint32_t)a, (uint32_t)n);
    tour[0] = (uint16_t)cur;
    visited[cur] = 1;
    int64_t fsteps = 0, fnodes = 0;
    for (int k = 1; k < n; ++k) {
        int fb = 0;
        int v = orc_select_next(c, cur, visited, it, (uint32_t)a, (uint32_t)k, &fb);
        if (fb) {
            fsteps += 1;
            fnodes += n - k; /* unvisited nodes enumerated */
        }
        tour[k] = (uint16_t)v;
        visited[v] = 1;
        cur = v;
    }
    c->lengths[a] = orc_tour_length(n, c->dist, tour);
    c->fb_steps[a] = fsteps;
    c->fb_nodes[a] = fnodes;
}

void orc_construct(orc_colony* c, uint32_t it, int nthreads) {
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        uint8_t* visited = (uint8_t*)malloc((size_t)c->n);
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < c->ants; ++a) construct_ant(c, it, a, visited);
        free(visited);
    }
}

void orc_two_opt(orc_colony* c, int nthreads) {
    if (c->ls_nn <= 0) return;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int a = 0; a < c->ants; ++a)
        c->lengths[a] = orc_two_opt_tour(c->n, c->dist, c->lsnn, c->ls_nn, c->tours + (size_t)a * c->n);
}

/* Alg. 1 after construction: iteration best; global best and limits if it
 * improved; evaporation tau <- max((1-rho) tau, tau_min); deposit of
 * 1/C_ib on both directions of the iteration best's edges (or, with the
 * global-best deposit that Sec. 2.1 allows, 1/C_gb on the global best's,
 * the global best being updated first); every stored trail clamped to
 * tau_max. On an asymmetric instance the tour's edge (i,j) is its arc from
 * i to the successor j, and only tau_ij receives the deposit. */
void orc_update(orc_colony* c) {
    int n = c->n, cl = c->cl;
    int ib = 0;
    for (int a = 1; a < c->ants; ++a)
        if (c->lengths[a] < c->lengths[ib]) ib = a;
    int64_t C_ib = c->lengths[ib];
    const uint16_t* ibt = c->tours + (size_t)ib * n;
    c->ib_ant = ib;
    c->ib_len = C_ib;
    if (!c->has_gb || C_ib < c->gb_len) {
        c->has_gb = 1;
        c->gb_len = C_ib;
        memcpy(c->gb_tour, ibt, sizeof(uint16_t) * (size_t)n);
        orc_limits(c->rho, c->gb_len, n, c->pdec, &c->tmin, &c->tmax);
    }
    const uint16_t* dep = c->deposit == ORC_DEPOSIT_GLOBAL_BEST ? c->gb_tour : ibt;
    int64_t C_dep = c->deposit == ORC_DEPOSIT_GLOBAL_BEST ? c->gb_len : C_ib;
    int* succ = (int*)malloc(sizeof(int) * (size_t)n);
    int* pred = (int*)malloc(sizeof(int) * (size_t)n);
    for (int k = 0; k < n; ++k) {
        succ[dep[k]] = dep[(k + 1) % n];
        pred[dep[(k + 1) % n]] = dep[k];
    }
    float keep = 1.0f - c->rho;
    float delta = (float)(1.0 / (double)C_dep);
    float tmin = c->tmin, tmax = c->tmax;
    if (c->pher_mode == ORC_PHER_DENSE) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                float* t = &c->tau[(size_t)i * n + j];
                float v = keep * *t;
                if (v < tmin) v = tmin;
                if (j == succ[i] || (!c->directed && j == pred[i])) v = v + delta;
                if (v > tmax) v = tmax;
                *t = v;
            }
    } else {
        for (int i = 0; i < n; ++i)
            for (int r = 0; r < cl; ++r) {
                int j = c->cand[(size_t)i * cl + r];
                float* t = &c->tau[(size_t)i * cl + r];
                float v = keep * *t;
                if (v < tmin) v = tmin;
                if (j == succ[i] || (!c->directed && j == pred[i])) v = v + delta;
                if (v > tmax) v = tmax;
                *t = v;
            }
    }
    free(succ);
    free(pred);
}

void orc_iterate(orc_colony* c, uint32_t it, int nthreads) {
    orc_prepare_choice(c);
    orc_construct(c, it, nthreads);
    orc_two_opt(c, nthreads);
    orc_update(c);
}

/* ---- accessors ---- */
int orc_set_select(orc_colony* c, int mode) {
    if (mode != ORC_SELECT_WRS && mode != ORC_SELECT_PRWM) return -1;
    c->select = mode;
    return 0;
}
int orc_set_problem(orc_colony* c, int mode) {
    if (mode != ORC_PROBLEM_TSP && mode != ORC_PROBLEM_ATSP) return -1;
    if (mode == ORC_PROBLEM_ATSP && c->ls_nn > 0) return -1;
    c->directed = mode == ORC_PROBLEM_ATSP;
    return 0;
}
int orc_set_deposit(orc_colony* c, int mode) {
    if (mode != ORC_DEPOSIT_ITERATION_BEST && mode != ORC_DEPOSIT_GLOBAL_BEST) return -1;
    c->deposit = mode;
    return 0;
}
int orc_n(const orc_colony* c) { return c->n; }
int orc_cl(const orc_colony* c) { return c->cl; }
void orc_get_tours(const orc_colony* c, uint16_t* out) {
    memcpy(out, c->tours, sizeof(uint16_t) * (size_t)c->ants * c->n);
}
void orc_get_lengths(const orc_colony* c, int64_t* out) {
    memcpy(out, c->lengths, sizeof(int64_t) * (size_t)c->ants);
}
static size_t ntau(const orc_colony* c) {
    return c->pher_mode == ORC_PHER_DENSE ? (size_t)c->n * c->n : (size_t)c->n * c->cl;
}
void orc_get_pheromone(const orc_colony* c, float* out) { memcpy(out, c->tau, sizeof(float) * ntau(c)); }
void orc_set_pheromone(orc_colony* c, const float* in) { memcpy(c->tau, in, sizeof(float) * ntau(c)); }
void orc_get_choice(const orc_colony* c, float* out) {
    if (c->choice) memcpy(out, c->choice, sizeof(float) * (size_t)c->n * c->n);
}
void orc_get_chc(const orc_colony* c, float* out) { memcpy(out, c->chc, sizeof(float) * (size_t)c->n * c->cl); }
void orc_get_cand(const orc_colony* c, uint16_t* out) {
    memcpy(out, c->cand, sizeof(uint16_t) * (size_t)c->n * c->cl);
}
void orc_get_heuristic(const orc_colony* c, float* out) {
    int n = c->n;
    if (c->pher_mode == ORC_PHER_DENSE && c->heur) {
        memcpy(out, c->heur, sizeof(float) * (size_t)n * n);
        return;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            out[(size_t)i * n + j] = (i == j) ? 0.0f : heur_of(c->dist[(size_t)i * n + j], c->beta);
}
/* Replaces the dense heuristic matrix (eta^beta, n*n) used from the next
 * choice_info on, e.g. by a learned heuristic; -1 in candidate-only mode,
 * which keeps no matrix. */
int orc_set_heuristic(orc_colony* c, const float* heur) {
    if (c->pher_mode != ORC_PHER_DENSE || !c->heur) return -1;
    memcpy(c->heur, heur, sizeof(float) * (size_t)c->n * c->n);
    return 0;
}
void orc_get_fallback(const orc_colony* c, int64_t* steps, int64_t* nodes) {
    memcpy(steps, c->fb_steps, sizeof(int64_t) * (size_t)c->ants);
    memcpy(nodes, c->fb_nodes, sizeof(int64_t) * (size_t)c->ants);
}
void orc_restore(orc_colony* c, const float* limits, int64_t gb_len, const uint16_t* gb_tour) {
    c->tmin = limits[0];
    c->tmax = limits[1];
    c->has_gb = gb_len >= 0;
    c->gb_len = gb_len;
    if (gb_len >= 0) memcpy(c->gb_tour, gb_tour, sizeof(uint16_t) * (size_t)c->n);
}
void orc_get_limits(const orc_colony* c, float* limits) {
    limits[0] = c->tmin;
    limits[1] = c->tmax;
}
int64_t orc_get_best(const orc_colony* c, uint16_t* gb_tour) {
    if (gb_tour && c->has_gb) memcpy(gb_tour, c->gb_tour, sizeof(uint16_t) * (size_t)c->n);
    return c->has_gb ? c->gb_len : -1;
}
int64_t orc_get_nn_tour(const orc_colony* c, uint16_t* tour) {
    if (tour) memcpy(tour, c->nn_tour, sizeof(uint16_t) * (size_t)c->n);
    return c->nn_len;
}
void orc_get_iteration_best(const orc_colony* c, int64_t* ib) {
    ib[0] = c->ib_ant;
    ib[1] = c->ib_len;
}
