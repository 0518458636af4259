// C ABI of libmmas: parameter checks, the workspace layout, and the call
// sequence of Alg. 1 on one HIP stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "internal.hpp"

static_assert(sizeof(mmas_params) == 64 && offsetof(mmas_params, problem) == 56, "mmas_params layout");

using mmas::Shape;
using mmas::Views;

struct mmas_ctx {
    mmas_params p;
    Shape s;
    Views v;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    size_t off[MMAS_BUF_COUNT];
    size_t len[MMAS_BUF_COUNT];
    size_t off_succ, off_pred, off_nnd, off_inv, off_cinv;
    bool choice_stale;
    bool constructed;
    // per-call timing (mmas_set_timing): event pairs not yet read, and the totals
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spare;
    double ms[MMAS_TIMING_KINDS] = {0, 0, 0, 0};
    int64_t calls[MMAS_TIMING_KINDS] = {0, 0, 0, 0};
    ~mmas_ctx();
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool params_ok(const mmas_params* p) {
    if (!p) return false;
    if (p->n < 3 || p->n > 65535) return false;
    if (p->ants < 1) return false;
    if (p->cand_len < 0 || p->cand_len > 64) return false;
    if (p->alpha < 0 || p->alpha > 8 || p->beta < 0 || p->beta > 8) return false;
    if (!(p->rho > 0.0f && p->rho < 1.0f)) return false;
    if (!(p->p_best > 0.0 && p->p_best < 1.0)) return false;
    if (p->tabu != MMAS_TABU_BITMASK && p->tabu != MMAS_TABU_COMPACT && p->tabu != MMAS_TABU_LIST) return false;
    if (p->pher_mode != MMAS_PHER_DENSE && p->pher_mode != MMAS_PHER_CANDIDATES) return false;
    const int cl = p->cand_len < p->n - 1 ? p->cand_len : p->n - 1;
    if (p->pher_mode == MMAS_PHER_CANDIDATES && cl == 0) return false;
    if (p->ls_nn < 0 || p->ls_nn > 32 || p->ls_nn > p->n - 1) return false;
    if (p->deposit != MMAS_DEPOSIT_ITERATION_BEST && p->deposit != MMAS_DEPOSIT_GLOBAL_BEST) return false;
    if (p->problem != MMAS_PROBLEM_TSP && p->problem != MMAS_PROBLEM_ATSP) return false;
    if (p->problem == MMAS_PROBLEM_ATSP && p->ls_nn != 0) return false;
    return true;
}

Shape shape_of(const mmas_params* p) {
    Shape s{};
    s.n = p->n;
    s.ants = p->ants;
    s.cl = p->cand_len < p->n - 1 ? p->cand_len : p->n - 1;
    s.alpha = p->alpha;
    s.beta = p->beta;
    s.ls_nn = p->ls_nn;
    s.pher = p->pher_mode;
    s.tabu = p->tabu;
    s.deposit = p->deposit;
    s.directed = p->problem == MMAS_PROBLEM_ATSP ? 1 : 0;
    s.rho = p->rho;
    s.pdec = std::pow(p->p_best, 1.0 / (double)p->n);
    s.seed = p->seed;
    s.ants_per_block = 4;
    s.table_rows = -1;
    s.lanes_per_ant = 64;
    s.construct_waves = 0;
    s.two_opt_waves = 0;  // by the instance size (launch_two_opt)
    return s;
}

// Byte sizes of every view, then their offsets (256-byte aligned).
size_t layout(const Shape& s, size_t* off, size_t* len, size_t* off_succ, size_t* off_pred, size_t* off_nnd,
              size_t* off_inv, size_t* off_cinv) {
    const size_t n = (size_t)s.n, cl = (size_t)s.cl, ants = (size_t)s.ants;
    const bool dense = s.pher == MMAS_PHER_DENSE;
    len[MMAS_BUF_DIST] = 4 * n * n;
    len[MMAS_BUF_PHEROMONE] = dense ? 4 * n * n : 4 * n * cl;
    len[MMAS_BUF_CHOICE] = dense ? 4 * n * n : 0;
    len[MMAS_BUF_CHC] = 4 * n * cl;
    len[MMAS_BUF_CAND] = 2 * n * cl;
    len[MMAS_BUF_HEUR] = dense ? 4 * n * n : 4 * n * cl;
    len[MMAS_BUF_TOURS] = 2 * n * ants;
    len[MMAS_BUF_LENGTHS] = 8 * ants;
    len[MMAS_BUF_GB_TOUR] = 2 * n;
    len[MMAS_BUF_NN_TOUR] = 2 * n;
    len[MMAS_BUF_FALLBACK] = 16 * ants;
    len[MMAS_BUF_STATE] = sizeof(mmas_device_state);
    len[MMAS_BUF_LSNN] = 2 * n * (size_t)s.ls_nn;
    size_t pos = 0;
    for (int b = 0; b < MMAS_BUF_COUNT; ++b) {
        off[b] = pos;
        pos = align_up(pos + len[b]);
    }
    *off_succ = pos;
    pos = align_up(pos + 2 * n);
    *off_pred = pos;
    pos = align_up(pos + 2 * n);
    *off_nnd = pos;  // d(i, nn[i][r]) of the 2-opt lists
    pos = align_up(pos + 4 * n * (size_t)s.ls_nn);
    *off_inv = pos;  // 1 / chc along the candidate lists
    pos = align_up(pos + 4 * n * cl);
    *off_cinv = pos;  // 1 / choice_info, dense trails
    pos = align_up(pos + (dense ? 4 * n * n : 0));
    return pos;
}

template <class T>
T* at(char* base, size_t off, size_t len) {
    return len ? reinterpret_cast<T*>(base + off) : nullptr;
}

thread_local char g_last_error[256] = "";

// Folds every pending event pair into the totals (waits for each stop event).
hipError_t fold_timing(mmas_ctx* c) {
    hipError_t first = hipSuccess;
    for (auto& p : c->pending) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(p.second.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.second.first, p.second.second);
        if (e == hipSuccess) {
            c->ms[p.first] += ms;
            c->calls[p.first] += 1;
        } else if (first == hipSuccess) {
            first = e;
        }
        c->spare.push_back(p.second);
    }
    c->pending.clear();
    return first;
}

// Brackets one enqueued call with events when timing is on. Used as
//   TimedCall t(c, kind); ...launch...; return t.done(status);
struct TimedCall {
    mmas_ctx* c;
    int kind;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    TimedCall(mmas_ctx* ctx, int k) : c(ctx), kind(k) {
        if (!c->timing) return;
        if (c->pending.size() >= 1024) (void)fold_timing(c);  // bounded memory
        if (!c->spare.empty()) {
            ev = c->spare.back();
            c->spare.pop_back();
        } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
            ev = {nullptr, nullptr};
            return;
        }
        if (hipEventRecord(ev.first, c->stream) != hipSuccess) ev = {nullptr, nullptr};
    }
    void done(bool launched) {
        if (!ev.first) return;
        if (launched && hipEventRecord(ev.second, c->stream) == hipSuccess)
            c->pending.push_back({kind, ev});
        else
            c->spare.push_back(ev);
        ev = {nullptr, nullptr};
    }
};

mmas_status hip_status(hipError_t e) { return e == hipSuccess ? MMAS_OK : mmas::hip_fail(e, "HIP call"); }

}  // namespace

namespace mmas {
mmas_status hip_fail(hipError_t e, const char* where) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    return MMAS_EHIP;
}

// The device views and constants of a context (for batches).
bool ctx_views(mmas_ctx* c, Views* v, Shape* s) {
    if (!c) return false;
    *v = c->v;
    *s = c->s;
    return true;
}
}  // namespace mmas

mmas_ctx::~mmas_ctx() {
    if (!pending.empty()) (void)hipStreamSynchronize(stream);
    for (auto& p : pending) spare.push_back(p.second);
    for (auto& p : spare) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
}

extern "C" {

size_t mmas_workspace_bytes(const mmas_params* p) {
    if (!params_ok(p)) return 0;
    Shape s = shape_of(p);
    size_t off[MMAS_BUF_COUNT], len[MMAS_BUF_COUNT], os, op, od, oi, oc;
    return layout(s, off, len, &os, &op, &od, &oi, &oc);
}

mmas_status mmas_create(const int32_t* dist_host, const mmas_params* p, void* dev_ws, size_t ws_bytes,
                        void* hip_stream, mmas_ctx** out) {
    if (!out) return MMAS_EINVAL;
    *out = nullptr;
    if (!dist_host || !params_ok(p) || !dev_ws) return MMAS_EINVAL;
    if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) return MMAS_EINVAL;
    Shape s = shape_of(p);
    mmas_ctx* c = new (std::nothrow) mmas_ctx();
    if (!c) return MMAS_EHIP;
    c->p = *p;
    c->s = s;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->ws = reinterpret_cast<char*>(dev_ws);
    c->ws_bytes = ws_bytes;
    const size_t need = layout(s, c->off, c->len, &c->off_succ, &c->off_pred, &c->off_nnd, &c->off_inv, &c->off_cinv);
    if (ws_bytes < need) {
        delete c;
        return MMAS_ENOSPACE;
    }
    {  // every tabu must fit in LDS (the list tabu takes 4n bytes per ant)
        int dev = 0, maxlds = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) {
            delete c;
            return mmas::hip_fail(e, "device query");
        }
        if (mmas::wide_lds_per_ant(s) > (size_t)maxlds ||
            (s.ls_nn > 0 && mmas::two_opt_lds_bytes(s, false) + mmas::kTwoOptStaticLds > (size_t)maxlds)) {
            delete c;
            return MMAS_EUNSUPPORTED;
        }
    }
    Views& v = c->v;
    char* b = c->ws;
    v.dist = at<int32_t>(b, c->off[MMAS_BUF_DIST], c->len[MMAS_BUF_DIST]);
    v.tau = at<float>(b, c->off[MMAS_BUF_PHEROMONE], c->len[MMAS_BUF_PHEROMONE]);
    v.choice = at<float>(b, c->off[MMAS_BUF_CHOICE], c->len[MMAS_BUF_CHOICE]);
    v.chc = at<float>(b, c->off[MMAS_BUF_CHC], c->len[MMAS_BUF_CHC]);
    v.cand = at<uint16_t>(b, c->off[MMAS_BUF_CAND], c->len[MMAS_BUF_CAND]);
    v.heur = at<float>(b, c->off[MMAS_BUF_HEUR], c->len[MMAS_BUF_HEUR]);
    v.tours = at<uint16_t>(b, c->off[MMAS_BUF_TOURS], c->len[MMAS_BUF_TOURS]);
    v.lengths = at<int64_t>(b, c->off[MMAS_BUF_LENGTHS], c->len[MMAS_BUF_LENGTHS]);
    v.gb_tour = at<uint16_t>(b, c->off[MMAS_BUF_GB_TOUR], c->len[MMAS_BUF_GB_TOUR]);
    v.nn_tour = at<uint16_t>(b, c->off[MMAS_BUF_NN_TOUR], c->len[MMAS_BUF_NN_TOUR]);
    v.fallback = at<int64_t>(b, c->off[MMAS_BUF_FALLBACK], c->len[MMAS_BUF_FALLBACK]);
    v.state = at<mmas_device_state>(b, c->off[MMAS_BUF_STATE], c->len[MMAS_BUF_STATE]);
    v.lsnn = at<uint16_t>(b, c->off[MMAS_BUF_LSNN], c->len[MMAS_BUF_LSNN]);
    v.chc_inv = c->len[MMAS_BUF_CHC] ? reinterpret_cast<float*>(b + c->off_inv) : nullptr;
    v.choice_inv = c->len[MMAS_BUF_CHOICE] ? reinterpret_cast<float*>(b + c->off_cinv) : nullptr;
    v.succ = reinterpret_cast<uint16_t*>(b + c->off_succ);
    v.pred = reinterpret_cast<uint16_t*>(b + c->off_pred);

    hipStream_t st = c->stream;
    const char* step = "copy of the distance matrix";
    hipError_t e = hipMemcpyAsync(v.dist, dist_host, c->len[MMAS_BUF_DIST], hipMemcpyHostToDevice, st);
    if (e == hipSuccess && (step = "state reset")) e = hipMemsetAsync(v.state, 0, sizeof(mmas_device_state), st);
    if (e == hipSuccess && (step = "validation")) e = mmas::launch_validate(v, s, st);
    if (e == hipSuccess && (step = "candidate lists")) e = mmas::launch_nearest(v.dist, s.n, s.cl, v.cand, st);
    if (e == hipSuccess && (step = "2-opt lists")) e = mmas::launch_nearest(v.dist, s.n, s.ls_nn, v.lsnn, st);
    if (e == hipSuccess && (step = "heuristic")) e = mmas::launch_heuristic(v, s, st);
    if (e == hipSuccess && (step = "2-opt list distances"))
        e = mmas::launch_two_opt_prepare(v, s, reinterpret_cast<int32_t*>(c->ws + c->off_nnd), st);
    if (e == hipSuccess && (step = "nearest-neighbour tour")) e = mmas::launch_nn_tour(v, s, st);
    if (e == hipSuccess && (step = "trail limits")) e = mmas::launch_init_trails(v, s, st);
    mmas_device_state hs;
    if (e == hipSuccess && (step = "state read")) e = hipMemcpyAsync(&hs, v.state, sizeof(hs), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && (step = "set-up synchronisation")) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete c;
        return mmas::hip_fail(e, step);
    }
    if (hs.flags != 0u || !std::isfinite(hs.tau_max) || !(hs.tau_min > 0.0f)) {
        delete c;
        return MMAS_EINVAL;
    }
    c->choice_stale = true;
    c->constructed = false;
    *out = c;
    return MMAS_OK;
}

mmas_status mmas_prepare_choice_info(mmas_ctx* c) {
    if (!c) return MMAS_EINVAL;
    if (!c->choice_stale) return MMAS_OK;
    TimedCall t(c, MMAS_TIMING_CHOICE);
    hipError_t e = mmas::launch_choice(c->v, c->s, c->stream);
    t.done(e == hipSuccess);
    if (e != hipSuccess) return hip_status(e);
    c->choice_stale = false;
    return MMAS_OK;
}

mmas_status mmas_construct(mmas_ctx* c, uint32_t iteration) {
    if (!c) return MMAS_EINVAL;
    mmas_status r = mmas_prepare_choice_info(c);
    if (r != MMAS_OK) return r;
    TimedCall t(c, MMAS_TIMING_CONSTRUCT);
    hipError_t e = mmas::launch_construct(c->v, c->s, iteration, c->stream);
    t.done(e == hipSuccess);
    if (e != hipSuccess) return hip_status(e);
    c->constructed = true;
    return MMAS_OK;
}

mmas_status mmas_set_launch(mmas_ctx* c, int32_t ants_per_block, int32_t table_rows, int32_t lanes_per_ant,
                            int32_t waves_per_ant) {
    if (!c) return MMAS_EINVAL;
    if (waves_per_ant != 0 && waves_per_ant != 1 && waves_per_ant != 2 && waves_per_ant != 4 && waves_per_ant != 8 &&
        waves_per_ant != 16)
        return MMAS_EINVAL;
    if (ants_per_block != 0 && ants_per_block != 1 && ants_per_block != 2 && ants_per_block != 4 &&
        ants_per_block != 8 && ants_per_block != 16)
        return MMAS_EINVAL;
    if (table_rows < -1) return MMAS_EINVAL;
    if (lanes_per_ant != 0 && lanes_per_ant != 32 && lanes_per_ant != 64) return MMAS_EINVAL;
    c->s.ants_per_block = ants_per_block == 0 ? 4 : ants_per_block;
    c->s.table_rows = table_rows;
    c->s.lanes_per_ant = lanes_per_ant == 0 ? 64 : lanes_per_ant;
    c->s.construct_waves = waves_per_ant;
    return MMAS_OK;
}

mmas_status mmas_set_selection(mmas_ctx* c, int32_t select) {
    if (!c || (select != MMAS_SELECT_WRS && select != MMAS_SELECT_PRWM)) return MMAS_EINVAL;
    if (select == MMAS_SELECT_PRWM && c->s.tabu != MMAS_TABU_BITMASK) return MMAS_EUNSUPPORTED;
    c->s.select = select;
    return MMAS_OK;
}

mmas_status mmas_set_two_opt_launch(mmas_ctx* c, int32_t waves_per_ant) {
    if (!c) return MMAS_EINVAL;
    if (waves_per_ant != 0 && waves_per_ant != 1 && waves_per_ant != 2 && waves_per_ant != 4 && waves_per_ant != 8 &&
        waves_per_ant != 16)
        return MMAS_EINVAL;
    c->s.two_opt_waves = waves_per_ant;
    return MMAS_OK;
}

mmas_status mmas_two_opt(mmas_ctx* c) {
    if (!c) return MMAS_EINVAL;
    if (c->s.ls_nn <= 0) return MMAS_EUNSUPPORTED;
    if (!c->constructed) return MMAS_ESTATE;
    TimedCall t(c, MMAS_TIMING_TWO_OPT);
    hipError_t e = mmas::launch_two_opt(c->v, c->s, reinterpret_cast<const int32_t*>(c->ws + c->off_nnd), c->stream);
    t.done(e == hipSuccess);
    return hip_status(e);
}

mmas_status mmas_update_pheromone(mmas_ctx* c) {
    if (!c) return MMAS_EINVAL;
    if (!c->constructed) return MMAS_ESTATE;
    TimedCall t(c, MMAS_TIMING_UPDATE);
    hipError_t e = mmas::launch_update(c->v, c->s, c->stream);
    t.done(e == hipSuccess);
    if (e != hipSuccess) return hip_status(e);
    c->choice_stale = false;  // refreshed by the fused pass
    c->constructed = false;   // these tours have deposited; the next update needs new ones
    return MMAS_OK;
}

mmas_status mmas_best(mmas_ctx* c, int32_t* tour_host, int64_t* len_host) {
    if (!c || !len_host) return MMAS_EINVAL;
    mmas_device_state hs;
    std::vector<uint16_t> t(tour_host ? (size_t)c->s.n : 0);
    hipError_t e = hipMemcpyAsync(&hs, c->v.state, sizeof(hs), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && tour_host)
        e = hipMemcpyAsync(t.data(), c->v.gb_tour, 2 * (size_t)c->s.n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_status(e);
    *len_host = hs.gb_len;
    if (tour_host)
        for (int k = 0; k < c->s.n; ++k) tour_host[k] = hs.gb_len >= 0 ? (int32_t)t[k] : -1;
    return MMAS_OK;
}

mmas_status mmas_buffer(mmas_ctx* c, int which, void** dev_ptr, size_t* bytes) {
    if (!c || which < 0 || which >= MMAS_BUF_COUNT) return MMAS_EINVAL;
    if (dev_ptr) *dev_ptr = c->len[which] ? c->ws + c->off[which] : nullptr;
    if (bytes) *bytes = c->len[which];
    return MMAS_OK;
}

mmas_status mmas_read(mmas_ctx* c, int which, void* host_dst, size_t bytes) {
    if (!c || which < 0 || which >= MMAS_BUF_COUNT || !host_dst) return MMAS_EINVAL;
    if (bytes != c->len[which]) return MMAS_EINVAL;
    if (bytes == 0) return MMAS_OK;
    hipError_t e = hipMemcpyAsync(host_dst, c->ws + c->off[which], bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_status(e);
}

mmas_status mmas_set_pheromone(mmas_ctx* c, const float* host_src) {
    if (!c || !host_src) return MMAS_EINVAL;
    const size_t count = c->len[MMAS_BUF_PHEROMONE] / sizeof(float);
    for (size_t e = 0; e < count; ++e)
        if (!std::isfinite(host_src[e]) || host_src[e] < 0.0f) return MMAS_EINVAL;
    hipError_t e = hipMemcpyAsync(c->v.tau, host_src, c->len[MMAS_BUF_PHEROMONE], hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_status(e);
    c->choice_stale = true;
    return MMAS_OK;
}

mmas_status mmas_restore(mmas_ctx* c, const float* tau_host, const mmas_device_state* state_host,
                         const uint16_t* gb_tour_host) {
    if (!c || !tau_host || !state_host) return MMAS_EINVAL;
    const mmas_device_state in = *state_host;
    if (!std::isfinite(in.tau_min) || !std::isfinite(in.tau_max) || !(in.tau_min > 0.0f) ||
        !(in.tau_min <= in.tau_max) || in.gb_len < -1)
        return MMAS_EINVAL;
    const int n = c->s.n;
    if (in.gb_len >= 0) {
        if (!gb_tour_host) return MMAS_EINVAL;
        std::vector<char> seen((size_t)n, 0);
        for (int k = 0; k < n; ++k) {
            const int v = gb_tour_host[k];
            if (v >= n || seen[(size_t)v]) return MMAS_EINVAL;
            seen[(size_t)v] = 1;
        }
    }
    mmas_status r = mmas_set_pheromone(c, tau_host);  // validates, copies, synchronises
    if (r != MMAS_OK) return r;
    mmas_device_state cur;
    hipError_t e = hipMemcpyAsync(&cur, c->v.state, sizeof(cur), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_status(e);
    mmas_device_state st = in;
    st.nn_len = cur.nn_len;
    st.flags = cur.flags;
    e = hipMemcpyAsync(c->v.state, &st, sizeof(st), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && in.gb_len >= 0)
        e = hipMemcpyAsync(c->v.gb_tour, gb_tour_host, 2 * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_status(e);
}

mmas_status mmas_set_learned_heuristic(mmas_ctx* c, const uint16_t* knn_dev, const float* score_dev) {
    if (!c || !knn_dev || !score_dev || c->s.n < 17) return MMAS_EINVAL;
    if (c->s.directed) return MMAS_EUNSUPPORTED;
    const Shape& s = c->s;
    hipError_t e = mmas::launch_install(c->v.dist, knn_dev, score_dev, c->v.cand, s.n, s.cl, s.beta,
                                        s.pher == MMAS_PHER_DENSE ? 1 : 0, c->v.heur, c->stream);
    if (e != hipSuccess) return hip_status(e);
    c->choice_stale = true;
    return MMAS_OK;
}

mmas_status mmas_synchronize(mmas_ctx* c) {
    if (!c) return MMAS_EINVAL;
    return hip_status(hipStreamSynchronize(c->stream));
}

mmas_status mmas_set_timing(mmas_ctx* c, int32_t on) {
    if (!c) return MMAS_EINVAL;
    c->timing = on != 0;
    return MMAS_OK;
}

mmas_status mmas_read_timing(mmas_ctx* c, double* ms_host, int64_t* calls_host, int32_t reset) {
    if (!c) return MMAS_EINVAL;
    const hipError_t e = fold_timing(c);
    for (int k = 0; k < MMAS_TIMING_KINDS; ++k) {
        if (ms_host) ms_host[k] = c->ms[k];
        if (calls_host) calls_host[k] = c->calls[k];
        if (reset) {
            c->ms[k] = 0.0;
            c->calls[k] = 0;
        }
    }
    return hip_status(e);
}

void mmas_destroy(mmas_ctx* c) {
    if (!c) return;
    // the caller may free the workspace right after this call
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

const char* mmas_last_error(void) { return g_last_error; }

const char* mmas_status_str(mmas_status s) {
    switch (s) {
        case MMAS_OK: return "ok";
        case MMAS_EINVAL: return "invalid argument";
        case MMAS_EUNSUPPORTED: return "unsupported";
        case MMAS_ENOSPACE: return "workspace too small";
        case MMAS_EHIP: return "HIP error";
        case MMAS_ESTATE: return "call out of order";
    }
    return "unknown status";
}

}  // extern "C"
