// Batched MMAS: many instances of uneven size advance one iteration per step
// with three launches for all of them (persistent construction over a tile
// queue, per-instance best and limits, fused update of every row), optionally
// captured once into a hipGraph. Each instance is an ordinary context living
// in its own part of the batch workspace, so its results are those of the
// single-instance calls with the same parameters and iteration numbers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace mmas {
// defined in mmas.hip
bool ctx_views(mmas_ctx* c, Views* v, Shape* s);
}  // namespace mmas

struct mmas_batch {
    int count;
    hipStream_t stream;
    char* ws;
    std::vector<mmas_ctx*> ctx;
    std::vector<mmas::BatchItem> items;
    std::vector<int> order;  // instances by decreasing n
    mmas::BatchItem* d_items;
    int* d_row_start;
    mmas::BatchTile* d_tiles;
    uint32_t* d_it;
    uint32_t* d_queue;
    int total_rows;
    int max_tiles;
    int tabu, pher;
    int per_ant;        // largest per-ant LDS region over the instances (current tabu)
    int per_ant_tabu[3];  // the same for the bitmask, the compact and the list tabu
    int table_request;  // table_bytes as last asked for (-1: all that fits)
    int ants_per_block;
    int lanes_per_ant;
    bool pair_ok;       // every instance has 1 <= cl <= 32
    int table_bytes;
    int ntiles;
    int grid;
    std::vector<mmas::BatchTile> tiles;
    hipGraph_t graph;
    hipGraphExec_t exec;
    // per-launch timing of the construction (mmas_batch_set_timing): event
    // pairs not yet read, spare pairs, and the totals
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending, spare;
    double construct_ms = 0.0;
    int64_t construct_calls = 0;
};

namespace {

constexpr size_t kAlign = 256;
// LDS the persistent construction kernel declares statically (its tile index)
constexpr int kStaticLds = 64;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Header {
    size_t items, row_start, tiles, counters, end;
};

Header header_layout(int count, size_t total_ants) {
    Header h{};
    size_t pos = 0;
    h.items = pos;
    pos = align_up(pos + sizeof(mmas::BatchItem) * (size_t)count);
    h.row_start = pos;
    pos = align_up(pos + sizeof(int) * (size_t)(count + 1));
    h.tiles = pos;
    pos = align_up(pos + sizeof(mmas::BatchTile) * total_ants);  // worst case: one ant per tile
    h.counters = pos;
    pos = align_up(pos + 2 * sizeof(uint32_t));
    h.end = pos;
    return h;
}

__global__ void k_reset_queue(uint32_t* q) {
    if (threadIdx.x == 0) *q = 0u;
}

mmas_status rebuild_tiles(mmas_batch* b) {
    b->tiles.clear();
    for (int i : b->order) {
        const int ants = b->items[i].s.ants;
        for (int a0 = 0; a0 < ants; a0 += b->ants_per_block) b->tiles.push_back(mmas::BatchTile{i, a0});
    }
    b->ntiles = (int)b->tiles.size();
    hipError_t e = hipMemcpyAsync(b->d_tiles, b->tiles.data(), sizeof(mmas::BatchTile) * b->tiles.size(),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return mmas::hip_fail(e, "tile table");
    const int lds = b->table_bytes + b->ants_per_block * b->per_ant;
    int g = mmas::batch_construct_grid(b->tabu, b->pher, b->ants_per_block, b->lanes_per_ant, lds);
    if (g <= 0) return MMAS_EUNSUPPORTED;
    b->grid = std::min(g, b->ntiles);
    return MMAS_OK;
}

mmas_status launch_step(mmas_batch* b) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (b->timing) {
        if (!b->spare.empty()) {
            ev = b->spare.back();
            b->spare.pop_back();
        } else {
            hipError_t ce = hipEventCreate(&ev.first);
            if (ce == hipSuccess) ce = hipEventCreate(&ev.second);
            if (ce != hipSuccess) return mmas::hip_fail(ce, "timing events");
        }
        const hipError_t re = hipEventRecord(ev.first, b->stream);
        if (re != hipSuccess) return mmas::hip_fail(re, "timing event record");
    }
    hipError_t e = mmas::launch_batch_construct(b->d_items, b->d_tiles, b->ntiles, b->d_queue, b->d_it, b->tabu,
                                                b->pher, b->ants_per_block, b->lanes_per_ant, b->table_bytes,
                                                b->per_ant, b->grid, b->stream);
    if (b->timing) {
        if (e == hipSuccess) e = hipEventRecord(ev.second, b->stream);
        if (e == hipSuccess)
            b->pending.push_back(ev);
        else
            b->spare.push_back(ev);
    }
    if (e != hipSuccess) return mmas::hip_fail(e, "batched construction launch");
    e = mmas::launch_batch_update(b->d_items, b->count, b->d_row_start, b->total_rows, b->d_it, b->d_queue, b->stream);
    return e == hipSuccess ? MMAS_OK : mmas::hip_fail(e, "batched update launch");
}

// The tabu of every construction (the device reads no tabu field; the host
// copies follow for the LDS sizes). The caller sets the launch shape again.
void apply_tabu(mmas_batch* b, int tabu) {
    b->tabu = tabu;
    b->per_ant = b->per_ant_tabu[tabu];
    for (auto& it : b->items) it.s.tabu = tabu;
}

// Adds up the timed launches that have finished (waits for them).
hipError_t fold_timing(mmas_batch* b) {
    hipError_t first = hipSuccess;
    for (auto& ev : b->pending) {
        hipError_t e = hipEventSynchronize(ev.second);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
        if (e == hipSuccess) {
            b->construct_ms += ms;
            b->construct_calls += 1;
        } else if (first == hipSuccess) {
            first = e;
        }
        b->spare.push_back(ev);
    }
    b->pending.clear();
    return first;
}

void drop_graph(mmas_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

mmas_status mmas_batch_workspace_bytes(int32_t count, const mmas_params* params, size_t* bytes) {
    if (count < 1 || !params || !bytes) return MMAS_EINVAL;
    size_t total_ants = 0, sub = 0;
    for (int i = 0; i < count; ++i) {
        const size_t w = mmas_workspace_bytes(&params[i]);
        if (w == 0) return MMAS_EINVAL;
        sub += align_up(w);
        total_ants += (size_t)params[i].ants;
    }
    *bytes = header_layout(count, total_ants).end + sub;
    return MMAS_OK;
}

mmas_status mmas_batch_create(int32_t count, const int32_t* const* dists_host, const mmas_params* params, void* dev_ws,
                              size_t ws_bytes, void* hip_stream, mmas_batch** out) {
    if (!out) return MMAS_EINVAL;
    *out = nullptr;
    if (count < 1 || !dists_host || !params || !dev_ws) return MMAS_EINVAL;
    if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) return MMAS_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (!dists_host[i]) return MMAS_EINVAL;
        if (params[i].tabu != params[0].tabu || params[i].pher_mode != params[0].pher_mode) return MMAS_EINVAL;
        if (params[i].ls_nn != 0) return MMAS_EUNSUPPORTED;  // batches carry no local search
    }
    size_t need = 0;
    mmas_status r = mmas_batch_workspace_bytes(count, params, &need);
    if (r != MMAS_OK) return r;
    if (ws_bytes < need) return MMAS_ENOSPACE;

    mmas_batch* b = new (std::nothrow) mmas_batch();
    if (!b) return MMAS_EHIP;
    b->count = count;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->ws = reinterpret_cast<char*>(dev_ws);
    b->tabu = params[0].tabu;
    b->pher = params[0].pher_mode;
    size_t total_ants = 0;
    for (int i = 0; i < count; ++i) total_ants += (size_t)params[i].ants;
    const Header h = header_layout(count, total_ants);
    b->d_items = reinterpret_cast<mmas::BatchItem*>(b->ws + h.items);
    b->d_row_start = reinterpret_cast<int*>(b->ws + h.row_start);
    b->d_tiles = reinterpret_cast<mmas::BatchTile*>(b->ws + h.tiles);
    b->d_it = reinterpret_cast<uint32_t*>(b->ws + h.counters);
    b->d_queue = b->d_it + 1;

    size_t pos = h.end;
    b->ctx.assign(count, nullptr);
    b->items.resize(count);
    std::vector<int> row_start(count + 1, 0);
    b->per_ant = 0;
    b->per_ant_tabu[0] = b->per_ant_tabu[1] = b->per_ant_tabu[2] = 0;
    for (int i = 0; i < count; ++i) {
        const size_t w = mmas_workspace_bytes(&params[i]);
        r = mmas_create(dists_host[i], &params[i], b->ws + pos, w, hip_stream, &b->ctx[i]);
        if (r == MMAS_OK) r = mmas_prepare_choice_info(b->ctx[i]);
        if (r != MMAS_OK) {
            for (mmas_ctx* c : b->ctx) mmas_destroy(c);
            delete b;
            return r;
        }
        pos += align_up(w);
        mmas::ctx_views(b->ctx[i], &b->items[i].v, &b->items[i].s);
        row_start[i + 1] = row_start[i] + b->items[i].s.n;
        b->per_ant = std::max(b->per_ant, (int)mmas::construct_lds_per_ant(b->items[i].s));
        for (int t = 0; t < 3; ++t) {
            mmas::Shape st = b->items[i].s;
            st.tabu = t;
            b->per_ant_tabu[t] = std::max(b->per_ant_tabu[t], (int)mmas::construct_lds_per_ant(st));
        }
    }
    b->total_rows = row_start[count];
    b->order.resize(count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return b->items[x].s.n > b->items[y].s.n; });
    const uint32_t zero[2] = {0u, 0u};
    hipError_t e = hipMemcpyAsync(b->d_items, b->items.data(), sizeof(mmas::BatchItem) * count, hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_row_start, row_start.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_it, zero, sizeof(zero), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        for (mmas_ctx* c : b->ctx) mmas_destroy(c);
        delete b;
        return mmas::hip_fail(e, "batch tables");
    }
    b->pair_ok = true;
    for (int i = 0; i < count; ++i) b->pair_ok = b->pair_ok && b->items[i].s.cl >= 1 && b->items[i].s.cl <= 32;
    b->ants_per_block = 4;
    b->lanes_per_ant = 64;
    b->table_request = -1;
    b->table_bytes = std::max(0, (mmas::max_lds_per_block() - kStaticLds - b->ants_per_block * b->per_ant) & ~15);
    r = rebuild_tiles(b);
    if (r != MMAS_OK) {
        for (mmas_ctx* c : b->ctx) mmas_destroy(c);
        delete b;
        return r;
    }
    *out = b;
    return MMAS_OK;
}

mmas_status mmas_batch_set_launch(mmas_batch* b, int32_t ants_per_block, int32_t table_bytes, int32_t lanes_per_ant) {
    if (!b) return MMAS_EINVAL;
    if (ants_per_block != 1 && ants_per_block != 2 && ants_per_block != 4 && ants_per_block != 8 &&
        ants_per_block != 16)
        return MMAS_EINVAL;
    if (lanes_per_ant != 0 && lanes_per_ant != 32 && lanes_per_ant != 64) return MMAS_EINVAL;
    if (table_bytes < -1) return MMAS_EINVAL;
    const int lanes = lanes_per_ant == 32 ? 32 : 64;
    if (lanes == 32 && (!b->pair_ok || ants_per_block < 2)) return MMAS_EUNSUPPORTED;
    const int budget = (mmas::max_lds_per_block() - kStaticLds - ants_per_block * b->per_ant) & ~15;
    if (budget < 0) return MMAS_EUNSUPPORTED;
    drop_graph(b);
    b->ants_per_block = ants_per_block;
    b->lanes_per_ant = lanes;
    b->table_request = table_bytes;
    b->table_bytes = table_bytes < 0 ? budget : std::min(budget, table_bytes & ~15);
    return rebuild_tiles(b);
}

mmas_status mmas_batch_set_tabu(mmas_batch* b, int32_t tabu) {
    if (!b || (tabu != MMAS_TABU_BITMASK && tabu != MMAS_TABU_COMPACT && tabu != MMAS_TABU_LIST)) return MMAS_EINVAL;
    const int keep = b->tabu;
    apply_tabu(b, tabu);
    mmas_status r = mmas_batch_set_launch(b, b->ants_per_block, b->table_request, b->lanes_per_ant);
    if (r != MMAS_OK) apply_tabu(b, keep);
    return r;
}

mmas_status mmas_batch_tune(mmas_batch* b, int32_t* ants_per_block, int32_t* table_bytes, int32_t* lanes_per_ant,
                            int32_t* tabu) {
    if (!b) return MMAS_EINVAL;
    struct Cand {
        int apb, tb, lanes, tabu;
    };
    std::vector<Cand> cands;
    for (int t : {MMAS_TABU_BITMASK, MMAS_TABU_COMPACT, MMAS_TABU_LIST})
        for (int lanes : {64, 32}) {
            if (lanes == 32 && !b->pair_ok) continue;
            for (int apb : {4, 8, 16}) {
                const int budget = mmas::max_lds_per_block() - kStaticLds - apb * b->per_ant_tabu[t];
                if (budget < 0) continue;
                cands.push_back({apb, -1, lanes, t});
                cands.push_back({apb, 0, lanes, t});
            }
        }
    hipEvent_t e0, e1;
    hipError_t ee = hipEventCreate(&e0);
    if (ee == hipSuccess) ee = hipEventCreate(&e1);
    if (ee != hipSuccess) return mmas::hip_fail(ee, "tuner events");
    float best_ms = 1e30f;
    Cand best = cands.empty() ? Cand{4, -1, 64, b->tabu} : cands[0];
    mmas_status r = MMAS_OK;
    for (const Cand& c : cands) {
        apply_tabu(b, c.tabu);
        r = mmas_batch_set_launch(b, c.apb, c.tb, c.lanes);
        if (r != MMAS_OK) break;
        // construction only: it writes tours and lengths, never the trails
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && r == MMAS_OK; ++rep) {
            k_reset_queue<<<1, 64, 0, b->stream>>>(b->d_queue);
            (void)hipEventRecord(e0, b->stream);
            ee = mmas::launch_batch_construct(b->d_items, b->d_tiles, b->ntiles, b->d_queue, b->d_it, b->tabu, b->pher,
                                              b->ants_per_block, b->lanes_per_ant, b->table_bytes, b->per_ant, b->grid,
                                              b->stream);
            if (ee != hipSuccess) r = mmas::hip_fail(ee, "tuner launch");
            (void)hipEventRecord(e1, b->stream);
            ee = hipEventSynchronize(e1);
            if (ee != hipSuccess) r = mmas::hip_fail(ee, "tuner synchronisation");
            (void)hipEventElapsedTime(&ms, e0, e1);  // the second repetition counts
        }
        if (r == MMAS_OK && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    k_reset_queue<<<1, 64, 0, b->stream>>>(b->d_queue);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != MMAS_OK) return r;
    apply_tabu(b, best.tabu);
    r = mmas_batch_set_launch(b, best.apb, best.tb, best.lanes);
    if (r != MMAS_OK) return r;
    if (tabu) *tabu = b->tabu;
    if (ants_per_block) *ants_per_block = b->ants_per_block;
    if (table_bytes) *table_bytes = b->table_bytes;
    if (lanes_per_ant) *lanes_per_ant = b->lanes_per_ant;
    ee = hipStreamSynchronize(b->stream);
    return ee == hipSuccess ? MMAS_OK : mmas::hip_fail(ee, "tuner synchronisation");
}

mmas_status mmas_batch_capture(mmas_batch* b) {
    if (!b) return MMAS_EINVAL;
    if (b->stream == nullptr) return MMAS_EUNSUPPORTED;  // the null stream cannot be captured
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return mmas::hip_fail(e, "capture begin");
    mmas_status r = launch_step(b);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (r != MMAS_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return r != MMAS_OK ? r : mmas::hip_fail(e, "capture end");
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return mmas::hip_fail(e, "graph instantiation");
    }
    return MMAS_OK;
}

mmas_status mmas_batch_step(mmas_batch* b) {
    if (!b) return MMAS_EINVAL;
    if (b->exec && !b->timing) {
        const hipError_t e = hipGraphLaunch(b->exec, b->stream);
        return e == hipSuccess ? MMAS_OK : mmas::hip_fail(e, "graph launch");
    }
    return launch_step(b);
}

mmas_status mmas_batch_iteration(mmas_batch* b, uint32_t* iteration) {
    if (!b || !iteration) return MMAS_EINVAL;
    hipError_t e = hipMemcpyAsync(iteration, b->d_it, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? MMAS_OK : mmas::hip_fail(e, "iteration read");
}

mmas_status mmas_batch_context(mmas_batch* b, int32_t index, mmas_ctx** ctx) {
    if (!b || !ctx || index < 0 || index >= b->count) return MMAS_EINVAL;
    *ctx = b->ctx[index];
    return MMAS_OK;
}

mmas_status mmas_batch_set_timing(mmas_batch* b, int32_t on) {
    if (!b) return MMAS_EINVAL;
    b->timing = on != 0;
    return MMAS_OK;
}

mmas_status mmas_batch_read_timing(mmas_batch* b, double* construct_ms, int64_t* calls, int32_t reset) {
    if (!b) return MMAS_EINVAL;
    const hipError_t e = fold_timing(b);
    if (construct_ms) *construct_ms = b->construct_ms;
    if (calls) *calls = b->construct_calls;
    if (reset) {
        b->construct_ms = 0.0;
        b->construct_calls = 0;
    }
    return e == hipSuccess ? MMAS_OK : mmas::hip_fail(e, "timing read");
}

void mmas_batch_destroy(mmas_batch* b) {
    if (!b) return;
    // the caller may free the workspace right after this call: let every
    // step already enqueued (a graph replay included) finish first
    (void)hipStreamSynchronize(b->stream);
    for (auto& ev : b->pending) b->spare.push_back(ev);
    for (auto& ev : b->spare) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    drop_graph(b);
    for (mmas_ctx* c : b->ctx) mmas_destroy(c);
    delete b;
}

}  // extern "C"
