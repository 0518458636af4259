// Diagnostic entry points: the device logarithm and Philox draws on arrays,
// so that they can be compared with an independent implementation.
#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

__global__ __launch_bounds__(256) void k_eval_log(const float* __restrict__ u, float* __restrict__ out, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        out[i] = log_u01(u[i]);
}

__global__ __launch_bounds__(256) void k_eval_draws(uint64_t seed, const uint32_t* __restrict__ it,
                                                    const uint32_t* __restrict__ ant, const uint32_t* __restrict__ step,
                                                    const uint32_t* __restrict__ slot, uint32_t* __restrict__ out,
                                                    size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        const Words4 b = draw_block(seed, it[i], ant[i], step[i], slot[i]);
        out[i] = pick_word(b, slot[i] & 3u);
    }
}

int grid_for(size_t total) {
    size_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    return g < 1 ? 1 : (int)g;
}

}  // namespace
}  // namespace mmas

extern "C" mmas_status mmas_eval_log(const float* dev_u, float* dev_out, size_t count, void* hip_stream) {
    if (count == 0) return MMAS_OK;
    if (!dev_u || !dev_out) return MMAS_EINVAL;
    mmas::k_eval_log<<<mmas::grid_for(count), 256, 0, reinterpret_cast<hipStream_t>(hip_stream)>>>(dev_u, dev_out, count);
    return hipGetLastError() == hipSuccess ? MMAS_OK : MMAS_EHIP;
}

extern "C" mmas_status mmas_eval_draws(uint64_t seed, const uint32_t* dev_it, const uint32_t* dev_ant,
                                       const uint32_t* dev_step, const uint32_t* dev_slot, uint32_t* dev_out,
                                       size_t count, void* hip_stream) {
    if (count == 0) return MMAS_OK;
    if (!dev_it || !dev_ant || !dev_step || !dev_slot || !dev_out) return MMAS_EINVAL;
    mmas::k_eval_draws<<<mmas::grid_for(count), 256, 0, reinterpret_cast<hipStream_t>(hip_stream)>>>(
        seed, dev_it, dev_ant, dev_step, dev_slot, dev_out, count);
    return hipGetLastError() == hipSuccess ? MMAS_OK : MMAS_EHIP;
}

extern "C" mmas_status mmas_eval_tabu(int32_t tabu, int32_t n, const int32_t* dev_marks, int32_t count,
                                      uint8_t* dev_visited, uint16_t* dev_state, int32_t* dev_left,
                                      void* hip_stream) {
    if (tabu != MMAS_TABU_BITMASK && tabu != MMAS_TABU_COMPACT && tabu != MMAS_TABU_LIST) return MMAS_EINVAL;
    if (n < 1 || n > 8192 || count < 0 || count > n || (count > 0 && !dev_marks) || !dev_visited || !dev_state ||
        !dev_left)
        return MMAS_EINVAL;
    const hipError_t e = mmas::launch_eval_tabu(tabu, n, dev_marks, count, dev_visited, dev_state, dev_left,
                                                reinterpret_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? MMAS_OK : mmas::hip_fail(e, "eval tabu");
}
