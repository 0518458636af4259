// 2-opt local search on every ant's tour (placeholder until the kernel lands).
#include "internal.hpp"

namespace mmas {

size_t two_opt_lds_bytes(const Shape& s) { return 4 * (size_t)s.n; }

hipError_t launch_two_opt(const Views&, const Shape&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace mmas
