#include "common.h"
namespace eor {
hipError_t launch_precompute_fp32(const Context &, const double2 *, int64_t, const double *, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_precompute_bf16x3(const Context &, const double2 *, int64_t, const double *, hipStream_t) {
    return hipErrorNotSupported;
}
}
