// MTTKRP kernels for 128-bit linearized indices and f32 factors (all orders and ranks).
#include "mttkrp_impl.h"

namespace alto {

int launch_mt_k128_f32(const MtLaunch &a, hipStream_t s) { return launch_mt_n<u128, float>(a, s); }

}  // namespace alto
