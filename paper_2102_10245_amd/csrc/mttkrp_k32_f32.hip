// MTTKRP kernels for 32-bit linearized indices and f32 factors (all orders and ranks).
#include "mttkrp_impl.h"

namespace alto {

int launch_mt_k32_f32(const MtLaunch &a, hipStream_t s) { return launch_mt_n<uint32_t, float>(a, s); }

}  // namespace alto
