// MTTKRP kernels for 64-bit linearized indices and bf16 factors (all orders and ranks).
#include "mttkrp_impl.h"

namespace alto {

int launch_mt_k64_bf16(const MtLaunch &a, hipStream_t s) { return launch_mt_n<uint64_t, uint16_t>(a, s); }

}  // namespace alto
