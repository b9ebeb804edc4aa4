// Instantiates the plain and wide kernels of ring 3 (one file per ring: parallel builds).
#include "plain_impl.hpp"

namespace pyrit {
template int launch_plain_ring<3>(int, int, const PassArgs &, hipStream_t);
template int launch_wide_ring<3>(int, const WideArgs &, hipStream_t);
}
