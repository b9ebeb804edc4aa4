// Instantiates the plain and wide kernels of ring 1 (one file per ring: parallel builds).
#include "plain_impl.hpp"

namespace pyrit {
template int launch_plain_ring<1>(int, int, const PassArgs &, hipStream_t);
template int launch_wide_ring<1>(int, const WideArgs &, hipStream_t);
}
