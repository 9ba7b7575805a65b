// Contiguous x passes: plain real transforms and the fused product pass, float.
#include "ps_launch_impl.hpp"

namespace ps {
template bool mhd_supported<float>(int);
template hipError_t launch_x_c2r<float>(int, XArgs<float>, hipStream_t);
template hipError_t launch_x_r2c<float>(int, XArgs<float>, hipStream_t);
template hipError_t launch_x_prod<float>(int, bool, bool, int, XArgs<float>, hipStream_t);
}  // namespace ps
