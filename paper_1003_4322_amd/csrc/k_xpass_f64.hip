// Contiguous x passes: plain real transforms and the fused product pass, double.
#include "ps_launch_impl.hpp"

namespace ps {
template bool mhd_supported<double>(int);
template hipError_t launch_x_c2r<double>(int, XArgs<double>, hipStream_t);
template hipError_t launch_x_r2c<double>(int, XArgs<double>, hipStream_t);
template hipError_t launch_x_prod<double>(int, bool, bool, int, XArgs<double>, hipStream_t);
}  // namespace ps
