// Plain strided complex passes (y and z axes), double.
#include "ps_launch_impl.hpp"

namespace ps {
template hipError_t launch_strided<double>(int, int, int, StridedArgs<double>, hipStream_t);
}  // namespace ps
