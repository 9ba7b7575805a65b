// Plain strided complex passes (y and z axes), float.
#include "ps_launch_impl.hpp"

namespace ps {
template hipError_t launch_strided<float>(int, int, int, StridedArgs<float>, hipStream_t);
}  // namespace ps
