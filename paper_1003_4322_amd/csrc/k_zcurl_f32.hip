// Fused inverse z pass + spectral curl prologue, float.
#include "ps_launch_impl.hpp"

namespace ps {
template hipError_t launch_z_curl<float>(int, bool, bool, int, ZCurlArgs<float>, const DiskTiles*, hipStream_t);
template int z_curl_tx<float>(int, int);
}  // namespace ps
