// Fused inverse z pass + spectral curl prologue, double.
#include "ps_launch_impl.hpp"

namespace ps {
template hipError_t launch_z_curl<double>(int, bool, bool, int, ZCurlArgs<double>, const DiskTiles*, hipStream_t);
template int z_curl_tx<double>(int, int);
}  // namespace ps
