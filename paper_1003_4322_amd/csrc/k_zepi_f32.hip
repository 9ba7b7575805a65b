// Fused forward z pass + dealias / projection / induction / RK2 epilogue, float.
#include "ps_launch_impl.hpp"

namespace ps {
template hipError_t launch_z_epi<float>(int, bool, bool, int, ZEpiArgs<float>, const DiskTiles*, hipStream_t);
template int z_epi_tx<float>(int, int);
}  // namespace ps
