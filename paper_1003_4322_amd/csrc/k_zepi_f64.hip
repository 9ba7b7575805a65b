// Fused forward z pass + dealias / projection / induction / RK2 epilogue, double.
#include "ps_launch_impl.hpp"

namespace ps {
template hipError_t launch_z_epi<double>(int, bool, bool, int, ZEpiArgs<double>, const DiskTiles*, hipStream_t);
template int z_epi_tx<double>(int, int);
}  // namespace ps
