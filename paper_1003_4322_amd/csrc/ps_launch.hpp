// ps_launch.hpp -- host-side launchers of the gfx950 kernels (internal).
// Each launcher picks the compiled configuration for the grid size N, fills
// in the tile counts and enqueues one kernel on the given stream.
#pragma once

#include <hip/hip_runtime.h>

#include "ps_kernels.hpp"

namespace ps {

bool size_supported(int N);
template <typename T>
bool mhd_supported(int N);

template <typename T>
hipError_t launch_strided(int N, int dir, StridedArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_z_curl(int N, bool mhd, ZCurlArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_z_epi(int N, bool mhd, ZEpiArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_x_c2r(int N, XArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_x_r2c(int N, XArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_x_prod(int N, bool mhd, XArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_spectrum(SpecArgs<T> a, double* spec, double* totals, hipStream_t s);

}  // namespace ps
