// ps_launch.hpp -- host-side launchers of the gfx950 kernels (internal).
// Each launcher picks the compiled configuration for the length N of the axis
// its pass transforms (z passes: nz, y passes: ny, x passes: nx) and the
// requested variant, fills in the tile counts and enqueues one kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "ps_kernels.hpp"

namespace ps {

bool size_supported(int N);
template <typename T>
bool mhd_supported(int N);

// number of variants of a pass kind at size N ("y", "z", "z_curl", "z_epi", "x_prod")
int variant_count(const char* kind, int N, bool mhd);

template <typename T>
hipError_t launch_strided(int N, int dir, int var, StridedArgs<T> a, hipStream_t s);
// Tiles of a z pass whose first column meets the dealiasing disk
// Grid::disk(kx, ky), one device list per tile width (entries
// tile | ky << 16, ky-major).
struct DiskTiles {
  static constexpr int MAXTX = 16;
  const int* list[MAXTX + 1] = {};
  int count[MAXTX + 1] = {};
};
// tile width (columns per workgroup) of a z-pass variant
template <typename T>
int z_curl_tx(int N, int var);
template <typename T>
int z_epi_tx(int N, int var);

// els: MHD in the Elsasser (divergence) form -- z_curl transforms z+- without
// a curl, x_prod forms the products z+_i z-_j (less z+_2 z-_2 on the diagonal,
// eight fields), z_epi takes their divergence
template <typename T>
hipError_t launch_z_curl(int N, bool mhd, bool els, int var, ZCurlArgs<T> a, const DiskTiles* dt,
                         hipStream_t s);
template <typename T>
hipError_t launch_z_epi(int N, bool mhd, bool els, int var, ZEpiArgs<T> a, const DiskTiles* dt,
                        hipStream_t s);
template <typename T>
hipError_t launch_x_c2r(int N, XArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_x_r2c(int N, XArgs<T> a, hipStream_t s);
template <typename T>
hipError_t launch_x_prod(int N, bool mhd, bool els, int var, XArgs<T> a, hipStream_t s);
// Bytes of the library-held device scratch of ps_energy_spectrum_static:
// the partials of one box, nz * nshell * 2 + nz doubles (14.6 MB at
// 1024^3, the largest supported grid).
constexpr size_t SPEC_SCRATCH_BYTES = size_t(16) << 20;
// Device address of the current device's copy of that scratch (looked up
// once per device; call with `device` current).
hipError_t spectrum_scratch(int device, double** ptr);

// mhd: Eu(s), Eb(s), Hc(s) of an Elsasser state instead of E(s) (and Z, maxdiv)
template <typename T>
hipError_t launch_spectrum(SpecArgs<T> a, bool mhd, double* spec, double* totals, hipStream_t s);

}  // namespace ps
