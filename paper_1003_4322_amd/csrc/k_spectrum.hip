// Deterministic FP64 shell spectrum.
#include <cstring>

#include "ps_config.hpp"
#include "ps_launch.hpp"

namespace ps {

bool size_supported(int N) {
  switch (N) {
#define PS_CASE(NN) case NN:
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
    return true;
    default:
      return false;
  }
}

int variant_count(const char* kind, int N, bool mhd) {
  (void)mhd;
  if (!has_variants(N)) return 1;
  if (!strcmp(kind, "z_curl")) return NZCURL;
  if (!strcmp(kind, "z_epi")) return NZEPI;
  if (!strcmp(kind, "y") || !strcmp(kind, "z")) return NSTR;
  if (!strcmp(kind, "x_prod")) return NXPROD;
  return 1;
}

// Second stage: per-shell sums over planes in plane order, then the totals in
// shell order, all Neumaier-compensated (one workgroup).
__global__ __launch_bounds__(1024) void k_spec_final(const double* part, const double* pmax, int nplanes,
                                                     int nshell, double* spec, double* totals) {
  __shared__ double zs[1024];
  __shared__ double es[1024];
  NSum Et{0, 0}, Zt{0, 0};
  for (int s0 = 0; s0 < nshell; s0 += blockDim.x) {
    const int s = s0 + threadIdx.x;
    if (s < nshell) {
      NSum E{0, 0}, Z{0, 0};
      for (int p = 0; p < nplanes; ++p) {
        nadd(E, part[((long)p * nshell + s) * 2]);
        nadd(Z, part[((long)p * nshell + s) * 2 + 1]);
      }
      spec[s] = E.s + E.c;
      es[threadIdx.x] = E.s + E.c;
      zs[threadIdx.x] = Z.s + Z.c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = nshell - s0 < (int)blockDim.x ? nshell - s0 : (int)blockDim.x;
      for (int i = 0; i < n; ++i) {
        nadd(Et, es[i]);
        nadd(Zt, zs[i]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double mx = 0;
    for (int p = 0; p < nplanes; ++p) mx = fmax(mx, pmax[p]);
    totals[0] = Et.s + Et.c;
    totals[1] = Zt.s + Zt.c;
    totals[2] = mx;
  }
}


template <typename T>
hipError_t launch_spectrum(SpecArgs<T> a, double* spec, double* totals, hipStream_t s) {
  k_spec_planes<T><<<dim3(a.nz), dim3(256), 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_spec_final<<<dim3(1), dim3(1024), 0, s>>>(a.part, a.pmax, a.nz, a.nshell, spec, totals);
  return hipGetLastError();
}

template hipError_t launch_spectrum<float>(SpecArgs<float>, double*, double*, hipStream_t);
template hipError_t launch_spectrum<double>(SpecArgs<double>, double*, double*, hipStream_t);

}  // namespace ps
