// Deterministic FP64 shell spectra (energy and enstrophy; MHD energies and
// cross-helicity).
#include <cstring>
#include <map>
#include <mutex>

#include "ps_config.hpp"
#include "ps_launch.hpp"

namespace ps {

// Library-held scratch of the allocation-free spectrum entry point
// (ps_energy_spectrum_static): the per-plane partials of one box at a time.
// Each device the library runs on holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): it uses the device address that
// spectrum_scratch() looked up with the device current.
static __device__ __align__(256) double scratch[SPEC_SCRATCH_BYTES / sizeof(double)];

hipError_t spectrum_scratch(int device, double** ptr) {
  static std::mutex mu;
  static std::map<int, double*> addr;  // device -> address of its copy
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *ptr = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
  if (e != hipSuccess) return e;
  addr[device] = static_cast<double*>(p);
  *ptr = static_cast<double*>(p);
  return hipSuccess;
}

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
// shell order, all Neumaier-compensated (one workgroup).  Q = 2 (energy):
// spec[s] = E(s), totals = [sum E, sum Z, max over planes of pmax]; Q = 3
// (MHD): spec[q nshell + s] = quantity q of shell s, totals[q] = its sum.
template <int Q>
__global__ __launch_bounds__(1024) void k_spec_final(const double* part, const double* pmax, int nplanes,
                                                     int nshell, double* spec, double* totals) {
  __shared__ double sh[Q][1024];
  NSum tot[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) tot[q] = NSum{0, 0};
  for (int s0 = 0; s0 < nshell; s0 += blockDim.x) {
    const int s = s0 + threadIdx.x;
    if (s < nshell) {
      // planes in order; the loads of U planes are issued before their adds
      constexpr int U = 8;
      NSum e[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) e[q] = NSum{0, 0};
      int p = 0;
      for (; p + U <= nplanes; p += U) {
        double v[U][Q];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < Q; ++q) v[u][q] = part[((long)(p + u) * nshell + s) * Q + q];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < Q; ++q) nadd(e[q], v[u][q]);
      }
      for (; p < nplanes; ++p)
#pragma unroll
        for (int q = 0; q < Q; ++q) nadd(e[q], part[((long)p * nshell + s) * Q + q]);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const double v = e[q].s + e[q].c;
        sh[q][threadIdx.x] = v;
        if (Q == 3)
          spec[q * nshell + s] = v;
        else if (q == 0)
          spec[s] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = nshell - s0 < (int)blockDim.x ? nshell - s0 : (int)blockDim.x;
      for (int i = 0; i < n; ++i)
#pragma unroll
        for (int q = 0; q < Q; ++q) nadd(tot[q], sh[q][i]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) totals[q] = tot[q].s + tot[q].c;
    if (Q == 2) {
      double mx = 0;
      for (int p = 0; p < nplanes; ++p) mx = fmax(mx, pmax[p]);
      totals[2] = mx;
    }
  }
}


template <typename T>
hipError_t launch_spectrum(SpecArgs<T> a, bool mhd, double* spec, double* totals, hipStream_t s) {
  // at most one 64-shell window per wave, at most SPEC_NF fields
  if (a.nshell > 64 * SPEC_WAVES || (!mhd && a.nf > SPEC_NF)) return hipErrorInvalidValue;
  if (mhd)
    k_spec_planes<T, true><<<dim3(a.nz), dim3(SPEC_WAVES * 64), 0, s>>>(a);
  else
    k_spec_planes<T, false><<<dim3(a.nz), dim3(SPEC_WAVES * 64), 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mhd)
    k_spec_final<3><<<dim3(1), dim3(1024), 0, s>>>(a.part, a.pmax, a.nz, a.nshell, spec, totals);
  else
    k_spec_final<2><<<dim3(1), dim3(1024), 0, s>>>(a.part, a.pmax, a.nz, a.nshell, spec, totals);
  return hipGetLastError();
}

template hipError_t launch_spectrum<float>(SpecArgs<float>, bool, double*, double*, hipStream_t);
template hipError_t launch_spectrum<double>(SpecArgs<double>, bool, double*, double*, hipStream_t);

}  // namespace ps
