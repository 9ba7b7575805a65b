// Fused z passes: inverse + spectral curl, forward + dealias/projection/RK2.
#include "ps_config.hpp"
#include "ps_launch.hpp"

namespace ps {

template <typename T, int N>
static hipError_t z_curl_n(bool mhd, ZCurlArgs<T> a, hipStream_t s) {
  using C = StridedCfg<T, N>;
  using LC = LenCfg<N>;
  a.ntile = cdiv(N / 2 + 1, C::TX);
  const long grid = (long)a.ntile * N;
  if (mhd)
    k_z_curl<T, N, LC::TQ, C::TX, typename LC::RL, true><<<dim3((unsigned)grid), dim3(C::TX * LC::TQ), 0, s>>>(a);
  else
    k_z_curl<T, N, LC::TQ, C::TX, typename LC::RL, false><<<dim3((unsigned)grid), dim3(C::TX * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t z_epi_n(bool mhd, ZEpiArgs<T> a, hipStream_t s) {
  using C = StridedCfg<T, N>;
  using LC = LenCfg<N>;
  a.ntile = cdiv(N / 2 + 1, C::TX);
  const long grid = (long)a.ntile * N;
  if (mhd)
    k_z_epi<T, N, LC::TQ, C::TX, typename LC::RL, true><<<dim3((unsigned)grid), dim3(C::TX * LC::TQ), 0, s>>>(a);
  else
    k_z_epi<T, N, LC::TQ, C::TX, typename LC::RL, false><<<dim3((unsigned)grid), dim3(C::TX * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_z_curl(int N, bool mhd, ZCurlArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return z_curl_n<T, NN>(mhd, a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_z_epi(int N, bool mhd, ZEpiArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return z_epi_n<T, NN>(mhd, a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_z_curl<float>(int, bool, ZCurlArgs<float>, hipStream_t);
template hipError_t launch_z_curl<double>(int, bool, ZCurlArgs<double>, hipStream_t);
template hipError_t launch_z_epi<float>(int, bool, ZEpiArgs<float>, hipStream_t);
template hipError_t launch_z_epi<double>(int, bool, ZEpiArgs<double>, hipStream_t);

}  // namespace ps
