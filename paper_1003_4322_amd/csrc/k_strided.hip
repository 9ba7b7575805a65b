// Plain strided complex passes (y and z axes), every supported N, FP32/FP64.
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

template <typename T, int N>
static hipError_t strided_n(int dir, StridedArgs<T> a, hipStream_t s) {
  using C = StridedCfg<T, N>;
  using LC = LenCfg<N>;
  a.ntile = cdiv(a.ncols, C::TX);
  const long grid = (long)a.ntile * a.nlines * a.nf;
  if (grid <= 0) return hipSuccess;
  if (dir == FWD)
    k_strided<T, N, LC::TQ, C::TX, FWD, typename LC::RL><<<dim3((unsigned)grid), dim3(C::TX * LC::TQ), 0, s>>>(a);
  else
    k_strided<T, N, LC::TQ, C::TX, INV, typename LC::RL><<<dim3((unsigned)grid), dim3(C::TX * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_strided(int N, int dir, StridedArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return strided_n<T, NN>(dir, a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_strided<float>(int, int, StridedArgs<float>, hipStream_t);
template hipError_t launch_strided<double>(int, int, StridedArgs<double>, hipStream_t);

}  // namespace ps
