// Contiguous x passes: plain real transforms and the fused product pass.
#include "ps_config.hpp"
#include "ps_launch.hpp"

namespace ps {

template <typename T>
bool mhd_supported(int N) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return XCfg<T, NN>::MHD_OK;
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return false;
}

template <typename T, int N>
static hipError_t x_c2r_n(XArgs<T> a, hipStream_t s) {
  using X = XCfg<T, N>;
  using LC = LenCfg<N / 2>;
  const long grid = (a.rows * a.nf + X::G - 1) / X::G;
  k_x_c2r<T, N / 2, LC::TQ, X::G, typename LC::RL><<<dim3((unsigned)grid), dim3(X::G * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t x_r2c_n(XArgs<T> a, hipStream_t s) {
  using X = XCfg<T, N>;
  using LC = LenCfg<N / 2>;
  const long grid = (a.rows * a.nf + X::G - 1) / X::G;
  k_x_r2c<T, N / 2, LC::TQ, X::G, typename LC::RL><<<dim3((unsigned)grid), dim3(X::G * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t x_prod_n(bool mhd, XArgs<T> a, hipStream_t s) {
  using X = XCfg<T, N>;
  using LC = LenCfg<N / 2>;
  if (mhd) {
    if constexpr (X::MHD_OK) {
      const long grid = (a.rows + X::RB_MHD - 1) / X::RB_MHD;
      k_x_prod<T, N / 2, LC::TQ, X::RB_MHD, typename LC::RL, true>
          <<<dim3((unsigned)grid), dim3(12 * X::RB_MHD * LC::TQ), 0, s>>>(a);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  const long grid = (a.rows + X::RB_NS - 1) / X::RB_NS;
  k_x_prod<T, N / 2, LC::TQ, X::RB_NS, typename LC::RL, false>
      <<<dim3((unsigned)grid), dim3(6 * X::RB_NS * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_x_c2r(int N, XArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return x_c2r_n<T, NN>(a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_x_r2c(int N, XArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return x_r2c_n<T, NN>(a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_x_prod(int N, bool mhd, XArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return x_prod_n<T, NN>(mhd, a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template bool mhd_supported<float>(int);
template bool mhd_supported<double>(int);
template hipError_t launch_x_c2r<float>(int, XArgs<float>, hipStream_t);
template hipError_t launch_x_c2r<double>(int, XArgs<double>, hipStream_t);
template hipError_t launch_x_r2c<float>(int, XArgs<float>, hipStream_t);
template hipError_t launch_x_r2c<double>(int, XArgs<double>, hipStream_t);
template hipError_t launch_x_prod<float>(int, bool, XArgs<float>, hipStream_t);
template hipError_t launch_x_prod<double>(int, bool, XArgs<double>, hipStream_t);

}  // namespace ps
