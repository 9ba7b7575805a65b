// ps_config.hpp -- compile-time launch configurations per transform length.
//
// For each supported length L: the radix schedule of the Stockham engine and
// the number of threads TQ that cooperate on one transform (about eight
// complex values per thread per stage).  For the strided passes, TX is the
// number of adjacent kx columns per workgroup: 16 (128-byte rows) in FP32 and
// 8 in FP64, fewer where the LDS tile L*TX would exceed 64 KB.
#pragma once

#include "ps_device.hpp"

namespace ps {

template <int L>
struct LenCfg;
#define PS_LEN(L_, TQ_, ...)                     \
  template <>                                    \
  struct LenCfg<L_> {                            \
    using RL = Radices<__VA_ARGS__>;             \
    static constexpr int TQ = TQ_;               \
  };
PS_LEN(4, 1, 4)
PS_LEN(6, 1, 3, 2)
PS_LEN(8, 1, 8)
PS_LEN(12, 3, 4, 3)
PS_LEN(16, 4, 4, 4)
PS_LEN(24, 3, 8, 3)
PS_LEN(32, 4, 8, 4)
PS_LEN(48, 6, 4, 4, 3)
PS_LEN(64, 8, 8, 8)
PS_LEN(96, 12, 8, 4, 3)
PS_LEN(128, 16, 8, 4, 4)
PS_LEN(192, 24, 8, 8, 3)
PS_LEN(256, 32, 8, 8, 4)
PS_LEN(384, 48, 8, 4, 4, 3)
PS_LEN(512, 64, 8, 8, 8)
PS_LEN(768, 96, 8, 8, 4, 3)
PS_LEN(1024, 128, 8, 8, 4, 4)
#undef PS_LEN

// grid sizes with a compiled configuration
#define PS_FOR_EACH_N(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

template <typename T, int N>
struct StridedCfg {
  static constexpr int TQ = LenCfg<N>::TQ;
  static constexpr int TX0 = sizeof(T) == 4 ? 16 : 8;
  static constexpr int TXL = (65536 / (N * 2 * (int)sizeof(T)));  // LDS cap
  static constexpr int TX1 = TX0 < TXL ? TX0 : TXL;
  static constexpr int TX = (TX1 * TQ > 1024) ? 1024 / TQ : TX1;
  static_assert(TX >= 1, "tile");
};

template <typename T, int N>
struct XCfg {
  static constexpr int M = N / 2;
  static constexpr int TQ = LenCfg<M>::TQ;
  // plain passes: G rows per workgroup, ~256 threads
  static constexpr int G = (256 / TQ) < 1 ? 1 : 256 / TQ;
  // fused product pass: RB rows of every field per workgroup, <= ~384 threads
  static constexpr int RB_NS = (384 / (6 * TQ)) < 1 ? 1 : 384 / (6 * TQ);
  static constexpr int RB_MHD = (384 / (12 * TQ)) < 1 ? 1 : 384 / (12 * TQ);
  static constexpr bool MHD_OK = 12 * RB_MHD * (M + 1) * 2 * (int)sizeof(T) <= 65536;
};

}  // namespace ps
