// ps_launch_impl.hpp -- launcher definitions, included by one translation
// unit per pass kind and dtype (k_<pass>_<dtype>.hip).
#pragma once

#include <cstring>
#include <type_traits>
#include <utility>

#include "ps_config.hpp"
#include "ps_launch.hpp"

namespace ps {

template <int N, bool ALT>
using Sched = std::conditional_t<ALT, LenAlt<N>, LenCfg<N>>;

// run f<I>() for the I == var of 0..n-1
template <int... I, class F>
hipError_t pick(int var, std::integer_sequence<int, I...>, F&& f) {
  hipError_t r = hipErrorInvalidValue;
  ((var == I ? (void)(r = f(std::integral_constant<int, I>{})) : (void)0), ...);
  return r;
}

// ---------------- strided plain passes ----------------
template <typename T, int N, int I>
hipError_t strided_v(int dir, StridedArgs<T> a, hipStream_t s) {
  constexpr ZV v = STR_V[I];
  using LC = Sched<N, v.alt>;
  constexpr int TX = StridedTX<T, N, LC::TQ, v.sh>::value;
  a.ntile = cdiv(a.ncols, TX);
  // pruned passes: launch only the tiles whose first column kx = tile TX
  // is kept by the 2/3 rule (the kernel skips the others)
  if (a.prune)
    while (a.ntile > 0 && !a.g.disk((a.ntile - 1) * TX, 0)) --a.ntile;
  const long grid = (long)a.ntile * a.nlines * a.nf * a.nb;
  if (grid <= 0) return hipSuccess;
  // staged twiddles only where the transform has more than one stage
  constexpr bool TWS = v.tws && RadixInfo<typename LC::RL>::count > 1;
  if (dir == FWD)
    k_strided<T, N, LC::TQ, TX, FWD, typename LC::RL, waves_per_simd(v.minb, TX * LC::TQ), TWS>
        <<<dim3((unsigned)grid), dim3(TX * LC::TQ), 0, s>>>(a);
  else
    k_strided<T, N, LC::TQ, TX, INV, typename LC::RL, waves_per_simd(v.minb, TX * LC::TQ), TWS>
        <<<dim3((unsigned)grid), dim3(TX * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t strided_n(int dir, int var, StridedArgs<T> a, hipStream_t s) {
  if constexpr (has_variants(N))
    return pick(var, std::make_integer_sequence<int, NSTR>{},
                [&](auto I) { return strided_v<T, N, decltype(I)::value>(dir, a, s); });
  else
    return strided_v<T, N, 0>(dir, a, s);
}

template <typename T>
hipError_t launch_strided(int N, int dir, int var, StridedArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return strided_n<T, NN>(dir, var, a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

// ---------------- inverse z pass + curl ----------------
template <typename T, int N, int I>
constexpr int zcurl_tx_of() {
  constexpr ZV v = ZCURL_V[I];
  return StridedTX<T, N, Sched<N, v.alt>::TQ, v.sh>::value;
}
// schedule of a z-pass variant: radix-16 (alt), wide (a last radix of 4
// over twice the threads), or the default
template <int N, int I>
using ZepiSched = std::conditional_t<ZEPI_V[I].wide, LenWide<N>, Sched<N, ZEPI_V[I].alt>>;

template <typename T, int N, int I>
constexpr int zepi_tx_of() {
  return StridedTX<T, N, ZepiSched<N, I>::TQ, ZEPI_V[I].sh>::value;
}

// grid of a z pass: every tile, or only those in the disk list
template <int TX>
long z_grid(int ny, int ntile, int nb, bool listed, const DiskTiles* dt, const int*& tiles, int& ntl) {
  static_assert(TX <= DiskTiles::MAXTX, "disk tile lists cover widths up to 16");
  if (listed && dt && dt->list[TX]) {
    tiles = dt->list[TX];
    ntl = dt->count[TX];
    return (long)ntl * nb;
  }
  tiles = nullptr;
  ntl = 0;
  return (long)ntile * ny * nb;
}

template <typename T, int N, int I, bool MHD, bool ELS = false>
hipError_t z_curl_v(ZCurlArgs<T> a, const DiskTiles* dt, hipStream_t s) {
  constexpr ZV v = ZCURL_V[I];
  using LC = Sched<N, v.alt>;
  constexpr int TX = StridedTX<T, N, LC::TQ, v.sh>::value;
  constexpr int SPLIT = (MHD && !ELS) ? v.split : !MHD && ELS ? 1 : (v.split > 2 ? 2 : v.split);
  if (a.g.nz != N) return hipErrorInvalidValue;
  a.ntile = cdiv(a.g.nx / 2 + 1, TX);
  const long grid = z_grid<TX>(a.g.ny, a.ntile, a.nb, a.prune != 0, dt, a.tiles, a.ntl) * SPLIT;
  k_z_curl<T, N, LC::TQ, TX, typename LC::RL, MHD, SPLIT, v.direct, waves_per_simd(v.minb, TX * LC::TQ), ELS>
      <<<dim3((unsigned)grid), dim3(TX * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int N, int I>
hipError_t z_curl_m(bool mhd, bool els, ZCurlArgs<T> a, const DiskTiles* dt, hipStream_t s) {
  if (els) return mhd ? z_curl_v<T, N, I, true, true>(a, dt, s) : z_curl_v<T, N, I, false, true>(a, dt, s);
  return mhd ? z_curl_v<T, N, I, true>(a, dt, s) : z_curl_v<T, N, I, false>(a, dt, s);
}

template <typename T, int N>
hipError_t z_curl_n(bool mhd, bool els, int var, ZCurlArgs<T> a, const DiskTiles* dt, hipStream_t s) {
  if constexpr (has_variants(N))
    return pick(var, std::make_integer_sequence<int, NZCURL>{},
                [&](auto I) { return z_curl_m<T, N, decltype(I)::value>(mhd, els, a, dt, s); });
  else
    return z_curl_m<T, N, 0>(mhd, els, a, dt, s);
}

template <typename T>
hipError_t launch_z_curl(int N, bool mhd, bool els, int var, ZCurlArgs<T> a, const DiskTiles* dt,
                         hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return z_curl_n<T, NN>(mhd, els, var, a, dt, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
int z_curl_tx(int N, int var) {
  int tx = 0;
  switch (N) {
#define PS_CASE(NN)                                                                         \
  case NN:                                                                                  \
    if constexpr (has_variants(NN))                                                         \
      pick(var, std::make_integer_sequence<int, NZCURL>{}, [&](auto I) {                    \
        tx = zcurl_tx_of<T, NN, decltype(I)::value>();                                      \
        return hipSuccess;                                                                  \
      });                                                                                   \
    else                                                                                    \
      tx = zcurl_tx_of<T, NN, 0>();                                                         \
    break;
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return tx;
}

// ---------------- forward z pass + epilogue ----------------
template <typename T, int N, int I, bool MHD, bool ELS = false>
hipError_t z_epi_v(ZEpiArgs<T> a, const DiskTiles* dt, hipStream_t s) {
  constexpr ZV v = ZEPI_V[I];
  using LC = ZepiSched<N, I>;
  constexpr int TX = StridedTX<T, N, LC::TQ, v.sh>::value;
  constexpr int SPLIT = ELS && MHD && v.split >= 2 ? 2 : 1;
  if (a.g.nz != N) return hipErrorInvalidValue;
  a.ntile = cdiv(a.g.nx / 2 + 1, TX);
  const long grid = z_grid<TX>(a.g.ny, a.ntile, a.nb, a.prune && a.mode != 0, dt, a.tiles, a.ntl) * SPLIT;
  k_z_epi<T, N, LC::TQ, TX, typename LC::RL, MHD, waves_per_simd(v.minb, TX * LC::TQ), ELS, SPLIT>
      <<<dim3((unsigned)grid), dim3(TX * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int N, int I>
hipError_t z_epi_m(bool mhd, bool els, ZEpiArgs<T> a, const DiskTiles* dt, hipStream_t s) {
  if (els) return mhd ? z_epi_v<T, N, I, true, true>(a, dt, s) : z_epi_v<T, N, I, false, true>(a, dt, s);
  return mhd ? z_epi_v<T, N, I, true>(a, dt, s) : z_epi_v<T, N, I, false>(a, dt, s);
}

template <typename T, int N>
hipError_t z_epi_n(bool mhd, bool els, int var, ZEpiArgs<T> a, const DiskTiles* dt, hipStream_t s) {
  if constexpr (has_variants(N))
    return pick(var, std::make_integer_sequence<int, NZEPI>{},
                [&](auto I) { return z_epi_m<T, N, decltype(I)::value>(mhd, els, a, dt, s); });
  else
    return z_epi_m<T, N, 0>(mhd, els, a, dt, s);
}

template <typename T>
hipError_t launch_z_epi(int N, bool mhd, bool els, int var, ZEpiArgs<T> a, const DiskTiles* dt,
                        hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return z_epi_n<T, NN>(mhd, els, var, a, dt, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
int z_epi_tx(int N, int var) {
  int tx = 0;
  switch (N) {
#define PS_CASE(NN)                                                                         \
  case NN:                                                                                  \
    if constexpr (has_variants(NN))                                                         \
      pick(var, std::make_integer_sequence<int, NZEPI>{}, [&](auto I) {                     \
        tx = zepi_tx_of<T, NN, decltype(I)::value>();                                       \
        return hipSuccess;                                                                  \
      });                                                                                   \
    else                                                                                    \
      tx = zepi_tx_of<T, NN, 0>();                                                          \
    break;
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return tx;
}

// ---------------- x passes ----------------
template <typename T, int N>
hipError_t x_c2r_n(XArgs<T> a, hipStream_t s) {
  using LC = LenCfg<N / 2>;
  using X = XCfg<T, N / 2, LC::TQ>;
  const long grid = (a.rows * a.nf * a.nb + X::G - 1) / X::G;
  k_x_c2r<T, N / 2, LC::TQ, X::G, typename LC::RL><<<dim3((unsigned)grid), dim3(X::G * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t x_r2c_n(XArgs<T> a, hipStream_t s) {
  using LC = LenCfg<N / 2>;
  using X = XCfg<T, N / 2, LC::TQ>;
  const long grid = (a.rows * a.nf * a.nb + X::G - 1) / X::G;
  k_x_r2c<T, N / 2, LC::TQ, X::G, typename LC::RL><<<dim3((unsigned)grid), dim3(X::G * LC::TQ), 0, s>>>(a);
  return hipGetLastError();
}

// packed form: full-length complex transforms, two real rows each
template <typename T, int N, int I>
hipError_t x_prod_pk_v(bool mhd, bool els, XArgs<T> a, hipStream_t s) {
  constexpr XV v = XPROD_V[I];
  using LC = Sched<N, v.sched == 1>;
  using X = XPkCfg<T, N, LC::TQ>;
  constexpr int LIM = v.big ? 81920 : 65536;
  using RLay = std::conditional_t<v.swz, LaySwz32, LayPad8>;
  constexpr int LP = v.ex ? Stockham<T, N, LC::TQ, FWD, typename LC::RL>::EX_SLOTS : RLay::slots(N);
  auto go = [&](auto mhd_c, auto els_c) -> hipError_t {
    constexpr bool M_ = decltype(mhd_c)::value, E_ = decltype(els_c)::value;
    constexpr int FI = xprod_fin(M_, E_), FO = xprod_fout(M_, E_);
    // short transforms: enough rows per workgroup for about 256 threads
    constexpr int want0 = M_ ? v.rb_mhd : v.rb_ns;
    constexpr int wfill = 256 / (X::w(FI, FO, 1) * LC::TQ) > want0 ? 256 / (X::w(FI, FO, 1) * LC::TQ) : want0;
    constexpr int RB = X::rb(FI, FO, wfill, LP, LIM);
    if constexpr (!X::fits(FI, FO, RB, LP, 163840)) {
      return hipErrorInvalidValue;
    } else {
      if (a.rows < RB) return hipErrorInvalidValue;  // the kernel assumes a box holds RB rows
      const long grid = (a.rows * a.nb + RB - 1) / RB;
      // dealiased input (kx <= (N - 1) / 3): the pruned form skips the slots
      // that hold only zeros or outputs nobody reads
      bool pruned = false;
      if constexpr (v.pr) pruned = a.kmax <= (N - 1) / 3;
      if (pruned)
        k_x_prod_pk<T, N, LC::TQ, RB, typename LC::RL, M_, E_, RLay, v.ex, v.pr>
            <<<dim3((unsigned)grid), dim3(xpk_slots(M_, E_, RB) * LC::TQ), 0, s>>>(a);
      else
        k_x_prod_pk<T, N, LC::TQ, RB, typename LC::RL, M_, E_, RLay, v.ex, false>
            <<<dim3((unsigned)grid), dim3(xpk_slots(M_, E_, RB) * LC::TQ), 0, s>>>(a);
      return hipGetLastError();
    }
  };
  using t_ = std::true_type;
  using f_ = std::false_type;
  if (mhd && els) return go(t_{}, t_{});
  if (mhd) return go(t_{}, f_{});
  if (els) return go(f_{}, t_{});
  return go(f_{}, f_{});
}

template <typename T, int N, int I>
hipError_t x_prod_v(bool mhd, bool els, XArgs<T> a, hipStream_t s) {
  constexpr XV v = XPROD_V[I];
  if constexpr (v.pk) return x_prod_pk_v<T, N, I>(mhd, els, a, s);
  using LC = std::conditional_t<v.sched == 2, LenWide<N / 2>, Sched<N / 2, v.sched == 1>>;
  using X = XCfg<T, N / 2, LC::TQ>;
  constexpr int LIM = v.big ? 81920 : 65536;  // LDS bytes per workgroup
  auto go = [&](auto mhd_c, auto els_c, auto rb_c) {
    constexpr bool M_ = decltype(mhd_c)::value, E_ = decltype(els_c)::value;
    constexpr int RB = decltype(rb_c)::value;
    const long grid = (a.rows * a.nb + RB - 1) / RB;
    using RLay = std::conditional_t<v.swz, LaySwz32, LayPad8>;
    k_x_prod<T, N / 2, LC::TQ, RB, typename LC::RL, M_, E_, RLay, LIM>
        <<<dim3((unsigned)grid), dim3(xprod_slots(M_, E_) * RB * LC::TQ), 0, s>>>(a);
    return hipGetLastError();
  };
  using t_ = std::true_type;
  using f_ = std::false_type;
  // short rows (few threads per transform): enough rows per workgroup for
  // about 192 threads, so that small boxes still fill whole waves
  constexpr auto want = [](int slots, int rb) {
    const int w = 192 / (slots * LC::TQ);
    return w > rb ? w : rb;
  };
  // a variant whose configuration does not fit this size (threads or LDS)
  // runs as variant 0, so that every variant index is valid at every size
  if (mhd && els) {
    if constexpr (X::fits(8, 1))
      return go(t_{}, t_{}, std::integral_constant<int, X::rb(8, want(8, v.rb_mhd), LIM)>{});
    else if constexpr (I != 0)
      return x_prod_v<T, N, 0>(mhd, els, a, s);
    return hipErrorInvalidValue;
  }
  if (mhd) {
    if constexpr (X::MHD_OK)
      return go(t_{}, f_{}, std::integral_constant<int, X::rb(12, want(12, v.rb_mhd), LIM)>{});
    else if constexpr (I != 0)
      return x_prod_v<T, N, 0>(mhd, els, a, s);
    return hipErrorInvalidValue;
  }
  if (els) {
    if constexpr (X::launchable(5))
      return go(f_{}, t_{}, std::integral_constant<int, X::rb(5, want(5, v.rb_ns), LIM)>{});
    else if constexpr (I != 0)
      return x_prod_v<T, N, 0>(mhd, els, a, s);
    return hipErrorInvalidValue;
  }
  if constexpr (X::launchable(6))
    return go(f_{}, f_{}, std::integral_constant<int, X::rb(6, want(6, v.rb_ns), LIM)>{});
  else if constexpr (I != 0)
    return x_prod_v<T, N, 0>(mhd, els, a, s);
  return hipErrorInvalidValue;
}

template <typename T, int N>
hipError_t x_prod_n(bool mhd, bool els, int var, XArgs<T> a, hipStream_t s) {
  if constexpr (has_variants(N))
    return pick(var, std::make_integer_sequence<int, NXPROD>{},
                [&](auto I) { return x_prod_v<T, N, decltype(I)::value>(mhd, els, a, s); });
  else
    return x_prod_v<T, N, 0>(mhd, els, a, s);
}

template <typename T>
bool mhd_supported(int N) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return XCfg<T, NN / 2, LenCfg<NN / 2>::TQ>::MHD_OK;
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return false;
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
hipError_t launch_x_prod(int N, bool mhd, bool els, int var, XArgs<T> a, hipStream_t s) {
  switch (N) {
#define PS_CASE(NN) \
  case NN:          \
    return x_prod_n<T, NN>(mhd, els, var, a, s);
    PS_FOR_EACH_N(PS_CASE)
#undef PS_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace ps
