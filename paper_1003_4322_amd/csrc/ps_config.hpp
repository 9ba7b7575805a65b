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

// Alternate schedules with radix-16 stages (fewer LDS exchanges, 16 values
// per thread), used by the kernel variants for N >= 256.
template <int L>
struct LenAlt : LenCfg<L> {};
#define PS_ALT(L_, TQ_, ...)                     \
  template <>                                    \
  struct LenAlt<L_> {                            \
    using RL = Radices<__VA_ARGS__>;             \
    static constexpr int TQ = TQ_;               \
  };
PS_ALT(128, 8, 16, 8)
PS_ALT(192, 12, 16, 4, 3)
PS_ALT(256, 16, 16, 16)
PS_ALT(384, 24, 16, 8, 3)
PS_ALT(512, 32, 16, 8, 4)
PS_ALT(768, 48, 16, 16, 3)
PS_ALT(1024, 64, 16, 8, 8)
#undef PS_ALT

// Wide schedules: a last radix of 4 over twice the threads (four values per
// thread at the end, whole waves for any number of rows at M = 256); product
// pass variants only.
template <int L>
struct LenWide : LenCfg<L> {};
#define PS_WIDE(L_, TQ_, ...)                    \
  template <>                                    \
  struct LenWide<L_> {                           \
    using RL = Radices<__VA_ARGS__>;             \
    static constexpr int TQ = TQ_;               \
  };
PS_WIDE(256, 64, 4, 4, 4, 4)
PS_WIDE(512, 128, 8, 4, 4, 4)
#undef PS_WIDE

#undef PS_LEN

// grid sizes with a compiled configuration
#define PS_FOR_EACH_N(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// Tile width of a strided pass: 16 columns (FP32) or 8 (FP64), halved SH
// times, capped by 64 KB of LDS and 1024 threads.
template <typename T, int N, int TQ, int SH>
struct StridedTX {
  static constexpr int TX0 = (sizeof(T) == 4 ? 16 : 8) >> SH;
  static constexpr int TXL = (65536 / (N * 2 * (int)sizeof(T)));
  static constexpr int TX1 = TX0 < TXL ? TX0 : TXL;
  static constexpr int TX2 = (TX1 * TQ > 1024) ? 1024 / TQ : TX1;
  static constexpr int value = TX2 < 1 ? 1 : TX2;
};

constexpr bool has_variants(int N) { return N >= 256; }

// x passes: rows live in LDS with the padded layout (pad8, M + M/8 + 1 slots)
// or, in the fused pass's swizzled variants, LaySwz32 (32 (M/32 + 1) slots);
// the fused pass also stages twiddles (2M values).
template <typename T, int M, int TQ>
struct XCfg {
  // LDS slots per row: the larger of the padded and swizzled layouts
  static constexpr int SLOTS = (M + M / 8 + 1) > 32 * (M / 32 + 1) ? (M + M / 8 + 1) : 32 * (M / 32 + 1);
  static constexpr int G = (256 / TQ) < 1 ? 1 : 256 / TQ;  // plain passes: rows per workgroup
  // lim: LDS bytes per workgroup (64 KB; 80 KB for two workgroups per CU)
  static constexpr bool fits(int f, int rb, int lim = 65536) {
    return (f * rb * SLOTS + 2 * M) * 2 * (int)sizeof(T) <= lim && f * rb * TQ <= 1024;
  }
  static constexpr int rb(int f, int want, int lim = 65536) {
    int r = want < 1 ? 1 : want;
    while (r > 1 && !fits(f, r, lim)) r >>= 1;
    return r;
  }
  static constexpr bool MHD_OK = fits(12, 1, 65536);
  // launch limits alone: 1024 threads and the 160 KB of LDS a gfx950
  // workgroup may hold (rows that overflow 64 KB cost occupancy, not
  // correctness)
  static constexpr bool launchable(int f) {
    return (f * SLOTS + 2 * M) * 2 * (int)sizeof(T) <= 163840 && f * TQ <= 1024;
  }
};

// Packed x pass (k_x_prod_pk): W = max(ceil(FIN rb / 2), ceil(FOUT rb / 2))
// complex transforms of length N, TQ threads each; LDS of W rows of `slots`
// plus N staged twiddles.
// lp: LDS slots per transform.
template <typename T, int N, int TQ>
struct XPkCfg {
  static constexpr int w(int fin, int fout, int rb) {
    const int a = (fin * rb + 1) / 2, b = (fout * rb + 1) / 2;
    return a > b ? a : b;
  }
  static constexpr bool fits(int fin, int fout, int rb, int lp, int lim) {
    return (w(fin, fout, rb) * lp + N) * 2 * (int)sizeof(T) <= lim && w(fin, fout, rb) * TQ <= 1024;
  }
  // an even number of grid rows, so that every transform pairs one field on
  // two grid rows (two different fields, such as u and its curl, can differ
  // in size by |k|, and the smaller would carry the larger one's rounding)
  static constexpr int rb(int fin, int fout, int want, int lp, int lim) {
    int r = 2;
    while (2 * r <= want) r *= 2;  // a power of two, at least 2
    while (r > 2 && !fits(fin, fout, r, lp, lim)) r >>= 1;
    return r;
  }
};

// Kernel variant tables.  Strided-pass variants: tile shift, z_curl split and
// direct gather, minimum workgroups per CU asked of the register allocator,
// alternate (radix-16) schedule.  Product-pass variants: rows per workgroup,
// schedule.
struct ZV {
  int sh;       // tile width shift
  int split;    // z_curl: workgroups per tile sharing the output groups (1, 2 or 4; NS caps at 2);
                // z_epi: 2 = z+ and z- updated by two workgroups (Elsasser form only)
  int minb;     // workgroups per CU the register allocator must leave room for (1: no request)
  bool alt;     // radix-16 schedule
  bool direct;  // z_curl: gather inputs per output field instead of holding them in registers
  bool wide = false;  // wide schedule (LenWide: a last radix of 4 over twice the threads)
  bool tws = false;   // strided passes: twiddles staged in LDS beside the tile
};
struct XV {
  int rb_ns, rb_mhd;  // rows per workgroup (reduced while the LDS tile would not fit)
  int sched;          // 0 LenCfg, 1 radix-16 (LenAlt), 2 wide (LenWide)
  bool swz;           // rows in LDS swizzled (LaySwz32) instead of padded (LayPad8)
  bool big = false;   // up to 80 KB of LDS per workgroup (two per CU) instead of 64 KB
  bool pk = false;    // packed form (k_x_prod_pk): two real rows per complex transform of length N
  bool ex = false;    // packed form: per-exchange LDS layouts (LayEx) and rows in natural order
  bool pr = false;    // packed form on dealiased input (kx <= (N - 1) / 3): the slots of
                      // zeros and of unread outputs skipped (falls back when kmax is larger)
};
constexpr ZV ZCURL_V[] = {{1, 1, 1, false, false}, {1, 2, 1, false, false}, {1, 2, 2, false, false},
                          {1, 2, 1, true, false},  {1, 1, 1, false, true},  {0, 2, 1, true, false},
                          {0, 1, 1, true, false}};
constexpr ZV ZEPI_V[] = {{0, 1, 1, false}, {1, 1, 1, false}, {1, 1, 2, false}, {1, 1, 1, true},
                         {2, 1, 1, false}, {1, 2, 1, false}, {1, 2, 2, false}, {2, 2, 1, false},
                         {0, 1, 1, false, false, true}, {1, 1, 1, false, false, true},
                         {1, 1, 2, false, false, true}, {2, 1, 1, false, false, true}};
constexpr ZV STR_V[] = {{0, 1, 1, false}, {1, 1, 1, false}, {0, 1, 1, true}, {1, 1, 1, true},
                        {0, 1, 1, true, false, false, true}, {0, 1, 1, false, false, false, true}};
constexpr XV XPROD_V[] = {{2, 1, 0, false}, {4, 2, 0, false}, {4, 2, 1, false}, {2, 1, 1, false},
                          {2, 1, 0, true},  {4, 2, 0, true},  {1, 1, 2, true},  {1, 1, 2, false},
                          {8, 4, 0, true, true}, {8, 4, 0, false, true}, {4, 2, 2, true, true},
                          // packed form
                          {2, 2, 0, false, false, true, true}, {4, 4, 0, false, true, true, true},
                          {2, 2, 0, true, false, true}, {4, 4, 0, true, true, true},
                          {2, 2, 1, false, false, true, true}, {4, 4, 1, false, true, true, true},
                          {8, 8, 0, false, true, true, true},
                          // packed, dealiased input
                          {2, 2, 0, false, false, true, true, true}, {8, 8, 0, false, true, true, true, true},
                          {2, 2, 0, true, false, true, false, true}};
constexpr int NZCURL = sizeof(ZCURL_V) / sizeof(ZV);
// waves per SIMD that minb workgroups of `threads` threads occupy (4 SIMDs per CU)
constexpr int waves_per_simd(int minb, int threads) {
  const int w = minb * ((threads + 63) / 64) / 4;
  return w < 1 ? 1 : w;
}
constexpr int NZEPI = sizeof(ZEPI_V) / sizeof(ZV);
constexpr int NSTR = sizeof(STR_V) / sizeof(ZV);
constexpr int NXPROD = sizeof(XPROD_V) / sizeof(XV);

}  // namespace ps
