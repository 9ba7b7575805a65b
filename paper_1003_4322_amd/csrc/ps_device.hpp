// ps_device.hpp -- device-side building blocks for the gfx950 pseudospectral
// kernels: interleaved complex values, small-radix DFT butterflies and a
// Stockham autosort FFT engine that stages its exchanges through LDS.
//
// The transform computed is the plain DFT of the method's Fourier-Galerkin
// discretisation (Sec. 2 of the paper: every field is a truncated Fourier
// series and its derivatives, products and transforms are evaluated through
// fast Fourier transforms).  The engine reaches the DFT exactly up to
// rounding; twiddles are read from tables computed on the host in extended
// precision and rounded once to the working type.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ps {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> mk(T a, T b) { return C2<T>{a, b}; }
template <typename T>
__device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b) { return C2<T>{a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b) { return C2<T>{a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> operator*(T s, C2<T> a) { return C2<T>{s * a.x, s * a.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return C2<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) {
  return C2<T>{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ C2<T> conj(C2<T> a) { return C2<T>{a.x, -a.y}; }
// multiply by +i and -i
template <typename T>
__device__ __forceinline__ C2<T> mul_i(C2<T> a) { return C2<T>{-a.y, a.x}; }
// c ? x : y on values
template <typename T>
__device__ __forceinline__ C2<T> sel(bool c, C2<T> x, C2<T> y) { return c ? x : y; }
// streaming store (non-temporal hint): for outputs far larger than the caches
// that the next pass reads back from HBM anyway
template <typename T>
__device__ __forceinline__ void store_nt(C2<T>* p, C2<T> v) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  V2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<V2*>(p));
}
template <typename T>
__device__ __forceinline__ C2<T> mul_mi(C2<T> a) { return C2<T>{a.y, -a.x}; }
template <typename T>
__device__ __forceinline__ C2<T> zero2() { return C2<T>{T(0), T(0)}; }

// Direction: FWD computes sum x_j exp(-2 pi i j k / n), INV uses exp(+...).
enum { FWD = 0, INV = 1 };

// multiply by -i (FWD) or +i (INV): the quarter-turn of the DFT kernel
template <int DIR, typename T>
__device__ __forceinline__ C2<T> rot4(C2<T> a) { return DIR == FWD ? mul_mi(a) : mul_i(a); }

// twiddle w(e) = exp(-+ 2 pi i e / L) from a table tw[e] = exp(-2 pi i e / L)
template <int DIR, typename T>
__device__ __forceinline__ C2<T> tw_apply(C2<T> a, C2<T> w) { return DIR == FWD ? cmul(a, w) : cmulc(a, w); }

// ---------------------------------------------------------------------------
// Small DFTs in registers.  dft<R, DIR>(a) replaces a[0..R) by its R-point DFT.
// ---------------------------------------------------------------------------
template <int R, int DIR, typename T>
struct Dft;

template <int DIR, typename T>
struct Dft<2, DIR, T> {
  __device__ __forceinline__ static void run(C2<T>* a) {
    C2<T> t = a[0] - a[1];
    a[0] = a[0] + a[1];
    a[1] = t;
  }
};

template <int DIR, typename T>
struct Dft<3, DIR, T> {
  __device__ __forceinline__ static void run(C2<T>* a) {
    const T c = T(-0.5);
    const T s = T(0.86602540378443864676372317075293618);  // sin(2 pi / 3)
    C2<T> t1 = a[1] + a[2];
    C2<T> t2 = a[1] - a[2];
    C2<T> m = a[0] + c * t1;
    // FWD: y1 = m - i s t2, y2 = m + i s t2
    C2<T> r = s * (DIR == FWD ? mul_mi(t2) : mul_i(t2));
    a[0] = a[0] + t1;
    a[1] = m + r;
    a[2] = m - r;
  }
};

template <int DIR, typename T>
struct Dft<4, DIR, T> {
  __device__ __forceinline__ static void run(C2<T>* a) {
    C2<T> t0 = a[0] + a[2];
    C2<T> t1 = a[0] - a[2];
    C2<T> t2 = a[1] + a[3];
    C2<T> t3 = rot4<DIR>(a[1] - a[3]);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
  }
};

template <int DIR, typename T>
struct Dft<8, DIR, T> {
  __device__ __forceinline__ static void run(C2<T>* a) {
    const T h = T(0.70710678118654752440084436210484904);
    C2<T> e[4] = {a[0], a[2], a[4], a[6]};
    C2<T> o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, DIR, T>::run(e);
    Dft<4, DIR, T>::run(o);
    // o[k] *= W8^k, W8 = exp(-+ i pi / 4)
    {
      C2<T> v = o[1];
      // FWD: (1 - i)/sqrt2 ; INV: (1 + i)/sqrt2
      o[1] = DIR == FWD ? C2<T>{h * (v.x + v.y), h * (v.y - v.x)} : C2<T>{h * (v.x - v.y), h * (v.y + v.x)};
      o[2] = rot4<DIR>(o[2]);
      v = o[3];
      // FWD: (-1 - i)/sqrt2 ; INV: (-1 + i)/sqrt2
      o[3] = DIR == FWD ? C2<T>{h * (v.y - v.x), -h * (v.x + v.y)} : C2<T>{-h * (v.x + v.y), h * (v.x - v.y)};
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = e[k] + o[k];
      a[k + 4] = e[k] - o[k];
    }
  }
};

// multiply by w16^m = exp(-+ 2 pi i m / 16), m a compile-time constant
template <int m, int DIR, typename T>
__device__ __forceinline__ C2<T> w16(C2<T> v) {
  constexpr double C[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                            -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  constexpr int ms = m & 15;
  constexpr T c = (T)C[ms];
  constexpr T sn = (T)C[(ms + 12) & 15];  // sin(2 pi m / 16) = cos(2 pi (m - 4) / 16)
  if constexpr (ms == 0) return v;
  if constexpr (ms == 4) return rot4<DIR>(v);
  if constexpr (ms == 8) return C2<T>{-v.x, -v.y};
  // FWD: v * (c - i sn); INV: v * (c + i sn)
  if constexpr (DIR == FWD)
    return C2<T>{c * v.x + sn * v.y, c * v.y - sn * v.x};
  else
    return C2<T>{c * v.x - sn * v.y, c * v.y + sn * v.x};
}

// radix 16 as 4 x 4: inner 4-point DFTs over a[4 n1 + n2], twiddle
// w16^{n2 k1}, outer 4-point DFTs over n2; output index k1 + 4 k2.
template <int DIR, typename T>
struct Dft<16, DIR, T> {
  __device__ __forceinline__ static void run(C2<T>* a) {
    C2<T> b[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      C2<T> t[4] = {a[n2], a[4 + n2], a[8 + n2], a[12 + n2]};
      Dft<4, DIR, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) b[n2][k1] = t[k1];
    }
    b[1][1] = w16<1, DIR>(b[1][1]);
    b[1][2] = w16<2, DIR>(b[1][2]);
    b[1][3] = w16<3, DIR>(b[1][3]);
    b[2][1] = w16<2, DIR>(b[2][1]);
    b[2][2] = w16<4, DIR>(b[2][2]);
    b[2][3] = w16<6, DIR>(b[2][3]);
    b[3][1] = w16<3, DIR>(b[3][1]);
    b[3][2] = w16<6, DIR>(b[3][2]);
    b[3][3] = w16<9, DIR>(b[3][3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C2<T> t[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
      Dft<4, DIR, T>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
    }
  }
};

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(C2<T>* a) { Dft<R, DIR, T>::run(a); }

// The same DFTs with the inputs whose bit is set in ZM known to be zero at
// compile time: the additions with them are left out (the compiler may not
// drop x + 0 itself, which differs from x for x = -0).  Radix 4 and 8; other
// radices fall back to the full DFT.
template <typename T>
__device__ __forceinline__ C2<T> neg2(C2<T> a) { return C2<T>{-a.x, -a.y}; }
template <int R, int DIR, unsigned ZM, typename T>
struct DftZ {
  __device__ __forceinline__ static void run(C2<T>* a) { Dft<R, DIR, T>::run(a); }
};
template <int DIR, unsigned ZM, typename T>
struct DftZ<4, DIR, ZM, T> {
  __device__ __forceinline__ static void run(C2<T>* a) {
    constexpr bool z0 = ZM & 1u, z1 = ZM & 2u, z2 = ZM & 4u, z3 = ZM & 8u;
    C2<T> t0, t1, t2, t3;
    if constexpr (z0 && z2) {
      t0 = zero2<T>(), t1 = zero2<T>();
    } else if constexpr (z2) {
      t0 = a[0], t1 = a[0];
    } else if constexpr (z0) {
      t0 = a[2], t1 = neg2(a[2]);
    } else {
      t0 = a[0] + a[2], t1 = a[0] - a[2];
    }
    if constexpr (z1 && z3) {
      t2 = zero2<T>(), t3 = zero2<T>();
    } else if constexpr (z3) {
      t2 = a[1], t3 = rot4<DIR>(a[1]);
    } else if constexpr (z1) {
      t2 = a[3], t3 = rot4<DIR>(neg2(a[3]));
    } else {
      t2 = a[1] + a[3], t3 = rot4<DIR>(a[1] - a[3]);
    }
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
  }
};
template <int DIR, unsigned ZM, typename T>
struct DftZ<8, DIR, ZM, T> {
  __device__ __forceinline__ static void run(C2<T>* a) {
    // even inputs 0, 2, 4, 6 and odd inputs 1, 3, 5, 7 of the 2 x 4 split
    constexpr unsigned ze = (ZM & 1u) | ((ZM >> 1) & 2u) | ((ZM >> 2) & 4u) | ((ZM >> 3) & 8u);
    constexpr unsigned zo = ((ZM >> 1) & 1u) | ((ZM >> 2) & 2u) | ((ZM >> 3) & 4u) | ((ZM >> 4) & 8u);
    const T h = T(0.70710678118654752440084436210484904);
    C2<T> e[4] = {a[0], a[2], a[4], a[6]};
    C2<T> o[4] = {a[1], a[3], a[5], a[7]};
    DftZ<4, DIR, ze, T>::run(e);
    DftZ<4, DIR, zo, T>::run(o);
    {
      C2<T> v = o[1];
      o[1] = DIR == FWD ? C2<T>{h * (v.x + v.y), h * (v.y - v.x)} : C2<T>{h * (v.x - v.y), h * (v.y + v.x)};
      o[2] = rot4<DIR>(o[2]);
      v = o[3];
      o[3] = DIR == FWD ? C2<T>{h * (v.y - v.x), -h * (v.x + v.y)} : C2<T>{-h * (v.x + v.y), h * (v.x - v.y)};
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = e[k] + o[k];
      a[k + 4] = e[k] - o[k];
    }
  }
};

// A first-stage loader whose slots with a bit set in ZM are zero at compile
// time (the loader of the slot is not called); the Stockham engine then uses
// DftZ for the first stage when each thread does one butterfly there.
template <unsigned ZM, class F>
struct LdZ {
  F f;
  __device__ __forceinline__ auto operator()(int slot, int idx) const {
    using V = decltype(f(slot, idx));
    if constexpr (ZM == 0)
      return f(slot, idx);
    else
      return slot < 32 && ((ZM >> slot) & 1u) ? V{} : f(slot, idx);
  }
};
template <unsigned ZM, class F>
__device__ __forceinline__ LdZ<ZM, F> ld_zero(F f) {
  return LdZ<ZM, F>{f};
}
template <class L>
struct LdZeroMask {
  static constexpr unsigned value = 0;
};
template <unsigned ZM, class F>
struct LdZeroMask<LdZ<ZM, F>> {
  static constexpr unsigned value = ZM;
};

// ---------------------------------------------------------------------------
// Radix schedules
// ---------------------------------------------------------------------------
template <int... Rs>
struct Radices {};

template <class RL>
struct RadixInfo;
template <int R0, int... Rs>
struct RadixInfo<Radices<R0, Rs...>> {
  static constexpr int first = R0;
  static constexpr int count = 1 + sizeof...(Rs);
  static constexpr int product = R0 * RadixInfo<Radices<Rs...>>::product;
  static constexpr int last = RadixInfo<Radices<Rs...>>::count == 0 ? R0 : RadixInfo<Radices<Rs...>>::last;
};
template <>
struct RadixInfo<Radices<>> {
  static constexpr int first = 1;
  static constexpr int count = 0;
  static constexpr int product = 1;
  static constexpr int last = 1;
};

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// LDS layouts of one transform's exchange buffer: element idx lives at
// lds[Lay::off(idx, ls)].  LayStride serves column tiles (ls = tile width);
// LayPad8 serves contiguous rows and inserts one pad slot after every 8
// elements, so the stride-R scatter of the first Stockham stage hits
// distinct LDS banks.
// SPLIT 2: off(a + c) = off(a) + offc(c) always; 1: whenever c % 8 == 0, or
// a % 8 == 0 and c < 8; 0: never.  The transforms use it to move the constant
// part of an unrolled index into the LDS instruction's offset.
struct LayStride {
  static constexpr int SPLIT = 2;
  __device__ __forceinline__ static int off(int i, int ls) { return i * ls; }
  __device__ __forceinline__ static int offc(int c, int ls) { return c * ls; }
};
struct LayPad8 {
  static constexpr int SPLIT = 1;
  __host__ __device__ static constexpr int slots(int M) { return M + M / 8 + 1; }
  __device__ __forceinline__ static int off(int i, int) { return i + (i >> 3); }
  __device__ __forceinline__ static int offc(int c, int) { return c + c / 8; }
};
__host__ __device__ constexpr int pad8(int i) { return i + (i >> 3); }
// rows, swizzled: element i at i ^ h(i / 32) with h(b) = (b & 7) | ((b & 6) << 2),
// a permutation inside every 32-element block.  For the radix-8 schedules it
// gives 32 distinct bank pairs to each of: 32 consecutive elements, the
// stride-8 scatter of a first radix-8 stage, and the scatter of a second one
// (pad8 wraps the first of these across 35 slots, so three lanes collide).
struct LaySwz32 {
  static constexpr int SPLIT = 0;
  __host__ __device__ static constexpr int slots(int M) { return 32 * (M / 32 + 1); }
  __device__ __forceinline__ static int off(int i, int) {
    const int b = i >> 5;
    return i ^ ((b & 7) | ((b & 6) << 2));
  }
  __device__ __forceinline__ static int offc(int c, int) { return c; }
};
// column tiles (TX columns side by side): row idx of the tile padded by one
// row per eight, so that a first stage writing rows j R + m from lanes of
// consecutive j spreads over the LDS banks instead of hitting one
struct LayColPad8 {
  static constexpr int SPLIT = 1;
  __device__ __forceinline__ static int off(int i, int ls) { return (i + (i >> 3)) * ls; }
  __device__ __forceinline__ static int offc(int c, int ls) { return (c + c / 8) * ls; }
};

// Per-exchange layout: the buffer a stage of span NS and radix R writes (and
// the next stage reads) keeps element i at i + P floor(i / B), P = NS and
// B = max(NS R, W) while NS < W, plain otherwise, where W = 256 bytes (the
// 64 four-byte LDS banks) over the element size: 32 complex floats, 16
// complex doubles.  Over any W consecutive threads the stage's writes (base
// (j / NS) NS R + j % NS, plus m NS) and the next stage's reads
// (j + m L / R') fall in distinct groups of banks, and every access of a
// thread is its base plus a constant: offc(c) when c % B == 0 (reads at
// stride L / R'), m NS when B % (NS R) == 0 (writes).
template <int NS, int R, int W = 32>
struct LayEx {
  static constexpr int P = NS < W ? NS : 0;
  static constexpr int B = NS * R > W ? NS * R : W;
  __host__ __device__ static constexpr int off(int i) { return P ? i + P * (i / B) : i; }
  __host__ __device__ static constexpr int offc(int c) { return P ? c + P * (c / B) : c; }
  static constexpr bool read_splits(int c) { return P == 0 || c % B == 0; }
  static constexpr bool write_splits = P == 0 || B % (NS * R) == 0;
  __host__ __device__ static constexpr int slots(int L) { return off(L - 1) + 1; }
};

// ---------------------------------------------------------------------------
// Stockham autosort FFT of length L done by TQ cooperating threads.
//
// Stage with radix R after Ns points have been combined: butterfly j
// (0 <= j < L/R) reads x[j + m L/R], m < R, multiplies input m by
// w^{m (j mod Ns)} with w = exp(-+ 2 pi i / (Ns R)), takes the R-point DFT
// and writes output m to position (j div Ns) Ns R + (j mod Ns) + m Ns.
// The result comes out in natural order.  Thread q runs butterflies
// j = q + TQ b.  The first stage reads its inputs through a caller functor
// ld(slot, idx); intermediate stages exchange through LDS (element idx at
// lds[Lay::off(idx, ls)]); the last stage leaves its outputs in registers:
// v[b * Rlast + m] holds output index q + TQ b + m (L / Rlast) (valid when
// q + TQ b < L / Rlast).
//
// Barrier discipline: every stage that writes LDS first waits until all
// threads finished reading the previous contents, so consecutive transforms
// (and in-place exchanges) can reuse one LDS buffer.
// ---------------------------------------------------------------------------
// Twiddle sources of the Stockham stages.  A stage of span NS and radix R
// multiplies input m of butterfly j by w^(m (j mod NS) L / (NS R)),
// w = exp(-2 pi i / L).
// TwTable: tw[e * twmul] = exp(-2 pi i e / (L twmul)), the plain table.
template <typename T>
struct TwTable {
  const C2<T>* tw;
  int twmul;
  template <int L, int NS, int R>
  __device__ __forceinline__ C2<T> get(int m, int k) const {
    return tw[(m * k * (L / (NS * R))) * twmul];
  }
};
// TwStaged: every stage's factors in the order the threads read them, the
// stage of span NS at offset NS - 1 (the spans before it sum to NS - 1), entry
// (m - 1) NS + k; consecutive k are consecutive words, so the reads of a wave
// fall in distinct LDS banks.  L - 1 entries in all.
template <typename T>
struct TwStaged {
  const C2<T>* t;
  template <int L, int NS, int R>
  __device__ __forceinline__ C2<T> get(int m, int k) const {
    return t[(NS - 1) + (m - 1) * NS + k];
  }
};
// entry idx of the TwStaged layout, found stage by stage with the span NS a
// compile-time constant (the divisions by NS are shifts or constant divisions)
template <typename T, int L, int NS, int R, int... Rest>
__device__ __forceinline__ void fill_staged_at(C2<T>* dst, const C2<T>* tw, int twmul, int idx) {
  if (idx < NS * R - 1) {
    const int r = idx - (NS - 1), m = 1 + r / NS, k = r % NS;
    dst[idx] = tw[(m * k * (L / (NS * R))) * twmul];
  } else if constexpr (sizeof...(Rest) > 0) {
    fill_staged_at<T, L, NS * R, Rest...>(dst, tw, twmul, idx);
  }
}
// fill dst[0, L - 1) with the TwStaged layout of schedule RL from a plain table
template <typename T, int L, int... Rs>
__device__ __forceinline__ void fill_staged(C2<T>* dst, const C2<T>* tw, int twmul, int tid, int nt,
                                            Radices<Rs...>) {
  for (int idx = tid; idx < L - 1; idx += nt) fill_staged_at<T, L, 1, Rs...>(dst, tw, twmul, idx);
}

// Exchange through LDS among the lanes of one wave.  A wave's LDS operations
// complete in the order it issues them, so no s_barrier is needed; the
// wavefront-scope fences and the wave barrier only keep the compiler from
// moving LDS accesses across this point.  Every lane of the wave must reach it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WAVE (the run_* template argument): every transform is done by lanes of a
// single wave (the group of TQ threads lies in one wave) in an LDS buffer of
// its own, so the exchanges after the first need only wave_lds_sync.  The
// first stage's pre-write barrier stays a workgroup barrier, because a first
// stage may gather from other transforms' buffers (a product of fields).
template <typename T, int L, int TQ, int DIR, class RL>
struct Stockham {
  static constexpr int R1 = RadixInfo<RL>::first;
  static constexpr int RL_ = RadixInfo<RL>::last;
  static constexpr int NSTAGE = RadixInfo<RL>::count;
  static_assert(RadixInfo<RL>::product == L, "radix schedule must multiply to L");
  // register slots: enough for the widest stage
  template <class RR>
  struct MaxSlots;
  template <int... Rs>
  struct MaxSlots<Radices<Rs...>> {
    static constexpr int value = [] {
      int m = 0;
      int rs[] = {Rs...};
      for (int r : rs) {
        int s = cdiv(L / r, TQ) * r;
        m = s > m ? s : m;
      }
      return m;
    }();
  };
  static constexpr int SLOTS = MaxSlots<RL>::value;
  // lanes whose accesses one LDS cycle (64 four-byte banks) serves
  static constexpr int EXW = 256 / (int)sizeof(C2<T>);
  static constexpr int FIRST_SLOTS = cdiv(L / R1, TQ) * R1;
  static constexpr int LAST_NB = cdiv(L / RL_, TQ);

  // index of first-stage input for (slot) -- used by callers that preload
  __device__ __forceinline__ static int first_index(int q, int slot) {
    const int b = slot / R1, m = slot % R1;
    return q + TQ * b + m * (L / R1);
  }
  __device__ __forceinline__ static bool first_valid(int q, int slot) {
    return (L / R1) % TQ == 0 || q + TQ * (slot / R1) < L / R1;
  }
  // output index of last-stage slot
  __device__ __forceinline__ static int last_index(int q, int slot) {
    const int b = slot / RL_, m = slot % RL_;
    return q + TQ * b + m * (L / RL_);
  }
  __device__ __forceinline__ static bool last_valid(int q, int slot) {
    return (L / RL_) % TQ == 0 || q + TQ * (slot / RL_) < L / RL_;
  }

  // act = false: the thread only takes part in the barriers (its group has no
  // transform to do); v is left undefined
  template <int NS, int R, bool FIRST, bool LAST, class Lay, bool WAVE, class TW, class Ld>
  __device__ __forceinline__ static void stage(C2<T> (&v)[SLOTS], C2<T>* lds, int ls, int q, const TW& tw,
                                               Ld& ld, bool act) {
    constexpr int NB = cdiv(L / R, TQ);
    constexpr bool EXACT = (L / R) % TQ == 0;
    if (act) {
      // ---- gather inputs
      constexpr bool SPLIT_G = Lay::SPLIT == 2 || (Lay::SPLIT == 1 && (L / R) % 8 == 0);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = q + TQ * b;
        const bool ok = EXACT || j < L / R;
        const int ja = Lay::off(j, ls);
#pragma unroll
        for (int m = 0; m < R; ++m) {
          const int idx = j + m * (L / R);
          if constexpr (FIRST) {
            v[b * R + m] = ok ? ld(b * R + m, idx) : zero2<T>();
          } else {
            const int o = SPLIT_G ? ja + Lay::offc(m * (L / R), ls) : Lay::off(idx, ls);
            v[b * R + m] = ok ? lds[o] : zero2<T>();
          }
        }
      }
      // ---- twiddle and butterfly
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = q + TQ * b;
        C2<T>* a = &v[b * R];
        if constexpr (NS > 1) {
          const int k = j % NS;
#pragma unroll
          for (int m = 1; m < R; ++m) a[m] = tw_apply<DIR>(a[m], tw.template get<L, NS, R>(m, k));
        }
        // slots the loader makes zero (one butterfly per thread: slot = m)
        if constexpr (FIRST && NB == 1 && LdZeroMask<Ld>::value != 0)
          DftZ<R, DIR, LdZeroMask<Ld>::value, T>::run(a);
        else
          dft<R, DIR>(a);
      }
    }
    if constexpr (!LAST) {
      constexpr bool SPLIT_W = Lay::SPLIT == 2 || (Lay::SPLIT == 1 && (NS % 8 == 0 || (NS == 1 && R % 8 == 0)));
      // all reads of the previous LDS contents are done
      if constexpr (WAVE && !FIRST)
        wave_lds_sync();
      else
        __syncthreads();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = q + TQ * b;
        if (act && (EXACT || j < L / R)) {
          const int base = (j / NS) * NS * R + (j % NS);
          const int ba = Lay::off(base, ls);
#pragma unroll
          for (int m = 0; m < R; ++m) {
            const int o = SPLIT_W ? ba + Lay::offc(m * NS, ls) : Lay::off(base + m * NS, ls);
            lds[o] = v[b * R + m];
          }
        }
      }
      // writes visible before the next stage gathers
      if constexpr (WAVE)
        wave_lds_sync();
      else
        __syncthreads();
    }
  }

  template <int NS, class Lay, bool WAVE, class TW, class Ld, int R, int... Rest>
  __device__ __forceinline__ static void chain(C2<T> (&v)[SLOTS], C2<T>* lds, int ls, int q, const TW& tw,
                                               Ld& ld, bool act, Radices<R, Rest...>) {
    stage<NS, R, NS == 1, sizeof...(Rest) == 0, Lay, WAVE>(v, lds, ls, q, tw, ld, act);
    if constexpr (sizeof...(Rest) > 0) chain<NS * R, Lay, WAVE>(v, lds, ls, q, tw, ld, act, Radices<Rest...>{});
  }

  // ---- the same with a layout of its own per exchange (LayEx): stage
  // (NS, R) gathers through the layout of the exchange before it (LR) and
  // writes through LayEx<NS, R>.  One transform per buffer, unit stride.
  template <int NS, int R, bool FIRST, bool LAST, class LR, bool WAVE, class TW, class Ld>
  __device__ __forceinline__ static void stage_ex(C2<T> (&v)[SLOTS], C2<T>* lds, int q, const TW& tw, Ld& ld,
                                                  bool act) {
    using LW = LayEx<NS, R, EXW>;
    constexpr int NB = cdiv(L / R, TQ);
    constexpr bool EXACT = (L / R) % TQ == 0;
    if (act) {
      constexpr bool SPLIT_G = FIRST || LR::read_splits(L / R);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = q + TQ * b;
        const bool ok = EXACT || j < L / R;
        if constexpr (FIRST) {
#pragma unroll
          for (int m = 0; m < R; ++m) v[b * R + m] = ok ? ld(b * R + m, j + m * (L / R)) : zero2<T>();
        } else {
          const int ja = LR::off(j);
#pragma unroll
          for (int m = 0; m < R; ++m) {
            const int o = SPLIT_G ? ja + LR::offc(m * (L / R)) : LR::off(j + m * (L / R));
            v[b * R + m] = ok ? lds[o] : zero2<T>();
          }
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = q + TQ * b;
        C2<T>* a = &v[b * R];
        if constexpr (NS > 1) {
          const int k = j % NS;
#pragma unroll
          for (int m = 1; m < R; ++m) a[m] = tw_apply<DIR>(a[m], tw.template get<L, NS, R>(m, k));
        }
        // slots the loader makes zero (one butterfly per thread: slot = m)
        if constexpr (FIRST && NB == 1 && LdZeroMask<Ld>::value != 0)
          DftZ<R, DIR, LdZeroMask<Ld>::value, T>::run(a);
        else
          dft<R, DIR>(a);
      }
    }
    if constexpr (!LAST) {
      // all reads of the previous LDS contents are done
      if constexpr (WAVE && !FIRST)
        wave_lds_sync();
      else
        __syncthreads();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = q + TQ * b;
        if (act && (EXACT || j < L / R)) {
          const int base = (j / NS) * NS * R + (j % NS);
          const int ba = LW::off(base);
#pragma unroll
          for (int m = 0; m < R; ++m) lds[LW::write_splits ? ba + m * NS : LW::off(base + m * NS)] = v[b * R + m];
        }
      }
      // writes visible before the next stage gathers
      if constexpr (WAVE)
        wave_lds_sync();
      else
        __syncthreads();
    }
  }
  template <int NS, class LR, bool WAVE, class TW, class Ld, int R, int... Rest>
  __device__ __forceinline__ static void chain_ex(C2<T> (&v)[SLOTS], C2<T>* lds, int q, const TW& tw, Ld& ld,
                                                  bool act, Radices<R, Rest...>) {
    stage_ex<NS, R, NS == 1, sizeof...(Rest) == 0, LR, WAVE>(v, lds, q, tw, ld, act);
    if constexpr (sizeof...(Rest) > 0)
      chain_ex<NS * R, LayEx<NS, R, EXW>, WAVE>(v, lds, q, tw, ld, act, Radices<Rest...>{});
  }
  template <bool WAVE = false, class TW, class Ld>
  __device__ __forceinline__ static void run_ex(C2<T> (&v)[SLOTS], C2<T>* lds, int q, const TW& tw, Ld ld,
                                                bool act = true) {
    static_assert(!WAVE || (TQ <= 64 && 64 % TQ == 0), "WAVE needs each transform inside one wave");
    chain_ex<1, LayEx<1, 1, EXW>, WAVE>(v, lds, q, tw, ld, act, RL{});
  }
  // LDS slots of one transform's buffer under run_ex (the exchanges, and the
  // natural-order copy callers keep after the last stage)
  template <class RR>
  struct ExSlots;
  template <int... Rs>
  struct ExSlots<Radices<Rs...>> {
    static constexpr int value = [] {
      int rs[] = {Rs...};
      int m = L, ns = 1;
      for (int r : rs) {
        const int p = ns < EXW ? ns : 0, b = ns * r > EXW ? ns * r : EXW;
        const int sl = (p ? (L - 1) + p * ((L - 1) / b) : L - 1) + 1;
        m = sl > m ? sl : m;
        ns *= r;
      }
      return m;
    }();
  };
  static constexpr int EX_SLOTS = ExSlots<RL>::value;

  // tw: table of exp(-2 pi i e / (L * twmul)), e < L * twmul.
  template <class Lay = LayStride, class Ld>
  __device__ __forceinline__ static void run(C2<T> (&v)[SLOTS], C2<T>* lds, int ls, int q,
                                             const C2<T>* __restrict__ tw, int twmul, Ld ld) {
    chain<1, Lay, false>(v, lds, ls, q, TwTable<T>{tw, twmul}, ld, true, RL{});
  }
  // any twiddle source (TwTable, TwStaged); act as in stage()
  template <class Lay, bool WAVE = false, class TW, class Ld>
  __device__ __forceinline__ static void run_tw(C2<T> (&v)[SLOTS], C2<T>* lds, int ls, int q, const TW& tw,
                                                Ld ld, bool act = true) {
    static_assert(!WAVE || (TQ <= 64 && 64 % TQ == 0), "WAVE needs each transform inside one wave");
    chain<1, Lay, WAVE>(v, lds, ls, q, tw, ld, act, RL{});
  }
};

// ---------------------------------------------------------------------------
// Wavenumbers
// ---------------------------------------------------------------------------
// signed wavenumber of a ky/kz storage index (N/2 -> -N/2)
__device__ __forceinline__ int wav(int i, int N) { return i < N / 2 ? i : i - N; }
// derivative wavenumber: zero at the Nyquist index
__device__ __forceinline__ int dwav(int i, int N) { return 2 * i == N ? 0 : wav(i, N); }
__device__ __forceinline__ int dwavx(int i, int N) { return 2 * i == N ? 0 : i; }

// A box's grid: axis lengths and the 2/3 rule on it.  A mode is kept when
// (3 kx/nx)^2 + (3 ky/ny)^2 + (3 kz/nz)^2 < 1 (the sphere 9|k|^2 < N^2 of the
// cube, stretched with the grid), tested in integers as
// 9 (kx^2 wx + ky^2 wy + kz^2 wz) < lim with w_a = (M / n_a)^2, lim = M^2,
// M = lcm(nx, ny, nz).  Every term stays below 6.75 M^2 < 2^31 for M <= 3072,
// the largest lcm of the supported lengths.
struct Grid {
  int nx, ny, nz;
  int wx, wy, wz, lim;
  // (kx, ky) pencil inside the disk the z passes keep
  __host__ __device__ bool disk(int kx, int ky) const { return 9 * (kx * kx * wx + ky * ky * wy) < lim; }
  // weighted |k_perp|^2 of a pencil, and the full test from it
  __host__ __device__ int perp(int kx, int ky) const { return kx * kx * wx + ky * ky * wy; }
  __host__ __device__ bool keep_p(int perp2, int kz) const { return 9 * (perp2 + kz * kz * wz) < lim; }
  __host__ __device__ bool keep(int kx, int ky, int kz) const { return keep_p(perp(kx, ky), kz); }
};

inline Grid make_grid(int nx, int ny, int nz) {
  auto gcd = [](int a, int b) {
    while (b) {
      const int t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  int M = nx / gcd(nx, ny) * ny;
  M = M / gcd(M, nz) * nz;
  Grid g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.wx = (M / nx) * (M / nx);
  g.wy = (M / ny) * (M / ny);
  g.wz = (M / nz) * (M / nz);
  g.lim = M * M;
  return g;
}

}  // namespace ps
