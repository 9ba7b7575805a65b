// ps_kernels.hpp -- gfx950 kernels of the pseudospectral step.
//
// The step evaluates the nonlinear term of the incompressible Navier-Stokes
// (Eq. 1-2 of the paper) or MHD equations by the Fourier-Galerkin
// pseudospectral method of Sec. 2: the spectral state is transformed to
// physical space, products are formed there and transformed back, then
// projected onto divergence-free fields and dealiased (the 2/3 rule).  The
// 3D real transforms are done one axis per kernel ("pass"), as the paper's
// slab algorithm does per axis (Fig. 1), but on one GPU the whole box is
// local, so no transpose ever leaves the device:
//
//   z pass  strided complex FFT along kz (columns: (ky, kx), stride N*pitch)
//   y pass  strided complex FFT along ky (columns: (z, kx),  stride pitch)
//   x pass  contiguous real<->half-complex FFT along x (rows of N reals)
//
// A strided pass reads a tile of TX adjacent kx columns per workgroup, so
// every global access is a TX-element contiguous segment; the column FFTs
// run through the Stockham engine with LDS exchanges (the in-LDS transpose
// replaces the paper's cache-blocked local transpose of Sec. 3).
//
// Fusion (each is one kernel, data touch HBM once per pass):
//   inverse z pass + spectral curl prologue       (state -> u, w [, b, j]);
//                  MHD in the Elsasser form: z+- transformed as they are
//   x pass: inverse real FFTs + products (u x w [+ j x b, u x b], or the
//                  eight z+_i z-_j less the isotropic part) + forward real FFTs
//   forward z pass + 1/(nx ny nz) + dealias + projection (+ induction curl, or the
//                  divergence of the Elsasser products) + Coriolis term
//                  + explicit midpoint RK2 stage update
// Pruned launches skip every pencil and mode the 2/3 rule makes zero; box
// lengths enter through the per-axis factors 2 pi / L of the wavenumbers.
#pragma once
#include <type_traits>

#include "ps_device.hpp"

namespace ps {

// Workgroups are handed to the 8 XCDs round robin; remap so that each XCD
// receives a contiguous range of logical tiles (neighbouring tiles share
// cache lines at misaligned row starts, and each XCD has its own L2).
__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = bid & 7, i = bid >> 3;
  return x * q + (x < r ? x : r) + i;
}

// LDS tile of TX columns of length L, padded (LayColPad8) when the padded
// tile plus EXTRA further values fits in 64 KB.
template <typename T, int L, int TX, int EXTRA>
struct ColTile {
  static constexpr int ROWS_PAD = pad8(L - 1) + 1;
  static constexpr bool PAD = (ROWS_PAD * TX + EXTRA) * (int)sizeof(C2<T>) <= 65536;
  static constexpr int ROWS = PAD ? ROWS_PAD : L;
  using Lay = std::conditional_t<PAD, LayColPad8, LayStride>;
  // a table of L twiddles fits beside the tile without lowering the number
  // of workgroups that fit in a CU's 160 KB of LDS (a workgroup may hold up
  // to 80 KB of it here, two per CU)
  static constexpr int BYTES = ROWS * TX * (int)sizeof(C2<T>);
  static constexpr bool TW_FITS =
      BYTES + L * (int)sizeof(C2<T>) <= 81920 &&
      163840 / (BYTES + L * (int)sizeof(C2<T>)) == 163840 / BYTES;
};

// ---------------------------------------------------------------------------
// Strided complex pass (plain), used for y and z.
// Box b, field f, line l, column c (0 <= c < ncols), element idx:
//   in[b * in_bs + f * in_fs + l * in_ls + c + idx * in_es]
// ---------------------------------------------------------------------------
template <typename T>
struct StridedArgs {
  const C2<T>* in;
  C2<T>* out;
  const C2<T>* tw;  // exp(-2 pi i e / L), e < L
  long in_fs, in_ls, in_es;
  long out_fs, out_ls, out_es;
  long in_bs, out_bs;  // box strides (ensembles of equal-size boxes)
  int ncols, ntile, nlines, nf, nb;
  // dealias pruning of a y pass (columns kx, elements ky): 0 none; 1 input
  // zero outside the disk g.disk(kx, ky) (inverse pass); 2 only outputs
  // inside the disk are needed (forward pass).  Tiles whose every kx lies
  // beyond the 2/3 rule are skipped.
  int prune;
  Grid g;
  int nt;  // inverse passes: streaming stores (set when the output far exceeds the caches)
};

// TWS: the transform's twiddles staged in LDS beside the tile (TwStaged)
// instead of read from the table in global memory at every stage.
template <typename T, int L, int TQ, int TX, int DIR, class RL, int MINW = 1, bool TWS = false>
__global__ __launch_bounds__(TX* TQ, MINW) void k_strided(StridedArgs<T> a) {
  using E = Stockham<T, L, TQ, DIR, RL>;
  using CT = ColTile<T, L, TX, 0>;
  __shared__ C2<T> smem[CT::ROWS * TX + (TWS ? L : 0)];
  const int tid = threadIdx.x, c = tid % TX, q = tid / TX;
  int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = blk % a.ntile;
  blk /= a.ntile;
  const int line = blk % a.nlines;
  blk /= a.nlines;
  const int f = blk % a.nf, box = blk / a.nf;
  const int col = tile * TX + c;
  if (a.prune && !a.g.disk(tile * TX, 0)) return;  // whole tile outside
  const bool ok = col < a.ncols && (!a.prune || a.g.disk(col, 0));
  auto in_disk = [&](int idx) { return a.g.disk(col, wav(idx, L)); };
  const C2<T>* in = a.in + box * a.in_bs + f * a.in_fs + line * a.in_ls + col;
  C2<T>* out = a.out + box * a.out_bs + f * a.out_fs + line * a.out_ls + col;
  C2<T> v[E::SLOTS];
  auto ld = [&](int, int idx) { return ok && (a.prune != 1 || in_disk(idx)) ? in[idx * a.in_es] : zero2<T>(); };
  if constexpr (TWS) {
    // read only from the second stage on: the first stage's barrier before
    // its LDS writes orders the fill before every read
    static_assert(E::NSTAGE > 1, "a single-stage transform has no twiddles to stage");
    fill_staged<T, L>(smem + CT::ROWS * TX, a.tw, 1, tid, TX * TQ, RL{});
    E::template run_tw<typename CT::Lay>(v, smem + c, TX, q, TwStaged<T>{smem + CT::ROWS * TX}, ld);
  } else {
    E::template run<typename CT::Lay>(v, smem + c, TX, q, a.tw, 1, ld);
  }
  if constexpr (E::NSTAGE == 1) __syncthreads();  // in place: all reads before any write
#pragma unroll
  for (int s = 0; s < E::LAST_NB * E::RL_; ++s) {
    const int idx = E::last_index(q, s);
    if (ok && E::last_valid(q, s) && (a.prune != 2 || in_disk(idx))) {
      // inverse passes write whole columns that only the next pass reads:
      // streaming stores when they far exceed the caches (measured faster
      // there; slower for the forward pass's scattered disk outputs and for
      // outputs the last-level cache can hold)
      if (DIR == INV && a.nt)
        store_nt(out + idx * a.out_es, v[s]);
      else
        out[idx * a.out_es] = v[s];
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse z pass with the spectral curl prologue.
// NS : in = u^ (3 fields)  -> out = [u, w]            (6 fields)
// MHD: in = z+^, z-^ (6)   -> out = [u, w, b, j]      (12 fields)
// with u = (z+ + z-)/2, b = (z+ - z-)/2, w = i k_d x u, j = i k_d x b.
// Column (kx, ky) is fixed per thread; idx is kz.
// ---------------------------------------------------------------------------
template <typename T>
struct ZCurlArgs {
  const C2<T>* in;
  C2<T>* out;
  const C2<T>* tw;
  long in_fs, in_pitch;   // field stride, kx pitch of the input (line = ky)
  long out_fs, out_pitch;
  long in_bs, out_bs;     // box strides
  Grid g;                 // the box's grid (the transform runs along z, length nz)
  int ntile, nb;
  int prune;  // 1: state zero outside the 2/3 sphere; only disk columns are produced
  // pruned launches: the ntl tiles (tile | ky << 16) that meet the disk, so
  // that no workgroup is spent on, and no XCD is left idle by, empty tiles
  const int* tiles;
  int ntl;
  T sx, sy, sz;  // box factors 2 pi / L: physical wavenumber = s * index
  int nt;        // streaming stores of the output (set when it far exceeds the caches)
};

// tile, ky and box of a z-pass workgroup
struct ZTile {
  int tile, ky, box;
};
__device__ __forceinline__ ZTile z_tile(int blk, int ntile, int ny, const int* tiles, int ntl) {
  if (tiles) {
    const int e = tiles[blk % ntl];
    return {e & 0xffff, e >> 16, blk / ntl};
  }
  return {blk % ntile, (blk / ntile) % ny, blk / (ntile * ny)};
}

// Output groups: 0 u, 1 w = curl u (NS and MHD), 2 b, 3 j = curl b (MHD).
// SPLIT > 1 hands the groups of a tile to SPLIT workgroups (adjacent block
// ids, so they share the tile's input lines in L2).  Without DIRECT the
// workgroup first loads the base fields (u, and b for MHD) its groups derive
// from into registers; with DIRECT every output field gathers what it needs
// straight from memory in the first FFT stage (re-reads hit the cache), which
// keeps register use, and so occupancy, near that of a plain FFT.  The
// transforms' twiddles are staged in LDS (TwStaged) when that costs no occupancy.
//
// ELS (divergence form): no curl is needed; the state's fields (MHD: z+, z-;
// NS: u) are transformed as they are, SPLIT workgroups sharing them (MHD:
// SPLIT 1 or 2; NS: 1).
template <typename T, int L, int TQ, int TX, class RL, bool MHD, int SPLIT, bool DIRECT, int MINW = 1,
          bool ELS = false>
__global__ __launch_bounds__(TX* TQ, MINW) void k_z_curl(ZCurlArgs<T> a) {
  using E = Stockham<T, L, TQ, INV, RL>;
  using CT = ColTile<T, L, TX, 0>;
  using Lay = typename CT::Lay;
  constexpr int NS_ = E::FIRST_SLOTS;
  constexpr int NG = MHD ? 4 : 2;
  static_assert(NG % SPLIT == 0 && (!ELS || (MHD ? SPLIT <= 2 : SPLIT == 1)), "split must divide the output groups");
  constexpr int GPP = NG / SPLIT;
  constexpr bool TWL = CT::TW_FITS;
  __shared__ C2<T> smem[CT::ROWS * TX + (TWL ? L : 0)];
  const int tid = threadIdx.x, c = tid % TX, q = tid / TX;
  const int blk0 = xcd_remap(blockIdx.x, gridDim.x);
  const int part = blk0 % SPLIT, blk = blk0 / SPLIT;
  const Grid& g = a.g;
  const ZTile zt = z_tile(blk, a.ntile, g.ny, a.prune ? a.tiles : nullptr, a.ntl);
  const int tile = zt.tile, ky = zt.ky, box = zt.box;
  const int col = tile * TX + c;
  const int kyw = wav(ky, g.ny);
  if (a.prune && !g.disk(tile * TX, kyw)) return;  // tile outside the disk
  const bool ok = col < g.nx / 2 + 1 && (!a.prune || g.disk(col, kyw));
  const long in_es = (long)g.ny * a.in_pitch, out_es = (long)g.ny * a.out_pitch;
  const C2<T>* in = a.in + box * a.in_bs + ky * a.in_pitch + col;
  C2<T>* out = a.out + box * a.out_bs + ky * a.out_pitch + col;
  const T kx = a.sx * (T)dwavx(col, g.nx), kyd = a.sy * (T)dwav(ky, g.ny);
  const int kperp2 = g.perp(col, kyw);
  if constexpr (TWL) {
    fill_staged<T, L>(smem + CT::ROWS * TX, a.tw, 1, tid, TX * TQ, RL{});
    __syncthreads();
  }
  const auto tw = [&] {
    if constexpr (TWL)
      return TwStaged<T>{smem + CT::ROWS * TX};
    else
      return TwTable<T>{a.tw, 1};
  }();
  // element kz of the column is stored (nonzero) input
  auto live = [&](int kzi) { return ok && (!a.prune || g.keep_p(kperp2, wav(kzi, L))); };
  // component f of u (sign +1) or b (sign -1) at kz row offset off
  auto base_at = [&](int f, long off, T sign) -> C2<T> {
    if constexpr (MHD)
      return T(0.5) * (in[f * a.in_fs + off] + sign * in[(3 + f) * a.in_fs + off]);
    else
      return in[f * a.in_fs + off];
  };
  // component comp of group grp (even: the base itself, odd: its curl) from
  // a getter g(f) of the base's components at wavenumber index kzi
  auto field_of = [&](int grp, int comp, int kzi, auto g) -> C2<T> {
    if ((grp & 1) == 0) return g(comp);
    const T kz = a.sz * (T)dwav(kzi, L);
    C2<T> r;
    if (comp == 0)
      r = kyd * g(2) - kz * g(1);
    else if (comp == 1)
      r = kz * g(0) - kx * g(2);
    else
      r = kx * g(1) - kyd * g(0);
    return mul_i(r);
  };
  auto store = [&](C2<T> (&v)[E::SLOTS], int fout) {
    if constexpr (E::NSTAGE == 1) __syncthreads();
#pragma unroll
    for (int s = 0; s < E::LAST_NB * E::RL_; ++s)
      if (ok && E::last_valid(q, s)) {
        C2<T>* o = out + fout * a.out_fs + E::last_index(q, s) * out_es;
        if (a.nt)
          store_nt(o, v[s]);
        else
          *o = v[s];
      }
  };

  if constexpr (ELS) {
    constexpr int PER = (MHD ? 6 : 3) / SPLIT;
#pragma unroll 1
    for (int fo = part * PER; fo < (part + 1) * PER; ++fo) {
      C2<T> v[E::SLOTS];
      E::template run_tw<Lay>(v, smem + c, TX, q, tw, [&](int, int kzi) -> C2<T> {
        return live(kzi) ? in[fo * a.in_fs + (long)kzi * in_es] : zero2<T>();
      });
      store(v, fo);
    }
  } else if constexpr (DIRECT) {
    // one output field per iteration, kept rolled so that no load address
    // or coefficient of another field stays live across the FFT
#pragma unroll 1
    for (int fo = part * 3 * GPP; fo < (part + 1) * 3 * GPP; ++fo) {
      const int grp = fo / 3, comp = fo % 3;
      const T sign = (MHD && grp >= 2) ? T(-1) : T(1);
      const bool curl = grp & 1;
      // curl component comp = ka g(ca) - kb g(cb), with kz in one of ka, kb
      const int ca = comp == 0 ? 2 : comp == 1 ? 0 : 1;
      const int cb = comp == 0 ? 1 : comp == 1 ? 2 : 0;
      const T kA = comp == 0 ? kyd : kx, kB = comp == 1 ? kx : kyd;
      C2<T> v[E::SLOTS];
      E::template run_tw<Lay>(v, smem + c, TX, q, tw, [&](int, int kzi) -> C2<T> {
        if (!live(kzi)) return zero2<T>();
        const long off = (long)kzi * in_es;
        if (!curl) return base_at(comp, off, sign);
        const T kz = a.sz * (T)dwav(kzi, L);
        const T ka = comp == 1 ? kz : kA, kb = comp == 0 ? kz : kB;
        return mul_i(ka * base_at(ca, off, sign) - kb * base_at(cb, off, sign));
      });
      store(v, fo);
    }
  } else {
    // hold the base fields in registers, indexed by first-stage slot
    auto load = [&](C2<T> (&dst)[3][NS_], T sign) {
#pragma unroll
      for (int s = 0; s < NS_; ++s) {
        const int kzi = E::first_index(q, s);
        const bool v = E::first_valid(q, s) && live(kzi);
        const long off = (long)kzi * in_es;
#pragma unroll
        for (int f = 0; f < 3; ++f) dst[f][s] = v ? base_at(f, off, sign) : zero2<T>();
      }
    };
    auto emit = [&](C2<T> (&src)[3][NS_], int grp, int comp) {
      C2<T> v[E::SLOTS];
      E::template run_tw<Lay>(v, smem + c, TX, q, tw, [&](int s, int kzi) -> C2<T> {
        return field_of(grp, comp, kzi, [&](int f) { return src[f][s]; });
      });
      store(v, 3 * grp + comp);
    };
    if constexpr (MHD && SPLIT == 1) {
      C2<T> u[3][NS_], b[3][NS_];
      load(u, T(1));
      load(b, T(-1));
#pragma unroll
      for (int f = 0; f < 12; ++f) {
        if (f < 6)
          emit(u, f / 3, f % 3);
        else
          emit(b, f / 3, f % 3);
      }
    } else {
      // groups [g0, g0 + GPP) all derive from one base field
      const int g0 = part * GPP;
      C2<T> w[3][NS_];
      load(w, (MHD && g0 >= 2) ? T(-1) : T(1));
#pragma unroll
      for (int gi = 0; gi < GPP; ++gi)
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) emit(w, g0 + gi, comp);
    }
  }
}

// ---------------------------------------------------------------------------
// Forward z pass with the nonlinear-term epilogue.
// in: products transformed along x and y (NS: u x w; MHD: u x w + j x b, u x b)
// N^ = D(k) P(k) F[n] / n3;  MHD: N+- = D(k) [P(k) F[nL] +- i k_d x F[e]] / n3
// (n3 = nx ny nz, D the 2/3 rule of the grid)
// mode 0: out = N^
// mode 1: out (= z*) = z^n + h (N^ - V(z^n))          h = dt/2
// mode 2: st0 (= z^n, in place) = z^n + h (N^ - V(z*)), h = dt; z* = st1
// V(z) = nu |k|^2 z (NS);  V(z+-) = |k|^2 (nua z+- + nub z-+) (MHD)
// In a rotating frame V also holds the projected Coriolis term P(k)(2 Omega x u),
// u = z (NS) or (z+ + z-)/2 (MHD, added to both Elsasser equations).
// ---------------------------------------------------------------------------
template <typename T>
struct ZEpiArgs {
  const C2<T>* in;
  C2<T>* out;
  const C2<T>* st0;
  const C2<T>* st1;
  const C2<T>* tw;
  long in_fs, in_pitch;
  long out_fs, out_pitch;  // out, st0 and st1 share this layout
  long in_bs, out_bs;      // box strides
  T scale, h, nua, nub;
  Grid g;  // the box's grid (the transform runs along z, length nz)
  int ntile, mode, nb;
  int prune;  // 1: only modes inside the 2/3 sphere are read or updated (mode 0 still writes zeros)
  const int* tiles;  // as in ZCurlArgs; used by pruned launches with mode != 0
  int ntl;
  // rotating frame (modes 1, 2): w2 = 2 Omega; the RHS gains -P(k)(w2 x u)
  // at every k != 0, u the velocity of the state the viscous term acts on
  T w2x, w2y, w2z;
  int rot;
  T sx, sy, sz;  // box factors 2 pi / L: physical wavenumber = s * index (D stays on the index)
};

//
// ELS (MHD, Elsasser form): in = the products T_ij = z+_i z-_j less
// delta_ij z+_2 z-_2 (field 3 i + j for the eight pairs other than (2, 2),
// whose entry is zero) transformed along x and y; with a_i = sum_j k_j T^_ij
// and c_i = sum_j k_j T^_ji (derivative wavenumbers),
//   N+ = -i D(k) P(k) a / n3,  N- = -i D(k) P(k) c / n3,
// the divergence form of -(z-+ . grad) z+-, equal to the form above for
// solenoidal z+- (the isotropic part left out adds a gradient to a and c,
// which P(k) removes).  a and c are accumulated field by field.
template <typename T, int L, int TQ, int TX, class RL, bool MHD, int MINW = 1, bool ELS = false, int SPLIT = 1>
__global__ __launch_bounds__(TX* TQ, MINW) void k_z_epi(ZEpiArgs<T> a) {
  using E = Stockham<T, L, TQ, FWD, RL>;
  static_assert(SPLIT == 1 || (ELS && MHD && SPLIT == 2), "only the Elsasser form splits z+ from z-");
  constexpr int NF = MHD ? 6 : 3;       // state fields
  constexpr int NOUT = NF / SPLIT;      // state fields this workgroup updates
  constexpr int NO = E::LAST_NB * E::RL_;
  using CT = ColTile<T, L, TX, 0>;
  constexpr bool TWL = CT::TW_FITS;
  __shared__ C2<T> smem[CT::ROWS * TX + (TWL ? L : 0)];
  const int tid = threadIdx.x, c = tid % TX, q = tid / TX;
  const int blk0 = xcd_remap(blockIdx.x, gridDim.x);
  const int part = blk0 % SPLIT, blk = blk0 / SPLIT;  // part 0: z+ (a), part 1: z- (c)
  const Grid& g = a.g;
  const ZTile zt = z_tile(blk, a.ntile, g.ny, a.prune && a.mode != 0 ? a.tiles : nullptr, a.ntl);
  const int tile = zt.tile, ky = zt.ky, box = zt.box;
  const int col = tile * TX + c;
  const int kyw0 = wav(ky, g.ny);
  if (a.prune && a.mode != 0 && !g.disk(tile * TX, kyw0)) return;
  const bool ok = col < g.nx / 2 + 1;
  const bool disk = !a.prune || g.disk(col, kyw0);
  const long in_es = (long)g.ny * a.in_pitch, out_es = (long)g.ny * a.out_pitch;
  const C2<T>* in = a.in + box * a.in_bs + ky * a.in_pitch + col;
  if constexpr (TWL) {
    fill_staged<T, L>(smem + CT::ROWS * TX, a.tw, 1, tid, TX * TQ, RL{});
    __syncthreads();
  }
  const auto tw = [&] {
    if constexpr (TWL)
      return TwStaged<T>{smem + CT::ROWS * TX};
    else
      return TwTable<T>{a.tw, 1};
  }();
  // first-stage loader of input field f
  auto ld_of = [&](int f) {
    return [&, f](int, int idx) { return ok && disk ? in[f * a.in_fs + idx * in_es] : zero2<T>(); };
  };

  // NS / rotational MHD: r[f] = transformed input field f.
  // Elsasser: r[0..2] = a (unsplit or part 0), r[3..5] = c (unsplit); with
  // SPLIT = 2, part 1 keeps c in r[0..2].
  constexpr int NR = ELS ? (MHD ? 3 * (2 / SPLIT) : 3) : NF;
  C2<T> r[NR][NO];
  if constexpr (ELS && !MHD) {
    // NS divergence form: the five products S_00 - S_22, S_11 - S_22, S_01,
    // S_02, S_12 of S_ij = u_i u_j (symmetric, less its isotropic part);
    // r = a, a_i = sum_j k_j S_ij
    const T kxd0 = a.sx * (T)dwavx(col, g.nx), kyd0 = a.sy * (T)dwav(ky, g.ny);
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int s = 0; s < NO; ++s) r[f][s] = zero2<T>();
#pragma unroll 1
    for (int f = 0; f < 5; ++f) {
      // (i, j) of product f; the diagonal ones (f < 2) feed a_i only
      const int i3 = f < 2 ? f : f == 4 ? 1 : 0;
      const int j3 = f < 2 ? f : f == 2 ? 1 : 2;
      C2<T> v[E::SLOTS];
      E::template run_tw<typename CT::Lay>(v, smem + c, TX, q, tw, ld_of(f));
#pragma unroll
      for (int s = 0; s < NO; ++s) {
        const T kzd0 = a.sz * (T)dwav(E::last_index(q, s), L);
        const T kj = j3 == 0 ? kxd0 : j3 == 1 ? kyd0 : kzd0;
        const T ki = i3 == 0 ? kxd0 : i3 == 1 ? kyd0 : kzd0;
        const bool off = f >= 2;
        r[0][s] = r[0][s] + ((i3 == 0 ? kj : T(0)) + (off && j3 == 0 ? ki : T(0))) * v[s];
        r[1][s] = r[1][s] + ((i3 == 1 ? kj : T(0)) + (off && j3 == 1 ? ki : T(0))) * v[s];
        r[2][s] = r[2][s] + ((i3 == 2 ? kj : T(0)) + (off && j3 == 2 ? ki : T(0))) * v[s];
      }
    }
  } else if constexpr (ELS) {
    const T kxd0 = a.sx * (T)dwavx(col, g.nx), kyd0 = a.sy * (T)dwav(ky, g.ny);
#pragma unroll
    for (int f = 0; f < NR; ++f)
#pragma unroll
      for (int s = 0; s < NO; ++s) r[f][s] = zero2<T>();
    if constexpr (SPLIT == 1) {
      // one rolled loop over the eight products, so that a single transform's
      // loads and temporaries are live at a time: a_i += k_j T_ij and
      // c_j += k_i T_ij through selects on the loop's (i, j)
#pragma unroll 1
      for (int f = 0; f < 8; ++f) {  // (2, 2) is zero
        const int i3 = f / 3, j3 = f % 3;
        C2<T> v[E::SLOTS];
        E::template run_tw<typename CT::Lay>(v, smem + c, TX, q, tw, ld_of(f));
#pragma unroll
        for (int s = 0; s < NO; ++s) {
          const T kzd0 = a.sz * (T)dwav(E::last_index(q, s), L);
          const T kj = j3 == 0 ? kxd0 : j3 == 1 ? kyd0 : kzd0;
          const T ki = i3 == 0 ? kxd0 : i3 == 1 ? kyd0 : kzd0;
          r[0][s] = r[0][s] + (i3 == 0 ? kj : T(0)) * v[s];
          r[1][s] = r[1][s] + (i3 == 1 ? kj : T(0)) * v[s];
          r[2][s] = r[2][s] + (i3 == 2 ? kj : T(0)) * v[s];
          r[3][s] = r[3][s] + (j3 == 0 ? ki : T(0)) * v[s];
          r[4][s] = r[4][s] + (j3 == 1 ? ki : T(0)) * v[s];
          r[5][s] = r[5][s] + (j3 == 2 ? ki : T(0)) * v[s];
        }
      }
    } else {
      // part 0: a_i = sum_j k_j T_ij;  part 1: c_j = sum_i k_i T_ij
#pragma unroll 1
      for (int f = 0; f < 8; ++f) {  // (2, 2) is zero
        const int i3 = f / 3, j3 = f % 3;
        const int t = part == 0 ? i3 : j3, m = part == 0 ? j3 : i3;
        C2<T> v[E::SLOTS];
        E::template run_tw<typename CT::Lay>(v, smem + c, TX, q, tw, ld_of(f));
#pragma unroll
        for (int s = 0; s < NO; ++s) {
          const T kzd0 = a.sz * (T)dwav(E::last_index(q, s), L);
          const T km = m == 0 ? kxd0 : m == 1 ? kyd0 : kzd0;
          r[0][s] = r[0][s] + (t == 0 ? km : T(0)) * v[s];
          r[1][s] = r[1][s] + (t == 1 ? km : T(0)) * v[s];
          r[2][s] = r[2][s] + (t == 2 ? km : T(0)) * v[s];
        }
      }
    }
  } else {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      C2<T> v[E::SLOTS];
      E::template run_tw<typename CT::Lay>(v, smem + c, TX, q, tw, ld_of(f));
#pragma unroll
      for (int s = 0; s < NO; ++s) r[f][s] = v[s];
    }
  }
  if (!ok) return;  // no barrier follows

  const long base = box * a.out_bs + ky * a.out_pitch + col;
  const int ikx = col, iky = wav(ky, g.ny);
  const int kperp2 = g.perp(ikx, iky);
  const T kxd = a.sx * (T)dwavx(col, g.nx), kyd = a.sy * (T)dwav(ky, g.ny);
#pragma unroll
  for (int s = 0; s < NO; ++s) {
    if (!E::last_valid(q, s)) continue;
    const int kzi = E::last_index(q, s);
    const int ikz = wav(kzi, L);
    const long k2i = (long)ikx * ikx + (long)iky * iky + (long)ikz * ikz;
    const bool sphere = g.keep_p(kperp2, ikz);
    if (a.prune && !sphere && a.mode != 0) continue;  // stays zero
    const bool keep = k2i > 0 && sphere;
    // physical wavenumber (projector, |k|^2); keep / sphere use the index
    const T kx = a.sx * (T)ikx, ky_ = a.sy * (T)iky, kz = a.sz * (T)ikz;
    const T k2 = kx * kx + ky_ * ky_ + kz * kz;
    C2<T> nh[NOUT];
    if constexpr (ELS) {
      const T ik2 = keep ? T(1) / k2 : T(0);
#pragma unroll
      for (int h = 0; h < NOUT / 3; ++h) {
        // -i P(k) applied to the accumulated divergence, scaled
        C2<T> n0 = a.scale * r[3 * h][s], n1 = a.scale * r[3 * h + 1][s], n2 = a.scale * r[3 * h + 2][s];
        const C2<T> kn = kx * n0 + ky_ * n1 + kz * n2;
        nh[3 * h] = keep ? mul_i((kx * ik2) * kn - n0) : zero2<T>();
        nh[3 * h + 1] = keep ? mul_i((ky_ * ik2) * kn - n1) : zero2<T>();
        nh[3 * h + 2] = keep ? mul_i((kz * ik2) * kn - n2) : zero2<T>();
      }
    } else if (keep) {
      const T ik2 = T(1) / k2;
      C2<T> n0 = a.scale * r[0][s], n1 = a.scale * r[1][s], n2 = a.scale * r[2][s];
      const C2<T> kn = kx * n0 + ky_ * n1 + kz * n2;
      n0 = n0 - (kx * ik2) * kn;
      n1 = n1 - (ky_ * ik2) * kn;
      n2 = n2 - (kz * ik2) * kn;
      if constexpr (MHD) {
        const C2<T> e0 = a.scale * r[3][s], e1 = a.scale * r[4][s], e2 = a.scale * r[5][s];
        const T kzd = a.sz * (T)dwav(kzi, L);
        const C2<T> c0 = mul_i(kyd * e2 - kzd * e1);
        const C2<T> c1 = mul_i(kzd * e0 - kxd * e2);
        const C2<T> c2 = mul_i(kxd * e1 - kyd * e0);
        nh[0] = n0 + c0; nh[1] = n1 + c1; nh[2] = n2 + c2;
        nh[3] = n0 - c0; nh[4] = n1 - c1; nh[5] = n2 - c2;
      } else {
        nh[0] = n0; nh[1] = n1; nh[2] = n2;
      }
    } else {
#pragma unroll
      for (int f = 0; f < NOUT; ++f) nh[f] = zero2<T>();
    }
    const long pos = base + kzi * out_es;
    const int fo0 = part * NOUT;  // first state field written here
    if (a.mode == 0) {
#pragma unroll
      for (int f = 0; f < NOUT; ++f) a.out[(fo0 + f) * a.out_fs + pos] = nh[f];
    } else {
      const C2<T>* zv = a.mode == 1 ? a.st0 : a.st1;  // field the viscous term acts on
      C2<T> zz[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) zz[f] = zv[f * a.out_fs + pos];
      C2<T>* dst = a.mode == 1 ? a.out : const_cast<C2<T>*>(a.st0);
      C2<T> cor[3] = {zero2<T>(), zero2<T>(), zero2<T>()};
      if (a.rot && k2i > 0) {
        C2<T> u[3];
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) u[c3] = MHD ? T(0.5) * (zz[c3] + zz[(c3 + 3) % NF]) : zz[c3];
        const C2<T> w0 = a.w2y * u[2] - a.w2z * u[1];
        const C2<T> w1 = a.w2z * u[0] - a.w2x * u[2];
        const C2<T> w2 = a.w2x * u[1] - a.w2y * u[0];
        const C2<T> kw = (T(1) / k2) * (kx * w0 + ky_ * w1 + kz * w2);
        cor[0] = w0 - kx * kw;
        cor[1] = w1 - ky_ * kw;
        cor[2] = w2 - kz * kw;
      }
#pragma unroll
      for (int f = 0; f < NOUT; ++f) {
        // this field and (MHD) its Elsasser partner, with static indices
        // (choices by value: a conditional between lvalues makes the compiler
        // select an address, which puts zz in scratch memory)
        const C2<T> self = sel(SPLIT == 2 && part == 1, zz[(f + 3) % NF], zz[f]);
        const C2<T> z0 = a.mode == 1 ? self : C2<T>(a.st0[(fo0 + f) * a.out_fs + pos]);
        C2<T> vis = (a.nua * k2) * self;
        if constexpr (MHD) {
          const C2<T> other = SPLIT == 2 ? sel(part == 1, zz[f], zz[(f + 3) % NF]) : zz[f < 3 ? f + 3 : f - 3];
          vis = vis + (a.nub * k2) * other;
        }
        vis = vis + cor[f % 3];
        dst[(fo0 + f) * a.out_fs + pos] = z0 + a.h * (nh[f] - vis);
      }
    }
    // one mode at a time, so the scheduler does not hold every mode's
    // results in registers before the first store
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ---------------------------------------------------------------------------
// Contiguous x pass.  A row holds N reals or N/2+1 complex coefficients.
// Half-length method: with M = N/2, z[n] = x[2n] + i x[2n+1],
//   inverse: Z[k] = (X[k] + X[k+M]) + i e^{+2 pi i k/N} (X[k] - X[k+M]),
//            X[k+M] = conj X[M-k], and Re X[0], Re X[M] at k = 0;
//            z = unnormalised inverse M-point DFT of Z.
//   forward: Z = M-point DFT of z;
//            X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) e^{-2 pi i k/N} (Z[k] - conj Z[M-k]),
//            Z[M] := Z[0].
// The table tw has length N (the M-point transform reads every other entry).
// ---------------------------------------------------------------------------
// Rows in LDS use the padded layout (element i at pad8(i)); RowLen(M) slots
// hold M+1 values.
__host__ __device__ constexpr int row_slots(int M) { return pad8(M) + 1; }
// rows of LDS (and thread groups) per grid row of the fused product pass
__host__ __device__ constexpr int xprod_slots(bool mhd, bool els) { return els ? (mhd ? 8 : 5) : mhd ? 12 : 6; }

template <typename T, class Lay = LayPad8>
__device__ __forceinline__ C2<T> c2r_pre(const C2<T>* buf, int k, int M, const C2<T>* __restrict__ tw) {
  // branch-free: at k = 0 the pair is (Re X[0], Re X[M]) (M - k = M there)
  C2<T> xk = buf[Lay::off(k, 1)], xm = conj(buf[Lay::off(M - k, 1)]);
  xk.y = k == 0 ? T(0) : xk.y;
  xm.y = k == 0 ? T(0) : xm.y;
  return (xk + xm) + mul_i(cmulc(xk - xm, tw[k]));  // conj(tw[k]) = e^{+2 pi i k/N}
}

// the same straight from a row in global memory whose coefficients above kmax are zero
template <typename T>
__device__ __forceinline__ C2<T> c2r_pre_g(const C2<T>* src, int k, int M, int kmax, const C2<T>* tw) {
  // branch-free: every load stays inside the row, zeros come from selects
  const int km = M - k;
  C2<T> xk = src[k < kmax ? k : kmax], xm = conj(src[km < kmax ? km : kmax]);
  xk = sel(k <= kmax, xk, zero2<T>());
  xm = sel(km <= kmax, xm, zero2<T>());
  xk.y = k == 0 ? T(0) : xk.y;
  xm.y = k == 0 ? T(0) : xm.y;
  return (xk + xm) + mul_i(cmulc(xk - xm, tw[k]));
}

template <typename T, class Lay = LayPad8>
__device__ __forceinline__ C2<T> r2c_post(const C2<T>* buf, int k, int M, const C2<T>* __restrict__ tw) {
  const C2<T> zk = buf[Lay::off(k == M ? 0 : k, 1)];
  const C2<T> zm = conj(buf[Lay::off(k == 0 ? 0 : M - k, 1)]);
  const C2<T> e = T(0.5) * (zk + zm);
  const C2<T> o = T(0.5) * mul_mi(zk - zm);
  return e + cmul(o, tw[k]);
}

template <typename T>
struct XArgs {
  const C2<T>* in;   // complex rows (pitch in_pitch) or real rows viewed as M complex
  C2<T>* out;
  const C2<T>* tw;   // length N
  long in_fs, in_pitch, out_fs, out_pitch;  // per-row pitch in complex elements
  long in_bs, out_bs;  // box strides
  long rows;         // rows per field (ny nz)
  int nf, nb;
  int kmax;  // fused passes: coefficients kx > kmax are zero on input and not needed on output
  int nt;    // fused pass: streaming stores for the output (set when it far exceeds the caches)
};

// plain inverse: complex rows (pitch in_pitch) -> real rows (N reals, pitch out_pitch complex = M)
template <typename T, int M, int TQ, int G, class RL>
__global__ __launch_bounds__(G* TQ) void k_x_c2r(XArgs<T> a) {
  using E = Stockham<T, M, TQ, INV, RL>;
  constexpr int LP = row_slots(M);
  __shared__ C2<T> smem[G * LP];
  const int tid = threadIdx.x, g = tid / TQ, q = tid % TQ;
  const long row0 = (long)xcd_remap(blockIdx.x, gridDim.x) * G;
  const long total = a.rows * a.nf * a.nb;
  for (int i = tid; i < G * (M + 1); i += G * TQ) {
    const int gg = i / (M + 1), k = i % (M + 1);
    const long row = row0 + gg;
    C2<T> val = zero2<T>();
    if (row < total) {
      const long fb = row / a.rows, r = row % a.rows;
      const long f = fb % a.nf, b = fb / a.nf;
      val = a.in[b * a.in_bs + f * a.in_fs + r * a.in_pitch + k];
    }
    smem[gg * LP + pad8(k)] = val;
  }
  __syncthreads();
  C2<T>* buf = smem + g * LP;
  C2<T> v[E::SLOTS];
  E::template run<LayPad8>(v, buf, 1, q, a.tw, 2, [&](int, int k) { return c2r_pre(buf, k, M, a.tw); });
  const long row = row0 + g;
  if (row >= total) return;
  const long fb = row / a.rows, r = row % a.rows;
  const long f = fb % a.nf, b = fb / a.nf;
  C2<T>* out = a.out + b * a.out_bs + f * a.out_fs + r * a.out_pitch;
#pragma unroll
  for (int s = 0; s < E::LAST_NB * E::RL_; ++s)
    if (E::last_valid(q, s)) out[E::last_index(q, s)] = v[s];
}

// plain forward: real rows (as M complex, pitch in_pitch) -> complex rows (M+1, pitch out_pitch)
template <typename T, int M, int TQ, int G, class RL>
__global__ __launch_bounds__(G* TQ) void k_x_r2c(XArgs<T> a) {
  using E = Stockham<T, M, TQ, FWD, RL>;
  constexpr int LP = row_slots(M);
  __shared__ C2<T> smem[G * LP];
  const int tid = threadIdx.x, g = tid / TQ, q = tid % TQ;
  const long row0 = (long)xcd_remap(blockIdx.x, gridDim.x) * G;
  const long total = a.rows * a.nf * a.nb;
  const long row = row0 + g;
  const bool ok = row < total;
  const long fb = ok ? row / a.rows : 0, r = ok ? row % a.rows : 0;
  const C2<T>* in = a.in + (fb / a.nf) * a.in_bs + (fb % a.nf) * a.in_fs + r * a.in_pitch;
  C2<T>* buf = smem + g * LP;
  C2<T> v[E::SLOTS];
  E::template run<LayPad8>(v, buf, 1, q, a.tw, 2, [&](int, int n) { return ok ? in[n] : zero2<T>(); });
  __syncthreads();
#pragma unroll
  for (int s = 0; s < E::LAST_NB * E::RL_; ++s)
    if (E::last_valid(q, s)) buf[pad8(E::last_index(q, s))] = v[s];
  __syncthreads();
  for (int i = tid; i < G * (M + 1); i += G * TQ) {
    const int gg = i / (M + 1), k = i % (M + 1);
    const long rw = row0 + gg;
    if (rw < total) {
      const long fb = rw / a.rows, rr = rw % a.rows;
      a.out[(fb / a.nf) * a.out_bs + (fb % a.nf) * a.out_fs + rr * a.out_pitch + k] =
          r2c_post(smem + gg * LP, k, M, a.tw);
    }
  }
}

// fused: FIN complex input fields -> inverse real FFTs -> cross products ->
// forward real FFTs -> FOUT complex output fields.  RB rows per workgroup.
// NS : in [u0 u1 u2 w0 w1 w2]             out [u x w]
// MHD: in [u0..2 w0..2 b0..2 j0..2]       out [u x w + j x b, u x b]
//
// ELS, NS (divergence form): input u (fields 0-2); outputs the five fields of
// S_ij = u_i u_j less its isotropic part delta_ij S_22: S_00 - S_22,
// S_11 - S_22, S_01, S_02, S_12 (symmetric; the gradient removed is again
// annihilated by P(k)).
// ELS, MHD (Elsasser form): inputs z+ (fields 0-2) and z- (3-5); outputs the
// eight fields of the stress T_ij = z+_i z-_j less its isotropic part
// delta_ij T_22, as field 3 i + j: T_00 - T_22, T_01, T_02, T_10,
// T_11 - T_22, T_12, T_20, T_21 (T_22 - T_22 = 0 is not stored).  The part
// removed contributes the gradient -i k T^_22 to both N+ and N-, which the
// projection P(k) annihilates.
template <typename T, int M, int TQ, int RB, class RL, bool MHD, bool ELS = false, class RLay = LayPad8,
          int LDSLIM = 65536>
__global__ __launch_bounds__(xprod_slots(MHD, ELS) * RB * TQ) void k_x_prod(XArgs<T> a) {
  constexpr int FIN = ELS ? (MHD ? 6 : 3) : MHD ? 12 : 6, FOUT = ELS ? (MHD ? 8 : 5) : MHD ? 6 : 3;
  constexpr int G = xprod_slots(MHD, ELS) * RB, NT = G * TQ;
  using EI = Stockham<T, M, TQ, INV, RL>;
  using EF = Stockham<T, M, TQ, FWD, RL>;
  constexpr int LP = RLay::slots(M);
  // rows of every field, then twiddles: the M + 1 factors e^{-2 pi i k/N} of
  // the half-length pre- and post-processing followed by the transforms' M - 1
  // factors in the bank-friendly staged order, or (when that would not fit in
  // LDSLIM bytes) the plain table of length N = 2M, which serves both
  constexpr bool STAGED = (G * LP + 2 * M) * (int)sizeof(C2<T>) <= LDSLIM;
  // a group of TQ <= 64 threads lies in one wave: wave-level exchanges
  constexpr bool XW = TQ <= 64 && 64 % TQ == 0;
  __shared__ C2<T> smem[G * LP + 2 * M];
  C2<T>* twl = smem + G * LP;
  const int tid = threadIdx.x, g = tid / TQ, q = tid % TQ;
  const int f = g / RB, rb = g % RB;  // group g owns field f of row rb (slot g)
  const long row = (long)xcd_remap(blockIdx.x, gridDim.x) * RB + rb;
  const bool rok = row < a.rows * a.nb;
  const long rr = rok ? row : 0;
  const long boxi = rr / a.rows, rloc = rr % a.rows;
  for (int i = tid; i < (STAGED ? M + 1 : 2 * M); i += NT) twl[i] = a.tw[i];
  if constexpr (STAGED) fill_staged<T, M>(twl + M + 1, a.tw, 2, tid, NT, RL{});
  const auto twf = [&] {
    if constexpr (STAGED)
      return TwStaged<T>{twl + M + 1};
    else
      return TwTable<T>{twl, 2};
  }();
  C2<T>* buf = smem + g * LP;
  const bool in_act = f < FIN;
  const C2<T>* src = a.in + boxi * a.in_bs + (in_act ? f : 0) * a.in_fs + rloc * a.in_pitch;
  if (!ELS && in_act) {
    for (int k = q; k <= M; k += TQ) buf[RLay::off(k, 1)] = rok && k <= a.kmax ? src[k] : zero2<T>();
  }
  __syncthreads();
  // ---- inverse real FFTs, physical values back into the same slot.  ELS: the
  // first stage gathers its pre-processed inputs straight from the row in HBM.
  {
    C2<T> v[EI::SLOTS];
    if constexpr (ELS)
      EI::template run_tw<RLay, XW>(
          v, buf, 1, q, twf,
          [&](int, int k) { return rok ? c2r_pre_g(src, k, M, a.kmax, twl) : zero2<T>(); }, in_act);
    else
      EI::template run_tw<RLay, XW>(v, buf, 1, q, twf, [&](int, int k) { return c2r_pre<T, RLay>(buf, k, M, twl); },
                                   in_act);
    __syncthreads();
    if (in_act) {
#pragma unroll
      for (int s = 0; s < EI::LAST_NB * EI::RL_; ++s)
        if (EI::last_valid(q, s)) buf[RLay::off(EI::last_index(q, s), 1)] = v[s];
    }
  }
  __syncthreads();
  // ---- products; each C2 holds two neighbouring grid points.  ELS: formed
  // in the first stage of the forward transforms instead (below).
  for (int i = tid; !ELS && i < RB * M; i += NT) {
    const int r = i / M, n = i % M;
    auto at = [&](int ff) -> C2<T>& { return smem[(ff * RB + r) * LP + RLay::off(n, 1)]; };
    const C2<T> u0 = at(0), u1 = at(1), u2 = at(2);
    const C2<T> w0 = at(3), w1 = at(4), w2 = at(5);
    auto cx = [](C2<T> a1, C2<T> a2, C2<T> b1, C2<T> b2) {  // a1 b2 - a2 b1 per point
      return C2<T>{a1.x * b2.x - a2.x * b1.x, a1.y * b2.y - a2.y * b1.y};
    };
    C2<T> n0 = cx(u1, u2, w1, w2), n1 = cx(u2, u0, w2, w0), n2 = cx(u0, u1, w0, w1);
    if constexpr (MHD) {
      const C2<T> b0 = at(6), b1 = at(7), b2 = at(8);
      const C2<T> j0 = at(9), j1 = at(10), j2 = at(11);
      n0 = n0 + cx(j1, j2, b1, b2);
      n1 = n1 + cx(j2, j0, b2, b0);
      n2 = n2 + cx(j0, j1, b0, b1);
      at(3) = cx(u1, u2, b1, b2);
      at(4) = cx(u2, u0, b2, b0);
      at(5) = cx(u0, u1, b0, b1);
    }
    at(0) = n0;
    at(1) = n1;
    at(2) = n2;
  }
  if constexpr (!ELS) __syncthreads();
  // ---- forward real FFTs of the FOUT product fields; the other groups only
  // join the barriers (with RB even their waves skip the work entirely)
  const bool active = f < FOUT;
  {
    C2<T> v[EF::SLOTS];
    if constexpr (ELS) {
      // MHD: T_ij = z+_i z-_j, i = f / 3, j = f % 3, less z+_2 z-_2 on the
      // diagonal (f = 0, 4).  NS: S_ij = u_i u_j for (i, j) = (0, 0), (1, 1),
      // (0, 1), (0, 2), (1, 2), less u_2 u_2 on the diagonal (f = 0, 1).
      // Every read happens before the first stage's barrier, so overwriting
      // the input slots after it is safe.
      const int fi = MHD ? f / 3 : (f < 2 ? f : f == 4 ? 1 : 0);
      const int fj = MHD ? 3 + f % 3 : (f < 2 ? f : f == 2 ? 1 : 2);
      const C2<T>* ra = smem + (fi * RB + rb) * LP;
      const C2<T>* rm = smem + (fj * RB + rb) * LP;
      const C2<T>* ra2 = smem + (2 * RB + rb) * LP;
      const C2<T>* rm2 = smem + ((MHD ? 5 : 2) * RB + rb) * LP;
      const bool diag = MHD ? f % 4 == 0 : f < 2;
      EF::template run_tw<RLay, XW>(
          v, buf, 1, q, twf,
          [&](int, int n) {
            const C2<T> x = ra[RLay::off(n, 1)], y = rm[RLay::off(n, 1)];
            C2<T> t{x.x * y.x, x.y * y.y};
            if (diag) {
              const C2<T> x2 = ra2[RLay::off(n, 1)], y2 = rm2[RLay::off(n, 1)];
              t = C2<T>{t.x - x2.x * y2.x, t.y - x2.y * y2.y};
            }
            return t;
          },
          active);
    } else {
      EF::template run_tw<RLay, XW>(v, buf, 1, q, twf, [&](int, int n) { return buf[RLay::off(n, 1)]; }, active);
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int s = 0; s < EF::LAST_NB * EF::RL_; ++s)
        if (EF::last_valid(q, s)) buf[RLay::off(EF::last_index(q, s), 1)] = v[s];
    }
  }
  __syncthreads();
  if (active && rok) {
    C2<T>* dst = a.out + boxi * a.out_bs + f * a.out_fs + rloc * a.out_pitch;
    for (int k = q; k <= M && k <= a.kmax; k += TQ) {
      const C2<T> x = r2c_post<T, RLay>(buf, k, M, twl);
      if (a.nt)
        store_nt(dst + k, x);
      else
        dst[k] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused x pass, packed form: two real rows per complex transform of the full
// length N (z = x + i y), instead of one half-length transform with twiddled
// pre- and post-processing per real row.
//   inverse: for k = 0..N-1, Z[k] = X[k] + i Y[k] from the stored half spectra
//            (X[N-k] = conj X[k] above N/2; only the real parts of the k = 0
//            and k = N/2 bins, the pass-order convention), z = inverse DFT_N(Z);
//            then x = Re z and y = Im z are the two physical rows;
//   forward: z = p + i q for two product rows p, q, Z = DFT_N(z);
//            P[k] = (Z[k] + conj Z[N-k]) / 2, Q[k] = -i (Z[k] - conj Z[N-k]) / 2.
// Real rows are numbered r = f RB + rb (field f, grid row rb of the
// workgroup, RB even); transform c carries real rows 2c and 2c + 1, one field
// on two grid rows.  Transforms of
// the inverse phase leave the physical rows in their LDS slots; the forward
// phase forms each product from them in its first stage (ProdTerms) and
// reuses the slots after the first stage's barrier.
// ---------------------------------------------------------------------------
// Products of the fused pass as sums of at most four terms s * f_a * f_b of
// physical input fields (field numbering as k_x_prod's inputs and outputs).
struct PTerm {
  int a, b, s;  // s = 0: unused slot
};
struct ProdDef {
  PTerm t[4];
};
__host__ __device__ constexpr ProdDef prod_def(bool mhd, bool els, int fo) {
  if (els && mhd) {  // T_ij = z+_i z-_j (fields 0-2, 3-5), less z+_2 z-_2 on the diagonal
    const int i = fo / 3, j = fo % 3;
    if (i == j) return ProdDef{{{i, 3 + j, 1}, {2, 5, -1}, {0, 0, 0}, {0, 0, 0}}};
    return ProdDef{{{i, 3 + j, 1}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}}};
  }
  if (els) {  // S_00 - S_22, S_11 - S_22, S_01, S_02, S_12 of S = u u
    if (fo == 0) return ProdDef{{{0, 0, 1}, {2, 2, -1}, {0, 0, 0}, {0, 0, 0}}};
    if (fo == 1) return ProdDef{{{1, 1, 1}, {2, 2, -1}, {0, 0, 0}, {0, 0, 0}}};
    if (fo == 2) return ProdDef{{{0, 1, 1}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}}};
    if (fo == 3) return ProdDef{{{0, 2, 1}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}}};
    return ProdDef{{{1, 2, 1}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}}};
  }
  // rotational: inputs u (0-2), w (3-5) [, b (6-8), j (9-11)];
  // component c of a x b is a_{c+1} b_{c+2} - a_{c+2} b_{c+1}
  const int c = fo % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
  if (!mhd) return ProdDef{{{c1, 3 + c2, 1}, {c2, 3 + c1, -1}, {0, 0, 0}, {0, 0, 0}}};
  if (fo < 3)  // u x w + j x b
    return ProdDef{{{c1, 3 + c2, 1}, {c2, 3 + c1, -1}, {9 + c1, 6 + c2, 1}, {9 + c2, 6 + c1, -1}}};
  return ProdDef{{{c1, 6 + c2, 1}, {c2, 6 + c1, -1}, {0, 0, 0}, {0, 0, 0}}};  // u x b
}
__host__ __device__ constexpr int xprod_fin(bool mhd, bool els) { return els ? (mhd ? 6 : 3) : mhd ? 12 : 6; }
__host__ __device__ constexpr int xprod_fout(bool mhd, bool els) { return els ? (mhd ? 8 : 5) : mhd ? 6 : 3; }
// complex transforms (workgroup slots) of the packed pass for RB grid rows
__host__ __device__ constexpr int xpk_ninv(bool mhd, bool els, int rb) { return (xprod_fin(mhd, els) * rb + 1) / 2; }
__host__ __device__ constexpr int xpk_nfwd(bool mhd, bool els, int rb) { return (xprod_fout(mhd, els) * rb + 1) / 2; }
__host__ __device__ constexpr int xpk_slots(bool mhd, bool els, int rb) {
  return xpk_ninv(mhd, els, rb) > xpk_nfwd(mhd, els, rb) ? xpk_ninv(mhd, els, rb) : xpk_nfwd(mhd, els, rb);
}

// Slots of the first inverse stage (radix R1, one butterfly per thread: slot
// m covers k = m N / R1 .. + N / R1 - 1) and of the last forward stage (radix
// RL, output m the same range) that lie entirely between KM and N - KM: with
// kx <= KM on input (the 2/3 rule) the former are zero, and the latter are
// never read by the split into real spectra.
template <int N, int R, int TQ, int KM>
__host__ __device__ constexpr unsigned xpk_mid_slots() {
  unsigned z = 0;
  if (N / R != TQ) return 0;  // more than one butterfly per thread
  for (int m = 0; m < R; ++m) {
    const int lo = m * (N / R), hi = lo + N / R - 1;
    if (lo > KM && N - hi > KM) z |= 1u << m;
  }
  return z;
}

// EX: the Stockham exchanges use per-exchange layouts (LayEx, immediate
// offsets) and rows are kept in natural order; otherwise every exchange and
// row uses RLay.  PR: the input holds kx <= (N - 1) / 3 only (the launcher
// checks a.kmax), so the slots xpk_mid_slots names are skipped.
template <typename T, int N, int TQ, int RB, class RL, bool MHD, bool ELS, class RLay, bool EX, bool PR = false>
__global__ __launch_bounds__(xpk_slots(MHD, ELS, RB) * TQ) void k_x_prod_pk(XArgs<T> a) {
  static_assert(RB % 2 == 0, "a transform pairs one field on two grid rows");
  constexpr int FIN = xprod_fin(MHD, ELS), FOUT = xprod_fout(MHD, ELS);
  constexpr int NI = xpk_ninv(MHD, ELS, RB), NO = xpk_nfwd(MHD, ELS, RB), W = xpk_slots(MHD, ELS, RB);
  constexpr int NT = W * TQ;
  using EI = Stockham<T, N, TQ, INV, RL>;
  using EF = Stockham<T, N, TQ, FWD, RL>;
  constexpr unsigned ZIN = PR ? xpk_mid_slots<N, EI::R1, TQ, (N - 1) / 3>() : 0u;
  constexpr unsigned ZOUT = PR ? xpk_mid_slots<N, EF::RL_, TQ, (N - 1) / 3>() : 0u;
  constexpr int LP = EX ? EI::EX_SLOTS : RLay::slots(N);
  // a transform's TQ <= 64 threads lie in one wave: wave-level exchanges
  constexpr bool XW = TQ <= 64 && 64 % TQ == 0;
  // element n of a row kept between the phases
  auto roff = [](int n) { return EX ? n : RLay::off(n, 1); };
  __shared__ C2<T> smem[W * LP + N];
  C2<T>* tws = smem + W * LP;  // the transforms' twiddles, staged (TwStaged layout)
  const int tid = threadIdx.x, q = tid % TQ;
  // the transform index is uniform over a wave when a transform spans whole
  // waves: keep it in a scalar register (row pointers and product terms
  // then cost scalar, not vector, instructions)
  const int c = TQ % 64 == 0 ? __builtin_amdgcn_readfirstlane(tid / TQ) : tid / TQ;
  // grid rows of the workgroup: row0 + rb, rb < RB, in boxes of a.rows rows
  // (one division per workgroup; a.rows >= RB)
  const unsigned rows = (unsigned)a.rows, nrows = (unsigned)(a.rows * a.nb);
  const unsigned row0 = (unsigned)xcd_remap(blockIdx.x, gridDim.x) * RB;
  const unsigned box0 = row0 / rows, loc0 = row0 - box0 * rows;
  auto row_of = [&](int rb, unsigned& box, unsigned& loc) {
    box = box0;
    loc = loc0 + rb;
    if (loc >= rows) {
      loc -= rows;
      ++box;
    }
    return row0 + rb < nrows;
  };
  fill_staged<T, N>(tws, a.tw, 1, tid, NT, RL{});
  __syncthreads();
  const TwStaged<T> tw{tws};
  C2<T>* buf = smem + c * LP;
  // row pointer of input real row r (field r / RB, grid row r % RB), or null
  auto in_row = [&](int r) -> const C2<T>* {
    unsigned box, loc;
    if (r >= FIN * RB || !row_of(r % RB, box, loc)) return nullptr;
    return a.in + (long)box * a.in_bs + (long)(r / RB) * a.in_fs + (long)loc * a.in_pitch;
  };
  auto fft = [&](auto E, C2<T>(&v)[decltype(E)::SLOTS], auto ld, bool act) {
    using EE = decltype(E);
    if constexpr (EX)
      EE::template run_ex<XW>(v, buf, q, tw, ld, act);
    else
      EE::template run_tw<RLay, XW>(v, buf, 1, q, tw, ld, act);
  };
  // ---- inverse: Z = X + i Y from the stored half spectra, in the first stage
  {
    const C2<T>* sx = in_row(2 * c);
    const C2<T>* sy = in_row(2 * c + 1);
    const bool act = c < NI;
    C2<T> v[EI::SLOTS];
    fft(EI{}, v,
        ld_zero<ZIN>([&](int, int k) -> C2<T> {
          const bool up = k > N / 2;
          const int kk = up ? N - k : k;           // stored index
          const bool real_bin = kk == 0 || 2 * kk == N;
          const bool live = kk <= a.kmax;
          C2<T> x = sx && live ? sx[kk] : zero2<T>();
          C2<T> y = sy && live ? sy[kk] : zero2<T>();
          const T xi = real_bin ? T(0) : (up ? -x.y : x.y);
          const T yi = real_bin ? T(0) : (up ? -y.y : y.y);
          return C2<T>{x.x - yi, xi + y.x};
        }),
        act);
    __syncthreads();
    if (act) {
#pragma unroll
      for (int s = 0; s < EI::LAST_NB * EI::RL_; ++s)
        if (EI::last_valid(q, s)) buf[roff(EI::last_index(q, s))] = v[s];
    }
  }
  __syncthreads();
  // ---- forward: products of the physical rows, two per transform.  With RB
  // even, transform c carries product field fo on grid rows rb and rb + 1
  // (rb = 2c mod RB), and input field f on those two rows sits in one slot as
  // (x, y): each term of the pair is one component-wise product of two slots.
  const bool fact = c < NO;
  {
    const int fo = (2 * c) / RB, rb2 = ((2 * c) % RB) / 2;
    C2<T> v[EF::SLOTS];
    fft(EF{}, v,
        [&](int, int n) -> C2<T> {
          C2<T> acc = zero2<T>();
          if (2 * c >= FOUT * RB) return acc;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const PTerm pt = prod_def(MHD, ELS, fo).t[t];
            if (pt.s != 0) {
              const C2<T> x = smem[(pt.a * (RB / 2) + rb2) * LP + roff(n)];
              const C2<T> y = smem[(pt.b * (RB / 2) + rb2) * LP + roff(n)];
              acc = C2<T>{acc.x + T(pt.s) * x.x * y.x, acc.y + T(pt.s) * x.y * y.y};
            }
          }
          return acc;
        },
        fact);
    __syncthreads();
    if (fact) {
#pragma unroll
      for (int s = 0; s < EF::LAST_NB * EF::RL_; ++s)
        if (!((ZOUT >> s) & 1u) && EF::last_valid(q, s)) buf[roff(EF::last_index(q, s))] = v[s];
    }
  }
  __syncthreads();
  if (!fact) return;
  // ---- split the two spectra and store kx = 0 .. min(N/2, kmax)
  const int kend = a.kmax < N / 2 ? a.kmax : N / 2;
  C2<T>* dst[2] = {nullptr, nullptr};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int p = 2 * c + h;
    unsigned box, loc;
    if (p < FOUT * RB && row_of(p % RB, box, loc))
      dst[h] = a.out + (long)box * a.out_bs + (long)(p / RB) * a.out_fs + (long)loc * a.out_pitch;
  }
  for (int k = q; k <= kend; k += TQ) {
    const C2<T> zk = buf[roff(k)];
    const C2<T> zm = conj(buf[roff(k == 0 ? 0 : N - k)]);
    const C2<T> P = T(0.5) * (zk + zm);
    const C2<T> Q = T(0.5) * mul_mi(zk - zm);
    if (a.nt) {
      if (dst[0]) store_nt(dst[0] + k, P);
      if (dst[1]) store_nt(dst[1] + k, Q);
    } else {
      if (dst[0]) dst[0][k] = P;
      if (dst[1]) dst[1][k] = Q;
    }
  }
}

// ---------------------------------------------------------------------------
// Shell spectra, deterministic.  Kernel 1: one workgroup per kz plane.
// The shells are cut into windows of 64 (window w: shells 64 w .. 64 w + 63,
// lane l of a wave owning shell 64 w + l), and each window gets R =
// SPEC_WAVES / (number of windows) waves, wave r of a window visiting the
// rows ky = r, r + R, ... in order.  The modes of a row whose shells fall in
// the window form one contiguous kx range (the shell of (kx, ky, kz) does not
// decrease with kx); the wave reads it in chunks of 64 consecutive kx, one
// mode per lane (the next chunk's loads issued before the current chunk is
// summed), sums each shell's run within the chunk by a segmented scan across
// the lanes, and hands each run's sum to the shell's lane, which adds it to Q
// Neumaier-compensated sums.  The R partial sums of a shell are then added
// in the order r = 0 .. R - 1.  Every shell's terms are thus added in one
// fixed order.  Kernel 2 sums the per-plane partials over planes in order.
// No atomics, so results are bitwise reproducible.
//   energy (Q = 2): E(s) = 1/2 sum w |f|^2 and Z(s) = 1/2 sum w |k|^2 |f|^2
//                   over nf fields, plus max |k_d . f| per plane;
//   MHD    (Q = 3): with u = (z+ + z-)/2, b = (z+ - z-)/2 (fields 0-2, 3-5):
//                   Eu(s) = 1/2 sum w |u|^2, Eb(s) = 1/2 sum w |b|^2,
//                   Hc(s) = 1/2 sum w Re(u . conj b).
// ---------------------------------------------------------------------------
constexpr int SPEC_WAVES = 16;  // waves per workgroup; nshell <= 64 SPEC_WAVES
constexpr int SPEC_NF = 6;      // fields a spectrum reads at most
struct NSum {
  double s, c;
};
__device__ __forceinline__ void nadd(NSum& a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}

__device__ __forceinline__ long isqrt_floor(long n) {  // n >= 0
  long r = (long)sqrt((double)n);
  while (r > 0 && r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r;
}

template <typename T>
struct SpecArgs {
  const C2<T>* f;
  double* part;     // [nz][nshell][Q] per plane
  double* pmax;     // [nz] max |k_d . f| per plane (energy spectrum only)
  long fs, pitch;   // field stride, kx pitch
  int nx, ny, nz, nf, nshell;
  double sx, sy, sz;  // box factors 2 pi / L (enstrophy and divergence; shells stay on the index)
};

// shell of |k|^2 = k2: the smallest s with 4 k2 < (2 s + 1)^2
__device__ __forceinline__ int shell_of_k2(long k2) { return (int)((isqrt_floor(4 * k2) + 1) / 2); }

template <typename T, bool MHD>
__global__ __launch_bounds__(SPEC_WAVES * 64) void k_spec_planes(SpecArgs<T> a) {
  constexpr int Q = MHD ? 3 : 2;
  const int kz = blockIdx.x, NX = a.nx, NY = a.ny, H = NX / 2 + 1;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int nwin = (a.nshell + 63) / 64, R = SPEC_WAVES / nwin;  // nwin <= SPEC_WAVES (host check)
  const int win = wv % nwin, grp = wv / nwin;
  const bool active = grp < R;
  const int s0 = 64 * win, own = s0 + lane;  // this lane's shell
  const long izw = wav(kz, a.nz);
  const double kzd = a.sz * dwav(kz, a.nz);
  const double qz2 = a.sz * a.sz * (double)(izw * izw);
  const int nf = MHD ? 6 : a.nf;
  __shared__ double seg[SPEC_WAVES][64][Q];
  __shared__ double red[SPEC_WAVES * 64];
  double (*sg)[Q] = seg[wv];
#pragma unroll
  for (int qq = 0; qq < Q; ++qq) sg[lane][qq] = 0.0;
  wave_lds_sync();
  NSum acc[Q];
#pragma unroll
  for (int qq = 0; qq < Q; ++qq) acc[qq] = NSum{0, 0};
  double mx = 0;
  // shells s0 .. s1 of the window: 4|k|^2 in [lo2, hi2)
  const int s1 = s0 + 63 < a.nshell - 1 ? s0 + 63 : a.nshell - 1;
  const long lo2 = (long)(2 * s0 - 1) * (2 * s0 - 1);
  const long hi2 = (long)(2 * s1 + 1) * (2 * s1 + 1);
  // the wave's chunks in order: row ky (kx range ..kx1, ky^2 + kz^2 = A),
  // first kx base; uniform over the wave
  int ky = grp - R;
  long base = 0, kx1 = -1, A = 0;
  auto advance = [&]() -> bool {
    base += 64;
    while (base > kx1) {
      ky += R;
      if (ky >= NY) return false;
      const long iyw = wav(ky, NY);
      A = iyw * iyw + izw * izw;
      const long A4 = 4 * A;
      kx1 = -1;
      if (A4 >= hi2) continue;
      long kx0 = 0;
      if (s0 > 0 && lo2 - A4 > 0) {  // smallest kx with 4 kx^2 >= lo2 - A4
        const long B = lo2 - A4;
        long t = isqrt_floor(B);
        if (t * t < B) ++t;
        kx0 = (t + 1) / 2;
      }
      kx1 = isqrt_floor(hi2 - A4 - 1) / 2;  // largest kx with 4 kx^2 < hi2 - A4
      if (kx1 > H - 1) kx1 = H - 1;
      base = kx0;
    }
    return true;
  };
  auto load = [&](C2<T>(&x)[SPEC_NF]) {
    const long kx = base + lane;
    const C2<T>* row = a.f + (long)kz * NY * a.pitch + (long)ky * a.pitch + kx;
#pragma unroll
    for (int ff = 0; ff < SPEC_NF; ++ff) x[ff] = kx <= kx1 && ff < nf ? row[ff * a.fs] : zero2<T>();
  };
  bool have = active && advance();
  C2<T> cur[SPEC_NF];
  if (have) load(cur);
  while (have) {
    const int cky = ky;
    const long ckx = base + lane, ckx1 = kx1, cA = A;
    have = advance();
    C2<T> nxt[SPEC_NF];
    if (have) load(nxt);  // in flight while this chunk is summed
    const bool live = ckx <= ckx1;
    const int sh = live ? shell_of_k2(ckx * ckx + cA) : s1 + 1;  // past the window: its own segment
    double v[Q];
#pragma unroll
    for (int qq = 0; qq < Q; ++qq) v[qq] = 0.0;
    if (live) {
      const double w = (ckx == 0 || 2 * ckx == NX) ? 0.5 : 1.0;  // (1/2) * weight
      if constexpr (MHD) {
        double eu = 0, eb = 0, hc = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const C2<T> zp = cur[c], zm = cur[3 + c];
          const double ux = 0.5 * ((double)zp.x + (double)zm.x), uy = 0.5 * ((double)zp.y + (double)zm.y);
          const double bx = 0.5 * ((double)zp.x - (double)zm.x), by = 0.5 * ((double)zp.y - (double)zm.y);
          eu += ux * ux + uy * uy;
          eb += bx * bx + by * by;
          hc += ux * bx + uy * by;
        }
        v[0] = w * eu;
        v[1] = w * eb;
        v[2] = w * hc;
      } else {
        double e = 0;
#pragma unroll
        for (int ff = 0; ff < SPEC_NF; ++ff)
          e += (double)cur[ff].x * (double)cur[ff].x + (double)cur[ff].y * (double)cur[ff].y;
        const long iyw = wav(cky, NY);
        const double q2 = a.sx * a.sx * (double)(ckx * ckx) + a.sy * a.sy * (double)(iyw * iyw) + qz2;
        v[0] = w * e;
        v[1] = w * q2 * e;
        const double kxd = a.sx * dwavx((int)ckx, NX), kyd = a.sy * dwav(cky, NY);
#pragma unroll
        for (int ff = 0; ff + 2 < SPEC_NF; ff += 3) {
          if (ff + 2 < nf) {
            const double dx = kxd * cur[ff].x + kyd * cur[ff + 1].x + kzd * cur[ff + 2].x;
            const double dy = kxd * cur[ff].y + kyd * cur[ff + 1].y + kzd * cur[ff + 2].y;
            const double d = sqrt(dx * dx + dy * dy);
            mx = d > mx ? d : mx;
          }
        }
      }
    }
    // inclusive segmented scan over the lanes (segments: equal shells,
    // contiguous because sh does not decrease with the lane)
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
      const int shd = __shfl_up(sh, d, 64);
#pragma unroll
      for (int qq = 0; qq < Q; ++qq) {
        const double vd = __shfl_up(v[qq], d, 64);
        if (lane >= d && shd == sh) v[qq] += vd;
      }
    }
    const int shn = __shfl_down(sh, 1, 64);
    if (live && (lane == 63 || shn != sh)) {  // last lane of its run
#pragma unroll
      for (int qq = 0; qq < Q; ++qq) sg[sh - s0][qq] = v[qq];
    }
    wave_lds_sync();
#pragma unroll
    for (int qq = 0; qq < Q; ++qq) {
      nadd(acc[qq], sg[lane][qq]);  // + 0 where this chunk has no run of the shell
      sg[lane][qq] = 0.0;
    }
    wave_lds_sync();
#pragma unroll
    for (int ff = 0; ff < SPEC_NF; ++ff) cur[ff] = nxt[ff];
  }
  // the R partials of each shell, in row-group order
  __syncthreads();
#pragma unroll
  for (int qq = 0; qq < Q; ++qq) sg[lane][qq] = acc[qq].s + acc[qq].c;
  __syncthreads();
  if (active && grp == 0 && own < a.nshell) {
    double* p = a.part + ((long)kz * a.nshell + own) * Q;
#pragma unroll
    for (int qq = 0; qq < Q; ++qq) {
      NSum t{0, 0};
      for (int r = 0; r < R; ++r) nadd(t, seg[win + r * nwin][lane][qq]);
      p[qq] = t.s + t.c;
    }
  }
  if constexpr (!MHD) {
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) a.pmax[kz] = red[0];
  }
}

}  // namespace ps
