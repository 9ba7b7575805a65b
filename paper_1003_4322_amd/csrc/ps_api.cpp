// ps_api.cpp -- C ABI of libps.so: plans, workspace layout, pass sequencing,
// graph capture of the RK2 step and per-kernel timing.
//
// One plan covers one box or an ensemble of independent boxes.  Consecutive
// boxes of equal size form a class; every pass runs as one launch per class
// (or, as a baseline, one launch per box).  A box of size N with F fields
// uses, inside its class's part of the caller's workspace:
//   zstar  F half spectra, dense pitch H = N/2+1       (RK2 midpoint state)
//   work   2F half spectra, pitch P (H rounded up to 128 bytes)
//          (physical-space passes: u, w [, b, j] and then the products)
//   spec   N * nshell * 3 + N doubles                  (spectrum partials)
// laid out [zstar of all boxes][work of all boxes][spec of all boxes].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <new>
#include <string>
#include <vector>

#include "../../include/ps.h"
#include "ps_launch.hpp"

namespace {

thread_local std::string g_last_error;

ps_status fail(ps_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

struct Box {
  int nx = 0, ny = 0, nz = 0;
  size_t real_off = 0, cplx_off = 0;  // element offsets in user field sets
  int nshell = 0;
  int cls = 0, idx = 0;  // class and index within it
};

// a run of consecutive boxes of equal grid
struct Class {
  int nx = 0, ny = 0, nz = 0, first = 0, nb = 0;
  ps::Grid g{};   // axis lengths and the 2/3 rule
  long H = 0, P = 0;
  long nc = 0;    // nz*ny*H   valid complex values per field
  long ncp = 0;   // nz*ny*P   pitched complex values per field
  long n3 = 0;    // nx*ny*nz
  int nshell = 0;
  // counts inside the 2/3 rule (half storage): modes, (kx, ky) columns, kx values
  long n_sphere = 0, n_disk = 0, kx_keep = 0;
  size_t real_off = 0, cplx_off = 0;   // of the first box
  size_t ws_off = 0;                   // byte offset of the class workspace
  size_t zs_box = 0, work_box = 0, spec_box = 0;  // bytes per box
  // device twiddle tables of lengths nx, ny and nz, owned by the plan
  void* twx = nullptr;
  void* twy = nullptr;
  void* twz = nullptr;
  const ps::DiskTiles* dt = nullptr;  // z-pass disk tile lists, owned by the plan
  bool same_grid(int x, int y, int z) const { return nx == x && ny == y && nz == z; }
};

// length of the axis a pass kind transforms ("z_curl", "z_epi", "z": z;
// "y": y; "x_prod": x)
int axis_len(const Class& c, const char* kind) {
  if (!strcmp(kind, "y")) return c.ny;
  if (!strcmp(kind, "x_prod")) return c.nx;
  return c.nz;
}

struct TimingRec {
  int kind;
  hipEvent_t a, b;
  double bytes;
};

struct KindStat {
  std::string name;
  double ms = 0;
  long launches = 0;
  double bytes = 0;  // summed over launches (a kind's launches may move different amounts)
};

long shell_of(long k2) {
  long s = (long)std::floor(std::sqrt((double)k2));
  while (s > 0 && 4 * k2 < (2 * s - 1) * (2 * s - 1)) --s;
  while (4 * k2 >= (2 * s + 1) * (2 * s + 1)) ++s;
  return s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct ps_plan_s {
  int nfields = 0;
  ps_dtype dtype = PS_F32;
  int device = 0;
  std::vector<Box> boxes;
  std::vector<Class> classes;
  bool per_box = false;  // baseline: one launch per box instead of per class
  bool prune = false;    // dealias-sphere pruning of the step (state zero outside the sphere)
  bool els = false;      // MHD nonlinear term in the Elsasser (divergence) form
  double omega[3] = {0, 0, 0};  // frame rotation (Coriolis term of the step)
  double bs[3] = {1, 1, 1};     // box factors 2 pi / L per axis (x, y, z)
  std::map<int, void*> tables;
  std::map<long, ps::DiskTiles> dtiles;  // per grid: z-pass tiles meeting the 2/3 disk
  std::vector<void*> dbufs;             // device lists behind dtiles
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  // z-slab pipeline of the y / x / y passes: helper streams and fork/join events
  static constexpr int NAUX = 3;
  hipStream_t aux[NAUX] = {};
  hipEvent_t ev_fork = nullptr, ev_join[NAUX] = {};
  void* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  size_t real_total = 0, cplx_total = 0;
  // graph cache for one RK2 step
  bool graphs = true;
  hipGraphExec_t gexec = nullptr;
  std::string gkey;
  // kernel variants per pass kind (chosen by ps_plan_autotune or by hand)
  std::map<std::string, int> var;
  // timing
  bool timing = false;
  std::vector<TimingRec> pending;
  std::vector<KindStat> stats;
  std::map<std::string, int> kind_index;
  // blow-up monitor of ps_rk2_step: energy check every mon_every steps
  int mon_every = 0;
  double mon_growth = 0;
  double* diag = nullptr;  // device: spectra (sum of nshell) then 3 totals per box, owned
  // timing launches of the last ps_plan_autotune (0: its result came from the cache)
  int tune_timed = -1;
  // this device's copy of the library-held spectrum scratch
  double* scratch = nullptr;
};

namespace {

size_t csize(const ps_plan_s* p) { return p->dtype == PS_F32 ? 8 : 16; }

const char* const KINDS[] = {"y", "z", "z_curl", "z_epi", "x_prod", "batch", "prune", "form", "pipe", "overlap"};
// "pipe" variant v: the y / x / y passes run as z-slabs: 2^v slabs over the
// three helper streams for v = 1..3, 2^v slabs one after another on the plan's
// stream for v = 4..6, and 2^(v-3) slabs as two chains (even and odd slabs) on
// two helper streams for v = 7..9
constexpr int NPIPE = 10, PIPE_SERIAL = 4, PIPE_TWO = 7;
struct PipeShape {
  int slabs;    // z-slabs (before capping at the box's planes)
  int streams;  // 0: in order on the plan's stream; else helper streams
};
PipeShape pipe_shape(int v) {
  if (v <= 0) return {1, 0};
  if (v < PIPE_SERIAL) return {1 << v, 3};
  if (v < PIPE_TWO) return {1 << v, 0};
  return {1 << (v - 3), 2};
}

int var_of(const ps_plan_s* p, const char* kind) {
  auto it = p->var.find(kind);
  return it == p->var.end() ? 0 : it->second;
}
size_t rsize(const ps_plan_s* p) { return p->dtype == PS_F32 ? 4 : 8; }

template <typename T>
std::vector<ps::C2<T>> make_table(int N) {
  std::vector<ps::C2<T>> t(N);
  const long double tp = 6.283185307179586476925286766559005768L;
  for (int e = 0; e < N; ++e) {
    long double a = tp * (long double)e / (long double)N;
    t[e].x = (T)cosl(a);
    t[e].y = (T)(-sinl(a));
  }
  return t;
}

ps_status hip_fail(hipError_t e, const char* what) {
  return fail(PS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// device pointer with at least `bytes` accessible from it
ps_status check_dev(const void* ptr, size_t bytes, const char* name) {
  if (!ptr) return fail(PS_ERR_ARG, std::string(name) + " is NULL");
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(PS_ERR_ARG, std::string(name) + " is not a HIP device pointer");
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return fail(PS_ERR_ARG, std::string(name) + " is not device memory");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(PS_ERR_ARG, std::string(name) + ": cannot query its allocation");
  }
  const size_t off = (const char*)ptr - (const char*)base;
  if (off + bytes > size) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %zu bytes needed but only %zu remain in its allocation", name, bytes,
             size - off);
    return fail(PS_ERR_ARG, buf);
  }
  return PS_OK;
}

int kind_of(ps_plan_s* p, const char* name) {
  auto it = p->kind_index.find(name);
  if (it != p->kind_index.end()) return it->second;
  int k = (int)p->stats.size();
  KindStat s;
  s.name = name;
  p->stats.push_back(s);
  p->kind_index[name] = k;
  return k;
}

// Enqueue one launch (a callable returning hipError_t) on stream s, with
// optional timing events.
template <class F>
ps_status enqueue(ps_plan_s* p, hipStream_t s, const char* kind, double bytes, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (p->timing) {
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
      return fail(PS_ERR_HIP, "hipEventCreate failed");
    hipEventRecord(a, s);
  }
  hipError_t e = launch(s);
  if (e != hipSuccess) {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    return hip_fail(e, kind);
  }
  if (p->timing) {
    hipEventRecord(b, s);
    p->pending.push_back({kind_of(p, kind), a, b, bytes});
  }
  return PS_OK;
}

// ---------------------------------------------------------------------------
// Pass sequences for one box
// ---------------------------------------------------------------------------
template <typename T>
struct Seq {
  ps_plan_s* p;
  const Class& b;
  int b0, nb;  // boxes [b0, b0 + nb) of the class
  hipStream_t s;
  using C = ps::C2<T>;
  const C* twx() const { return (const C*)b.twx; }
  const C* twy() const { return (const C*)b.twy; }
  const C* twz() const { return (const C*)b.twz; }
  int nf() const { return p->nfields; }
  long st_bs() const { return nf() * b.nc; }      // state / zstar box stride
  long wk_bs() const { return 2 * nf() * b.ncp; }  // work box stride
  C* zstar() const { return (C*)((char*)p->ws + b.ws_off) + b0 * st_bs(); }
  C* work() const { return (C*)((char*)p->ws + b.ws_off + b.zs_box * b.nb) + b0 * wk_bs(); }
  double* spec_part(int i) const {
    return (double*)((char*)p->ws + b.ws_off + (b.zs_box + b.work_box) * b.nb + (b0 + i) * b.spec_box);
  }
  double cs() const { return (double)sizeof(C); }

  // strided pass in place on the first nfl fields of every box, line = z;
  // nz >= 0: only the z-planes [z0, z0 + nz)
  ps_status ypass(C* x, long pitch, long bs, int nfl, int dir, int prune = 0, int z0 = 0, int nz = -1) {
    if (nz < 0) nz = b.nz;
    ps::StridedArgs<T> a{};
    a.prune = prune;
    a.g = b.g;
    a.out = x + (long)z0 * b.ny * pitch; a.in = a.out; a.tw = twy();
    a.in_fs = a.out_fs = (long)b.nz * b.ny * pitch;
    a.in_ls = a.out_ls = (long)b.ny * pitch;
    a.in_es = a.out_es = pitch;
    a.in_bs = a.out_bs = bs;
    a.ncols = (int)b.H; a.nlines = nz; a.nf = nfl; a.nb = nb;
    const double full = (double)b.nz * b.ny * b.kx_keep, disk = (double)b.nz * b.n_disk;
    const double frac = (double)nz / b.nz;
    const double bytes = frac * (prune == 0 ? 2.0 * nfl * nb * b.nc * cs() : (double)nfl * nb * (full + disk) * cs());
    // streaming stores once the written columns (every ky of the kept kx)
    // exceed the 256 MB last-level cache
    a.nt = (double)nfl * nb * nz * b.ny * (prune ? b.kx_keep : b.H) * cs() > 268435456.0;
    const int v = var_of(p, "y");
    return enqueue(p, s, dir == ps::FWD ? "y_fwd" : "y_inv", bytes,
                   [&](hipStream_t st) { return ps::launch_strided<T>(b.ny, dir, v, a, st); });
  }
  ps_status zpass(const C* in, long in_pitch, long in_bs, C* out, long out_pitch, long out_bs, int dir) {
    ps::StridedArgs<T> a{};
    a.g = b.g;
    a.in = in; a.out = out; a.tw = twz();
    a.in_fs = (long)b.nz * b.ny * in_pitch; a.out_fs = (long)b.nz * b.ny * out_pitch;
    a.in_ls = in_pitch; a.out_ls = out_pitch;
    a.in_es = (long)b.ny * in_pitch; a.out_es = (long)b.ny * out_pitch;
    a.in_bs = in_bs; a.out_bs = out_bs;
    a.ncols = (int)b.H; a.nlines = b.ny; a.nf = nf(); a.nb = nb;
    const double bytes = 2.0 * nf() * nb * b.nc * cs();
    const int v = var_of(p, "z");
    return enqueue(p, s, dir == ps::FWD ? "z_fwd" : "z_inv", bytes,
                   [&](hipStream_t st) { return ps::launch_strided<T>(b.nz, dir, v, a, st); });
  }

  ps_status r2c(const T* real_in, C* out) {
    ps::XArgs<T> a{};
    a.in = (const C*)real_in; a.out = out; a.tw = twx();
    a.in_pitch = b.nx / 2; a.in_fs = (long)b.nz * b.ny * (b.nx / 2); a.in_bs = nf() * a.in_fs;
    a.out_pitch = b.H; a.out_fs = b.nc; a.out_bs = st_bs();
    a.rows = (long)b.ny * b.nz; a.nf = nf(); a.nb = nb;
    const double bytes = nf() * nb * (b.n3 * (double)sizeof(T) + b.nc * cs());
    ps_status st = enqueue(p, s, "x_r2c", bytes, [&](hipStream_t q) { return ps::launch_x_r2c<T>(b.nx, a, q); });
    if (st) return st;
    if ((st = ypass(out, b.H, st_bs(), nf(), ps::FWD))) return st;
    return zpass(out, b.H, st_bs(), out, b.H, st_bs(), ps::FWD);
  }

  ps_status c2r(const C* in, T* real_out) {
    C* w = work();
    ps_status st = zpass(in, b.H, st_bs(), w, b.P, wk_bs(), ps::INV);
    if (st) return st;
    if ((st = ypass(w, b.P, wk_bs(), nf(), ps::INV))) return st;
    ps::XArgs<T> a{};
    a.in = w; a.out = (C*)real_out; a.tw = twx();
    a.in_pitch = b.P; a.in_fs = b.ncp; a.in_bs = wk_bs();
    a.out_pitch = b.nx / 2; a.out_fs = (long)b.nz * b.ny * (b.nx / 2); a.out_bs = nf() * a.out_fs;
    a.rows = (long)b.ny * b.nz; a.nf = nf(); a.nb = nb;
    const double bytes = nf() * nb * (b.n3 * (double)sizeof(T) + b.nc * cs());
    return enqueue(p, s, "x_c2r", bytes, [&](hipStream_t q) { return ps::launch_x_c2r<T>(b.nx, a, q); });
  }

  // the five passes of one right-hand side evaluation
  // fields of each stage: state, physical inputs of the products, products
  bool els(bool) const { return p->els; }
  int nphys(bool mhd) const { return p->els ? (mhd ? 6 : 3) : (mhd ? 12 : 6); }
  int nprod(bool mhd) const { return p->els ? (mhd ? 8 : 5) : (mhd ? 6 : 3); }

  ps_status pass_zcurl(const C* src, bool mhd) {
    const int nin = mhd ? 6 : 3, nphys = this->nphys(mhd);
    ps::ZCurlArgs<T> ca{};
    ca.in = src; ca.out = work(); ca.tw = twz();
    ca.in_fs = b.nc; ca.in_pitch = b.H; ca.out_fs = b.ncp; ca.out_pitch = b.P; ca.g = b.g;
    ca.in_bs = st_bs(); ca.out_bs = wk_bs(); ca.nb = nb;
    ca.prune = p->prune;
    ca.sx = (T)p->bs[0]; ca.sy = (T)p->bs[1]; ca.sz = (T)p->bs[2];
    const int v = var_of(p, "z_curl");
    const double bytes = p->prune ? ((double)nin * b.n_sphere + (double)nphys * b.n_disk * b.nz) * nb * cs()
                                  : (double)(nin + nphys) * nb * b.nc * cs();
    // streaming stores once the output far exceeds the caches (measured: z_curl
    // at 512^3 FP64 0.82 -> 0.74 ms, FP32 unchanged)
    const double out_bytes = (double)nphys * nb * (p->prune ? (double)b.n_disk * b.nz : (double)b.nc) * cs();
    ca.nt = out_bytes > 268435456.0;
    return enqueue(p, s, "z_curl", bytes,
                   [&](hipStream_t q) { return ps::launch_z_curl<T>(b.nz, mhd, els(mhd), v, ca, b.dt, q); });
  }
  ps_status pass_xprod(bool mhd, int z0 = 0, int nz = -1) {
    if (nz < 0) nz = b.nz;
    const int nphys = this->nphys(mhd), nprod = this->nprod(mhd);
    ps::XArgs<T> xa{};
    xa.out = work() + (long)z0 * b.ny * b.P; xa.in = xa.out; xa.tw = twx();
    xa.in_pitch = xa.out_pitch = b.P; xa.in_fs = xa.out_fs = b.ncp;
    xa.in_bs = xa.out_bs = wk_bs();
    xa.rows = (long)nz * b.ny; xa.nf = nphys; xa.nb = nb;
    xa.kmax = p->prune ? (int)b.kx_keep - 1 : b.nx / 2;
    // streaming stores once the product rows written exceed the 256 MB
    // last-level cache
    xa.nt = (double)nprod * nb * nz * b.ny * (xa.kmax + 1) * cs() > 268435456.0;
    const int v = var_of(p, "x_prod");
    const double per = (double)nz / b.nz * (p->prune ? (double)b.nz * b.ny * b.kx_keep : (double)b.nc);
    return enqueue(p, s, "x_prod", (double)(nphys + nprod) * nb * per * cs(),
                   [&](hipStream_t q) { return ps::launch_x_prod<T>(b.nx, mhd, els(mhd), v, xa, q); });
  }
  ps_status pass_zepi(bool mhd, int mode, C* out, const C* st0, const C* st1, T h, T nua, T nub) {
    const int nprod = this->nprod(mhd), nst = mhd ? 6 : 3;
    ps::ZEpiArgs<T> ea{};
    ea.in = work(); ea.out = out; ea.st0 = st0; ea.st1 = st1; ea.tw = twz();
    ea.in_fs = b.ncp; ea.in_pitch = b.P; ea.out_fs = b.nc; ea.out_pitch = b.H;
    ea.in_bs = wk_bs(); ea.out_bs = st_bs(); ea.nb = nb;
    ea.scale = (T)(1.0 / (double)b.n3);
    ea.h = h; ea.nua = nua; ea.nub = nub; ea.g = b.g; ea.mode = mode;
    ea.rot = mode != 0 && (p->omega[0] != 0 || p->omega[1] != 0 || p->omega[2] != 0);
    ea.w2x = (T)(2 * p->omega[0]); ea.w2y = (T)(2 * p->omega[1]); ea.w2z = (T)(2 * p->omega[2]);
    ea.prune = p->prune;
    ea.sx = (T)p->bs[0]; ea.sy = (T)p->bs[1]; ea.sz = (T)p->bs[2];
    const int nrw = mode == 0 ? 0 : (mode == 1 ? 1 : 2);
    const int v = var_of(p, "z_epi");
    double bytes = (double)(nprod + nst + nrw * nst) * nb * b.nc * cs();
    if (p->prune)
      bytes = ((double)nprod * b.n_disk * b.nz +
               (mode == 0 ? (double)nst * b.nc : (double)(1 + nrw) * nst * b.n_sphere)) * nb * cs();
    return enqueue(p, s, "z_epi", bytes,
                   [&](hipStream_t q) { return ps::launch_z_epi<T>(b.nz, mhd, els(mhd), v, ea, b.dt, q); });
  }

  // nonlinear right-hand side, epilogue mode 0/1/2 (see k_z_epi)
  // inverse y, products, forward y on the z-planes [z0, z0 + nz): every plane's
  // chain is independent of the others' (only the z passes couple planes)
  ps_status yxy(bool mhd, int z0, int nz) {
    ps_status st = ypass(work(), b.P, wk_bs(), nphys(mhd), ps::INV, p->prune ? 1 : 0, z0, nz);
    if (!st) st = pass_xprod(mhd, z0, nz);
    if (!st) st = ypass(work(), b.P, wk_bs(), nprod(mhd), ps::FWD, p->prune ? 2 : 0, z0, nz);
    return st;
  }

  ps_status rhs(const C* src, bool mhd, int mode, C* out, const C* st0, const C* st1, T h, T nua, T nub) {
    ps_status st = pass_zcurl(src, mhd);
    if (st) return st;
    const PipeShape ps = pipe_shape(var_of(p, "pipe"));
    const int slabs = std::min(ps.slabs, b.nz);
    if (slabs <= 1) {
      if ((st = yxy(mhd, 0, b.nz))) return st;
    } else if (ps.streams == 0) {
      // slabs in order on the plan's stream: each slab's chain (inverse y,
      // products, forward y) works on data the previous pass of the chain
      // has just left in the last-level cache
      for (int i = 0; i < slabs; ++i) {
        const int z0 = (int)((long)i * b.nz / slabs), z1 = (int)((long)(i + 1) * b.nz / slabs);
        if ((st = yxy(mhd, z0, z1 - z0))) return st;
      }
    } else {
      // fork the slabs over the helper streams (their memory-bound y passes
      // overlap other slabs' compute-bound product pass), then join; with two
      // chains of small slabs, the two slabs in flight together can still
      // stay in the last-level cache
      const int k = std::min({slabs, ps.streams, ps_plan_s::NAUX});
      hipError_t e = hipEventRecord(p->ev_fork, s);
      for (int i = 0; i < k && e == hipSuccess; ++i) e = hipStreamWaitEvent(p->aux[i], p->ev_fork, 0);
      if (e != hipSuccess) return hip_fail(e, "slab fork");
      for (int i = 0; i < slabs; ++i) {
        Seq<T> q{p, b, b0, nb, p->aux[i % k]};
        const int z0 = (int)((long)i * b.nz / slabs), z1 = (int)((long)(i + 1) * b.nz / slabs);
        if ((st = q.yxy(mhd, z0, z1 - z0))) return st;
      }
      for (int i = 0; i < k && e == hipSuccess; ++i) {
        e = hipEventRecord(p->ev_join[i], p->aux[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_join[i], 0);
      }
      if (e != hipSuccess) return hip_fail(e, "slab join");
    }
    return pass_zepi(mhd, mode, out, st0, st1, h, nua, nub);
  }

  // one launch of pass `kind` on the plan's buffers (tuning); only the
  // workspace is written
  ps_status tune_launch(const char* kind, const C* state, bool mhd) {
    if (!strcmp(kind, "z_curl")) return pass_zcurl(state, mhd);
    if (!strcmp(kind, "y")) return ypass(work(), b.P, wk_bs(), nphys(mhd), ps::INV, p->prune ? 1 : 0);
    if (!strcmp(kind, "x_prod")) return pass_xprod(mhd);
    // as in the step's two stages: mode 1 (z* <- state) and mode 2, which
    // reads two state-sized buffers and updates one in place: here z*
    // (updated) and the caller's state (only read)
    if (!strcmp(kind, "z_epi")) {
      ps_status st = pass_zepi(mhd, 1, zstar(), state, nullptr, T(0), T(0), T(0));
      return st ? st : pass_zepi(mhd, 2, nullptr, zstar(), state, T(0), T(0), T(0));
    }
    // a whole right-hand side in the first stage's mode (writes z* only)
    if (!strcmp(kind, "step")) return rhs(state, mhd, 1, zstar(), state, nullptr, T(0), T(0), T(0));
    return fail(PS_ERR_ARG, std::string("no tuning launch for kind ") + kind);
  }

  ps_status rk2(C* state, bool mhd, double nu, double eta, double dt) {
    const T nua = (T)(mhd ? 0.5 * (nu + eta) : nu), nub = (T)(mhd ? 0.5 * (nu - eta) : 0.0);
    C* zs = zstar();
    ps_status st = rhs(state, mhd, 1, zs, state, nullptr, (T)(0.5 * dt), nua, nub);
    if (st) return st;
    return rhs(zs, mhd, 2, nullptr, state, zs, (T)dt, nua, nub);
  }

  // energy spectrum of nfl fields (mhd false) or the MHD quantities of the
  // six Elsasser fields (mhd true) of box i of the class
  ps_status spectrum(int i, const C* f, int nfl, bool mhd, double* spec, double* totals) {
    ps::SpecArgs<T> a{};
    a.f = f; a.part = spec_part(i); a.pmax = a.part + (long)b.nz * b.nshell * (mhd ? 3 : 2);
    a.fs = b.nc; a.pitch = b.H; a.nx = b.nx; a.ny = b.ny; a.nz = b.nz; a.nf = nfl; a.nshell = b.nshell;
    a.sx = p->bs[0]; a.sy = p->bs[1]; a.sz = p->bs[2];
    return enqueue(p, s, "spectrum", nfl * b.nc * cs(),
                   [&](hipStream_t q) { return ps::launch_spectrum<T>(a, mhd, spec, totals, q); });
  }
};

// Run f(seq, first_box_index) over the plan: one Seq per class, or per box
// in the one-box-per-launch baseline.
template <typename T, class F>
ps_status for_each_launch(ps_plan_s* p, hipStream_t s, F&& f) {
  for (auto& c : p->classes) {
    if (p->per_box) {
      for (int i = 0; i < c.nb; ++i) {
        Seq<T> q{p, c, i, 1, s};
        if (ps_status st = f(q, c.first + i)) return st;
      }
    } else {
      Seq<T> q{p, c, 0, c.nb, s};
      if (ps_status st = f(q, c.first)) return st;
    }
  }
  return PS_OK;
}

ps_status validate_plan(ps_plan p) {
  if (!p) return fail(PS_ERR_ARG, "plan is NULL");
  return PS_OK;
}

ps_status need_ws(ps_plan p) {
  if (!p->ws || p->ws_bytes < p->ws_need)
    return fail(PS_ERR_STATE, "no (or too small) workspace: call ps_plan_set_workspace");
  return PS_OK;
}

ps_status set_device(ps_plan p) {
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return PS_OK;
}

void free_plan(ps_plan p) {
  if (!p) return;
  for (auto& r : p->pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->cap) hipStreamDestroy(p->cap);
  for (auto& a : p->aux)
    if (a) hipStreamDestroy(a);
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  for (auto& e : p->ev_join)
    if (e) hipEventDestroy(e);
  for (auto& kv : p->tables) hipFree(kv.second);
  for (void* d : p->dbufs) hipFree(d);
  if (p->diag) hipFree(p->diag);
  delete p;
}

// For every tile width a z-pass variant of the class's z length can use, the
// list of tiles (tile | ky << 16, ky-major, tile fastest) whose first column
// lies inside the disk Grid::disk(kx, ky); the kernels skip exactly the other
// tiles.
template <typename T>
ps_status upload_disk_tiles(ps_plan p, const Class& c) {
  const long key = ((long)c.nx << 22) | ((long)c.ny << 11) | c.nz;
  if (p->dtiles.count(key)) return PS_OK;
  ps::DiskTiles& dt = p->dtiles[key];
  const bool mhd = p->nfields == 6;
  std::set<int> widths;
  for (int v = 0; v < ps::variant_count("z_curl", c.nz, mhd); ++v) widths.insert(ps::z_curl_tx<T>(c.nz, v));
  for (int v = 0; v < ps::variant_count("z_epi", c.nz, mhd); ++v) widths.insert(ps::z_epi_tx<T>(c.nz, v));
  for (int tx : widths) {
    if (tx < 1 || tx > ps::DiskTiles::MAXTX) return fail(PS_ERR_STATE, "z-pass tile width out of range");
    std::vector<int> list;
    const long ntile = (c.H + tx - 1) / tx;
    for (long ky = 0; ky < c.ny; ++ky) {
      const int kyw = (int)(ky < c.ny / 2 ? ky : ky - c.ny);
      for (long t = 0; t < ntile; ++t)
        if (c.g.disk((int)(t * tx), kyw)) list.push_back((int)(t | ky << 16));
    }
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, std::max<size_t>(list.size(), 1) * sizeof(int));
    if (e != hipSuccess) return fail(PS_ERR_NOMEM, std::string("disk tile list: ") + hipGetErrorString(e));
    p->dbufs.push_back(d);
    if (!list.empty()) {
      e = hipMemcpy(d, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "disk tile upload");
    }
    dt.list[tx] = (const int*)d;
    dt.count[tx] = (int)list.size();
  }
  return PS_OK;
}

template <typename T>
ps_status upload_table(ps_plan p, int N) {
  if (p->tables.count(N)) return PS_OK;
  auto t = make_table<T>(N);
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, t.size() * sizeof(t[0]));
  if (e != hipSuccess) return fail(PS_ERR_NOMEM, std::string("twiddle table: ") + hipGetErrorString(e));
  e = hipMemcpy(d, t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(d);
    return hip_fail(e, "twiddle upload");
  }
  p->tables[N] = d;
  return PS_OK;
}

template <typename F>
ps_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(PS_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(PS_ERR_HIP, "unexpected exception");
  }
}

// dispatch on the plan's dtype
template <class F>
ps_status by_type(ps_plan p, F&& f) {
  if (p->dtype == PS_F32) return f((float*)nullptr);
  return f((double*)nullptr);
}

ps_status sync_timing(ps_plan p) {
  for (auto& r : p->pending) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e, "timing event");
    KindStat& k = p->stats[r.kind];
    k.ms += ms;
    k.launches += 1;
    k.bytes += r.bytes;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  p->pending.clear();
  return PS_OK;
}

// FP64 energy of every box of `state` (all of the plan's fields), read back
// to the host: e[i] for box i.  Synchronises the plan's stream.
template <typename T>
ps_status box_energies(ps_plan p, const void* state, std::vector<double>& e) {
  const size_t nb = p->boxes.size();
  size_t so = 0;
  for (auto& b : p->boxes) so += b.nshell;
  double* tot = p->diag + so;
  so = 0;
  for (size_t i = 0; i < nb; ++i) {
    auto& b = p->boxes[i];
    Seq<T> q{p, p->classes[b.cls], 0, p->classes[b.cls].nb, p->stream};
    ps_status st = q.spectrum(b.idx, (const ps::C2<T>*)state + b.cplx_off, p->nfields, false, p->diag + so,
                              tot + 3 * i);
    if (st) return st;
    so += b.nshell;
  }
  std::vector<double> t(3 * nb);
  hipError_t er = hipMemcpyAsync(t.data(), tot, t.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (er == hipSuccess) er = hipStreamSynchronize(p->stream);
  if (er != hipSuccess) return hip_fail(er, "monitor read-back");
  e.resize(nb);
  for (size_t i = 0; i < nb; ++i) e[i] = t[3 * i];
  return PS_OK;
}

// Persistent autotune cache (file named by PS_TUNE_CACHE): one line per key,
// "key<TAB>kind=v,kind=v,...".  The key names everything the timings depend
// on: device architecture, HIP runtime, the library build, model, dtype,
// fields, every size class and the variants that are not tuned.
std::string tune_key(ps_plan p, bool mhd) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
  int rt = 0;
  (void)hipRuntimeGetVersion(&rt);
  char buf[160];
  snprintf(buf, sizeof buf, "%s|hip%d|%s|%s|%s|nf%d", arch.c_str(), rt, ps_build_hash(), mhd ? "mhd" : "ns",
           p->dtype == PS_F32 ? "f32" : "f64", p->nfields);
  std::string k = buf;
  for (auto& c : p->classes) {
    snprintf(buf, sizeof buf, "|%dx%dx%d*%d", c.nx, c.ny, c.nz, c.nb);
    k += buf;
  }
  for (const char* kind : {"form", "prune", "batch", "overlap"}) {
    snprintf(buf, sizeof buf, "|%s=%d", kind, var_of(p, kind));
    k += buf;
  }
  return k;
}

// kinds the autotuner chooses (per pass, then the slab pipeline per right-hand side)
const char* const TUNED[] = {"z_curl", "y", "x_prod", "z_epi", "pipe"};
constexpr int NTUNED = sizeof(TUNED) / sizeof(TUNED[0]);

bool tune_cache_lookup(ps_plan p, const std::string& key) {
  const char* path = getenv("PS_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  std::map<std::string, int> found;
  bool hit = false;
  char line[4096];
  while (fgets(line, sizeof line, f)) {
    char* tab = strchr(line, '\t');
    if (!tab || std::string(line, tab) != key) continue;
    std::map<std::string, int> v;
    bool ok = true;
    for (char* tok = strtok(tab + 1, ",\n"); tok; tok = strtok(nullptr, ",\n")) {
      char* eq = strchr(tok, '=');
      if (!eq) { ok = false; break; }
      const std::string kind(tok, eq);
      const int val = atoi(eq + 1);
      if (val < 0 || val >= ps_plan_variant_count(p, kind.c_str())) { ok = false; break; }
      v[kind] = val;
    }
    for (const char* kind : TUNED) ok = ok && v.count(kind);
    if (ok) {  // the last valid line for the key wins
      found = v;
      hit = true;
    }
  }
  fclose(f);
  if (hit)
    for (auto& kv : found) p->var[kv.first] = kv.second;
  return hit;
}

void tune_cache_store(ps_plan p, const std::string& key) {
  const char* path = getenv("PS_TUNE_CACHE");
  if (!path || !*path) return;
  std::string line = key + "\t";
  for (int i = 0; i < NTUNED; ++i) {
    char buf[64];
    snprintf(buf, sizeof buf, "%s%s=%d", i ? "," : "", TUNED[i], var_of(p, TUNED[i]));
    line += buf;
  }
  line += "\n";
  FILE* f = fopen(path, "a");
  if (!f) return;  // a cache that cannot be written only costs the next plan its timing runs
  fwrite(line.data(), 1, line.size(), f);
  fclose(f);
}

}  // namespace

extern "C" {

const char* ps_status_string(ps_status s) {
  switch (s) {
    case PS_OK: return "ok";
    case PS_ERR_ARG: return "invalid argument";
    case PS_ERR_SIZE: return "unsupported size";
    case PS_ERR_NOMEM: return "out of memory";
    case PS_ERR_HIP: return "HIP runtime error";
    case PS_ERR_STATE: return "invalid plan state";
    case PS_ERR_DIVERGED: return "diverged";
  }
  return "unknown status";
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

#ifndef PS_SRC_HASH
#define PS_SRC_HASH "unknown"
#endif
const char* ps_build_hash(void) { return PS_SRC_HASH; }

}  // extern "C"

namespace {

// boxes of grids dims[3 i .. 3 i + 2] = (nx, ny, nz)
ps_status create_plan(ps_plan* out, int nbox, const int* dims, int nfields, ps_dtype dtype) {
  return guarded([&]() -> ps_status {
    if (!out) return fail(PS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nfields != 3 && nfields != 6) return fail(PS_ERR_SIZE, "nfields must be 3 (NS) or 6 (MHD)");
    if (dtype != PS_F32 && dtype != PS_F64) return fail(PS_ERR_ARG, "dtype must be PS_F32 or PS_F64");
    for (int i = 0; i < 3 * nbox; ++i)
      if (!ps::size_supported(dims[i])) {
        char buf[128];
        snprintf(buf, sizeof buf, "unsupported axis length %d (box %d)", dims[i], i / 3);
        return fail(PS_ERR_SIZE, buf);
      }
    ps_plan p = new ps_plan_s();
    p->nfields = nfields;
    p->dtype = dtype;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "hipGetDevice");
    }
    const size_t cs = csize(p);
    size_t roff = 0, coff = 0;
    for (int i = 0; i < nbox; ++i) {
      Box b;
      b.nx = dims[3 * i];
      b.ny = dims[3 * i + 1];
      b.nz = dims[3 * i + 2];
      b.real_off = roff;
      b.cplx_off = coff;
      roff += (size_t)nfields * b.nx * b.ny * b.nz;
      coff += (size_t)nfields * b.nz * b.ny * (b.nx / 2 + 1);
      {
        const long hx = b.nx / 2, hy = b.ny / 2, hz = b.nz / 2;
        b.nshell = (int)shell_of(hx * hx + hy * hy + hz * hz) + 1;
      }
      if (p->classes.empty() || !p->classes.back().same_grid(b.nx, b.ny, b.nz)) {
        Class c;
        c.nx = b.nx;
        c.ny = b.ny;
        c.nz = b.nz;
        c.g = ps::make_grid(c.nx, c.ny, c.nz);
        c.first = i;
        c.nb = 0;
        c.H = c.nx / 2 + 1;
        const long align = 128 / (long)cs;
        c.P = (c.H + align - 1) / align * align;
        c.nc = (long)c.nz * c.ny * c.H;
        c.ncp = (long)c.nz * c.ny * c.P;
        c.n3 = (long)c.nx * c.ny * c.nz;
        c.nshell = b.nshell;
        {
          auto w = [](long i, long n) { return (int)(i < n / 2 ? i : i - n); };
          for (long kx = 0; kx < c.H; ++kx)
            for (long ky = 0; ky < c.ny; ++ky) {
              if (!c.g.disk((int)kx, w(ky, c.ny))) continue;
              ++c.n_disk;
              const int pp = c.g.perp((int)kx, w(ky, c.ny));
              for (long kz = 0; kz < c.nz; ++kz) c.n_sphere += c.g.keep_p(pp, w(kz, c.nz));
            }
          while (c.kx_keep < c.H && c.g.disk((int)c.kx_keep, 0)) ++c.kx_keep;
        }
        c.real_off = b.real_off;
        c.cplx_off = b.cplx_off;
        c.zs_box = (size_t)nfields * c.nc * cs;
        c.work_box = (size_t)2 * nfields * c.ncp * cs;
        c.spec_box = align256(((size_t)c.nz * c.nshell * 3 + c.nz) * sizeof(double));
        p->classes.push_back(c);
      }
      b.cls = (int)p->classes.size() - 1;
      b.idx = p->classes.back().nb++;
      p->boxes.push_back(b);
    }
    size_t ws = 0;
    for (auto& c : p->classes) {
      c.ws_off = ws;
      ws += align256((c.zs_box + c.work_box) * c.nb) + c.spec_box * c.nb;
    }
    p->ws_need = ws;
    p->real_total = roff;
    p->cplx_total = coff;
    for (auto& c : p->classes) {
      ps_status st = PS_OK;
      for (int n : {c.nx, c.ny, c.nz})
        if (!st) st = dtype == PS_F32 ? upload_table<float>(p, n) : upload_table<double>(p, n);
      if (!st) st = dtype == PS_F32 ? upload_disk_tiles<float>(p, c) : upload_disk_tiles<double>(p, c);
      if (st) {
        free_plan(p);
        return st;
      }
      c.twx = p->tables[c.nx];
      c.twy = p->tables[c.ny];
      c.twz = p->tables[c.nz];
      c.dt = &p->dtiles[((long)c.nx << 22) | ((long)c.ny << 11) | c.nz];
    }
    // the rotational form by default: valid for any input; the divergence
    // form (fewer transforms) needs a solenoidal, truncated state and is set
    // by the caller
    // measured defaults at 512^3 (the autotuner refines them per workload),
    // set where some box's pass has variants
    const std::pair<const char*, int> defaults[] = {
        {"z_curl", 0},
        {"z_epi", nfields == 6 ? 5 : 2},  // MHD (Elsasser): z+ and z- in two workgroups
        {"x_prod", dtype == PS_F32 ? (nfields == 6 ? 8 : 4) : 7},
        {"y", dtype == PS_F32 ? 2 : 0}};
    for (auto& d : defaults)
      if (ps_plan_variant_count(p, d.first) > d.second) p->var[d.first] = d.second;
    {
      size_t nsh = 0;
      for (auto& b : p->boxes) nsh += b.nshell;
      e = hipMalloc(&p->diag, (nsh + 3 * p->boxes.size()) * sizeof(double));
      if (e != hipSuccess) {
        p->diag = nullptr;
        free_plan(p);
        return fail(PS_ERR_NOMEM, std::string("diagnostics buffer: ") + hipGetErrorString(e));
      }
    }
    // set-up of the allocation-free spectrum entry point: the address of
    // this device's copy of its scratch (looked up once per device)
    e = ps::spectrum_scratch(p->device, &p->scratch);
    if (e != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "hipGetSymbolAddress (spectrum scratch)");
    }
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    for (int i = 0; i < ps_plan_s::NAUX && e == hipSuccess; ++i)
      e = hipStreamCreateWithFlags(&p->aux[i], hipStreamNonBlocking);  // default priority
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    for (int i = 0; i < ps_plan_s::NAUX && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&p->ev_join[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "hipStreamCreate");
    }
    *out = p;
    return PS_OK;
  });
}

}  // namespace

extern "C" {

ps_status ps_plan_create_batch(ps_plan* out, int nbox, const int* Ns, int nfields, ps_dtype dtype) {
  return guarded([&]() -> ps_status {
    if (!out) return fail(PS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nbox < 1 || !Ns) return fail(PS_ERR_ARG, "need nbox >= 1 and a size array");
    std::vector<int> dims(3 * (size_t)nbox);
    for (int i = 0; i < nbox; ++i) dims[3 * i] = dims[3 * i + 1] = dims[3 * i + 2] = Ns[i];
    return create_plan(out, nbox, dims.data(), nfields, dtype);
  });
}

ps_status ps_plan_create(ps_plan* out, int N, int nfields, ps_dtype dtype) {
  return ps_plan_create_batch(out, 1, &N, nfields, dtype);
}

ps_status ps_plan_create_grid(ps_plan* out, int nx, int ny, int nz, int nfields, ps_dtype dtype) {
  const int dims[3] = {nx, ny, nz};
  return create_plan(out, 1, dims, nfields, dtype);
}

ps_status ps_plan_destroy(ps_plan p) {
  if (!p) return PS_OK;
  return guarded([&]() -> ps_status {
    hipSetDevice(p->device);
    free_plan(p);
    return PS_OK;
  });
}

ps_status ps_plan_set_stream(ps_plan p, void* stream) {
  if (ps_status st = validate_plan(p)) return st;
  p->stream = (hipStream_t)stream;
  return PS_OK;
}

size_t ps_plan_workspace_bytes(ps_plan p) { return p ? p->ws_need : 0; }

ps_status ps_plan_set_workspace(ps_plan p, void* dev, size_t bytes) {
  if (ps_status st = validate_plan(p)) return st;
  if (bytes < p->ws_need) return fail(PS_ERR_NOMEM, "workspace smaller than ps_plan_workspace_bytes");
  if (((uintptr_t)dev & 255) != 0) return fail(PS_ERR_ARG, "workspace must be 256-byte aligned");
  if (ps_status st = check_dev(dev, p->ws_need, "workspace")) return st;
  p->ws = dev;
  p->ws_bytes = bytes;
  if (p->gexec) {
    hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey.clear();
  }
  return PS_OK;
}

ps_status ps_plan_box_offsets(ps_plan p, int box, size_t* real_off, size_t* cplx_off) {
  if (ps_status st = validate_plan(p)) return st;
  if (box < 0 || box >= (int)p->boxes.size()) return fail(PS_ERR_ARG, "box index out of range");
  if (real_off) *real_off = p->boxes[box].real_off;
  if (cplx_off) *cplx_off = p->boxes[box].cplx_off;
  return PS_OK;
}

int ps_num_shells(ps_plan p, int box) {
  if (!p || box < 0 || box >= (int)p->boxes.size()) return PS_ERR_ARG;
  return p->boxes[box].nshell;
}

ps_status ps_fft_r2c(ps_plan p, const void* real_in, void* cplx_out) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (ps_status st = check_dev(real_in, p->real_total * rsize(p), "real_in")) return st;
    if (ps_status st = check_dev(cplx_out, p->cplx_total * csize(p), "cplx_out")) return st;
    if (ps_status st = set_device(p)) return st;
    return by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      return for_each_launch<T>(p, p->stream, [&](Seq<T>& q, int bi) {
        const Box& b = p->boxes[bi];
        return q.r2c((const T*)real_in + b.real_off, (ps::C2<T>*)cplx_out + b.cplx_off);
      });
    });
  });
}

ps_status ps_fft_c2r(ps_plan p, const void* cplx_in, void* real_out) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (ps_status st = need_ws(p)) return st;
    if (ps_status st = check_dev(cplx_in, p->cplx_total * csize(p), "cplx_in")) return st;
    if (ps_status st = check_dev(real_out, p->real_total * rsize(p), "real_out")) return st;
    if (ps_status st = set_device(p)) return st;
    return by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      return for_each_launch<T>(p, p->stream, [&](Seq<T>& q, int bi) {
        const Box& b = p->boxes[bi];
        return q.c2r((const ps::C2<T>*)cplx_in + b.cplx_off, (T*)real_out + b.real_off);
      });
    });
  });
}

static ps_status nonlinear(ps_plan p, const void* in, void* out, bool mhd) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (p->nfields != (mhd ? 6 : 3))
      return fail(PS_ERR_ARG, mhd ? "MHD needs a plan with nfields = 6" : "NS needs a plan with nfields = 3");
    if (ps_status st = need_ws(p)) return st;
    if (ps_status st = check_dev(in, p->cplx_total * csize(p), "input")) return st;
    if (ps_status st = check_dev(out, p->cplx_total * csize(p), "output")) return st;
    if (ps_status st = set_device(p)) return st;
    return by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      for (auto& c : p->classes)
        if (mhd && !ps::mhd_supported<T>(c.nx)) return fail(PS_ERR_SIZE, "MHD not supported at this nx and dtype");
      return for_each_launch<T>(p, p->stream, [&](Seq<T>& q, int bi) {
        const Box& b = p->boxes[bi];
        ps::C2<T>* o = (ps::C2<T>*)out + b.cplx_off;
        return q.rhs((const ps::C2<T>*)in + b.cplx_off, mhd, 0, o, nullptr, nullptr, T(0), T(0), T(0));
      });
    });
  });
}

ps_status ps_nonlinear_ns(ps_plan p, const void* uhat, void* nhat) { return nonlinear(p, uhat, nhat, false); }
ps_status ps_nonlinear_mhd(ps_plan p, const void* zhat, void* nhat) { return nonlinear(p, zhat, nhat, true); }

ps_status ps_rk2_step(ps_plan p, void* state, ps_model m, double nu, double eta, double dt, int nsteps) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (m != PS_NS && m != PS_MHD) return fail(PS_ERR_ARG, "model must be PS_NS or PS_MHD");
    const bool mhd = m == PS_MHD;
    if (p->nfields != (mhd ? 6 : 3)) return fail(PS_ERR_ARG, "model does not match the plan's nfields");
    if (nsteps < 0) return fail(PS_ERR_ARG, "nsteps < 0");
    if (!std::isfinite(nu) || !std::isfinite(eta) || !std::isfinite(dt))
      return fail(PS_ERR_ARG, "nu, eta and dt must be finite");
    if (ps_status st = need_ws(p)) return st;
    if (ps_status st = check_dev(state, p->cplx_total * csize(p), "state")) return st;
    if (ps_status st = set_device(p)) return st;
    if (nsteps == 0) return PS_OK;
    return by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      for (auto& c : p->classes)
        if (mhd && !ps::mhd_supported<T>(c.nx)) return fail(PS_ERR_SIZE, "MHD not supported at this nx and dtype");
      auto one_step = [&](hipStream_t s) -> ps_status {
        return for_each_launch<T>(p, s, [&](Seq<T>& q, int bi) {
          return q.rk2((ps::C2<T>*)state + p->boxes[bi].cplx_off, mhd, nu, eta, dt);
        });
      };
      // the blow-up monitor: energies at the start, then after every
      // mon_every steps and after the last one
      std::vector<double> e0, e1;
      const int every = p->mon_every > 0 ? p->mon_every : nsteps;
      if (p->mon_every > 0) {
        if (ps_status st = box_energies<T>(p, state, e0)) return st;
        for (size_t i = 0; i < e0.size(); ++i)
          if (!std::isfinite(e0[i])) return fail(PS_ERR_DIVERGED, "initial energy is not finite");
      }
      auto check = [&](int done) -> ps_status {
        if (p->mon_every <= 0) return PS_OK;
        if (ps_status st = box_energies<T>(p, state, e1)) return st;
        for (size_t i = 0; i < e1.size(); ++i)
          if (!std::isfinite(e1[i]) || e1[i] > p->mon_growth * e0[i]) {
            char buf[200];
            snprintf(buf, sizeof buf, "box %zu: energy %.6g after %d of %d steps (%.6g at the start)", i, e1[i],
                     done, nsteps, e0[i]);
            return fail(PS_ERR_DIVERGED, buf);
          }
        return PS_OK;
      };
      if (!p->graphs || p->timing) {
        for (int i = 0; i < nsteps; ++i) {
          if (ps_status st = one_step(p->stream)) return st;
          if ((i + 1) % every == 0 || i + 1 == nsteps)
            if (ps_status st = check(i + 1)) return st;
        }
        return PS_OK;
      }
      char key[256];
      snprintf(key, sizeof key, "%p|%d|%.17g|%.17g|%.17g|%p", state, (int)m, nu, eta, dt, p->ws);
      if (!p->gexec || p->gkey != key) {
        if (p->gexec) {
          hipGraphExecDestroy(p->gexec);
          p->gexec = nullptr;
        }
        hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        ps_status st = one_step(p->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p->cap, &g);
        if (st) {
          if (g) hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) {
          p->gexec = nullptr;
          return hip_fail(e, "hipGraphInstantiate");
        }
        p->gkey = key;
      }
      for (int i = 0; i < nsteps; ++i) {
        hipError_t e = hipGraphLaunch(p->gexec, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        if ((i + 1) % every == 0 || i + 1 == nsteps)
          if (ps_status st = check(i + 1)) return st;
      }
      return PS_OK;
    });
  });
}

ps_status ps_plan_set_monitor(ps_plan p, int every, double growth) {
  if (ps_status st = validate_plan(p)) return st;
  if (every < 0) return fail(PS_ERR_ARG, "every < 0");
  if (every > 0 && !(growth > 1.0 && std::isfinite(growth)))
    return fail(PS_ERR_ARG, "growth must be finite and > 1");
  p->mon_every = every;
  p->mon_growth = growth;
  return PS_OK;
}

ps_status ps_energy_spectrum_static(ps_plan p, const void* fhat, int nfields, double* spec_dev,
                                    double* totals_dev) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (nfields < 1 || nfields > p->nfields) return fail(PS_ERR_ARG, "nfields out of range");
    if (!p->scratch) return fail(PS_ERR_STATE, "the library scratch of this device was not set up");
    size_t nsh = 0;
    for (auto& b : p->boxes) {
      nsh += b.nshell;
      const size_t need = ((size_t)b.nz * b.nshell * 2 + b.nz) * sizeof(double);
      if (need > ps::SPEC_SCRATCH_BYTES) {
        char buf[200];
        snprintf(buf, sizeof buf, "box of %d x %d x %d needs %zu bytes of scratch; the library holds %zu",
                 b.nx, b.ny, b.nz, need, ps::SPEC_SCRATCH_BYTES);
        return fail(PS_ERR_SIZE, buf);
      }
    }
    const Class& lc = p->classes.back();
    if (ps_status st = check_dev(fhat, p->cplx_total * csize(p) - (size_t)(p->nfields - nfields) *
                                           lc.nc * csize(p), "fhat"))
      return st;
    if (ps_status st = check_dev(spec_dev, nsh * sizeof(double), "spec")) return st;
    if (ps_status st = check_dev(totals_dev, 3 * p->boxes.size() * sizeof(double), "totals")) return st;
    if (ps_status st = set_device(p)) return st;
    return by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      size_t so = 0;
      for (size_t i = 0; i < p->boxes.size(); ++i) {
        const Box& b = p->boxes[i];
        const Class& c = p->classes[b.cls];
        // boxes run one after another on the plan's stream, each reusing the
        // scratch after the previous box's last kernel has read it; every
        // entry is written before it is read, so nothing is cleared
        ps::SpecArgs<T> a{};
        a.f = (const ps::C2<T>*)fhat + b.cplx_off;
        a.part = p->scratch;
        a.pmax = a.part + (long)b.nz * b.nshell * 2;
        a.fs = c.nc; a.pitch = c.H; a.nx = b.nx; a.ny = b.ny; a.nz = b.nz; a.nf = nfields; a.nshell = b.nshell;
        a.sx = p->bs[0]; a.sy = p->bs[1]; a.sz = p->bs[2];
        const hipError_t e = ps::launch_spectrum<T>(a, false, spec_dev + so, totals_dev + 3 * i, p->stream);
        if (e != hipSuccess) return hip_fail(e, "spectrum (static scratch)");
        so += b.nshell;
      }
      return PS_OK;
    });
  });
}

ps_status ps_mhd_spectrum(ps_plan p, const void* zhat, double* spec_dev, double* totals_dev) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (p->nfields != 6) return fail(PS_ERR_ARG, "MHD diagnostics need a plan with nfields = 6");
    if (ps_status st = need_ws(p)) return st;
    size_t nsh = 0;
    for (auto& b : p->boxes) nsh += b.nshell;
    if (ps_status st = check_dev(zhat, p->cplx_total * csize(p), "zhat")) return st;
    if (ps_status st = check_dev(spec_dev, 3 * nsh * sizeof(double), "spec")) return st;
    if (ps_status st = check_dev(totals_dev, 3 * p->boxes.size() * sizeof(double), "totals")) return st;
    if (ps_status st = set_device(p)) return st;
    return by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      size_t so = 0;
      for (size_t i = 0; i < p->boxes.size(); ++i) {
        auto& b = p->boxes[i];
        Seq<T> q{p, p->classes[b.cls], 0, p->classes[b.cls].nb, p->stream};
        ps_status st = q.spectrum(b.idx, (const ps::C2<T>*)zhat + b.cplx_off, 6, true, spec_dev + 3 * so,
                                  totals_dev + 3 * i);
        if (st) return st;
        so += b.nshell;
      }
      return PS_OK;
    });
  });
}

ps_status ps_energy_spectrum(ps_plan p, const void* fhat, int nfields, double* spec_dev, double* totals_dev) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (nfields < 1 || nfields > p->nfields) return fail(PS_ERR_ARG, "nfields out of range");
    if (ps_status st = need_ws(p)) return st;
    size_t nsh = 0;
    for (auto& b : p->boxes) nsh += b.nshell;
    // the input holds nfields fields per box at the plan's box offsets
    const Class& lc = p->classes.back();
    if (ps_status st = check_dev(fhat, p->cplx_total * csize(p) - (size_t)(p->nfields - nfields) *
                                           lc.nc * csize(p), "fhat"))
      return st;
    if (ps_status st = check_dev(spec_dev, nsh * sizeof(double), "spec")) return st;
    if (ps_status st = check_dev(totals_dev, 3 * p->boxes.size() * sizeof(double), "totals")) return st;
    if (ps_status st = set_device(p)) return st;
    return by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      size_t so = 0;
      for (size_t i = 0; i < p->boxes.size(); ++i) {
        auto& b = p->boxes[i];
        Seq<T> q{p, p->classes[b.cls], 0, p->classes[b.cls].nb, p->stream};
        ps_status st = q.spectrum(b.idx, (const ps::C2<T>*)fhat + b.cplx_off, nfields, false, spec_dev + so,
                                  totals_dev + 3 * i);
        if (st) return st;
        so += b.nshell;
      }
      return PS_OK;
    });
  });
}

ps_status ps_plan_set_variant(ps_plan p, const char* kind, int v) {
  if (ps_status st = validate_plan(p)) return st;
  if (!kind) return fail(PS_ERR_ARG, "kind is NULL");
  bool known = false;
  for (const char* k : KINDS) known |= !strcmp(k, kind);
  if (!known) return fail(PS_ERR_ARG, std::string("unknown pass kind ") + kind);
  const int n = ps_plan_variant_count(p, kind);
  if (v < 0 || v >= n) return fail(PS_ERR_ARG, "variant out of range");
  p->var[kind] = v;
  p->per_box = var_of(p, "batch") == 1;
  p->prune = var_of(p, "prune") == 1;
  p->els = var_of(p, "form") == 1;
  if (p->gexec) {
    hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey.clear();
  }
  return PS_OK;
}

ps_status ps_plan_set_rotation(ps_plan p, double ox, double oy, double oz) {
  if (ps_status st = validate_plan(p)) return st;
  if (!std::isfinite(ox) || !std::isfinite(oy) || !std::isfinite(oz))
    return fail(PS_ERR_ARG, "rotation vector must be finite");
  p->omega[0] = ox;
  p->omega[1] = oy;
  p->omega[2] = oz;
  if (p->gexec) {  // the captured step holds the old coefficients
    hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey.clear();
  }
  return PS_OK;
}

ps_status ps_plan_set_box(ps_plan p, double Lx, double Ly, double Lz) {
  if (ps_status st = validate_plan(p)) return st;
  if (!(Lx > 0 && Ly > 0 && Lz > 0) || !std::isfinite(Lx) || !std::isfinite(Ly) || !std::isfinite(Lz))
    return fail(PS_ERR_ARG, "box lengths must be positive and finite");
  const double two_pi = 6.283185307179586476925286766559;
  p->bs[0] = two_pi / Lx;
  p->bs[1] = two_pi / Ly;
  p->bs[2] = two_pi / Lz;
  if (p->gexec) {
    hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->gkey.clear();
  }
  return PS_OK;
}

int ps_plan_get_variant(ps_plan p, const char* kind) {
  if (!p || !kind) return PS_ERR_ARG;
  return var_of(p, kind);
}

int ps_plan_variant_count(ps_plan p, const char* kind) {
  if (!p || !kind) return PS_ERR_ARG;
  if (!strcmp(kind, "batch") || !strcmp(kind, "prune")) return 2;
  if (!strcmp(kind, "form") || !strcmp(kind, "overlap")) return 2;
  if (!strcmp(kind, "pipe")) return NPIPE;
  int n = 1;
  for (auto& c : p->classes) n = std::max(n, ps::variant_count(kind, axis_len(c, kind), p->nfields == 6));
  return n;
}

ps_status ps_plan_autotune(ps_plan p, const void* state, ps_model m, int reps) {
  return guarded([&]() -> ps_status {
    if (ps_status st = validate_plan(p)) return st;
    if (m != PS_NS && m != PS_MHD) return fail(PS_ERR_ARG, "model must be PS_NS or PS_MHD");
    const bool mhd = m == PS_MHD;
    if (p->nfields != (mhd ? 6 : 3)) return fail(PS_ERR_ARG, "model does not match the plan's nfields");
    if (reps < 1) return fail(PS_ERR_ARG, "reps < 1");
    if (ps_status st = need_ws(p)) return st;
    if (ps_status st = check_dev(state, p->cplx_total * csize(p), "state")) return st;
    if (ps_status st = set_device(p)) return st;
    const std::string key = tune_key(p, mhd);
    if (tune_cache_lookup(p, key)) {
      p->tune_timed = 0;
      if (p->gexec) {
        hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
        p->gkey.clear();
      }
      return PS_OK;
    }
    int timed = 0;
    const bool timing = p->timing;
    p->timing = false;
    ps_status res = by_type(p, [&](auto* tag) -> ps_status {
      using T = std::remove_pointer_t<decltype(tag)>;
      size_t ci = 0;
      for (size_t i = 1; i < p->classes.size(); ++i)
        if (p->classes[i].n3 > p->classes[ci].n3) ci = i;
      const Class& b = p->classes[ci];
      Seq<T> q{p, b, 0, b.nb, p->stream};
      const auto* st = (const ps::C2<T>*)state + b.cplx_off;
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(PS_ERR_HIP, "hipEventCreate failed");
      ps_status out = PS_OK;
      // the passes are timed one at a time with the slab pipeline off (its
      // concurrent launches would blur the per-pass timings); the pipeline
      // setting is chosen afterwards on whole right-hand sides
      p->var["pipe"] = 0;
      // reps launches of variant v of `kind` (kind "pipe": right-hand sides)
      // between two events; ms = their time
      auto time_v = [&](const char* kind, int v, float& ms) -> ps_status {
        p->var[kind] = v;
        const char* launch = strcmp(kind, "pipe") ? kind : "step";
        ps_status o = PS_OK;
        hipEventRecord(e0, p->stream);
        for (int r = 0; r < reps && o == PS_OK; ++r, ++timed) o = q.tune_launch(launch, st, mhd);
        hipEventRecord(e1, p->stream);
        hipError_t e = hipEventSynchronize(e1);
        ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess && o == PS_OK) o = hip_fail(e, "autotune timing");
        return o;
      };
      for (const char* kind : TUNED) {
        const int n = strcmp(kind, "pipe") ? ps::variant_count(kind, axis_len(b, kind), mhd) : NPIPE;
        if (n <= 1) continue;
        // every variant once (after a warm-up launch), then the ones within
        // 10 % of the fastest again in FINAL interleaved rounds, each keeping
        // its best time: variants a few per cent apart are otherwise ranked
        // by clock and thermal drift over the sequence
        constexpr int FINAL = 3;
        std::vector<float> best_ms(n, 1e30f);
        for (int v = 0; v < n && out == PS_OK; ++v) {
          // pipeline settings whose slabs run concurrently on helper streams
          // are not considered (per-kernel timings of overlapping launches
          // would mean nothing), except the two-chain settings when the
          // caller has asked for them ("overlap" 1)
          if (!strcmp(kind, "pipe") && pipe_shape(v).streams != 0 &&
              !(var_of(p, "overlap") == 1 && v >= PIPE_TWO))
            continue;
          p->var[kind] = v;
          if ((out = q.tune_launch(strcmp(kind, "pipe") ? kind : "step", st, mhd))) break;  // warm-up
          out = time_v(kind, v, best_ms[v]);
        }
        const float first = *std::min_element(best_ms.begin(), best_ms.end());
        std::vector<int> fin;
        for (int v = 0; v < n; ++v)
          if (best_ms[v] <= 1.10f * first) fin.push_back(v);
        for (int r = 0; r < FINAL && fin.size() > 1 && out == PS_OK; ++r)
          for (size_t i = 0; i < fin.size() && out == PS_OK; ++i) {
            const int v = fin[(i + r) % fin.size()];
            float ms = 0;
            if ((out = time_v(kind, v, ms)) == PS_OK) best_ms[v] = std::min(best_ms[v], ms);
          }
        p->var[kind] = (int)(std::min_element(best_ms.begin(), best_ms.end()) - best_ms.begin());
        if (out) break;
      }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      return out;
    });
    p->timing = timing;
    p->tune_timed = timed;
    if (p->gexec) {
      hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
      p->gkey.clear();
    }
    if (res == PS_OK) tune_cache_store(p, key);
    return res;
  });
}

int ps_plan_autotune_timed(ps_plan p) {
  if (!p) return PS_ERR_ARG;
  return p->tune_timed;
}

ps_status ps_plan_set_timing(ps_plan p, int enable) {
  if (ps_status st = validate_plan(p)) return st;
  p->timing = enable != 0;
  return PS_OK;
}

ps_status ps_plan_set_graphs(ps_plan p, int enable) {
  if (ps_status st = validate_plan(p)) return st;
  p->graphs = enable != 0;
  return PS_OK;
}

ps_status ps_plan_timing_reset(ps_plan p) {
  if (ps_status st = validate_plan(p)) return st;
  ps_status st = sync_timing(p);
  p->stats.clear();
  p->kind_index.clear();
  return st;
}

int ps_plan_timing_count(ps_plan p) {
  if (!p) return PS_ERR_ARG;
  if (ps_status st = sync_timing(p)) return st;
  return (int)p->stats.size();
}

ps_status ps_plan_timing_get(ps_plan p, int idx, const char** name, double* total_ms, long* launches,
                             double* bytes_per_launch) {
  if (ps_status st = validate_plan(p)) return st;
  if (ps_status st = sync_timing(p)) return st;
  if (idx < 0 || idx >= (int)p->stats.size()) return fail(PS_ERR_ARG, "timing index out of range");
  const KindStat& k = p->stats[idx];
  if (name) *name = k.name.c_str();
  if (total_ms) *total_ms = k.ms;
  if (launches) *launches = k.launches;
  if (bytes_per_launch) *bytes_per_launch = k.launches ? k.bytes / (double)k.launches : 0.0;
  return PS_OK;
}

}  // extern "C"
