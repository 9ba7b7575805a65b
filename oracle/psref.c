/*
 * psref.c -- FP64 CPU oracle for the pseudospectral Navier-Stokes / MHD step.
 *
 * TEST INFRASTRUCTURE: see psref.h.  Written for a reader checking it against
 * the paper by eye: no blocking, fusion or reordering beyond what each
 * definition states.  Loops over pencils and planes are threaded with OpenMP
 * one loop level at a time, the loop-level threading the paper describes in
 * Sec. 3; the threading never changes a result.
 *
 * A compile-time switch PSREF_MUTANT=n (n > 0) plants one deliberate mistake
 * per n.  It exists only so the test suite can show that its pins catch
 * plausible mistakes; the default build (PSREF_MUTANT undefined or 0) has
 * none of them.
 */
#include "psref.h"

#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef PSREF_MUTANT
#define PSREF_MUTANT 0
#endif
#ifndef PSREF_SRC_HASH
#define PSREF_SRC_HASH "unknown"
#endif

/* hash of the sources this build was compiled from (set by the build step) */
const char *psref_build_hash(void) { return PSREF_SRC_HASH; }
#define MUT(n) (PSREF_MUTANT == (n))

typedef double complex cplx;

static const double TWO_PI = 6.28318530717958647692528676655900577;

/* ------------------------------------------------------------------------ */
/* Index conventions (Sec. 2, Fig. 1: a real nx x ny x nz grid, and its half */
/* spectrum (nx/2+1) x ny x nz after the real-to-complex transform; the     */
/* paper's cube is nx = ny = nz = N).                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  long nx, ny, nz;
  long H;   /* nx/2 + 1 kx values        */
  long nc;  /* nz ny H modes per field   */
  long n3;  /* nz ny nx points per field */
} grid;

static grid grid_of(int nx, int ny, int nz) {
  grid g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.H = nx / 2 + 1;
  g.nc = (long)nz * ny * g.H;
  g.n3 = (long)nz * ny * nx;
  return g;
}

/* signed wavenumber of storage index i along ky or kz (axis length N) */
static long wav(long i, long N) { return (i < N / 2) ? i : i - N; }

/* derivative wavenumber: odd derivatives of the Nyquist mode are zero */
static long dwav(long i, long N) {
  if (MUT(9)) return wav(i, N);
  return (2 * i == N) ? 0 : wav(i, N);
}

/* kx storage index -> wavenumber (kx = 0..nx/2) */
static long wavx(long i) { return i; }
static long dwavx(long i, long N) {
  if (MUT(9)) return i;
  return (2 * i == N) ? 0 : i;
}

/* Box lengths.  Sec. 5 notes the method works for boxes whose aspect ratio
 * is not unity; a box of lengths L has physical wavenumbers k = (2 pi / L) n
 * for the signed index n, so every derivative, the projector and |k|^2 in
 * the viscous and diagnostic terms carry the factors s = 2 pi / L.  The 2/3
 * rule stays on the index n: aliasing belongs to the grid, not the lengths.
 * Default: the 2 pi-periodic cube (s = 1). */
static double g_s[3] = {1.0, 1.0, 1.0};

int psref_set_box(double Lx, double Ly, double Lz) {
  if (!(Lx > 0 && Ly > 0 && Lz > 0) || !isfinite(Lx) || !isfinite(Ly) || !isfinite(Lz)) return -1;
  g_s[0] = TWO_PI / Lx;
  g_s[1] = TWO_PI / Ly;
  g_s[2] = TWO_PI / Lz;
  return 0;
}

/* 2/3-rule dealiasing as a truncation on the index n: keep
 *   (3 nx' / nx)^2 + (3 ny' / ny)^2 + (3 nz' / nz)^2 < 1,
 * the sphere 9 |n|^2 < N^2 of the cube, stretched with the grid (each axis
 * then keeps |n_a| < N_a / 3, the per-axis 2/3 rule).  Evaluated exactly in
 * integers after multiplying by (nx ny nz)^2 (128-bit: up to 2^76). */
static int dealias_keep(const grid *g, long ix, long iy, long iz) {
  typedef __int128 i128;
  const i128 X = g->nx, Y = MUT(17) ? g->nx : g->ny, Z = MUT(17) ? g->nx : g->nz;
  const i128 lhs = 9 * ((i128)ix * ix * Y * Y * Z * Z + (i128)iy * iy * X * X * Z * Z +
                        (i128)iz * iz * X * X * Y * Y);
  const i128 rhs = X * X * Y * Y * Z * Z;
  if (MUT(3)) return lhs <= rhs;
  return lhs < rhs;
}

/* ------------------------------------------------------------------------ */
/* One-dimensional DFT by recursive mixed-radix decimation in time.          */
/*   X[k] = sum_j x[j] exp(-+ 2 pi i j k / n)                                */
/* n = p m with p the smallest prime factor; x[r + p j] gives p sub-DFTs of  */
/* length m, combined as X[k] = sum_r W_n^{r k} Y_r[k mod m].                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int n;
  cplx *w; /* w[e] = exp(-2 pi i e / n), computed in FP64 */
} line_plan;

static int line_plan_init(line_plan *p, int n) {
  p->n = n;
  p->w = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  if (!p->w) return -3;
  for (int e = 0; e < n; ++e) {
    double a = TWO_PI * (double)e / (double)n;
    p->w[e] = cos(a) - I * sin(a);
  }
  return 0;
}

static void line_plan_free(line_plan *p) { free(p->w); p->w = NULL; }

static int smallest_factor(int n) {
  for (int p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

/* t: scratch of at least n entries, shared by all recursion levels (each
 * level combines only after its sub-transforms have returned) */
static void fft_rec(const line_plan *pl, int n, const cplx *x, long stride,
                    cplx *X, cplx *t, int inverse) {
  if (n == 1) {
    X[0] = x[0];
    return;
  }
  int p = smallest_factor(n), m = n / p;
  for (int r = 0; r < p; ++r)
    fft_rec(pl, m, x + (long)r * stride, stride * p, X + (long)r * m, t, inverse);
  int scale = pl->n / n;
  for (int q = 0; q < p; ++q) {
    for (int k = 0; k < m; ++k) {
      int kk = k + q * m;
      cplx s = 0;
      for (int r = 0; r < p; ++r) {
        long e = ((long)r * kk) % n;
        cplx w = pl->w[e * scale];
        if (inverse && !MUT(8)) w = conj(w);
        s += w * X[(long)r * m + k];
      }
      t[kk] = s;
    }
  }
  memcpy(X, t, sizeof(cplx) * (size_t)n);
}

/* in and out are separate buffers of length pl->n */
static void line_fft(const line_plan *pl, const cplx *in, cplx *out, int inverse) {
  cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)pl->n);
  fft_rec(pl, pl->n, in, 1, out, t, inverse);
  free(t);
}

/* one line plan per axis */
typedef struct {
  line_plan x, y, z;
} plans;

static int plans_init(plans *p, const grid *g) {
  p->x.w = p->y.w = p->z.w = NULL;
  if (line_plan_init(&p->x, (int)g->nx) || line_plan_init(&p->y, (int)g->ny) ||
      line_plan_init(&p->z, (int)g->nz)) {
    free(p->x.w);
    free(p->y.w);
    free(p->z.w);
    return -3;
  }
  return 0;
}

static void plans_free(plans *p) {
  line_plan_free(&p->x);
  line_plan_free(&p->y);
  line_plan_free(&p->z);
}

/* ------------------------------------------------------------------------ */
/* Three-dimensional real transforms (Sec. 2, Fig. 1): transforms along x,   */
/* then y, then z for the forward direction; the reverse for the inverse.    */
/* ------------------------------------------------------------------------ */

static int size_ok(int N) { return N >= 2 && N <= 4096 && (N % 2) == 0; }
static int grid_ok(int nx, int ny, int nz) { return size_ok(nx) && size_ok(ny) && size_ok(nz); }

/* complex transforms along y (or z) of one half-spectrum field */
static void pass_y(const line_plan *pl, const grid *g, cplx *X, int inverse) {
  const long H = g->H, ny = g->ny;
#pragma omp parallel
  {
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
    cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)ny);
#pragma omp for schedule(static)
    for (long zk = 0; zk < g->nz * H; ++zk) {
      long z = zk / H, kx = zk % H;
      for (long y = 0; y < ny; ++y) a[y] = X[(z * ny + y) * H + kx];
      line_fft(pl, a, b, inverse);
      for (long y = 0; y < ny; ++y) X[(z * ny + y) * H + kx] = b[y];
    }
    free(a);
    free(b);
  }
}

static void pass_z(const line_plan *pl, const grid *g, cplx *X, int inverse) {
  const long H = g->H, ny = g->ny, nz = g->nz;
#pragma omp parallel
  {
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)nz);
    cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)nz);
#pragma omp for schedule(static)
    for (long yk = 0; yk < ny * H; ++yk) {
      long ky = yk / H, kx = yk % H;
      for (long z = 0; z < nz; ++z) a[z] = X[(z * ny + ky) * H + kx];
      line_fft(pl, a, b, inverse);
      for (long z = 0; z < nz; ++z) X[(z * ny + ky) * H + kx] = b[z];
    }
    free(a);
    free(b);
  }
}

static void r2c_field(const plans *pl, const grid *g, const double *u, cplx *X) {
  const long H = g->H, nx = g->nx;
#pragma omp parallel
  {
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
    cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
#pragma omp for schedule(static)
    for (long row = 0; row < g->ny * g->nz; ++row) {
      for (long x = 0; x < nx; ++x) a[x] = u[row * nx + x];
      line_fft(&pl->x, a, b, 0);
      for (long kx = 0; kx < H; ++kx) X[row * H + kx] = b[kx];
    }
    free(a);
    free(b);
  }
  pass_y(&pl->y, g, X, 0);
  pass_z(&pl->z, g, X, 0);
}

/* Y is overwritten (used as the z/y-transformed intermediate) */
static void c2r_field_inplace(const plans *pl, const grid *g, cplx *Y, double *u) {
  const long H = g->H, nx = g->nx;
  pass_z(&pl->z, g, Y, 1);
  pass_y(&pl->y, g, Y, 1);
#pragma omp parallel
  {
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
    cplx *b = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
#pragma omp for schedule(static)
    for (long row = 0; row < g->ny * g->nz; ++row) {
      const cplx *y = Y + row * H;
      /* Hermitian extension of the kx line; the imaginary parts of the
       * kx = 0 and kx = nx/2 bins are dropped */
      a[0] = creal(y[0]);
      for (long k = 1; k < nx / 2; ++k) {
        a[k] = y[k];
        a[nx - k] = conj(y[k]);
      }
      a[nx / 2] = creal(y[nx / 2]);
      line_fft(&pl->x, a, b, 1);
      for (long x = 0; x < nx; ++x) u[row * nx + x] = creal(b[x]);
    }
    free(a);
    free(b);
  }
}

int psref_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int psref_fft_r2c(int nx, int ny, int nz, int nf, const double *in, double *out) {
  if (!in || !out || nf < 1) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  plans pl;
  if (plans_init(&pl, &g)) return -3;
  for (int f = 0; f < nf; ++f)
    r2c_field(&pl, &g, in + f * g.n3, (cplx *)out + f * g.nc);
  plans_free(&pl);
  return 0;
}

int psref_fft_c2r(int nx, int ny, int nz, int nf, const double *in, double *out) {
  if (!in || !out || nf < 1) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (size_t)g.nc);
  if (!Y) return -3;
  plans pl;
  if (plans_init(&pl, &g)) { free(Y); return -3; }
  for (int f = 0; f < nf; ++f) {
    memcpy(Y, (const cplx *)in + f * g.nc, sizeof(cplx) * (size_t)g.nc);
    c2r_field_inplace(&pl, &g, Y, out + f * g.n3);
  }
  plans_free(&pl);
  free(Y);
  return 0;
}

int psref_dft_at(int nx, int ny, int nz, const double *in, int nk, const int *kx, const int *ky,
                 const int *kz, double *out) {
  if (!in || !out || nk < 0 || (nk > 0 && (!kx || !ky || !kz))) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  for (int i = 0; i < nk; ++i)
    if (kx[i] < 0 || kx[i] > nx / 2 || ky[i] < 0 || ky[i] >= ny || kz[i] < 0 || kz[i] >= nz)
      return -1;
  const grid g = grid_of(nx, ny, nz);
  plans pl;
  if (plans_init(&pl, &g)) return -3;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < nk; ++i) {
    cplx s = 0;
    for (long z = 0; z < nz; ++z)
      for (long y = 0; y < ny; ++y)
        for (long x = 0; x < nx; ++x) {
          cplx w = pl.x.w[((long)kx[i] * x) % nx] * pl.y.w[((long)ky[i] * y) % ny] *
                   pl.z.w[((long)kz[i] * z) % nz];
          s += in[(z * ny + y) * nx + x] * w;
        }
    out[2 * i] = creal(s);
    out[2 * i + 1] = cimag(s);
  }
  plans_free(&pl);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Spectral operators (Sec. 2: derivatives in Fourier space; projection onto */
/* divergence-free fields; dealiasing of the quadratic term).                */
/* ------------------------------------------------------------------------ */

/* w = i k_d x u for one 3-vector field set of nc modes each */
static void curl_fields(const grid *g, const cplx *u, cplx *w) {
  const long H = g->H, nc = g->nc, ny = g->ny;
#pragma omp parallel for schedule(static)
  for (long kz = 0; kz < g->nz; ++kz)
    for (long ky = 0; ky < ny; ++ky)
      for (long kx = 0; kx < H; ++kx) {
        long m = (kz * ny + ky) * H + kx;
        const double *sc = MUT(16) ? (const double[3]){1, 1, 1} : g_s;
        double ax = sc[0] * dwavx(kx, g->nx), ay = sc[1] * dwav(ky, ny), az = sc[2] * dwav(kz, g->nz);
        cplx ux = u[m], uy = u[nc + m], uz = u[2 * nc + m];
        w[m] = I * (ay * uz - az * uy);
        w[nc + m] = I * (az * ux - ax * uz);
        w[2 * nc + m] = I * (ax * uy - ay * ux);
        if (MUT(1)) w[nc + m] = -w[nc + m];
      }
}

int psref_curl(int nx, int ny, int nz, const double *uhat, double *what) {
  if (!uhat || !what) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  curl_fields(&g, (const cplx *)uhat, (cplx *)what);
  return 0;
}

/* v <- D(k) P(k) v / (nx ny nz) for a 3-vector field set (P(0) v := 0) */
static void dealias_project(const grid *g, cplx *v) {
  const long H = g->H, nc = g->nc, ny = g->ny;
  const double inv = 1.0 / (double)g->n3;
#pragma omp parallel for schedule(static)
  for (long kz = 0; kz < g->nz; ++kz)
    for (long ky = 0; ky < ny; ++ky)
      for (long kx = 0; kx < H; ++kx) {
        long m = (kz * ny + ky) * H + kx;
        long ix = wavx(kx), iy = wav(ky, ny), iz = wav(kz, g->nz);
        long k2 = ix * ix + iy * iy + iz * iz;
        if (k2 == 0 || !dealias_keep(g, ix, iy, iz)) {
          v[m] = v[nc + m] = v[2 * nc + m] = 0;
          continue;
        }
        double ax = g_s[0] * ix, ay = g_s[1] * iy, az = g_s[2] * iz;
        double q2 = ax * ax + ay * ay + az * az;  /* physical |k|^2 */
        cplx vx = v[m], vy = v[nc + m], vz = v[2 * nc + m];
        cplx kv = ax * vx + ay * vy + az * vz;
        if (MUT(2)) kv = 0;
        double s = MUT(6) ? 1.0 : inv;
        v[m] = s * (vx - ax * kv / q2);
        v[nc + m] = s * (vy - ay * kv / q2);
        v[2 * nc + m] = s * (vz - az * kv / q2);
      }
}

/* n = a x b pointwise on real fields (3 components each) */
static void cross_real(long n3, const double *a, const double *b, double *n) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < n3; ++i) {
    double ax = a[i], ay = a[n3 + i], az = a[2 * n3 + i];
    double bx = b[i], by = b[n3 + i], bz = b[2 * n3 + i];
    n[i] = ay * bz - az * by;
    n[n3 + i] = az * bx - ax * bz;
    n[2 * n3 + i] = ax * by - ay * bx;
  }
}

/* c2r of a 3-field spectral set (input preserved) */
static int c2r3(const plans *pl, const grid *g, const cplx *in, double *out, cplx *tmp) {
  for (int f = 0; f < 3; ++f) {
    memcpy(tmp, in + f * g->nc, sizeof(cplx) * (size_t)g->nc);
    c2r_field_inplace(pl, g, tmp, out + f * g->n3);
  }
  return 0;
}

static void r2c3(const plans *pl, const grid *g, const double *in, cplx *out) {
  for (int f = 0; f < 3; ++f) r2c_field(pl, g, in + f * g->n3, out + f * g->nc);
}

static int nonlinear_ns(const grid *g, const cplx *uhat, cplx *nhat) {
  const long n3 = g->n3, nc = g->nc;
  cplx *what = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nc);
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)nc);
  double *u = (double *)malloc(sizeof(double) * 3 * (size_t)n3);
  double *w = (double *)malloc(sizeof(double) * 3 * (size_t)n3);
  plans pl;
  int rc = 0;
  if (!what || !tmp || !u || !w || plans_init(&pl, g)) {
    rc = -3;
    goto done;
  }
  curl_fields(g, uhat, what);               /* w^ = i k x u^            */
  c2r3(&pl, g, uhat, u, tmp);               /* u(x)                      */
  c2r3(&pl, g, what, w, tmp);               /* w(x)                      */
  if (MUT(10))
    cross_real(n3, w, u, u);                /* planted: operands swapped */
  else
    cross_real(n3, u, w, u);                /* u x w, written over u     */
  r2c3(&pl, g, u, nhat);                    /* F[u x w]                  */
  dealias_project(g, nhat);                 /* D P (.) / (nx ny nz)      */
  plans_free(&pl);
done:
  free(what);
  free(tmp);
  free(u);
  free(w);
  return rc;
}

int psref_nonlinear_ns(int nx, int ny, int nz, const double *uhat, double *nhat) {
  if (!uhat || !nhat) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  return nonlinear_ns(&g, (const cplx *)uhat, (cplx *)nhat);
}

static int nonlinear_mhd(const grid *g, const cplx *zp, cplx *np_) {
  const long H = g->H, n3 = g->n3, nc = g->nc, ny = g->ny;
  const cplx *zm = zp + 3 * nc;
  cplx *nm = np_ + 3 * nc;
  cplx *uh = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nc);
  cplx *bh = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nc);
  cplx *sh = (cplx *)malloc(sizeof(cplx) * 3 * (size_t)nc);
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)nc);
  double *u = (double *)malloc(sizeof(double) * 3 * (size_t)n3);
  double *b = (double *)malloc(sizeof(double) * 3 * (size_t)n3);
  double *w = (double *)malloc(sizeof(double) * 3 * (size_t)n3);
  double *j = (double *)malloc(sizeof(double) * 3 * (size_t)n3);
  plans pl;
  int rc = 0;
  if (!uh || !bh || !sh || !tmp || !u || !b || !w || !j || plans_init(&pl, g)) {
    rc = -3;
    goto done;
  }
  /* primitive variables u = (z+ + z-)/2, b = (z+ - z-)/2 */
  for (long m = 0; m < 3 * nc; ++m) {
    uh[m] = 0.5 * (zp[m] + zm[m]);
    bh[m] = 0.5 * (zp[m] - zm[m]);
  }
  c2r3(&pl, g, uh, u, tmp);
  c2r3(&pl, g, bh, b, tmp);
  curl_fields(g, uh, sh);                   /* w^ = i k x u^ */
  c2r3(&pl, g, sh, w, tmp);
  curl_fields(g, bh, sh);                   /* j^ = i k x b^ */
  c2r3(&pl, g, sh, j, tmp);
  /* Lorentz + advection part: u x w + j x b  (into w), induction e = u x b (into u) */
  cross_real(n3, u, w, w);
  cross_real(n3, j, b, j);
  for (long i = 0; i < 3 * n3; ++i) w[i] += j[i];
  cross_real(n3, u, b, u);
  r2c3(&pl, g, w, uh);                      /* F[u x w + j x b] */
  r2c3(&pl, g, u, bh);                      /* F[u x b]         */
  dealias_project(g, uh);                   /* D P (.) / (nx ny nz) */
  curl_fields(g, bh, sh);                   /* i k x F[u x b]   */
  {
    const double inv = 1.0 / (double)n3;
#pragma omp parallel for schedule(static)
    for (long kz = 0; kz < g->nz; ++kz)
      for (long ky = 0; ky < ny; ++ky)
        for (long kx = 0; kx < H; ++kx) {
          long m = (kz * ny + ky) * H + kx;
          long ix = wavx(kx), iy = wav(ky, ny), iz = wav(kz, g->nz);
          double d = dealias_keep(g, ix, iy, iz) ? inv : 0.0;
          double sg = MUT(7) ? -1.0 : 1.0;
          for (int c = 0; c < 3; ++c) {
            cplx a = uh[c * nc + m], e = d * sh[c * nc + m];
            np_[c * nc + m] = a + sg * e;
            nm[c * nc + m] = a - sg * e;
          }
        }
  }
  plans_free(&pl);
done:
  free(uh);
  free(bh);
  free(sh);
  free(tmp);
  free(u);
  free(b);
  free(w);
  free(j);
  return rc;
}

int psref_nonlinear_mhd(int nx, int ny, int nz, const double *zhat, double *nhat) {
  if (!zhat || !nhat) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  return nonlinear_mhd(&g, (const cplx *)zhat, (cplx *)nhat);
}

/* ------------------------------------------------------------------------ */
/* Galerkin triad sum: the dealiased quadratic term as the convolution of    */
/* Fourier coefficients, N(k) = D P sum_{p+q=k} u(p) x (i q x u(q)).  For a  */
/* dealiased input no alias reaches a kept mode, so this equals the          */
/* pseudospectral value there.                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  long K[3];     /* half-widths: |k_a| <= K[a] */
  long side[3];  /* 2K+1 */
  cplx *v;       /* [f][kz][ky][kx] over the box, full spectrum */
} full_cube;

/* effective full-spectrum coefficient seen by the inverse transform: the kx = 0
 * and kx = nx/2 planes are used through their Hermitian part */
static cplx eff_coef(const grid *g, const cplx *F, long ix, long iy, long iz) {
  const long H = g->H, ny = g->ny, nz = g->nz;
  long sx = ix < 0 ? -ix : ix;
  long syi, szi, myi, mzi;
  if (ix < 0) { iy = -iy; iz = -iz; }
  syi = (iy % ny + ny) % ny;
  szi = (iz % nz + nz) % nz;
  myi = ((-iy) % ny + ny) % ny;
  mzi = ((-iz) % nz + nz) % nz;
  cplx a = F[(szi * ny + syi) * H + sx];
  if (sx == 0 || 2 * sx == g->nx) {
    cplx b = F[(mzi * ny + myi) * H + sx];
    a = 0.5 * (a + conj(b));
  }
  return ix < 0 ? conj(a) : a;
}

static size_t cube_index(const full_cube *c, int f, long ix, long iy, long iz) {
  return (((size_t)f * c->side[2] + (iz + c->K[2])) * c->side[1] + (iy + c->K[1])) * c->side[0] +
         (ix + c->K[0]);
}

static int cube_build(const grid *g, int nf, const cplx *F, full_cube *c) {
  const long H = g->H, nc = g->nc, ny = g->ny, nz = g->nz;
  long K[3] = {0, 0, 0};
  for (int f = 0; f < nf; ++f)
    for (long kz = 0; kz < nz; ++kz)
      for (long ky = 0; ky < ny; ++ky)
        for (long kx = 0; kx < H; ++kx) {
          cplx a = F[f * nc + (kz * ny + ky) * H + kx];
          if (a != 0) {
            if (kx > K[0]) K[0] = kx;
            if (labs(wav(ky, ny)) > K[1]) K[1] = labs(wav(ky, ny));
            if (labs(wav(kz, nz)) > K[2]) K[2] = labs(wav(kz, nz));
          }
        }
  /* content at Nyquist indices is outside the Galerkin set and ignored */
  const long n[3] = {g->nx, ny, nz};
  size_t cnt = (size_t)nf;
  for (int a = 0; a < 3; ++a) {
    if (K[a] > n[a] / 2 - 1) K[a] = n[a] / 2 - 1;
    c->K[a] = K[a];
    c->side[a] = 2 * K[a] + 1;
    cnt *= (size_t)c->side[a];
  }
  c->v = (cplx *)calloc(cnt, sizeof(cplx));
  if (!c->v) return -3;
  for (int f = 0; f < nf; ++f)
    for (long iz = -K[2]; iz <= K[2]; ++iz)
      for (long iy = -K[1]; iy <= K[1]; ++iy)
        for (long ix = -K[0]; ix <= K[0]; ++ix)
          c->v[cube_index(c, f, ix, iy, iz)] = eff_coef(g, F + f * nc, ix, iy, iz);
  return 0;
}

static int cube_has(const full_cube *c, long ix, long iy, long iz) {
  return labs(ix) <= c->K[0] && labs(iy) <= c->K[1] && labs(iz) <= c->K[2];
}

static cplx cube_at(const full_cube *c, int f, long ix, long iy, long iz) {
  return cube_has(c, ix, iy, iz) ? c->v[cube_index(c, f, ix, iy, iz)] : 0;
}

static void cross_c(const cplx a[3], const cplx b[3], cplx o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* i q x v with the derivative wavenumber (Nyquist components zero) */
static void icurl_c(const grid *g, long qx, long qy, long qz, const cplx v[3], cplx o[3]) {
  double ax = (2 * labs(qx) == g->nx) ? 0.0 : g_s[0] * qx;
  double ay = (2 * labs(qy) == g->ny) ? 0.0 : g_s[1] * qy;
  double az = (2 * labs(qz) == g->nz) ? 0.0 : g_s[2] * qz;
  o[0] = I * (ay * v[2] - az * v[1]);
  o[1] = I * (az * v[0] - ax * v[2]);
  o[2] = I * (ax * v[1] - ay * v[0]);
}

int psref_nonlinear_at(int nx, int ny, int nz, int model, const double *fhat, int nk,
                       const int *kx, const int *ky, const int *kz, double *out) {
  if (!fhat || !out || nk < 0 || (nk > 0 && (!kx || !ky || !kz))) return -1;
  if (model != 0 && model != 1) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  for (int i = 0; i < nk; ++i)
    if (kx[i] < 0 || kx[i] > nx / 2 || ky[i] < 0 || ky[i] >= ny || kz[i] < 0 || kz[i] >= nz)
      return -1;
  const grid g = grid_of(nx, ny, nz);
  const int nf = model == 0 ? 3 : 6;
  full_cube c;
  if (cube_build(&g, nf, (const cplx *)fhat, &c)) return -3;
  const long *K = c.K;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < nk; ++i) {
    long ox = kx[i], oy = wav(ky[i], ny), oz = wav(kz[i], nz);
    cplx accL[3] = {0, 0, 0}, accE[3] = {0, 0, 0};
    /* the sum runs plane by plane in pz (each plane's terms summed on their
     * own, then the plane sums added), so that its rounding stays near
     * eps sqrt(terms per plane) even for the ~10^8 triads of a large grid */
    for (long pz = -K[2]; pz <= K[2]; ++pz) {
      cplx plL[3] = {0, 0, 0}, plE[3] = {0, 0, 0};
      for (long py = -K[1]; py <= K[1]; ++py)
        for (long px = -K[0]; px <= K[0]; ++px) {
          long qx = ox - px, qy = oy - py, qz = oz - pz;
          if (!cube_has(&c, qx, qy, qz)) continue;
          if (model == 0) {
            cplx up[3], uq[3], wq[3], t[3];
            for (int f = 0; f < 3; ++f) {
              up[f] = cube_at(&c, f, px, py, pz);
              uq[f] = cube_at(&c, f, qx, qy, qz);
            }
            if (up[0] == 0 && up[1] == 0 && up[2] == 0) continue;
            icurl_c(&g, qx, qy, qz, uq, wq);
            cross_c(up, wq, t);
            for (int f = 0; f < 3; ++f) plL[f] += t[f];
          } else {
            cplx up[3], bp[3], uq[3], bq[3], wq[3], jp[3], t1[3], t2[3], t3[3];
            for (int f = 0; f < 3; ++f) {
              cplx zpp = cube_at(&c, f, px, py, pz), zmp = cube_at(&c, 3 + f, px, py, pz);
              cplx zpq = cube_at(&c, f, qx, qy, qz), zmq = cube_at(&c, 3 + f, qx, qy, qz);
              up[f] = 0.5 * (zpp + zmp);
              bp[f] = 0.5 * (zpp - zmp);
              uq[f] = 0.5 * (zpq + zmq);
              bq[f] = 0.5 * (zpq - zmq);
            }
            icurl_c(&g, qx, qy, qz, uq, wq);  /* w(q) */
            icurl_c(&g, px, py, pz, bp, jp);  /* j(p) */
            cross_c(up, wq, t1);              /* u(p) x w(q) */
            cross_c(jp, bq, t2);              /* j(p) x b(q) */
            cross_c(up, bq, t3);              /* u(p) x b(q) */
            for (int f = 0; f < 3; ++f) {
              plL[f] += t1[f] + t2[f];
              plE[f] += t3[f];
            }
          }
        }
      for (int f = 0; f < 3; ++f) {
        accL[f] += plL[f];
        accE[f] += plE[f];
      }
    }
    long k2 = ox * ox + oy * oy + oz * oz;
    cplx res[6] = {0, 0, 0, 0, 0, 0};
    if (k2 != 0 && dealias_keep(&g, ox, oy, oz)) {
      double ax = g_s[0] * ox, ay = g_s[1] * oy, az = g_s[2] * oz;
      double q2 = ax * ax + ay * ay + az * az;
      cplx kv = ax * accL[0] + ay * accL[1] + az * accL[2];
      cplx pl_[3] = {accL[0] - ax * kv / q2, accL[1] - ay * kv / q2, accL[2] - az * kv / q2};
      if (model == 0) {
        for (int f = 0; f < 3; ++f) res[f] = pl_[f];
      } else {
        cplx ce[3];
        icurl_c(&g, ox, oy, oz, accE, ce);
        for (int f = 0; f < 3; ++f) {
          res[f] = pl_[f] + ce[f];
          res[3 + f] = pl_[f] - ce[f];
        }
      }
    }
    for (int f = 0; f < nf; ++f) {
      out[2 * ((long)i * nf + f)] = creal(res[f]);
      out[2 * ((long)i * nf + f) + 1] = cimag(res[f]);
    }
  }
  free(c.v);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Time advance.  The paper times a time-advance loop (Sec. 4) without      */
/* naming its integrator; the explicit midpoint second-order Runge-Kutta    */
/* method is used:                                                           */
/*   z* = z^n + (dt/2) F(z^n),   z^{n+1} = z^n + dt F(z*)                    */
/* F(u) = N(u) - nu |k|^2 u (NS);  for MHD in Elsasser variables             */
/* F(z+-) = N+-(z) - (nu+eta)/2 |k|^2 z+- - (nu-eta)/2 |k|^2 z-+.            */
/* Rotation (Sec. 5 says the code includes it; no equation is given): in a   */
/* frame rotating at Omega the momentum equation gains the Coriolis         */
/* acceleration -2 Omega x u, the centrifugal part going into the pressure; */
/* projected like every other term, P(k) at k = 0 read as 0, applied to     */
/* every mode (a linear term, like the viscous one).  For MHD it acts on    */
/* u = (z+ + z-)/2 and so enters both Elsasser equations; b is untouched.   */
/* ------------------------------------------------------------------------ */

/* F -= P(k) (2 Omega x u) at every mode, u the velocity of state z */
static void coriolis(const grid *g, int model, const cplx *z, cplx *F, const double *om) {
  const long H = g->H, nc = g->nc, ny = g->ny;
  const double f = MUT(14) ? 1.0 : 2.0;
#pragma omp parallel for schedule(static)
  for (long kz = 0; kz < g->nz; ++kz)
    for (long ky = 0; ky < ny; ++ky)
      for (long kx = 0; kx < H; ++kx) {
        long m = (kz * ny + ky) * H + kx;
        long ix = wavx(kx), iy = wav(ky, ny), iz = wav(kz, g->nz);
        long k2 = ix * ix + iy * iy + iz * iz;
        if (k2 == 0) continue;
        cplx u[3];
        for (int c = 0; c < 3; ++c)
          u[c] = model == 0 ? z[c * nc + m] : 0.5 * (z[c * nc + m] + z[(3 + c) * nc + m]);
        cplx a[3] = {f * (om[1] * u[2] - om[2] * u[1]), f * (om[2] * u[0] - om[0] * u[2]),
                     f * (om[0] * u[1] - om[1] * u[0])};
        double kk[3] = {g_s[0] * ix, g_s[1] * iy, g_s[2] * iz};
        double q2 = kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2];
        cplx ka = kk[0] * a[0] + kk[1] * a[1] + kk[2] * a[2];
        if (MUT(13)) ka = 0;
        for (int c = 0; c < 3; ++c) {
          cplx pa = a[c] - kk[c] * ka / q2;
          F[c * nc + m] -= pa;
          if (model == 1) F[(3 + c) * nc + m] -= pa;
        }
      }
}

static int rhs(const grid *g, int model, const cplx *z, cplx *F, double nu, double eta,
               const double *om) {
  const long H = g->H, nc = g->nc, ny = g->ny;
  int rc = model == 0 ? nonlinear_ns(g, z, F) : nonlinear_mhd(g, z, F);
  if (rc) return rc;
  const double a = model == 0 ? nu : 0.5 * (nu + eta);
  const double b = model == 0 ? 0.0 : (MUT(18) ? 0.5 * (eta - nu) : 0.5 * (nu - eta));
#pragma omp parallel for schedule(static)
  for (long kz = 0; kz < g->nz; ++kz)
    for (long ky = 0; ky < ny; ++ky)
      for (long kx = 0; kx < H; ++kx) {
        long m = (kz * ny + ky) * H + kx;
        long ix = wavx(kx), iy = wav(ky, ny), iz = wav(kz, g->nz);
        const double *sc = MUT(15) ? (const double[3]){1, 1, 1} : g_s;
        double k2 = sc[0] * sc[0] * ix * ix + sc[1] * sc[1] * iy * iy + sc[2] * sc[2] * iz * iz;
        if (model == 0) {
          for (int c = 0; c < 3; ++c) F[c * nc + m] -= a * k2 * z[c * nc + m];
        } else {
          for (int c = 0; c < 3; ++c) {
            cplx zp = z[c * nc + m], zm = z[(3 + c) * nc + m];
            F[c * nc + m] -= a * k2 * zp + b * k2 * zm;
            F[(3 + c) * nc + m] -= a * k2 * zm + b * k2 * zp;
          }
        }
      }
  if (om && (om[0] != 0 || om[1] != 0 || om[2] != 0)) coriolis(g, model, z, F, om);
  return 0;
}

int psref_rk2_step(int nx, int ny, int nz, int model, double *state, double nu, double eta,
                   double dt, int nsteps) {
  return psref_rk2_step_rot(nx, ny, nz, model, state, nu, eta, dt, nsteps, NULL);
}

int psref_rk2_step_rot(int nx, int ny, int nz, int model, double *state_, double nu, double eta,
                       double dt, int nsteps, const double *omega) {
  if (!state_ || nsteps < 0 || (model != 0 && model != 1)) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  const long nf = model == 0 ? 3 : 6;
  const long n = nf * g.nc;
  cplx *z = (cplx *)state_;
  cplx *zs = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  cplx *F = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  int rc = 0;
  if (!zs || !F) {
    rc = -3;
    goto done;
  }
  for (int s = 0; s < nsteps; ++s) {
    if ((rc = rhs(&g, model, z, F, nu, eta, omega))) goto done;
#pragma omp parallel for schedule(static)
    for (long m = 0; m < n; ++m) zs[m] = z[m] + (MUT(11) ? 1.0 : 0.5) * dt * F[m];
    if ((rc = rhs(&g, model, MUT(5) ? z : zs, F, nu, eta, omega))) goto done;
#pragma omp parallel for schedule(static)
    for (long m = 0; m < n; ++m) z[m] = z[m] + dt * F[m];
  }
done:
  free(zs);
  free(F);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Global quantities and spectra (Sec. 3: reductions over the grid).         */
/* FP64 with Neumaier-compensated summation, in a fixed order.               */
/* ------------------------------------------------------------------------ */

typedef struct {
  double s, c;
} nsum;

static void nadd(nsum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double nval(const nsum *a) { return a->s + a->c; }

/* smallest s >= 0 with 4 k2 < (2s+1)^2, i.e. |k| rounded to nearest */
static long shell_of(long k2) {
  long s = (long)floor(sqrt((double)k2));
  if (MUT(12)) return s;
  while (s > 0 && 4 * k2 < (2 * s - 1) * (2 * s - 1)) --s;
  while (4 * k2 >= (2 * s + 1) * (2 * s + 1)) ++s;
  return s;
}

int psref_num_shells(int nx, int ny, int nz) {
  if (!grid_ok(nx, ny, nz)) return -2;
  long hx = nx / 2, hy = ny / 2, hz = nz / 2;
  return (int)shell_of(hx * hx + hy * hy + hz * hz) + 1;
}

int psref_energy_spectrum(int nx, int ny, int nz, int nf, const double *fhat_, double *spec,
                          double *totals) {
  if (!fhat_ || !spec || !totals || nf < 1) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  const long H = g.H, nc = g.nc;
  const int ns = psref_num_shells(nx, ny, nz);
  const cplx *F = (const cplx *)fhat_;
  nsum *es = (nsum *)calloc((size_t)ns, sizeof(nsum));
  if (!es) return -3;
  nsum Z = {0, 0};
  double maxdiv = 0;
  for (long kz = 0; kz < nz; ++kz)
    for (long ky = 0; ky < ny; ++ky)
      for (long kx = 0; kx < H; ++kx) {
        long m = (kz * ny + ky) * H + kx;
        long ix = wavx(kx), iy = wav(ky, ny), iz = wav(kz, nz);
        long k2 = ix * ix + iy * iy + iz * iz;
        double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
        if (MUT(4) && 2 * kx == nx) w = 2.0;
        double e = 0;
        for (int f = 0; f < nf; ++f) {
          cplx a = F[f * nc + m];
          e += creal(a) * creal(a) + cimag(a) * cimag(a);
        }
        long s = shell_of(k2);  /* shells of the index |n| */
        double q2 = g_s[0] * g_s[0] * ix * ix + g_s[1] * g_s[1] * iy * iy + g_s[2] * g_s[2] * iz * iz;
        nadd(&es[s], 0.5 * w * e);
        nadd(&Z, 0.5 * w * q2 * e);
        for (int f = 0; f + 2 < nf; f += 3) {
          double ax = g_s[0] * dwavx(kx, nx), ay = g_s[1] * dwav(ky, ny), az = g_s[2] * dwav(kz, nz);
          cplx d = ax * F[f * nc + m] + ay * F[(f + 1) * nc + m] + az * F[(f + 2) * nc + m];
          if (cabs(d) > maxdiv) maxdiv = cabs(d);
        }
      }
  nsum E = {0, 0};
  for (int s = 0; s < ns; ++s) {
    spec[s] = nval(&es[s]);
    nadd(&E, spec[s]);
  }
  totals[0] = nval(&E);
  totals[1] = nval(&Z);
  totals[2] = maxdiv;
  free(es);
  return 0;
}

/* MHD global quantities of an Elsasser state (Sec. 3: global quantities by
 * reductions; Sec. 5: the MHD form of the solver).  With the primitive
 * fields u = (z+ + z-)/2 and b = (z+ - z-)/2 at every mode:
 *   Eu(s) = 1/2 sum_{shell(k)=s} w |u(k)|^2       kinetic energy
 *   Eb(s) = 1/2 sum_{shell(k)=s} w |b(k)|^2       magnetic energy
 *   Hc(s) = 1/2 sum_{shell(k)=s} w Re(u(k) . b(k)*)  cross-helicity
 * (the spectral form of the box averages 1/2 <|u|^2>, 1/2 <|b|^2> and
 * 1/2 <u . b>), with the weights and shells of psref_energy_spectrum.
 * spec holds [Eu(s)] then [Eb(s)] then [Hc(s)], each of nshell values;
 * totals = [Eu, Eb, Hc], each the compensated sum of its shells in order. */
int psref_mhd_spectrum(int nx, int ny, int nz, const double *zhat_, double *spec,
                       double *totals) {
  if (!zhat_ || !spec || !totals) return -1;
  if (!grid_ok(nx, ny, nz)) return -2;
  const grid g = grid_of(nx, ny, nz);
  const long H = g.H, nc = g.nc;
  const int ns = psref_num_shells(nx, ny, nz);
  const cplx *zp = (const cplx *)zhat_, *zm = zp + 3 * nc;
  nsum *acc = (nsum *)calloc((size_t)3 * ns, sizeof(nsum));
  if (!acc) return -3;
  const double half = MUT(20) ? 1.0 : 0.5;
  for (long kz = 0; kz < nz; ++kz)
    for (long ky = 0; ky < ny; ++ky)
      for (long kx = 0; kx < H; ++kx) {
        long m = (kz * ny + ky) * H + kx;
        long ix = wavx(kx), iy = wav(ky, ny), iz = wav(kz, nz);
        double w = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
        double eu = 0, eb = 0, hc = 0;
        for (int c = 0; c < 3; ++c) {
          cplx u = half * (zp[c * nc + m] + zm[c * nc + m]);
          cplx b = MUT(19) ? 0.5 * (zm[c * nc + m] - zp[c * nc + m])
                           : 0.5 * (zp[c * nc + m] - zm[c * nc + m]);
          eu += creal(u) * creal(u) + cimag(u) * cimag(u);
          eb += creal(b) * creal(b) + cimag(b) * cimag(b);
          hc += creal(u * conj(b));
        }
        long s = shell_of(ix * ix + iy * iy + iz * iz);
        nadd(&acc[s], 0.5 * w * eu);
        nadd(&acc[ns + s], 0.5 * w * eb);
        nadd(&acc[2 * ns + s], 0.5 * w * hc);
      }
  for (int q = 0; q < 3; ++q) {
    nsum t = {0, 0};
    for (int s = 0; s < ns; ++s) {
      spec[q * ns + s] = nval(&acc[q * ns + s]);
      nadd(&t, spec[q * ns + s]);
    }
    totals[q] = nval(&t);
  }
  free(acc);
  return 0;
}
