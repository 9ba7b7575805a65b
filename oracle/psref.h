/*
 * psref.h -- FP64 CPU oracle for the pseudospectral Navier-Stokes / MHD step.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library. The GPU
 * library never links, includes or calls it, and it shares no code with the
 * GPU library (no headers, tables or helpers).
 *
 * Source of every definition: Mininni, Rosenberg, Reddy & Pouquet, "A hybrid
 * MPI-OpenMP scheme for scalable parallel pseudospectral computations for
 * fluid turbulence", Sec. 2 (Eq. 1-2, the Fourier-Galerkin method, the
 * Hermitian half-spectrum storage of Fig. 1), Sec. 3 (loop-level threading
 * and reductions for spectra).  Where the paper defers to its references
 * (projection, dealiasing, the time integrator), the textbook reading is used
 * and stated at each function.
 *
 * Conventions (all arrays dense, C order), on an nx x ny x nz grid (the
 * paper's N^3 cube is nx = ny = nz = N):
 *   real fields      [f][z][y][x]            double,   x fastest, nx ny nz per field
 *   spectral fields  [f][kz][ky][kx]         complex double (re,im interleaved),
 *                                            kx = 0..nx/2 fastest, nz ny (nx/2+1) per field
 *   ky, kz index i   -> wavenumber i for i < n/2, i - n otherwise (n/2 -> -n/2),
 *                       n the axis length
 *   derivative wavenumber (odd derivatives): 0 at the Nyquist index n/2
 *   grid points      x_j = 2*pi*j/nx on [0, 2*pi) (likewise y, z)
 *   dealiasing       keep (3 kx/nx)^2 + (3 ky/ny)^2 + (3 kz/nz)^2 < 1, the
 *                    2/3-rule sphere 9|k|^2 < N^2 of the cube stretched with
 *                    the grid
 *
 * All functions return 0 on success and a negative code on bad arguments
 * (-1 null pointer / bad enum, -2 unsupported size, -3 out of memory).
 * Supported sizes: each of nx, ny, nz even, 2 <= n <= 4096.
 */
#ifndef PSREF_H
#define PSREF_H

#ifdef __cplusplus
extern "C" {
#endif

/* Hash of the sources (psref.c, psref.h) the library was built from. */
const char *psref_build_hash(void);

/* Number of OpenMP threads the oracle uses (<= 0: leave the runtime default).
 * Returns the number of threads that will be used. */
int psref_set_threads(int n);

/* Unnormalised forward 3D transform X(k) = sum_x u(x) exp(-i k.x) of nf real
 * fields, stored for kx = 0..nx/2. */
int psref_fft_r2c(int nx, int ny, int nz, int nf, const double *in, double *out);

/* Unnormalised inverse 3D transform of nf half spectra, in pass order:
 * inverse complex transforms along z then y on every kx plane, then
 * u(x) = Re Y_0 + 2 sum_{0<kx<nx/2} Re(Y_kx e^{i kx x}) + Re Y_{nx/2} (-1)^x.
 * The imaginary parts of the kx = 0 and kx = nx/2 bins are ignored. */
int psref_fft_c2r(int nx, int ny, int nz, int nf, const double *in, double *out);

/* Direct sum of the forward transform at nk selected bins (kx[i], ky[i],
 * kz[i] are storage indices). out: nk complex values. */
int psref_dft_at(int nx, int ny, int nz, const double *in, int nk, const int *kx,
                 const int *ky, const int *kz, double *out);

/* Spectral curl  w = i k_d x u  of one 3-component spectral vector. */
int psref_curl(int nx, int ny, int nz, const double *uhat, double *what);

/* Dealiased, projected nonlinear term of incompressible Navier-Stokes in
 * rotational form, nhat = D P F[u x w] / (nx ny nz) (3 fields in, 3 out). */
int psref_nonlinear_ns(int nx, int ny, int nz, const double *uhat, double *nhat);

/* MHD nonlinear terms for the Elsasser state (z+ = u + b, z- = u - b):
 * N+- = D [ P F[u x w + j x b] +- i k_d x F[u x b] ] / (nx ny nz)
 * (6 fields in: z+ then z-; 6 out: N+ then N-). */
int psref_nonlinear_mhd(int nx, int ny, int nz, const double *zhat, double *nhat);

/* Galerkin (direct triad sum) value of the same nonlinear terms at nk
 * selected storage indices.  model 0 = NS (uhat: 3 fields), 1 = MHD (6).
 * out: nk x (3 or 6) complex values, component-major per mode. */
int psref_nonlinear_at(int nx, int ny, int nz, int model, const double *fhat, int nk,
                       const int *kx, const int *ky, const int *kz, double *out);

/* Explicit midpoint RK2 steps, in place.  model 0 = NS (3 fields, viscosity
 * nu), 1 = MHD Elsasser (6 fields, viscosity nu, resistivity eta). */
int psref_rk2_step(int nx, int ny, int nz, int model, double *state, double nu, double eta,
                   double dt, int nsteps);

/* The same in a frame rotating at omega[3] (NULL or all zero: no rotation):
 * the momentum equation gains -P(k) (2 Omega x u) at every k != 0 (for MHD
 * with u = (z+ + z-)/2, added to both Elsasser fields). */
int psref_rk2_step_rot(int nx, int ny, int nz, int model, double *state, double nu,
                       double eta, double dt, int nsteps, const double *omega);

/* Box lengths (default 2 pi each): physical wavenumbers k = (2 pi / L) n in
 * every derivative, in the projector and in |k|^2 of the viscous term and
 * of the enstrophy; dealiasing and the spectral shells stay on the index n.
 * Process-wide setting.  Returns -1 for non-positive or non-finite L. */
int psref_set_box(double Lx, double Ly, double Lz);

/* Number of spectral shells: s((nx/2)^2 + (ny/2)^2 + (nz/2)^2) + 1. */
int psref_num_shells(int nx, int ny, int nz);

/* Shell energy spectrum E(s) = 1/2 sum_{shell(k)=s} w |f(k)|^2 over nf
 * fields, w = 1 on the kx = 0 and kx = nx/2 planes, 2 elsewhere, and the
 * totals [E, Z, maxdiv] with Z = 1/2 sum w |k|^2 |f|^2 and maxdiv the largest
 * |k_d . f| over consecutive component triples (0 if nf is not a multiple of
 * 3).  shell(k) = round(|k|) of the index, evaluated exactly in integers. */
int psref_energy_spectrum(int nx, int ny, int nz, int nf, const double *fhat, double *spec,
                          double *totals);

/* MHD global quantities of an Elsasser state (6 fields, z+ then z-), from
 * u = (z+ + z-)/2 and b = (z+ - z-)/2 at every mode, with the weights and
 * shells of psref_energy_spectrum:
 *   spec[s]            = Eu(s) = 1/2 sum_{shell(k)=s} w |u(k)|^2
 *   spec[nshell + s]   = Eb(s) = 1/2 sum_{shell(k)=s} w |b(k)|^2
 *   spec[2 nshell + s] = Hc(s) = 1/2 sum_{shell(k)=s} w Re(u(k) . conj b(k))
 * and totals = [Eu, Eb, Hc] (kinetic energy, magnetic energy,
 * cross-helicity: 1/2 <|u|^2>, 1/2 <|b|^2>, 1/2 <u . b> over the box). */
int psref_mhd_spectrum(int nx, int ny, int nz, const double *zhat, double *spec, double *totals);

#ifdef __cplusplus
}
#endif
#endif
