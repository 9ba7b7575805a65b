/*
 * ps.h -- C ABI of libps.so, the gfx950 (MI355X) pseudospectral hot path.
 *
 * What it computes (Mininni, Rosenberg, Reddy & Pouquet, "A hybrid MPI-OpenMP
 * scheme for scalable parallel pseudospectral computations for fluid
 * turbulence"):
 *   - Sec. 2, Eq. 1-2: incompressible Navier-Stokes  du/dt + u.grad u =
 *     -grad p + nu lap u,  div u = 0, in a 2 pi-periodic box, discretised by
 *     a truncated Fourier (Galerkin) expansion with the nonlinear term
 *     evaluated in physical space through FFTs, projected onto
 *     divergence-free fields and dealiased;
 *   - Sec. 5: the same code with a magnetic field (MHD), here in Elsasser
 *     variables z+- = u +- b;
 *   - Sec. 2 / Fig. 1: real-to-complex 3D transforms stored as half spectra
 *     of (N/2+1) x N x N complex values;
 *   - Sec. 3: global quantities and spectra computed by reductions;
 *   - Sec. 4: the main time-advance loop (its integrator is not named in the
 *     paper; this library uses explicit midpoint RK2).
 *
 * Layouts (all dense, C order, element = float/double or its complex pair):
 *   real field set     [box][f][z][y][x]        x fastest, N^3 reals per field
 *   spectral field set [box][f][kz][ky][kx]     kx = 0..N/2 fastest, complex
 *                      interleaved (re, im), N*N*(N/2+1) per field; identical
 *                      to numpy/torch rfftn of a [z][y][x] array.
 *   ky, kz index i <-> wavenumber i (i < N/2) or i - N (i >= N/2).
 *   Spectral coefficients of the solver state are normalised:
 *   u(x) = sum_k u_k exp(i k.x).  ps_fft_* are unnormalised.
 *
 * Ownership: every field pointer and the workspace are DEVICE memory owned by
 * the caller.  The plan owns only its twiddle tables, schedule, private
 * capture stream and cached graph, released by ps_plan_destroy.  After
 * ps_plan_create no call allocates device memory.
 *
 * Execution: calls are asynchronous on the plan's stream (ps_plan_set_stream;
 * default: the null stream).  Outputs are valid after the caller synchronises
 * that stream.  A plan is not thread-safe; distinct plans are independent.
 *
 * Errors: every call validates its arguments before launching anything and
 * returns a ps_status; nothing aborts, exits or throws across the ABI.
 * ps_last_error() gives the detail text of the calling thread's last failure.
 * Device pointers are checked to be device memory large enough for the
 * shape (PS_ERR_ARG otherwise).
 */
#ifndef PS_H
#define PS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_plan_s *ps_plan;

typedef enum { PS_F32 = 0, PS_F64 = 1 } ps_dtype;
typedef enum { PS_NS = 0, PS_MHD = 1 } ps_model;
typedef enum {
  PS_OK = 0,
  PS_ERR_ARG = -1,      /* null/invalid argument, host pointer, buffer too small */
  PS_ERR_SIZE = -2,     /* unsupported grid size or field count */
  PS_ERR_NOMEM = -3,    /* host or table allocation failed, workspace too small */
  PS_ERR_HIP = -4,      /* a HIP runtime call failed (detail in ps_last_error) */
  PS_ERR_STATE = -5,    /* call not valid in the plan's state (e.g. no workspace) */
  PS_ERR_DIVERGED = -6  /* the blow-up monitor found a non-finite or exploding energy */
} ps_status;

/* Plan for one N^3 box of nfields fields (3: NS velocity; 6: MHD z+, z-),
 * the 2 pi-periodic box of Sec. 2 discretised by N^3 points (Fig. 1).
 * N must be one of 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512,
 * 768, 1024 (even, 2^a 3^b).  Builds FP64-accurate twiddle tables on the
 * device of the current HIP device.  *out is set to NULL on failure. */
ps_status ps_plan_create(ps_plan *out, int N, int nfields, ps_dtype dtype);

/* Plan for an ensemble of nbox independent boxes of sizes N[0..nbox), all
 * with nfields fields; field sets are concatenated box after box.  Each box
 * is the problem of Sec. 2 on its own; the paper runs one box at a time, and
 * batching independent boxes is this library's addition. */
ps_status ps_plan_create_batch(ps_plan *out, int nbox, const int *N, int nfields,
                               ps_dtype dtype);

/* Plan for one box of nx x ny x nz points (Sec. 5 says the method applies to
 * domains whose aspect ratio is not unity; each length one of the sizes
 * above).  Real fields are [f][z][y][x] (nx fastest), half spectra
 * [f][kz][ky][kx <= nx/2]; the transforms are unnormalised and the nonlinear
 * terms carry 1/(nx ny nz).  The 2/3 rule keeps the modes with
 * (3 kx/nx)^2 + (3 ky/ny)^2 + (3 kz/nz)^2 < 1 (the sphere 9|k|^2 < N^2 below
 * when the lengths agree), the shells are round(|k|) of the index, and
 * ps_num_shells gives s((nx/2)^2 + (ny/2)^2 + (nz/2)^2) + 1 of them.  MHD
 * needs an nx that ps_plan_create would accept for MHD.  Everything below
 * applies with N read per axis. */
ps_status ps_plan_create_grid(ps_plan *out, int nx, int ny, int nz, int nfields,
                              ps_dtype dtype);

/* Releases the plan (not the caller's buffers).  NULL is a no-op. */
ps_status ps_plan_destroy(ps_plan p);

/* Stream (a hipStream_t passed as void*) on which all later calls enqueue
 * work.  NULL selects the null stream. */
ps_status ps_plan_set_stream(ps_plan p, void *stream);

/* Bytes of device workspace the plan needs (ensemble: all boxes). */
size_t ps_plan_workspace_bytes(ps_plan p);

/* Hands the plan a caller-owned device workspace of at least
 * ps_plan_workspace_bytes(p) bytes, 256-byte aligned. */
ps_status ps_plan_set_workspace(ps_plan p, void *dev, size_t bytes);

/* Element offsets of box `box` inside the concatenated real (in reals) and
 * spectral (in complex values) field sets. */
ps_status ps_plan_box_offsets(ps_plan p, int box, size_t *real_off, size_t *cplx_off);

/* Number of spectral shells of box `box`: s(3 (N/2)^2) + 1 with
 * s(k2) = round(sqrt(k2)); 444 at N = 512, 888 at N = 1024; < 0 on error. */
int ps_num_shells(ps_plan p, int box);

/* Unnormalised forward transform X(k) = sum_x u(x) exp(-i k.x) of every
 * field of every box (Sec. 2, Fig. 1).  real_in and cplx_out must not
 * overlap. */
ps_status ps_fft_r2c(ps_plan p, const void *real_in, void *cplx_out);

/* Unnormalised inverse transform in pass order (inverse complex transforms
 * along z, then y, then the real inverse along x, whose kx = 0 and kx = N/2
 * bins contribute their real parts).  cplx_in is preserved. */
ps_status ps_fft_c2r(ps_plan p, const void *cplx_in, void *real_out);

/* Navier-Stokes nonlinear term (Sec. 2, Eq. 1-2, rotational form):
 * nhat = D(k) P(k) F[u x w] / N^3 with u = c2r(uhat), w = c2r(i k x uhat),
 * D the 2/3-rule spherical truncation (keep 9|k|^2 < N^2), P(k) = I - k k^T/|k|^2
 * (P(0) = 0).  3 fields in, 3 out; the plan must have nfields = 3.  With the
 * default variants any input is valid (it need be neither solenoidal nor
 * dealiased); the "form" and "prune" variants below have preconditions. */
ps_status ps_nonlinear_ns(ps_plan p, const void *uhat, void *nhat);

/* MHD nonlinear terms for the Elsasser state (z+ then z-; plan nfields = 6).
 * Sec. 5 names the MHD form of the solver without its equations; the
 * quadratic terms of incompressible MHD are taken in rotational form, with
 * the transforms, projection and 2/3 rule Sec. 2 uses for Navier-Stokes:
 * N+- = D [ P F[u x w + j x b] +- i k x F[u x b] ] / N^3,
 * u = (z+ + z-)/2, b = (z+ - z-)/2, w = curl u, j = curl b.  With the
 * default variants any input is valid; the "form" and "prune" variants
 * below are faster and have preconditions. */
ps_status ps_nonlinear_mhd(ps_plan p, const void *zhat, void *nhat);

/* nsteps explicit midpoint RK2 steps in place on the spectral state (the
 * main time-advance loop of Sec. 4; the paper does not name its integrator):
 * z* = z + (dt/2) F(z), z <- z + dt F(z*), F = nonlinear term - viscous
 * term (NS: nu |k|^2 u; MHD: |k|^2 ((nu+eta)/2 z+- + (nu-eta)/2 z-+)).
 * One RK2 step is replayed from a captured HIP graph unless graphs are
 * disabled or kernel timing is on.  Needs a workspace. */
ps_status ps_rk2_step(ps_plan p, void *state, ps_model m, double nu, double eta, double dt,
                      int nsteps);

/* Blow-up monitor for ps_rk2_step (the time-advance loop of Sec. 4).  With
 * every > 0, each call computes the FP64 total energy of every box of the
 * state (ps_energy_spectrum over all fields) before its first step, after
 * every `every` steps and after its last step; the energies are read back to
 * the host, which synchronises the plan's stream.  The call stops and
 * returns PS_ERR_DIVERGED (detail: box, energy and step in ps_last_error) as
 * soon as some box's energy is not finite or exceeds `growth` times its value
 * at the start of the call; the state is then the one at that check.  every
 * = 0 (the default) switches the monitor off.  PS_ERR_ARG for every < 0 or,
 * with every > 0, growth not finite or not > 1. */
ps_status ps_plan_set_monitor(ps_plan p, int every, double growth);

/* Frame rotation for ps_rk2_step (Sec. 5 lists rotating flows among what the
 * code integrates; the paper gives no formula).  In a frame rotating at
 * angular velocity Omega = (ox, oy, oz) the momentum equation gains the
 * Coriolis acceleration -2 Omega x u (the centrifugal part is a gradient and
 * goes into the pressure), projected like every other term; F above gains
 * -P(k)(2 Omega x u) at every k != 0, with u = z (NS) or u = (z+ + z-)/2 (MHD,
 * added to both Elsasser equations; the induction equation is unchanged).
 * Default (0, 0, 0).  Affects ps_rk2_step only, not ps_nonlinear_*.  Drops
 * a cached graph.  PS_ERR_ARG for non-finite components. */
ps_status ps_plan_set_rotation(ps_plan p, double ox, double oy, double oz);

/* Box lengths (Sec. 5: the scheme also serves domains whose aspect ratio is
 * not unity).  Default 2 pi each.  A box of lengths (Lx, Ly, Lz) has physical
 * wavenumbers k = (2 pi / L) n for the signed storage index n; they enter the
 * curl, the projector P(k), the divergence form, |k|^2 of the viscous term,
 * the Coriolis term, and the enstrophy and divergence of
 * ps_energy_spectrum.  The 2/3 truncation and the spectral shells stay on
 * the index n (aliasing is a property of the grid).  The grid is N^3 in every
 * case.  Drops a cached graph.  PS_ERR_ARG for non-positive or non-finite L. */
ps_status ps_plan_set_box(ps_plan p, double Lx, double Ly, double Lz);

/* Shell spectrum of nfields fields per box (1 <= nfields <= plan nfields),
 * one of the global quantities Sec. 3 computes by reductions over the grid:
 * spec_dev[s] = 1/2 sum_{round(|k|)=s} w |f(k)|^2 (w = 1 on the kx = 0 and
 * kx = N/2 planes, 2 elsewhere) and totals_dev = [E, Z, maxdiv] with
 * Z = 1/2 sum w |k|^2 |f|^2 and maxdiv = max |k . f| over consecutive
 * component triples.  FP64, deterministic (fixed-order compensated sums).
 * Ensembles: per-box spectra concatenated, 3 totals per box.  Device output. */
ps_status ps_energy_spectrum(ps_plan p, const void *fhat, int nfields, double *spec_dev,
                             double *totals_dev);

/* ps_energy_spectrum for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments and the same results, bit for bit, but the
 * per-plane partials live in a device scratch array the library holds (16 MiB
 * per device, enough for every supported grid; one box at a time), so the
 * plan needs no workspace and the call allocates nothing.  Every call on a
 * device shares that device's scratch: calls that overlap on one device (on
 * different streams, or from different threads) race and must not be
 * issued.  PS_ERR_SIZE if a box's partials (nz nshell 2 + nz doubles) exceed
 * the scratch, PS_ERR_ARG as for ps_energy_spectrum. */
ps_status ps_energy_spectrum_static(ps_plan p, const void *fhat, int nfields, double *spec_dev,
                                    double *totals_dev);

/* Kinetic and magnetic energy and cross-helicity of an Elsasser state (plan
 * nfields = 6; Sec. 3 computes global quantities and spectra by reductions,
 * Sec. 5 runs the solver for MHD).  With u = (z+ + z-)/2 and b = (z+ - z-)/2
 * at every mode, and the weights and shells of ps_energy_spectrum:
 *   spec_dev[s] = Eu(s) = 1/2 sum_{round(|k|)=s} w |u(k)|^2,
 *   spec_dev[nshell + s] = Eb(s) (the same with b),
 *   spec_dev[2 nshell + s] = Hc(s) = 1/2 sum w Re(u(k) . conj b(k)),
 * totals_dev = [Eu, Eb, Hc] (each the sum of its shells).  FP64,
 * deterministic (fixed-order compensated sums).  Ensembles: 3 nshell values
 * and 3 totals per box, box after box.  Device output; needs a workspace. */
ps_status ps_mhd_spectrum(ps_plan p, const void *zhat, double *spec_dev, double *totals_dev);

/* Kernel variants.  Pass kinds: "y", "z" (plain strided passes), "z_curl",
 * "z_epi", "x_prod"; the tile width, radix schedule or register/LDS trade-off
 * of a pass (results are identical up to rounding order).  Kind "batch":
 * 0 = one launch per pass for each run of consecutive equal-size boxes
 * (default), 1 = one launch per box (baseline).  Kind "prune": 1 = the
 * step and the nonlinear terms skip everything the 2/3 rule makes zero (pencils
 * and modes outside the sphere 9|k|^2 < N^2 are neither read nor transformed);
 * valid when the input is zero outside that sphere (a dealiased state stays
 * dealiased under the step), and modes outside it are then left untouched by
 * ps_rk2_step (ps_nonlinear_* still writes zeros there).  Kind "form":
 * 0 = the rotational form of Sec. 2 (NS: u x w; MHD: u x w + j x b and u x b
 * of the primitive fields), the default, valid for any input; 1 = the
 * divergence form.  MHD (Elsasser variables): N+- = -i P(k) k_j F[z-+_j z+-_i]
 * from the products z+_i z-_j less their isotropic part delta_ij z+_2 z-_2,
 * a gradient that P(k) removes (eight products, so fourteen real transforms
 * per evaluation instead of eighteen).  NS: N = -i P(k) k_j F[u_i u_j] from
 * the five products of the symmetric u_i u_j less delta_ij u_2 u_2 (eight
 * real transforms instead of nine, and no curl).  Precondition of form 1:
 * the state is solenoidal (k . z = 0 for every 3-vector, in the box's
 * metric) AND zero outside the 2/3 sphere; it then agrees with form 0 up to
 * rounding (both sets of products are alias-free inside the sphere), and
 * every state ps_rk2_step makes from such a state is again such a state.
 * On other inputs the two forms compute different functions (they differ by
 * P(u div u) and by the aliases of the products); nothing checks the
 * precondition.  Kind "pipe" v: the inverse y pass, the product pass and
 * the forward y pass of each right-hand side run as 2^v slabs of z-planes
 * (each plane's chain is independent of the others'): for v = 1..3 spread
 * over helper streams, so that one slab's memory-bound y passes overlap
 * another's compute-bound product pass; for v = 4..6 one after another on
 * the plan's stream, so that each slab's chain finds its data in the
 * last-level cache; for v = 7..9, 2^(v-3) slabs (16, 32, 64) as two chains,
 * even and odd slabs, on two helper streams, so that the two slabs in flight
 * still fit the last-level cache while each fills the other's launch gaps;
 * 0 = one slab on the plan's stream (default; ps_plan_autotune chooses among
 * 0 and 4..6, the settings whose launches do not overlap, unless "overlap"
 * is 1).  Every setting computes the same step bit for bit.  Kind "overlap"
 * (0 default, 1): whether ps_plan_autotune may also choose the two-chain
 * settings 7..9, for a caller who wants the fastest step over per-kernel
 * timings (a launch's duration is no longer its own when two overlap); it
 * changes no arithmetic.  Setting a variant drops a cached graph. */
ps_status ps_plan_set_variant(ps_plan p, const char *kind, int variant);
int ps_plan_get_variant(ps_plan p, const char *kind);
int ps_plan_variant_count(ps_plan p, const char *kind);

/* Autotuner: times every variant of the RK2 passes (z_curl, y, x_prod, z_epi)
 * over reps launches on the caller's state for model m, times the variants
 * within 10 % of the fastest again in three interleaved rounds (each keeping
 * its best time, so that clock drift over the sequence does not rank them)
 * and keeps the fastest; then chooses the "pipe" setting (0 or 4..6, and
 * 7..9 when "overlap" is 1) the same way on whole right-hand sides
 * (evaluated in the first RK stage's mode).  Reads
 * state, writes only the workspace; synchronises the plan's stream.  Plan
 * time, like FFT planning, is not part of a step (Sec. 4 leaves planning out
 * of its timings).  When the environment variable PS_TUNE_CACHE names a
 * file, the tuned variants are kept there under a key of everything the
 * timings depend on (device architecture, HIP runtime version, this
 * library's build hash, model, dtype, fields, every size class, and the
 * "form", "prune", "batch" and "overlap" variants); a later call with the same
 * key takes them from the file and times nothing.  A file that cannot be
 * read or written only costs the timing runs. */
ps_status ps_plan_autotune(ps_plan p, const void *state, ps_model m, int reps);

/* Timing launches the last ps_plan_autotune made: 0 when its variants came
 * from the PS_TUNE_CACHE file, -1 before the first call; PS_ERR_ARG for a
 * NULL plan. */
int ps_plan_autotune_timed(ps_plan p);

/* Per-kernel timing with HIP events on the plan's stream (disables graph
 * replay while on).  Statistics accumulate until ps_plan_timing_reset. */
ps_status ps_plan_set_timing(ps_plan p, int enable);
ps_status ps_plan_set_graphs(ps_plan p, int enable);
ps_status ps_plan_timing_reset(ps_plan p);
/* Number of kernel kinds with statistics (synchronises pending events). */
int ps_plan_timing_count(ps_plan p);
/* Statistics of kind idx: name (static storage), total milliseconds, launch
 * count and algorithmic bytes moved per launch (reads + writes of the
 * values the pass must touch), averaged over the kind's launches (the two
 * RK stages' epilogues move different amounts). */
ps_status ps_plan_timing_get(ps_plan p, int idx, const char **name, double *total_ms,
                             long *launches, double *bytes_per_launch);

const char *ps_status_string(ps_status s);
const char *ps_last_error(void);

/* Hash of the sources and flags the library was built from (16 hex digits,
 * static storage); the binding compares it with the sources beside it. */
const char *ps_build_hash(void);

#ifdef __cplusplus
}
#endif
#endif
