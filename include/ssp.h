/*
 * ssp.h - C ABI of the MI355X spectral split-step Pade (SSSP) range-march library.
 *
 * The library marches the one-way (parabolic) wave equation in range with the spectral
 * split-step Pade method of Walsken, Ehrhardt and Petrov (arXiv 2511.03343):
 *   Sec. 2    u(r + dr) ~ e^{i k0 dr} R(X) u(r), R the [p/p] Pade approximant of
 *             exp(i sigma (sqrt(1+x) - 1)), sigma = k0 dr, X = (d_z^2 + k^2 - k0^2)/k0^2.
 *   Sec. 3    each Pade term (1 + b_j X)^{-1} is a diagonal solve in the sine basis when
 *             the sound speed is constant, and a Neumann series (eq. neumannseries) of
 *             transform -> diagonal scale -> inverse transform -> multiply by
 *             v(z) = (c0/c(z))^2 - 1 otherwise.
 *   Sec. 3.1  homogeneous Dirichlet boundaries at z = 0 and z = H: the transform is the
 *             orthonormal DST-I on the interior grid z_n = n H/(Nz+1), n = 1..Nz.  The
 *             same section's Neumann (cosine transform) and periodic (Fourier transform)
 *             boundaries are available through ssp_plan_create_bc.
 *   Alg. 1    the range march: for every step, every Pade term, then the carrier.
 *
 * All entry points are extern "C", return an ssp_status and never throw.  Pointers are
 * host pointers unless the name says "device".  The caller owns every array it passes;
 * the library copies host arrays in and out before returning.  A plan owns its device
 * memory (field, tables, profile, staging) and releases it in ssp_plan_destroy.  A plan is
 * not thread-safe; distinct plans may be used from different threads.  Every call runs on
 * the plan's HIP stream (default: the null stream; see SSP_OPT_STREAM) and the host calls
 * (ssp_march, ssp_get_field, ...) synchronise that stream before returning.
 *
 * Numerics: the field is complex FP32 (interleaved re, im), kept on the device in the sine
 * basis between calls.  Pade coefficients are computed on the host in extended
 * precision; sine-space multipliers and FFT twiddles are applied as double-float
 * (hi + lo FP32) products; the Neumann residual is accumulated in FP64; the carrier
 * phase exp(i k0 r) is formed in FP64.
 */
#ifndef SSP_H
#define SSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSP_OK = 0,
    SSP_W_NOT_CONVERGED = 1, /* march finished; some Neumann series stopped at
                                neumann_max with residual > tol (see ssp_stats) */
    SSP_E_INVAL = -1,        /* invalid argument (size, NULL, non-finite or <= 0 speed) */
    SSP_E_NOMEM = -2,        /* device or host allocation failed */
    SSP_E_DEVICE = -3,       /* HIP runtime error (message in ssp_last_error) */
    SSP_E_DIVERGED = -4,     /* a Neumann series grew or a value became non-finite; the
                                field is left at the last good step (ssp_stats.steps_done) */
    SSP_E_UNSTABLE = -5,     /* plan rejected: max_l |e^{i sigma} R(x_l)| > 1 + eps, eps the
                                plan's gain limit (SSP_OPT_GAIN_LIMIT, default 1e-6) */
    SSP_E_STATE = -6,        /* call out of order (e.g. march before a field was set) */
    SSP_E_UNIMPL = -7        /* size or option outside what this build supports */
} ssp_status;

typedef struct ssp_plan ssp_plan; /* opaque, library-owned */

/* Options for ssp_plan_set_option. */
enum {
    SSP_OPT_ROTATION = 1,  /* branch-cut rotation angle alpha (rad) of the Pade
                              approximant; 0 (default) = standard approximant.  Changing
                              it recomputes the coefficients and the stability check. */
    SSP_OPT_OUT_EVERY = 2, /* write an output every k-th step (default 1) */
    SSP_OPT_STREAM = 3,    /* value = (double)(uintptr_t)hipStream_t; 0 = null stream.
                              Use ssp_plan_set_stream to pass a pointer exactly. */
    SSP_OPT_ENGINE = 4,    /* transform engine of the march (SSP_ENGINE_*):
                              SSP_ENGINE_AUTO (default): the engine the autotuner measured
                              faster for the plan's (Nz, pade_order) class; SSP_ENGINE_FFT:
                              FFT-based transforms in the fused persistent kernel;
                              SSP_ENGINE_DENSE: every DST-I of the Neumann series is the
                              dense product S X on the matrix cores (Sec. 3.1: S is the
                              orthonormal DST-I matrix, symmetric and its own inverse) over
                              the whole batch of solves of one Nz; Dirichlet plans with
                              Nz <= ssp_max_dense_nz() only (SSP_E_UNIMPL otherwise).  The
                              engines differ in rounding only. */
    SSP_OPT_GRAPH = 5,     /* 1: ssp_march_device and ssp_march_batch_async record their
                              launches (march + outputs) in a HIP graph on the first call and
                              replay the graph on later calls with the same arguments; needs
                              a non-null stream (FFT engine).  0 (default): plain launches */
    SSP_OPT_VARIANT = 6,   /* engine layout of the fused march kernel: -1 (default) = the
                              layout the autotuner chose for this FFT length and transform
                              kind (chirp-z, direct Fourier, direct sine) on batches of one
                              length; -2 = the layout it chose for batches that mix lengths
                              (broadband and serving); 0, 1 or 2 = that
                              layout (falls back to 0 where the length has no such layout;
                              split lengths, P > 16384, have layout 0 only).
                              Layouts differ in rounding only; a solve's results do not
                              depend on what it is batched with. */
    SSP_OPT_PLAIN = 7,     /* 0 (default): fused persistent kernel; 1: plain form, one kernel
                              per transform / pointwise stage and a host-driven loop (FFT
                              engine, chirp-z plans, ssp_march of one plan) */
    SSP_OPT_FORM = 8,      /* SSP_FORM_PRODUCT (default): the Pade factors applied one after
                              the other, u <- g_j u + (1 - g_j)(1 + b_j X)^{-1} u, the same
                              approximant as the sum form of Sec. 2.  SSP_FORM_SUM (the
                              paper's form, u <- d0 u + sum_j d_j (1 + b_j X)^{-1} u) is not
                              built: sum_j |d_j| reaches 1e2 .. 4e3 at the benchmark
                              settings, and in FP32 that cancellation costs up to 12 bits
                              per step; setting it returns SSP_E_UNIMPL. */
    SSP_OPT_GAIN_LIMIT = 9, /* eps >= 0 of the stability check max_l |e^{i sigma} R(x_l)|
                              <= 1 + eps (default 1e-6: the rotated [4/4] approximant of the
                              homogeneous waveguide at sigma = 2.09 exceeds 1 by 4.5e-8,
                              i.e. 4.5e-5 over 1000 steps).  Setting it re-checks the
                              current coefficients; if they fail, SSP_E_UNSTABLE is returned
                              and the limit is left unchanged. */
    SSP_OPT_CONTRACTION_CHECK = 10 /* 1: before marching, estimate the spectral radius of
                              every factor's Neumann operator b_j L_j^{-1} V (see
                              ssp_plan_contraction; once per profile) and return
                              SSP_E_DIVERGED without marching if one is >= 1.  0 (default):
                              divergence is detected while marching. */
};

enum { SSP_ENGINE_FFT = 0, SSP_ENGINE_DENSE = 1, SSP_ENGINE_AUTO = 2 };
enum { SSP_FORM_PRODUCT = 0, SSP_FORM_SUM = 1 };

/* Analytic range-dependent environment evaluated on the device every step at the step's
 * mid-range r = (n - 1/2) dr:  c(r, z) = c_munk(z) + dc(r, z), with the Munk profile of
 * Sec. 4.1 eq. (Munk), c_munk = munk_c1 (1 + munk_eps (eta + e^{-eta} - 1)),
 * eta = 2 (z - munk_z1)/munk_z1, and a Gaussian eddy
 * dc = -eddy_amp exp(-((r - eddy_r0)/eddy_rr)^2 - ((z - eddy_z0)/eddy_rz)^2). */
typedef struct {
    double munk_c1, munk_eps, munk_z1;                   /* 1500, 0.00737, 1300 */
    double eddy_amp, eddy_r0, eddy_rr, eddy_z0, eddy_rz; /* eddy_amp = 0: no eddy */
} ssp_env;

/* Per-march statistics (filled by ssp_march / ssp_march_batch / ssp_read_stats). */
typedef struct {
    int64_t steps_done;       /* range steps completed by this call */
    int64_t step_index;       /* global step counter of the plan after the call */
    int64_t neumann_terms;    /* sum over steps and Pade factors of the terms m >= 1 */
    int32_t neumann_max_used; /* largest m reached by one series */
    int32_t not_converged;    /* number of (step, factor) series that hit neumann_max */
    double max_residual;      /* largest final ||term_m|| / ||w^(m)|| */
    int32_t status;           /* ssp_status of this solve */
    int32_t pad_;
} ssp_stats;

/* Boundary conditions at z = 0 and z = H (Sec. 3.1), each with its grid and transform:
 *   SSP_BC_DIRICHLET  u = 0;  z_n = n H/(Nz+1), n = 1..Nz (interior points);  orthonormal
 *                     DST-I, basis sin(l pi z/H), l = 1..Nz.  Nz + 1 a power of two with
 *                     2 (Nz + 1) in [128, 16384]: each DST-I is one FFT of length 2 (Nz + 1)
 *                     over the odd extension of the data (else chirp-z FFTs of length
 *                     >= 2 Nz - 1); such plans run the fused kernel as periodic direct
 *                     plans do (below)
 *   SSP_BC_NEUMANN    d_z u = 0;  z_n = n H/(Nz-1), n = 0..Nz-1 (both boundaries on the
 *                     grid);  basis cos(l pi z/H), l = 0..Nz-1, through the orthonormal DCT-I
 *                     C applied to the grid values with the two boundary values scaled by
 *                     1/sqrt(2) (forward C e u, inverse C a / e);  Neumann-series norms are
 *                     the norms of e u (trapezoidal weights)
 *   SSP_BC_PERIODIC   u(0) = u(H);  z_n = n H/Nz, n = 0..Nz-1;  orthonormal DFT (forward
 *                     e^{-2 pi i l n/Nz}/sqrt(Nz)), basis e^{2 pi i l' z/H}, l' = l for
 *                     l <= Nz/2 and l - Nz above.  Nz a power of two in [128, 16384]: the
 *                     transforms are direct FFTs of length Nz (else chirp-z ones of length
 *                     >= 2 Nz - 1); such plans run the fused kernel only
 *                     (SSP_OPT_PLAIN = 1 gives SSP_E_UNIMPL)
 * Every basis function is an eigenfunction of d_z^2 (eigenvalue -kappa_l^2, kappa_l = l pi/H
 * or 2 pi l'/H), which makes the isovelocity operator of every Pade term diagonal.  The
 * coefficient-space field kept on the device ("sine basis" below) is that of the plan's
 * basis. */
enum { SSP_BC_DIRICHLET = 0, SSP_BC_NEUMANN = 1, SSP_BC_PERIODIC = 2 };

/* Create a plan (Alg. 1 "compute d_j and b_j"; Sec. 2 Pade form; Sec. 3.1 grid).
 *   Nz           interior depth points, 2 <= Nz <= ssp_max_nz();  dz = H/(Nz+1)
 *   H            waveguide depth (m) > 0;  f  frequency (Hz) > 0
 *   c0           reference sound speed (m/s) > 0, k0 = 2 pi f / c0
 *   dr           range step (m) > 0
 *   pade_order   p in [1, 12]
 *   neumann_max  largest Neumann index M >= 0 (0: the m = 0 term only, Sec. 4.1 "M = 0")
 *   tol          > 0; a series stops at the first m >= 1 with ||term_m|| <= tol ||w^(m)||
 * The environment defaults to c = c0 (v = 0) until ssp_set_profile* is called.
 * Tables are uploaded synchronously.  The first plan on a device whose FFT length exceeds
 * the largest single-workgroup FFT (Nz > 8192 for chirp-z plans) also fills a shared
 * twiddle table on that device: one small kernel on the null stream, waited for (so do not
 * create such a plan while a stream capture that forbids null-stream work is in progress).
 * Errors: SSP_E_INVAL, SSP_E_UNSTABLE, SSP_E_UNIMPL (Nz too large), SSP_E_NOMEM,
 * SSP_E_DEVICE.  *out is set to NULL on error. */
ssp_status ssp_plan_create(int Nz, double H, double f, double c0, double dr, int pade_order,
                           int neumann_max, double tol, ssp_plan **out);
/* ssp_plan_create with the boundary condition bc (SSP_BC_*; Sec. 3.1): grid, transform and
 * eigenvalues as listed above; ssp_plan_create is bc = SSP_BC_DIRICHLET.  Sound-speed
 * tables and starters are sampled on the bc's grid; every entry point below works on any
 * bc except ssp_dst_dense_device (Dirichlet only).  Errors as ssp_plan_create, and
 * SSP_E_INVAL for an unknown bc. */
ssp_status ssp_plan_create_bc(int Nz, double H, double f, double c0, double dr, int pade_order,
                              int neumann_max, double tol, int bc, ssp_plan **out);
void ssp_plan_destroy(ssp_plan *plan); /* NULL-safe; releases device memory */
ssp_status ssp_plan_set_option(ssp_plan *plan, int key, double value);
ssp_status ssp_plan_set_stream(ssp_plan *plan, void *hip_stream);

/* Plan facts: sigma, k0, the Pade coefficients in product form (b_j and the combine
 * weights g_j = a_j/b_j, complex as re, im pairs, in application order), the constant C,
 * and the sum form (d0, d_j).  Arrays hold 2*p doubles; any pointer may be NULL. */
ssp_status ssp_plan_info(const ssp_plan *plan, double *sigma, double *k0, double *b,
                         double *g, double *C, double *d0, double *d);
int ssp_max_nz(void);

/* Engine of the plan's fused march: layout actually used (0, 1 or 2, see SSP_OPT_VARIANT),
 * threads per workgroup and the FFT length P: chirp-z length, Nz for periodic direct plans,
 * 2 (Nz + 1) for Dirichlet direct plans (any pointer may be NULL). */
ssp_status ssp_plan_engine(const ssp_plan *plan, int *variant, int *threads, int *fft_length);

/* Convergence of the Neumann series (Sec. 3: the series for (1 + b_j X)^{-1} converges when
 * K_j = b_j L_j^{-1} V is a contraction, L_j the isovelocity operator), per Pade factor j in
 * application order, for the plan's current profile (its first, middle and last tabulated
 * rows, or the analytic Munk profile alone and with the eddy at its centre range) and
 * absorber, evaluated on the host in FP64:
 *   bound[p]     max_l |b_j/(1 + b_j x_l)| max |v|: a norm bound (>= the spectral radius);
 *                below 1 the series converges geometrically for every input
 *   estimate[p]  the spectral radius of K_j by power iteration (iterations products with
 *                two FP64 DST-I each, the growth rate over the second half; largest over
 *                the sampled rows): >= 1 means the series diverges for generic inputs.
 *                Dirichlet plans only (NaN otherwise, or for iterations = 0).
 * Either pointer may be NULL.  Cost: 2 x iterations x p FFT pairs of length >= 2 Nz - 1 on
 * the host (about a second for Nz = 4096, 40 iterations, p = 6). */
ssp_status ssp_plan_contraction(ssp_plan *plan, int iterations, double *bound, double *estimate);

/* Host-only Pade coefficients (Sec. 2; Alg. 1 first step) for sigma = k0 dr, order p and
 * rotation alpha, in the library's factor order: b[2p], g[2p] (product-form weights
 * g_j = a_j/b_j), C[2], d0[2], d[2p] as (re, im) pairs; any output may be NULL.  Touches no
 * device.  Errors: SSP_E_INVAL (p outside [1, 12], non-finite sigma or alpha). */
ssp_status ssp_pade_coefficients(double sigma, int pade_order, double alpha, double *b,
                                 double *g, double *C, double *d0, double *d);

/* Sound speed per range step (Sec. 2: k = omega / c(r, z)).  c is [nsteps][Nz] m/s,
 * row i is used for global step step0 + 1 + i (steps count from 1).  nsteps = -1 gives one
 * row used for every step >= step0 + 1 (range-independent).  Values must be finite
 * and > 0 (SSP_E_INVAL otherwise).  The rows are converted to v = (c0/c)^2 - 1 in FP64
 * and stored on the device in FP32.  A later call replaces the profile. */
ssp_status ssp_set_profile(ssp_plan *plan, int step0, int nsteps, const double *c);
/* Analytic profile evaluated on the device each step (replaces any table). */
ssp_status ssp_set_profile_analytic(ssp_plan *plan, const ssp_env *env);

/* Complex absorbing potential (Sec. 3.1: an imaginary part of the wavenumber in a layer,
 * a simple absorbing boundary that lets a computational domain be truncated):
 * v -> v + i eta(z) on top of whatever profile is set, fixed in range.  eta [Nz] (doubles,
 * finite; eta >= 0 damps, typically zero above a bottom layer and rising inside it) is
 * stored on the device in FP32; NULL removes the absorber.  The Neumann series then runs in
 * complex v; a strong absorber raises the number of terms per series (and, past the
 * series' convergence radius, is reported as SSP_E_DIVERGED by the march). */
ssp_status ssp_set_absorber(ssp_plan *plan, const double *eta);

/* Normal-mode starters (Sec. 3.2): u(0, z) = sqrt(2 pi) sum_m Psi_m(zs) Psi_m(z)/sqrt(kappa_m)
 * for point sources at depths zs[0..nsrc-1] in (0, H), with the mode functions Psi_m (unit L2
 * norm over depth) and horizontal wavenumbers kappa_m of d_z^2 Psi + (k^2(z) - kappa^2) Psi = 0,
 * i.e. of the plan's own vertical operator: k0^2 (1 + X) Psi = kappa^2 Psi.  X is formed
 * densely in the sine basis in FP64 on the device and diagonalised there once for all sources
 * (rocSOLVER dsyevd; three Nz x Nz FP64 matrices of device memory during the call).  Modes:
 * the propagating ones (kappa^2 > 0), lowest first, at most max_modes of them (max_modes <= 0:
 * all).  c [Nz] is the sound speed on the plan's grid (m/s, finite, > 0).  Outputs: psi0
 * [nsrc][Nz] complex (re, im doubles; the starters are real), kappa [Nz] or NULL (the modes'
 * kappa_m, decreasing), n_modes or NULL.  Dirichlet plans with Nz <= 16384 only
 * (SSP_E_UNIMPL otherwise); SSP_E_DEVICE if the eigensolver fails.  Synchronous; the plan's
 * field is not touched (pass a starter to ssp_set_field, ssp_march or ssp_to_sine). */
ssp_status ssp_modal_starter(ssp_plan *plan, const double *c, int nsrc, const double *zs,
                             int max_modes, double *psi0, double *kappa, int *n_modes);

/* Starter: psi0 [Nz] complex (re, im doubles), physical space.  Resets the step
 * counter to 0 and r to 0.  The field is transformed to the sine basis on the device. */
ssp_status ssp_set_field(ssp_plan *plan, const double *psi0);
/* Current field in physical space including the carrier exp(i k0 r): [Nz] complex. */
ssp_status ssp_get_field(const ssp_plan *plan, double *psi);

/* March nsteps range steps from the resident field (Alg. 1).  psi0 may be NULL to
 * continue (resume) or [Nz] complex to (re)start.  Outputs at steps with
 * step_index % out_every == 0:  field_out [nout][Nz] complex (re, im doubles, carrier
 * included) and/or tl_out [nout][Nz] float, TL = -20 log10(|u|/sqrt(r)) dB re 1 m; either
 * may be NULL.  nout = number of output steps in this call (see ssp_count_outputs).
 * Returns SSP_OK, SSP_W_NOT_CONVERGED or SSP_E_DIVERGED (plus argument errors). */
ssp_status ssp_march(ssp_plan *plan, const double *psi0, int nsteps, double *field_out,
                     float *tl_out, ssp_stats *stats);
int ssp_count_outputs(const ssp_plan *plan, int nsteps);

/* Batched march: n plans advanced by nsteps in one persistent launch per FFT-size class.
 * The plans must differ only in their starter, profile and (for different FFT sizes)
 * grid; each plan keeps its own field, counter and statistics.  Outputs are written per
 * plan as in ssp_march (arrays of n pointers, entries may be NULL); stats [n] or NULL.
 * Returns the worst status over the plans (SSP_E_DIVERGED first): the outputs and statistics
 * of every plan are written in any case, and a plan that diverged keeps the field of its
 * last good step. */
ssp_status ssp_march_batch(ssp_plan *const *plans, int n, int nsteps, double *const *field_out,
                           float *const *tl_out, ssp_stats *stats);

/* ssp_march_batch with its own step count per plan (nsteps [n], each >= 0; a plan with 0
 * steps is left unchanged): the batch of a continuous-batching server, whose requests end
 * at different ranges.  Outputs, stats and the returned status as in ssp_march_batch. */
ssp_status ssp_march_batch_steps(ssp_plan *const *plans, int n, const int *nsteps,
                                 double *const *field_out, float *const *tl_out, ssp_stats *stats);

/* ssp_march_batch_steps without host copies, asynchronous on the first plan's stream: the
 * uneven batch of Sec. 4's broadband and serving workloads run from device memory.  The
 * plans' fields stay resident; d_tl_out[i] (device float, may be NULL, or the array NULL)
 * receives plan i's TL rows of the output steps reached, in order, with room for
 * nsteps[i]/out_every + 1 rows of Nz.  Groups of different FFT length run concurrently
 * (side streams forked from and joined into the stream).  With SSP_OPT_GRAPH on the first
 * plan and a non-null stream, the launches are recorded in a HIP graph on the first call and
 * replayed while plans, step counts, output arrays and stream are unchanged (FFT-engine
 * batches).  Statistics (and each plan's step counter on the host) are read with
 * ssp_batch_stats; every host call on a plan first waits for its pending batch.  Dense-engine
 * groups wait for their stream between terms (see SSP_ENGINE_DENSE). */
ssp_status ssp_march_batch_async(ssp_plan *const *plans, int n, const int *nsteps, float *const *d_tl_out);
/* Wait for the plans' pending batches and read their statistics (stats [n] or NULL); returns
 * the worst per-plan status. */
ssp_status ssp_batch_stats(ssp_plan *const *plans, int n, ssp_stats *stats);

/* Device-resident batch for serving and benchmarking (no host copies in the hot path):
 * B solves of one plan's grid and coefficients, each with its own state.  d_psi is a device
 * array [B][Nz] complex64 holding each solve's field in the library's sine-basis
 * representation (see ssp_to_sine / ssp_from_sine); d_step a device int64 [B] of step
 * counters (they may differ between solves); d_tl (may be NULL) a device float
 * [B][nsteps/out_every + 1][Nz] that receives, per solve, the TL rows of the output steps
 * reached in this call, in order; d_stats a device array of B ssp_stats (may be NULL).
 * The call is asynchronous on the plan's stream.  Scratch (per-solve state between Pade
 * factors, output snapshots) is owned by the plan and reused by later calls.  The plan's own
 * field and step counter are not touched.  A solve whose step has no row in a tabulated
 * profile (ssp_set_profile with nsteps > 0) stops there with status SSP_E_INVAL in its
 * statistics.  Dense-engine plans run without graph recording. */
ssp_status ssp_march_device(ssp_plan *plan, int B, void *d_psi, void *d_step, int nsteps,
                            void *d_tl, void *d_stats);
/* ssp_march_device for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments,
 * kernels and results (bitwise), with every scratch array (descriptors, per-solve state
 * between Pade factors, statistics when d_stats is NULL, output snapshots) carved from one
 * fixed device array of SSP_NOALLOC_SCRATCH_MIB MiB that the library holds on each device
 * it runs on until the process ends.  The call allocates nothing, copies nothing from the
 * host (the descriptors are written by a kernel) and is asynchronous on the plan's stream.
 * A batch whose scratch exceeds the array (5 S B complex values, S = P/2 >= Nz for the
 * plan's FFT length P, or S = Nz for a periodic grid whose length is an FFT length, plus Nz B
 * (nsteps/out_every + 1) for TL outputs) is rejected with SSP_E_INVAL; dense-engine plans
 * with SSP_E_UNIMPL.  Every call on a device shares that device's array, which keeps the
 * last call's contents: calls that overlap in time on one device (other streams, other
 * threads) race and must be serialised by the caller.  The statistics kept in the array
 * when d_stats is NULL are not readable by the caller. */
#define SSP_NOALLOC_SCRATCH_MIB 64
ssp_status ssp_march_device_noalloc(ssp_plan *plan, int B, void *d_psi, void *d_step, int nsteps,
                                    void *d_tl, void *d_stats);

/* physical complex64 [B][Nz] (device) -> sine-basis representation (device), in place ok */
ssp_status ssp_to_sine(ssp_plan *plan, int B, const void *d_phys, void *d_sine);
/* sine-basis representation -> physical field with carrier at the given step counters */
ssp_status ssp_from_sine(ssp_plan *plan, int B, const void *d_sine, const void *d_step,
                         void *d_phys);

/* Stand-alone batched orthonormal DST-I (Sec. 3.1) of B complex64 vectors of length Nz,
 * device in/out (may alias), asynchronous on the plan's stream.  For Neumann and periodic
 * plans: the forward transform of the plan's basis (grid values -> coefficients, as
 * listed with SSP_BC_*). */
ssp_status ssp_dst_device(ssp_plan *plan, int B, const void *d_in, void *d_out);

/* The same transform as a dense matrix product Y = S X on the matrix cores (Sec. 3.1: S is
 * the orthonormal DST-I matrix, symmetric and its own inverse).  Each complex vector is two
 * real columns of X; the product runs in fp16 MFMA with FP32 accumulation, every operand
 * split into high and low fp16 parts (three partial products) after exact power-of-two
 * scaling of S and of each column, so the relative error is about 2^-22 (a few 1e-7).
 * Device in/out [B][Nz] complex64 (may alias); asynchronous on the plan's stream.  The
 * plan builds S (2 x 2 bytes per entry, Nz rounded up to 128) and scratch for the split
 * operands on first use.  Nz > ssp_max_dense_nz() or a plan that is not Dirichlet ->
 * SSP_E_UNIMPL. */
ssp_status ssp_dst_dense_device(ssp_plan *plan, int B, const void *d_in, void *d_out);
int ssp_max_dense_nz(void);

const char *ssp_status_string(ssp_status s);
const char *ssp_last_error(void); /* thread-local detail of the last error */

#ifdef __cplusplus
}
#endif
#endif /* SSP_H */
