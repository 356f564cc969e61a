/*
 * mhd.h -- C ABI of the MI355X (gfx950) solver for forced, isothermal, resistive MHD
 * on a triply periodic grid (Vaisala et al., arXiv:2012.08758).
 *
 * What is computed (the paper's Section 4 model, Section 2 numerics):
 *   d ln(rho)/dt = -u.grad ln(rho) - div u                               (Eq. continuity)
 *   du/dt        = -(u.grad)u - cs^2 grad ln(rho) + j x B / rho
 *                  + nu [lap u + 1/3 grad div u + 2 S.grad ln(rho)] + f     (Eq. navierstokes)
 *   dA/dt        = u x B + eta lap A                                       (Eq. magnetic)
 * with B = curl A (+ B_ext), j = curl B (mu0 = 1), S the traceless rate of strain,
 * f the random helical / non-helical forcing of Eqs. forcing, fnorm, feigen;
 * sixth-order central first, second and mixed derivatives (stencil radius 3, the
 * axes and diagonals of Fig. stencils), advanced by the third-order 2N-storage
 * Runge-Kutta scheme (Williamson 1980 coefficients).
 *
 * Conventions for every call:
 *   - Return value is an mhd_status; MHD_OK = 0.  After a failure,
 *     mhd_last_error() gives a message (per thread).  No call throws.
 *   - Device work is enqueued on the HIP stream given at creation (NULL = the
 *     default stream) and is asynchronous unless stated.  Errors raised by
 *     device work surface at the next call that synchronises.
 *   - A context, batch or server is used by one host thread at a time, except
 *     the server calls marked thread-safe.
 *   - Field data are dense arrays of nx*ny*nz values at the run's precision
 *     (float for MHD_FP32, double for MHD_FP64), x fastest:
 *     index = i + nx*(j + ny*k).  Diagnostics are always double.
 *   - Grid points sit at x_i = i*L/N; the box is [0,L)^3, periodic.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MHD_OK = 0,
    MHD_E_INVALID = 1,     /* bad argument (message says which) */
    MHD_E_OOM = 2,         /* device or host allocation failed */
    MHD_E_DEVICE = 3,      /* HIP runtime error */
    MHD_E_NONFINITE = 4,   /* a diagnostic found NaN/Inf in the state */
    MHD_E_BUSY = 5,        /* resource in use (e.g. server slots / budget) */
    MHD_E_UNSUPPORTED = 6, /* valid request this build does not implement */
    MHD_E_NOTFOUND = 7     /* unknown run id */
} mhd_status;

enum { MHD_FP32 = 4, MHD_FP64 = 8 };

enum { MHD_LNRHO = 0, MHD_UX, MHD_UY, MHD_UZ, MHD_AX, MHD_AY, MHD_AZ, MHD_NFIELDS };

/* Parameters of one run (units of Section 4: L = 2 pi, cs = 1, rho0 = 1, mu0 = 1). */
typedef struct {
    int32_t nx, ny, nz;      /* grid points per axis, each >= 8 */
    int32_t precision;       /* MHD_FP32 or MHD_FP64 */
    double lx, ly, lz;       /* box size (> 0) */
    double cs;               /* isothermal sound speed (>= 0) */
    double nu, eta;          /* viscosity and magnetic diffusivity (>= 0) */
    double dt;               /* time step (> 0) */
    double bext[3];          /* imposed uniform field added to B (zero by default) */
    double upwind;           /* upwinding of the continuity advection (Section 4): 0 = off
                                (default), c > 0 adds c |u_a| delta6_a ln rho / (60 h_a) to the
                                ln rho right-hand side, i.e. for c = 1 each u_a d_a ln rho is
                                taken with the fifth-order stencil biased against the flow */
} mhd_params;

/* Forcing record of one step (Section 4, Eqs. forcing, fnorm, feigen):
 *   f(x) = Re{ N f_k exp[i(K.x + phi)] },  K_a = 2 pi k_a / L_a,  N = f0 cs sqrt(|K| cs / dt),
 *   f_k  = [K x (K x e) - i sigma |K| (K x e)] / [sqrt(1+sigma^2) K^2 sqrt(1 - (K.e)^2/K^2)].
 * e is a unit vector not parallel to k; f0 = 0 switches the forcing off for that step.
 * The record is held fixed over the three substeps of its step. */
typedef struct {
    int32_t k[3];
    int32_t pad;
    double e[3];
    double phi;
    double sigma;            /* helicity fraction in [0,1] (any real accepted) */
    double f0;
} mhd_forcing;

/* Global diagnostics of the state at the start of step `step` (time t = step * dt,
 * rounded once, so records do not depend on how the steps were split into calls):
 *   em = <|B|^2>/2, ek = <rho |u|^2>/2, urms = sqrt<|u|^2>, brms = sqrt<|B|^2>,
 *   umax = max |u|, lnrho_mean = <ln rho>, b_mean = <B>, nonfinite = number of
 * cells holding a NaN/Inf in any field.  B uses the same sixth-order curl as the
 * update.  Sums are FP64 at either precision, in a fixed order (deterministic). */
typedef struct {
    int64_t step;
    double t;
    double em, ek, urms, brms, umax, lnrho_mean;
    double b_mean[3];
    int64_t nonfinite;       /* cells holding a NaN or Inf in any field */
    double t_device;         /* device wall clock when this record was reduced on the device
                              * (seconds, arbitrary origin, constant rate): the difference of
                              * two records of a run is its measured time per step */
} mhd_diag;

typedef struct mhd_ctx mhd_ctx;
typedef struct mhd_batch mhd_batch;
typedef struct mhd_server mhd_server;

/* ---------------------------------------------------------------- single run */

/* Create a run and allocate its 14 device arrays (two buffer sets of 7 fields).
 * The state starts at zero.  hip_stream: a hipStream_t, or NULL. */
mhd_status mhd_create(const mhd_params *p, void *hip_stream, mhd_ctx **out);

/* Same, but the caller owns the memory: bufs[0..13] are device pointers to
 * nx*ny*nz values each (bufs[0..6] = state fields, bufs[7..13] = the second set).
 * The caller keeps them alive until mhd_destroy and does not touch them while
 * work is in flight. */
mhd_status mhd_create_borrowed(const mhd_params *p, void *const bufs[14], void *hip_stream,
                               mhd_ctx **out);

/* Synchronise and free everything the context owns.  NULL is accepted. */
mhd_status mhd_destroy(mhd_ctx *ctx);

/* Copy one field in (src) or out (dst).  on_device != 0: device pointer (stream-
 * ordered, asynchronous); 0: host pointer (synchronous). */
mhd_status mhd_set_field(mhd_ctx *ctx, int field, const void *src, int on_device);
mhd_status mhd_get_field(mhd_ctx *ctx, int field, void *dst, int on_device);

/* Section 4 initial condition: ln rho = 0, u = 0, A_c = a_noise * N(0,1) per cell,
 * from SplitMix64 stream (seed, 104 + c), Box-Muller on consecutive pairs. */
mhd_status mhd_init_seed(mhd_ctx *ctx, uint64_t seed, double a_noise);

/* Forcing schedule consumed by the following steps, one record per step.
 * Replaces any earlier schedule.  Steps beyond the schedule are an error. */
mhd_status mhd_set_forcing(mhd_ctx *ctx, const mhd_forcing *recs, int64_t n);

/* Random schedule generated on demand: step n draws k from the shell
 * kf-1/2 <= |k| <= kf+1/2, e uniform on the sphere and phi uniform in [-pi,pi)
 * from SplitMix64 stream (seed, 1), counters 8n .. 8n+5; sigma and f0 fixed. */
mhd_status mhd_set_forcing_random(mhd_ctx *ctx, double kf, double f0, double sigma,
                                  uint64_t seed);

/* No forcing for the following steps (the default). */
mhd_status mhd_clear_forcing(mhd_ctx *ctx);

/* Advance nsteps full RK3 steps (3 fused substeps each).  Each step also
 * records the diagnostics of its input state.  Asynchronous. */
mhd_status mhd_step(mhd_ctx *ctx, int64_t nsteps);

/* mhd_step with a HIP event recorded around every kernel launch on the run's
 * stream; synchronises.  kernel_ms[0..2]: mean duration of the substep-1, -2 and -3
 * kernels, kernel_ms[3]: of the diagnostic finalize kernel; step_ms[i] (nsteps
 * entries, may be NULL): wall time of step i from its first to its last event. */
mhd_status mhd_step_timed(mhd_ctx *ctx, int64_t nsteps, double kernel_ms[4], double *step_ms);

/* Record the diagnostics of the current state (one extra pass). Asynchronous. */
mhd_status mhd_reduce(mhd_ctx *ctx);

/* Copy out diagnostic records collected so far (oldest first), up to cap.
 * *n_out = number available (may exceed cap).  Synchronises. */
mhd_status mhd_get_diag(mhd_ctx *ctx, mhd_diag *out, int64_t cap, int64_t *n_out);
mhd_status mhd_clear_diag(mhd_ctx *ctx);

/* Step counter and time of the current state. */
mhd_status mhd_get_time(mhd_ctx *ctx, int64_t *step, double *t);

/* Block until queued work finishes; reports deferred device errors. */
mhd_status mhd_sync(mhd_ctx *ctx);

/* Device pointer of field `field` of the current state (valid until the next step). */
mhd_status mhd_field_ptr(mhd_ctx *ctx, int field, void **dptr);

/* Least-squares slope of ln(brms) against t over records [i0, i1) (Section 5.1:
 * B_rms ~ exp(lambda t)).  Host-only, FP64.  Needs i1 - i0 >= 2. */
mhd_status mhd_growth_rate(const mhd_diag *d, int64_t n, int64_t i0, int64_t i1,
                           double *lambda);

/* Magnetic power spectrum of the current state (Section 5.3).  B = curl A with the
 * sixth-order first derivative (plus b_ext); with B_hat(k) = sum_x B(x) exp(-i k.x),
 * shell s (s = 0 .. nshell-1) collects the wavevectors with s - 1/2 <= |k|/dk < s + 1/2,
 * dk = 2 pi / max(lx, ly, lz), and out[s] = V / (2 dk Ncell^2) * sum_{k in s} |B_hat(k)|^2,
 * so that sum_s out[s] dk = (1/2) int |B|^2 dV (V = lx ly lz, mu0 = 1).  Computed on the
 * run's stream in FP64 at either precision: an FFT of the three A components, the curl
 * applied as its Fourier symbol i kappa(k) x (kappa_a the modified wavenumber of the
 * first-derivative stencil), a deterministic shell sum.  Every grid side must be a product
 * of 2, 3, 5 and 7 and at most 4096 (else MHD_E_UNSUPPORTED).  Writes min(cap, nshell)
 * values to the host array out, the shell count to *nshell and the shell width to *dk
 * (either may be NULL); cap = 0 only queries nshell and dk (no device work).
 * Synchronises.  The first computing call allocates a device workspace of about
 * 48 (nx/2+1) ny nz bytes (mhd_spectrum_shells reports it), kept until mhd_destroy;
 * MHD_E_OOM if it does not fit. */
mhd_status mhd_spectrum(mhd_ctx *ctx, double *out, int32_t cap, int32_t *nshell, double *dk);

/* The magnetic spectrum of mhd_spectrum for callers that cannot allocate device memory
 * (code under stream capture, serving loops, harnesses that forbid hipMalloc): the
 * workspace is a static device array of 64 MiB that the library holds on each GPU it
 * runs on until the process ends (grids up to about 128^3; larger ones return
 * MHD_E_UNSUPPORTED before any device work).  out_dev is a device array of cap doubles
 * (caller-owned) that receives the first min(cap, nshell) shells on the run's stream;
 * the call neither allocates nor synchronises, and its result is ready once the stream
 * is.  *nshell and *dk as in mhd_spectrum (either may be NULL); cap = 0 only queries
 * them.  All calls on one GPU share the scratch: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller. */
mhd_status mhd_spectrum_noalloc(mhd_ctx *ctx, double *out_dev, int32_t cap, int32_t *nshell, double *dk);

/* Shell count, shell width and spectrum workspace bytes for runs of this size
 * (host-only).  MHD_E_UNSUPPORTED (outputs still written) if a side is not a product of
 * 2, 3, 5 and 7 at most 4096. */
mhd_status mhd_spectrum_shells(const mhd_params *p, int32_t *nshell, double *dk, size_t *workspace_bytes);

/* Growth rate of one spectral channel from samples (t_i, E_i), i < n: half the
 * least-squares slope of ln E against t (Section 5.1: E_B,k ~ exp(2 lambda_k t), so that
 * lambda_k and the B_rms rate agree).  Host-only, FP64.  Needs n >= 2, E_i > 0. */
mhd_status mhd_channel_growth_rate(const double *t, const double *e, int64_t n, double *lambda);

/* Thread-local message of the last failure ("" if none). */
const char *mhd_last_error(void);

/* The forcing record that mhd_set_forcing_random(kf, f0, sigma, seed) uses at
 * step n (host-only; no device work). */
mhd_status mhd_forcing_draw(double kf, double f0, double sigma, uint64_t seed, int64_t n,
                            mhd_forcing *out);

/* Number of compiled tile shapes, and shape i as "TXxTYxTZ/cz" (box tiles, with
 * "+ring" for the direct-to-LDS ring kernel and "+march" for the marching-slab kernel)
 * or "TXxTY+zm" (z-marching column tiles; "64x8+zm": FP32 only, substeps 2 and 3 on
 * 64x8 tiles, the first substep and the diagnostics on 32x8). */
int32_t mhd_num_tile_shapes(void);
mhd_status mhd_tile_shape_name(int32_t i, char *buf, size_t len);

/* Pin tile shape i for later contexts of this (grid, precision) (host-only; the
 * same table mhd_autotune writes).  i = -1 removes the pin. */
mhd_status mhd_set_tile_shape(const mhd_params *p, int32_t i);

/* Tile shape used for runs of this size and precision, in the same form (chosen by
 * the autotuner or the default table); writes into buf. */
mhd_status mhd_tile_config(const mhd_params *p, char *buf, size_t len);

/* Tile shape this context's launches use, in the same form (a context of a batch may
 * differ from mhd_tile_config: see mhd_batch_create). */
mhd_status mhd_ctx_tile_config(const mhd_ctx *ctx, char *buf, size_t len);

/* Try every compiled tile shape on a scratch run of this size and precision, time
 * `reps` steps of each on the given stream, and keep the fastest for later
 * contexts of the same (grid, precision).  best_ms: time per step of the winner. */
mhd_status mhd_autotune(const mhd_params *p, int reps, void *hip_stream, double *best_ms);

/* ---------------------------------------------------------------- batched ensemble */

/* A set of independent runs (any grid sizes, same or mixed precision) advanced
 * together: each substep of every run is one tile list, launched as one kernel per
 * (precision, tile shape) class.  Runs never wait on each other's data.  Each run
 * takes the tile shape it would take alone (so its state is bit for bit the same),
 * except that when the runs of one precision bring at least 2^22 cells together they
 * fill the chip, and every run of that precision takes the filled-chip shape (the
 * z-marching tile where its grid allows it, else the large ring tile) unless
 * mhd_autotune pinned a shape for it (its state then matches the run alone to the
 * parity bar, and the run alone on the same pinned shape bit for bit). */
mhd_status mhd_batch_create(const mhd_params *runs, int32_t n, void *hip_stream,
                            mhd_batch **out);
mhd_status mhd_batch_destroy(mhd_batch *b);

/* The context of run i (owned by the batch): use it to set fields, forcing and
 * read diagnostics.  Do not call mhd_step / mhd_destroy on it. */
mhd_status mhd_batch_ctx(mhd_batch *b, int32_t i, mhd_ctx **ctx);

/* Advance every run by nsteps.  use_graph != 0: the launches of all nsteps are
 * captured once into a HIP graph and replayed (the capture is reused while the
 * batch and nsteps are unchanged).  Asynchronous. */
mhd_status mhd_batch_run(mhd_batch *b, int64_t nsteps, int use_graph);

/* ---------------------------------------------------------------- serving */

typedef enum { MHD_RUN_QUEUED = 0, MHD_RUN_ACTIVE = 1, MHD_RUN_DONE = 2, MHD_RUN_FAILED = 3 } mhd_run_state;

typedef struct {
    int32_t state;          /* mhd_run_state */
    int32_t precision;
    int64_t steps_done;
    int64_t steps_total;
    double t_submit, t_admit, t_done;   /* seconds on the server clock */
    double em, brms;        /* last diagnostics */
} mhd_run_info;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int64_t ticks;
    int64_t step_samples;          /* per-run step latencies recorded */
    double lat_p50_ms, lat_p90_ms, lat_p99_ms;   /* per-step latency of active runs: for every
                                                  * run and step, the device-clock time between
                                                  * its consecutive diagnostic records */
    double queue_p50_s, queue_p99_s;             /* submit -> admit */
    double e2e_p50_s, e2e_p99_s;                 /* submit -> done */
    double busy_s, wall_s;
    double cell_substeps;          /* total work done */
    size_t hbm_in_use, hbm_peak;
} mhd_server_stats;

/* A request loop with continuous batching: runs are admitted (first come, first
 * served) while the sum of their device footprints stays within hbm_budget bytes
 * and a slot is free; every tick advances all active runs in batched launches;
 * finished runs leave and free their memory at tick boundaries.  Active runs are
 * grouped by precision, tile shape and power-of-two size class: the group with the
 * most cells advances steps_per_tick steps per tick, every other group about
 * steps_per_tick * (its cost ratio) steps (at most 512, never past a run's end), so
 * each group's share of a tick takes about as long and small runs progress at their
 * own speed.  The loop runs on its own host thread between mhd_server_start and _stop. */
mhd_status mhd_server_create(size_t hbm_budget, int32_t max_slots, int32_t steps_per_tick,
                             void *hip_stream, mhd_server **out);
mhd_status mhd_server_start(mhd_server *s);
/* Thread-safe.  Queue a run: initial condition from mhd_init_seed(seed, a_noise),
 * forcing from mhd_set_forcing_random(kf, f0, sigma, seed).  retain != 0: the final
 * state is copied to host memory when the run finishes, for mhd_server_get_field. */
mhd_status mhd_server_submit(mhd_server *s, const mhd_params *p, uint64_t seed, double a_noise,
                             double kf, double f0, double sigma, int64_t nsteps, int32_t retain,
                             int64_t *id);
/* Thread-safe. */
mhd_status mhd_server_poll(mhd_server *s, int64_t id, mhd_run_info *info);
/* Thread-safe.  Block until the run is done or failed, or timeout_s passes (MHD_E_BUSY). */
mhd_status mhd_server_wait(mhd_server *s, int64_t id, double timeout_s);
/* Thread-safe.  Copy a field of a finished run submitted with retain != 0 (host dst). */
mhd_status mhd_server_get_field(mhd_server *s, int64_t id, int field, void *dst);
/* Thread-safe.  Forget a finished run (frees its retained state). */
mhd_status mhd_server_release(mhd_server *s, int64_t id);
/* Thread-safe. */
mhd_status mhd_server_stats_get(mhd_server *s, mhd_server_stats *st);
/* Stop the loop after the current tick (queued and active runs stay). */
mhd_status mhd_server_stop(mhd_server *s);
mhd_status mhd_server_destroy(mhd_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MHD_H */
