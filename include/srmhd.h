/*
 * srmhd.h -- C ABI of libsrmhd.so: SSP Runge-Kutta steps of 3D ideal special-
 * relativistic MHD (flat space, Cartesian, periodic box) on an MI355X, with a
 * learned Newton guess and its training kernels.
 *
 * The method follows Del Zanna et al., "A GPU-Accelerated Modern Fortran
 * Version of the ECHO Code for Relativistic Magnetohydrodynamics" (arXiv
 * 2401.03008): the ideal SRMHD system and its conserved variables (Sec. 2),
 * the semi-discrete point-value scheme with face-staggered B and edge electric
 * fields, and the five parts of each Runge-Kutta substep -- INT + Newton
 * inversion, REC + upwind fluxes + stored fast speeds, DER, UCT, RK update with
 * a timestep from the global maximum of the speeds once per step (Sec. 3).
 * Formulas the paper leaves to its references are taken from the published
 * methods named at each entry point.
 *
 * Conventions for every entry point
 *   - Device pointers are HIP device addresses on the context's device; host
 *     pointers are marked (host).  Every grid array is nx*ny*nz doubles
 *     (nx*ny*(nz + 2 ghost_z) for a slab context), contiguous, x fastest:
 *     a[(k*ny + j)*nx + i].
 *   - bface[d] holds B_d on the +d face of each cell (x_{i+1/2} for d = 0).
 *   - The caller owns every buffer; the library allocates no device memory.
 *     Scratch comes from srmhd_buffers.work (size from srmhd_work_bytes), or
 *     for srmhd_mlp_forward_noalloc from a fixed static device array.
 *   - All GPU work is enqueued on the stream given to srmhd_create, in order;
 *     only calls documented as "syncs" wait for the stream.
 *   - Return value: SRMHD_OK (0) or a negative SRMHD_E_* code.  Argument
 *     errors are detected on the host before any launch.  Failures detected on
 *     the device set a device error word that the next syncing call returns.
 *     srmhd_last_error gives the message of the last failure of a context.
 *   - A context is used from one host thread at a time.
 */
#ifndef SRMHD_H
#define SRMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRMHD_OK 0
#define SRMHD_E_INVAL (-1)     /* bad argument or configuration */
#define SRMHD_E_HIP (-2)       /* a HIP runtime call failed */
#define SRMHD_E_C2P (-3)       /* Newton inversion failed in some cell */
#define SRMHD_E_NONFINITE (-4) /* non-finite conserved data or timestep */
#define SRMHD_E_STATE (-5)     /* call out of order (e.g. step before init) */

enum { SRMHD_HLL = 0, SRMHD_LLF = 1 };
enum { SRMHD_FP64 = 0, SRMHD_MIXED = 1 };
/* Newton guess: the previous inversion's W; the learned guess where no usable
 * previous W exists (W <= 0 or v^2(W) >= 1, e.g. after srmhd_set_state with
 * no W), the previous W elsewhere; a cold start from W0 = U; or the learned
 * guess first in every cell (the previous W where Newton from it fails). */
enum { SRMHD_GUESS_PREV = 0, SRMHD_GUESS_MLP = 1, SRMHD_GUESS_COLD = 2,
       SRMHD_GUESS_MLP_ALL = 3 };
/* Reconstruction (REC, Sec. 3): MP5 (Suresh & Huynh 1997), or linear with the
 * monotonized-central limiter of van Leer (1977), the second-order option of
 * the benchmark section. */
enum { SRMHD_REC_MP5 = 0, SRMHD_REC_MC = 1 };

/* Device error word bits (srmhd_diag.error_word). */
#define SRMHD_ERRBIT_C2P 1u       /* an inversion did not converge */
#define SRMHD_ERRBIT_NONFINITE 2u /* non-finite or unusable conserved input */
#define SRMHD_ERRBIT_DT 4u        /* timestep not finite and positive */
#define SRMHD_ERRBIT_PRESSURE 8u  /* recovered p <= 0 with no floor set */

typedef struct {
  int nx, ny, nz;   /* cells per direction, each >= 1 (1 makes a uniform
                       direction: a 2D or 1D box); nx*ny*nz < 2^31 */
  double lx, ly, lz;/* box lengths (> 0) */
  double gamma_ad;  /* adiabatic index, 1 < gamma_ad <= 2 (4/3 in all tests) */
  double cfl;       /* dt = cfl / max_cells sum_d max(a+,a-)_d/dx_d */
  double dt_fixed;  /* > 0: fixed dt instead of the CFL rule */
  int riemann;      /* SRMHD_HLL or SRMHD_LLF */
  int precision;    /* SRMHD_FP64, or SRMHD_MIXED: REC + face fluxes in FP32 */
  int guess;        /* SRMHD_GUESS_PREV, _COLD, _MLP or _MLP_ALL (the last
                       two need srmhd_set_mlp before the first step) */
  int newton_maxit; /* Newton iteration cap, 1..1000 (50) */
  double newton_tol;/* relative step tolerance on W (1e-14) */
  double pfloor;    /* pressure floor as a fraction of rho; 0 = none */
  int collect_stats;/* 1: Newton histogram / counters per inversion */
  int recon;        /* SRMHD_REC_MP5 (default) or SRMHD_REC_MC */
  int time_order;   /* 3: SSP-RK3 (default); 2: SSP-RK2 (Shu & Osher 1988),
                       U1 = U0 + dt L(U0), U = (U0 + U1 + dt L(U1))/2 */
  int high_order;   /* HO = YES of Sec. 3 (needs SRMHD_REC_MP5): sixth-order
                       INT (3, -25, 150, 150, -25, 3)/256 of the six nearest
                       faces; sixth-order DER of the face fluxes and of the
                       edge fields in the curl, d/dx f = (-9 f_{-5/2} + 125
                       f_{-3/2} - 2250 f_{-1/2} + 2250 f_{1/2} - 125 f_{3/2}
                       + 9 f_{5/2}) / (1920 dx); MP5 around the point-value
                       interpolation (3, -20, 90, 60, -5)/128.  div B in the
                       diagnostics is then the same sixth-order difference
                       of the face B, which the HO curl keeps constant. */
  int ghost_z;      /* 0: the box is periodic in z.  G > 0: the context holds
                       one z-slab of a larger box periodic in z, split into
                       slabs for domain decomposition (Sec. 3 decomposes over
                       ranks; the enlarged halo of the closing section lets
                       one exchange per Runge-Kutta stage suffice): nz and lz
                       are the slab's interior planes and length, and every
                       grid array holds nx*ny*(nz + 2G) values, the G planes
                       below and above the interior being ghost copies of the
                       neighbouring slabs' edge planes.  G >= 4 (>= 8 with
                       high_order): one stage's update of a plane reads the
                       state of the 4 planes below and 3 above it (8 and 7
                       with HO).  nz >= G.  x and y stay periodic.  Such a
                       context steps only through srmhd_stage_begin/_end,
                       with srmhd_halo_pack/_unpack after every stage. */
} srmhd_config;

typedef struct {
  double *cons[5];   /* D, Sx, Sy, Sz, U at cell centres (device) */
  double *bface[3];  /* staggered B_x, B_y, B_z (device) */
  double *guess_w;   /* per-cell Newton guess / converged W (device) */
  void *work;        /* scratch (device), >= srmhd_work_bytes, 256-B aligned */
  size_t work_bytes;
} srmhd_buffers;

typedef struct {
  double t;              /* simulated time */
  double dt;             /* last timestep */
  long step;             /* full RK steps taken */
  double amax;           /* last max_cells sum_d max(a+,a-)_d/dx_d */
  double divb_max;       /* max over cells |div_h B| (sixth-order differences
                            with high_order) */
  double sums[8];        /* sum over cells of D, Sx, Sy, Sz, U, Bx, By, Bz(face) */
  long newton_iters;     /* Newton iterations summed over inversions */
  long newton_calls;     /* inversions counted */
  long newton_hist[32];  /* histogram of per-inversion iteration counts */
  long c2p_failures;     /* inversions that did not converge */
  long recon_fallbacks;  /* face states replaced by first-order values */
  long floors;           /* pressure floors applied */
  long mlp_fallbacks;    /* learned-guess inversions redone from the old W */
  unsigned error_word;   /* SRMHD_ERRBIT_* accumulated since the last reset */
} srmhd_diag;

typedef struct srmhd_ctx srmhd_ctx;

/* Fill *cfg with the defaults: 32^3 unit box, gamma 4/3, cfl 0.5, HLL, FP64,
 * previous-W guess, maxit 50, tol 1e-14, no floor, stats on, MP5, SSP-RK3,
 * HO off. */
int srmhd_config_default(srmhd_config *cfg);

/* Size in bytes of the scratch a context with *cfg needs.  Validates *cfg;
 * no GPU call. */
int srmhd_work_bytes(const srmhd_config *cfg, size_t *bytes);

/* Create a context over caller-owned device buffers.  stream is a
 * hipStream_t (NULL = default stream); the current HIP device becomes the
 * context's device.  The library keeps the pointers, never frees them. */
int srmhd_create(const srmhd_config *cfg, const srmhd_buffers *buf,
                 void *stream, srmhd_ctx **out);

/* Set the state from cell-centred rho, vx, vy, vz, p (prim5, device) and
 * face B (bface, device; copied into the state's face arrays).  Conserved
 * variables follow Sec. 2 with centred B = INT of bface (face average, or
 * the sixth-order interpolation with high_order); the
 * guess W is set to rho h Gamma^2.  Resets t, step, counters and the error
 * word. */
int srmhd_init_from_prims(srmhd_ctx *ctx, const double *const prim5[5],
                          const double *const bface[3]);

/* Enqueue nsteps full SSP-RK3 (or, with time_order 2, SSP-RK2) steps (Shu &
 * Osher 1988) of the Sec. 3 scheme: per stage INT + Newton inversion, REC
 * (MP5 of Suresh & Huynh 1997, or linear MC) of rho, v, p and transverse
 * centred B, HLL/LLF face fluxes with the Del Zanna et al. (2003) fast-speed
 * bound, UCT edge fields (Londrillo & Del Zanna 2004), flux divergence and
 * curl (DER, sixth order with high_order); dt from the first stage's speeds.
 * Asynchronous; t and dt stay on the device. */
int srmhd_step(srmhd_ctx *ctx, int nsteps);

/* Spatial operator on the current state: INT + inversion, then
 * rhs[0..4] = -sum_d (Fhat(+d face) - Fhat(-d face))/dx_d at the centres and
 * rhs[5+d] = -(curl_h E)_d on the d faces (Sec. 3 semi-discrete equations);
 * *amax_dev (device, one double) receives max_cells sum_d max(a+,a-)_d/dx_d.
 * Updates the guess W.  Asynchronous. */
int srmhd_rhs(srmhd_ctx *ctx, double *const rhs[8], double *amax_dev);

/* INT + inversion of the current state into caller device arrays
 * prim[0..7] = rho, vx, vy, vz, p, Bcx, Bcy, Bcz.  Updates the guess W.
 * Asynchronous. */
int srmhd_get_primitives(srmhd_ctx *ctx, double *const prim[8]);

/* Diagnostics (host struct).  Syncs the stream.  Sums and div B use fixed-
 * order reductions (bitwise reproducible).  Returns SRMHD_E_C2P /
 * SRMHD_E_NONFINITE if the device error word is set (the struct is still
 * filled). */
int srmhd_get_diagnostics(srmhd_ctx *ctx, srmhd_diag *out);

/* Clear counters and the error word.  Asynchronous. */
int srmhd_reset_counters(srmhd_ctx *ctx);

/* Simulated time and step count (host values).  get syncs; set is
 * asynchronous. */
int srmhd_get_time(srmhd_ctx *ctx, double *t, long *step, double *dt);
int srmhd_set_time(srmhd_ctx *ctx, double t, long step);

/* The evolved state of the scheme (Sec. 3): the cell-centred conserved
 * variables D, S, U, the staggered face B, and the per-cell Newton guess W
 * that the next inversion of this state starts from (the converged W =
 * rho h Gamma^2 of the inversion before it), with the simulated time and
 * step count.  Together they are a checkpoint: a context given them
 * by srmhd_set_state continues bit for bit as the one they came from.
 *
 * srmhd_get_state copies the state into caller device arrays (cons[5],
 * bface[3], w; each nx*ny*nz doubles, the layout above; cons, bface or w may
 * be NULL to skip) and the time and step count into host values (t, step;
 * either may be NULL).  Syncs.  SRMHD_E_STATE before the state is set.
 *
 * srmhd_set_state copies cons[5] and bface[3] (device, required) into the
 * context's state and w (device) into its guess array; w = NULL means no
 * previous W: the next inversion starts from the learned guess (learned
 * form) or from U.  Sets t and the step count, clears the counters, the
 * running speed maximum and the error word.  The face B should be
 * divergence-free as the scheme keeps it; it is not checked.  Source arrays
 * may be the context's own (no copy).  Asynchronous. */
int srmhd_get_state(srmhd_ctx *ctx, double *const cons[5], double *const bface[3],
                    double *w, double *t, long *step);
int srmhd_set_state(srmhd_ctx *ctx, const double *const cons[5],
                    const double *const bface[3], const double *w, double t,
                    long step);

/* ---------------------------------------------------------------------
 * One Runge-Kutta stage in two halves, for a driver that splits a box into
 * z-slabs (config.ghost_z) and exchanges ghost planes between them once per
 * stage; on a periodic context (ghost_z = 0) the same sequence gives the
 * srmhd_step result bit for bit.  A step is stages 1..3 (SSP-RK3) or 1..2
 * (SSP-RK2), each stage_begin(s) followed by stage_end(s), in order;
 * anything else returns SRMHD_E_STATE.  Between stages, and after the last
 * one, the slabs exchange ghost planes (srmhd_halo_pack on each slab,
 * srmhd_halo_unpack on its neighbours).  Other entry points that touch the
 * state (step, rhs, get/set_state, get_primitives, init, harvest,
 * mlp_guess) return SRMHD_E_STATE while a step is under way.
 *
 * srmhd_stage_begin: INT + inversion of every plane, REC + upwind fluxes
 * and fast speeds (Sec. 3); in stage 1 also this slab's max over its
 * interior cells of sum_d max(a+,a-)_d/dx_d.  Asynchronous.
 *
 * srmhd_local_amax (after stage_begin(1)): that maximum into amax_dev
 * (device, one double), for a max-reduction over the slabs.  Asynchronous.
 *
 * srmhd_stage_end: in stage 1, dt = cfl / *amax_dev (device; the max over
 * all slabs; NULL = this slab's own maximum), or dt_fixed; then UCT, DER and
 * the stage's Runge-Kutta update.  amax_dev is ignored in later stages.
 * Asynchronous. */
int srmhd_stage_begin(srmhd_ctx *ctx, int stage);
int srmhd_local_amax(srmhd_ctx *ctx, double *amax_dev);
int srmhd_stage_end(srmhd_ctx *ctx, int stage, const double *amax_dev);

/* Ghost planes of a slab context (ghost_z = G > 0): the exchanged values are
 * the 9 state arrays D, Sx, Sy, Sz, U, face B_x, B_y, B_z and the Newton
 * guess W (G planes of each) of the current stage's state.
 * srmhd_halo_count: *n (host) = 9*G*nx*ny, the doubles of one side's buffer.
 * srmhd_halo_pack: side 0 = the G lowest interior planes (for the slab
 * below), side 1 = the G highest (for the slab above), into buf (device,
 * array-major: array a's planes at buf[a*G*nx*ny]).
 * srmhd_halo_unpack: buf into the ghost planes of side 0 (below the
 * interior) or 1 (above), from the neighbour's pack of its facing side.
 * SRMHD_E_STATE on a periodic context or between the halves of a stage.
 * Asynchronous on the context's stream; a buffer from another context's
 * stream needs the caller's ordering. */
int srmhd_halo_count(const srmhd_ctx *ctx, size_t *n);
int srmhd_halo_pack(srmhd_ctx *ctx, int side, double *buf);
int srmhd_halo_unpack(srmhd_ctx *ctx, int side, const double *buf);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch (adds a small host/queue overhead per launch; off by
 * default).  Classes, in order: 0 inversion, 1 face fluxes of the x and y
 * faces (one kernel), 2 face fluxes of the z faces, 3-5 UCT edge fields
 * E_x/E_y/E_z, 6 RK update, 7 timestep, 8 RK update fused with the inversion
 * of its result for the next stage (periodic boxes without HO, previous-W or
 * cold guess; class 0 then runs only where no stage before inverted the
 * state) (the learned guess's inference is part of class 0).
 * srmhd_get_kernel_times syncs and
 * returns the accumulated milliseconds and launch counts since timing was
 * last enabled (ms, launches: host arrays of SRMHD_NKCLASS). */
#define SRMHD_NKCLASS 9
int srmhd_kernel_timing(srmhd_ctx *ctx, int enable);
int srmhd_get_kernel_times(srmhd_ctx *ctx, double *ms, long *launches);

/* ---------------------------------------------------------------------
 * Learned Newton guess (not part of the paper; the inversion it seeds is the
 * Sec. 3 Newton step): a 5 -> 64 -> 64 -> 2 ReLU network, BF16 weights, FP32
 * accumulation on the matrix cores.  Inputs: the five invariants of a
 * conserved state on which the inversion depends, log(U/D), |S|/U, B^2/U,
 * tau^2/(S^2 B^2 + 1e-300), log D (tau = S.B), standardised.  Outputs: the
 * standardised log(p/D) and log Gamma of the converged inversion, giving
 * W0 = D Gamma + g/(g-1) p Gamma^2.  With SRMHD_GUESS_MLP the network seeds
 * Newton only in cells without a usable previous W (its guess is ~5e-3 from
 * the root, the previous stage's W ~1e-4: measured, it costs iterations
 * wherever a warm start exists), and a cold start from U is the fallback;
 * once every cell holds a W from a completed inversion (after
 * srmhd_init_from_prims, or after the first inversion that follows
 * srmhd_set_state) the form runs the previous-W kernels.  With
 * SRMHD_GUESS_MLP_ALL the network seeds every cell and the previous W is the
 * fallback.  The convergence test is unchanged, so results agree with the
 * plain form to the Newton tolerance.
 *
 * Parameter vector, FP32 master and BF16 copy in the same layout (rows are
 * output units): W1[64][5] | b1[64] | W2[64][64] | b2[64] | W3[2][64] | b3[2].
 * Training arrays are row-major: x (batch x 5), y and t (batch x 2).
 * ------------------------------------------------------------------- */
#define SRMHD_MLP_NPARAM 4674
#define SRMHD_MLP_OFF_W1 0
#define SRMHD_MLP_OFF_B1 320
#define SRMHD_MLP_OFF_W2 384
#define SRMHD_MLP_OFF_B2 4480
#define SRMHD_MLP_OFF_W3 4544
#define SRMHD_MLP_OFF_B3 4672

/* Use the network (device params: FP32 biases and BF16 weights, caller-owned,
 * kept by pointer; w_bf16 8-byte aligned, else SRMHD_E_INVAL) for the guess.
 * norm (host, 14 floats): feature means[5], feature std[5], output means[2],
 * output std[2].  Asynchronous. */
int srmhd_set_mlp(srmhd_ctx *ctx, const float *params, const uint16_t *w_bf16,
                  const float *norm);

/* Switch the Newton guess (SRMHD_GUESS_*; _MLP needs srmhd_set_mlp). */
int srmhd_set_guess(srmhd_ctx *ctx, int guess);

/* The learned guess of every cell of the current state, from the same
 * feature and inference code the learned-guess inversion runs (nothing is
 * inverted; the state and W are not modified).  out (device, 2*nx*ny*nz
 * floats): the network's de-standardised outputs, log(p/D) at out[id] and
 * log Gamma at out[ncell + id]; w0 (device, nx*ny*nz doubles, or NULL): the
 * guess W0 = D Gamma + g/(g-1) p Gamma^2 they give (with log Gamma clamped
 * at 0), or -1 where a feature is not finite.  Needs srmhd_set_mlp
 * (SRMHD_E_STATE otherwise).  Asynchronous. */
int srmhd_mlp_guess(srmhd_ctx *ctx, float *out, double *w0);

/* Training pairs from the current state: each cell is kept with probability
 * frac (counter-based hash of its index and seed), inverted from the stored W
 * (W not modified); feats (device, cap x 5) get its features, targets
 * (device, cap x 2) log(p/D) and log Gamma.  *n_out (host) = pairs written
 * (<= cap).  Syncs. */
int srmhd_harvest(srmhd_ctx *ctx, float *feats, float *targets, int cap,
                  double frac, unsigned seed, int *n_out);

/* Scratch (device, 256-B aligned) for one batch of forward + backward; 0 if
 * batch is out of range (1..524288). */
size_t srmhd_mlp_cache_bytes(int batch);

/* w_bf16 = round-to-nearest-even BF16 of params (n values). Asynchronous. */
int srmhd_mlp_quantize(const float *params, uint16_t *w_bf16, int n, void *stream);

/* y (batch x 2, device) = network(x); keeps activations in cache for the
 * backward pass.  All pointers device.  Asynchronous on stream. */
int srmhd_mlp_forward(const float *params, const uint16_t *w_bf16, const float *x,
                      float *y, void *cache, int batch, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward pass of srmhd_mlp_forward (same kernels, the same y bit for bit)
 * without the activation cache.  Its scratch is a static device array inside
 * the library, 18 MiB per GPU, held until the process ends, so batch is
 * limited to 1..65536 (SRMHD_E_INVAL beyond, before any launch, with the
 * message in srmhd_last_error(NULL)).  params, w_bf16, x, y: device, as in
 * srmhd_mlp_forward; stream: a hipStream_t of the current device.  No device
 * memory is allocated or freed.  Every call on a GPU shares that GPU's
 * scratch: calls that overlap on one GPU (different streams or host threads
 * without ordering) race; calls in order on one stream do not.
 * Asynchronous. */
#define SRMHD_MLP_NOALLOC_MAX_BATCH 65536
int srmhd_mlp_forward_noalloc(const float *params, const uint16_t *w_bf16,
                              const float *x, float *y, int batch, void *stream);

/* Mean squared error over the 2*batch outputs into *loss (device) and its
 * gradient with respect to y into cache.  Asynchronous. */
int srmhd_mlp_loss_grad(const float *y, const float *t, void *cache, float *loss,
                        int batch, void *stream);

/* grad (device, SRMHD_MLP_NPARAM floats) = d loss / d params, from the cache
 * of the last forward + loss_grad with the same batch.  Asynchronous. */
int srmhd_mlp_backward(const uint16_t *w_bf16, void *cache, float *grad, int batch,
                       void *stream);

/* One Adam step (Kingma & Ba 2015; t counts from 1) on the FP32 master
 * params with moments m, v; rewrites the BF16 copy.  Asynchronous. */
int srmhd_mlp_adam(float *params, uint16_t *w_bf16, float *m, float *v,
                   const float *grad, int n, float lr, float beta1, float beta2,
                   float eps, int t, void *stream);

/* Identifier of the sources the library was built from (sha256 prefix over
 * the HIP sources and this header, fixed at build time); a binding compares
 * it with the sources beside it to refuse a stale build. */
const char *srmhd_build_id(void);

/* Message of the last failure on ctx (NULL ctx: the last failure of
 * srmhd_create or of a call without a context). */
const char *srmhd_last_error(const srmhd_ctx *ctx);
const char *srmhd_strerror(int code);

/* Release the context (host memory only). Syncs the stream. */
void srmhd_destroy(srmhd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
