/*
 * tflbm.h -- C ABI of the MI355X (gfx950) thin-film lattice Boltzmann library.
 *
 * The library advances the D2Q9 film-height populations of the thin-film
 * lattice Boltzmann method of Zitz, Scagliarini, Maddu, Darhuber and Harting,
 * "A lattice Boltzmann method for thin liquid film hydrodynamics"
 * (arXiv:1810.07642), Sec. II, on a periodic nx x ny lattice (Sec. III):
 *
 *   f_l(x + c_l, t + 1) = f_l + omega (f_l^eq - f_l) + 3 w_l c_l . F_tot     (eq. "LBE")
 *   f^eq: shallow-water equilibrium with hydrostatic term g h^2/2            (eq. "equilibria")
 *   F_tot = -h grad p_film - nu alpha_delta(h) u + h (ax, ay)                (eqs. "force", "forcefric")
 *   p_film = -gamma (lap h + kappa(x) [(h_* / h)^n - (h_* / h)^m])                (eqs. "pfilm", "disjoiningP")
 *   kappa(x) = (1 - cos theta(x)) (n - 1)(m - 1) / ((n - m) h_*)
 *   alpha_delta(h) = 6 h / (2 h^2 + 6 delta h + 3 delta^2)                     (eq. "alphafric")
 *   grad, lap: isotropic D2Q9 stencils                                         (eqs. "derivative", "n_laplace")
 *   h = sum_l f_l, h u = sum_l c_l f_l, nu = (tau - 1/2)/3, omega = 1/tau.
 *
 * Readings of the printed equations (denominators of the equilibrium taken
 * with lattice speed 1, the Laplacian without the printed weights, the
 * disjoining sign that gives partial wetting) are those of the FP64 oracle
 * the library is tested against.
 *
 * Conventions common to every call:
 *  - All arrays passed in or out are row-major [ny][nx], x fastest, FP64,
 *    dense (row pitch nx), in HIP device memory unless a pointer is named h_*.
 *  - The library never allocates device memory for data (its only device
 *    memory of its own is the 8 KiB static reduction scratch per GPU of
 *    tflbm_mass_noalloc).  The caller
 *    allocates the workspace (tflbm_workspace_bytes), the adjoint workspace
 *    (tflbm_adj_bytes), checkpoints (tflbm_state_bytes) and captures
 *    (tflbm_capture_bytes), keeps them alive until the stream work that uses
 *    them has completed, and frees them.  The handle owns host memory and, on
 *    launch-bound lattices, up to two step graphs and the stream they were
 *    captured on (tflbm_step), released by tflbm_destroy.
 *  - Calls marked (async) enqueue work on `stream` and return at once;
 *    errors of already-launched kernels surface at the next blocking call.
 *    Calls marked (blocking) synchronise `stream`.
 *  - Return value: TFLBM_OK (0) or a negative TFLBM_E* code.  No exceptions
 *    and no abort cross the ABI.  A handle is not thread-safe: calls on one
 *    handle must be serialised by the caller.
 */
#ifndef TFLBM_H
#define TFLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *tflbm_stream_t; /* a hipStream_t; NULL = default stream */

enum {
  TFLBM_OK = 0,
  TFLBM_EINVAL = -1,     /* bad argument: dimensions, tau <= 1/2, h_* <= 0, null pointer, size */
  TFLBM_EUNSTABLE = -2,  /* tflbm_check_params only: 2 nu / delta^2 >= 2 (friction recurrence unstable near h -> 0) */
  TFLBM_EHIP = -3,       /* a HIP runtime error; tflbm_last_error() gives its text */
  TFLBM_ENONFINITE = -4, /* a step produced h <= 0 or a non-finite h */
  TFLBM_ESTATE = -5      /* call out of order (e.g. step before init, adjoint step before seed) */
};

/* Population storage forms.  Arithmetic is FP64 for TFLBM_FP64 and FP32 otherwise.
 *
 * Every form stores, and steps, the deviations d_l = f_l - E_l(href) of the
 * populations from the rest equilibrium at the reference height href,
 *   E_0(href) = href - 5 g href^2/6,  E_l(href) = g href^2/6 (axes), g href^2/24 (diagonals),
 * so that h = href + sum_l d_l and h u = sum_l c_l d_l.  The step is the same
 * map as on f (eq. "LBE"); only its rounding changes: FP32 resolves changes
 * of h relative to |h - href| instead of |h|.  href = 0 stores f itself.  Pick
 * href near the film height whose small changes matter (the mean of a nearly
 * flat film); a drop on a precursor film is best served by href = h_*.  For
 * TFLBM_FP32 and TFLBM_FP16S href is rounded to FP32 first.
 *
 * TFLBM_FP16S stores, per site, its height deviation s = h - href in FP32
 * and each moving population shifted by the rest equilibrium of the site
 * that emitted it, q_l = (f_l - E_l(h_src)) * 2^fp16_scale_log2, in FP16; the
 * rest population is implied (the nine values of a site add up to its s),
 * so mass is held in FP32 and tflbm_mass sums the s.  FP16 keeps about 3
 * significant digits of q_l: pick the scale so that the moving differences
 * stay above FP16's subnormal range (2^-14 after scaling) and below its
 * largest value (65504); h itself has FP32 resolution relative to
 * |h - href|, so on slow dynamics put href at the film height. */
enum { TFLBM_FP64 = 0, TFLBM_FP32 = 1, TFLBM_FP16S = 2 };

typedef struct tflbm_params {
  int32_t nx, ny;          /* periodic lattice size, >= 1 each, ny * roundup(nx, 64) < 2^31, and every row of
                              population, capture and adjoint records < 0x7fff0000 bytes (the kernels aim the
                              stores they drop past it): nx up to about 28.5 million in FP64, 53 million in
                              FP32 and FP16S */
  int32_t prec;            /* TFLBM_FP64, TFLBM_FP32 or TFLBM_FP16S */
  int32_t n_exp, m_exp;    /* disjoining exponents n != m, 1..32 (paper: 9 and 3) */
  int32_t fp16_scale_log2; /* TFLBM_FP16S scale exponent s, 0..24 */
  int32_t gamma_field;     /* 0, or 1: the surface tension is a per-site field given to tflbm_init_fields
                              (the workspace then holds two values per site instead of kappa) */
  double tau;              /* BGK relaxation time, > 1/2 */
  double gamma;            /* surface tension, >= 0 */
  double g;                /* gravity in the equilibrium's g h^2/2; < 0 destabilises */
  double hstar;            /* precursor film thickness h_* > 0 */
  double delta;            /* slip length, >= 0 */
  double ax, ay;           /* body acceleration: F = h (ax, ay) */
  double theta0;           /* uniform contact angle used when tflbm_init gets d_theta == NULL */
  double href;             /* reference height of the stored deviations (>= 0; 0 stores f) */
} tflbm_params;

typedef struct tflbm_sim tflbm_sim; /* opaque; host memory only */

/* Library version string. */
const char *tflbm_version(void);

/* Text of a TFLBM_E* code. */
const char *tflbm_strerror(int code);

/* Text of the last HIP error seen by any call on `sim` (or "" if none). */
const char *tflbm_last_error(const tflbm_sim *sim);

/* Fills *p with the defaults: tau 1, gamma 0.01, g 0, h_* 0.05, (n, m) = (9, 3),
 * delta 1, no body force, theta0 0, FP64, fp16 scale 2^12, href 0; nx = ny = 0. */
void tflbm_default_params(tflbm_params *p);

/* Validates *p without creating anything.  TFLBM_OK, TFLBM_EINVAL, or
 * TFLBM_EUNSTABLE for the warning-class friction bound 2 nu/delta^2 >= 2
 * (uniform-film velocity recurrence u_{t+1} = u_t (1 - nu alpha/h) needs
 * nu alpha/h < 2; its supremum over h > 0 is 2 nu/delta^2).  */
int tflbm_check_params(const tflbm_params *p);

/* Creates a handle for the lattice and parameters in *p (copied).  Performs
 * the TFLBM_EINVAL checks of tflbm_check_params; a TFLBM_EUNSTABLE warning
 * does not prevent creation.  *out receives the handle or NULL.
 * Launch-shape overrides, read from the environment here (fusion) and at
 * tflbm_init (row chunks), for measurement only; results do not depend on
 * them: TFLBM_FUSE=1, 2 or 3 (most forward steps per pass in tflbm_step and
 * tflbm_step_capture; by default three with tau = 1 on large lattices, else
 * two where the lattice is large enough for it to pay),
 * TFLBM_OMEGA1=0 (with tau = 1, the general collision stages instead of the
 * ones that keep no populations; the same bits), TFLBM_ADJ_FUSE=1 or 2 (the
 * same for the reverse steps of tflbm_adj_steps; by default two where the
 * lattice is large enough for it to pay), TFLBM_ROWS, TFLBM_ROWS2,
 * TFLBM_ROWS3, TFLBM_ADJ_ROWS, TFLBM_ADJ_ROWS2 (rows per chunk of the one-,
 * two- and three-step kernels),
 * TFLBM_GRAPH=0 or 1 (read at tflbm_init: whether tflbm_step replays blocks
 * of steps from graphs; by default on lattices of at most 2^20 sites). */
int tflbm_create(const tflbm_params *p, tflbm_sim **out);

/* Releases the handle: its host memory and, if tflbm_step captured any, its
 * step graphs and the stream it captured them on (after waiting for the
 * device).  No device memory is owned. */
void tflbm_destroy(tflbm_sim *sim);

/* Bytes of device workspace the handle needs: two population buffers, the
 * kappa field (or, with params.gamma_field, the per-site pair
 * (-gamma/6, -gamma kappa)), a status word and reduction partials.  Depends
 * only on the parameters. */
size_t tflbm_workspace_bytes(const tflbm_sim *sim);

/* Attaches a caller-allocated device workspace of `bytes` >= tflbm_workspace_bytes
 * bytes, 256-byte aligned.  Re-binding detaches the previous one, releases
 * the step graphs (which name it; after waiting for the device) and clears
 * the initialised state. */
int tflbm_bind(tflbm_sim *sim, void *d_ws, size_t bytes);

/* (async) Initial populations f_l = f_l^eq(h0, u = 0) (the equilibrium at
 * rest) and kappa from theta (Sec. II, eq. "disjoiningP").  d_h0: [ny][nx]
 * FP64, every value > 0 (checked on the device; reported by tflbm_check).
 * d_theta: [ny][nx] FP64 contact angles, or NULL for the uniform
 * params.theta0 (then the step reads no kappa field).  Sets the step count
 * to 0 and clears the status word; releases the step graphs of an earlier
 * init (after waiting for the device). */
int tflbm_init(tflbm_sim *sim, const double *d_h0, const double *d_theta, tflbm_stream_t stream);

/* (async) tflbm_init with a position-dependent surface tension gamma(x)
 * (Sec. II: the sentence after eq. "n_laplace" names such a field among those
 * the stencils act on).  It replaces gamma in the film pressure,
 *   p_film = -gamma(x) (lap h + kappa(x) f(h)),  F_film = -h grad p_film,
 * so the isotropic gradient acts on the product (no Marangoni stress is
 * added: the paper writes none).  d_gamma: [ny][nx] FP64, every value >= 0
 * and finite (checked on the device; reported by tflbm_check), or NULL for
 * params.gamma everywhere (then the steps are bit for bit those of a handle
 * without the field).  Needs params.gamma_field = 1 (TFLBM_EINVAL otherwise);
 * a handle with params.gamma_field = 1 reads the field in every step, also
 * after tflbm_init.  The reverse pass (tflbm_adj_seed) refuses such a handle
 * with TFLBM_EINVAL.  d_h0, d_theta as for tflbm_init. */
int tflbm_init_fields(tflbm_sim *sim, const double *d_h0, const double *d_theta, const double *d_gamma,
                      tflbm_stream_t stream);

/* (async) Advances nsteps >= 0 time steps of eq. "LBE".  On lattices whose
 * steps are bound by launch latency (at most 2^20 sites; TFLBM_GRAPH), whole
 * blocks of 64 steps go out as one graph launch on `stream` once the handle
 * has run 256 steps: the block's kernel launches are captured on first use,
 * once for each of the two buffer parities a block can start from, on a
 * stream the handle creates for it.
 * The results are the same bits as with plain launches.  Where `stream` is
 * itself being captured, or capturing fails, the steps are launched one by
 * one. */
int tflbm_step(tflbm_sim *sim, int64_t nsteps, tflbm_stream_t stream);

/* Number of step graphs the handle holds (0, 1 or 2: one per starting buffer
 * parity of a block); -1 for NULL. */
int tflbm_step_graphs(const tflbm_sim *sim);

/* Most time steps one pass of tflbm_step advances on this handle (1, 2 or 3:
 * several steps of eq. "LBE" applied to a row chunk before it is stored; 3
 * needs tau = 1 and a lattice large enough for it to pay; TFLBM_FUSE
 * overrides); EINVAL for NULL, ESTATE before tflbm_init. */
int tflbm_steps_per_pass(const tflbm_sim *sim);

/* Number of steps taken since tflbm_init (host counter). */
int64_t tflbm_step_count(const tflbm_sim *sim);

/* (async) Height h = sum_l f_l and velocity u = (sum_l c_l f_l)/h of the
 * current populations (the moments of Sec. II that define h and h u from the
 * populations), computed in FP64 from the stored values.  Each output is
 * [ny][nx] FP64 device memory; any of them may be NULL to skip it.
 * TFLBM_ESTATE before tflbm_init. */
int tflbm_read(const tflbm_sim *sim, double *d_h, double *d_ux, double *d_uy, tflbm_stream_t stream);

/* (blocking) Total mass sum_{x,l} f_l(x) in FP64 (deterministic two-pass
 * reduction) into *h_mass (host memory).  The method conserves it exactly in
 * real arithmetic (Sec. III B). */
int tflbm_mass(const tflbm_sim *sim, double *h_mass, tflbm_stream_t stream);

/* (async) For callers that cannot allocate device memory or synchronise (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the total mass of tflbm_mass, same deterministic two-pass FP64
 * reduction and same bits, written to device memory *d_mass (one double,
 * caller-owned) without synchronising.  Its 1024 partial sums live in a
 * static device array of the library (8 KiB per GPU, held until the process
 * ends; the partial count does not depend on the lattice, so every lattice
 * fits) instead of the workspace; no call allocates or frees anything.  Every
 * call on one GPU shares that array, and the previous call's partials are
 * overwritten: calls that overlap on one GPU (several streams, handles or
 * threads) race and must be serialised by the caller.  TFLBM_ESTATE before
 * tflbm_init, TFLBM_EINVAL for NULL pointers. */
int tflbm_mass_noalloc(const tflbm_sim *sim, double *d_mass, tflbm_stream_t stream);

/* (blocking) TFLBM_OK, or TFLBM_ENONFINITE if a step since tflbm_init met
 * h <= 0 or a non-finite h at an updated site (the height moment of Sec. II,
 * h = sum_l f_l, which divides the momentum in u = j/h and must stay positive
 * for the film pressure's (h_* / h)^n), or if h0 (or a surface tension field)
 * had an invalid value.  TFLBM_ESTATE before tflbm_init. */
int tflbm_check(const tflbm_sim *sim, tflbm_stream_t stream);

/* (blocking) Term-balance diagnostic (appendix, eq. "magnitude"): h_norms[0..7]
 * (host memory, 8 doubles) receive (N^-1 sum_x phi^2)^(1/2), N = nx ny, of the
 * x then the y components of the terms of the depth-averaged momentum
 * equation (eq. "hydro2") at the current pre-collision state:
 *   [0] -h d_x p_film        [1] -nu alpha_delta(h) u_x
 *   [2] nu lap(h u_x) + 2 nu d_x(div(h u))   [3] d_x(j_x u_x) + d_y(j_y u_x)
 *   [4..7] the same for y.
 * Derivatives are the isotropic stencils of the step (eqs. "derivative",
 * "n_laplace"); d_x(div j) applies the derivative stencil to the stencil
 * divergence.  Evaluated in FP64 from the stored populations and reduced in
 * a fixed order (deterministic).  TFLBM_ESTATE before tflbm_init. */
int tflbm_term_norms(const tflbm_sim *sim, double *h_norms, tflbm_stream_t stream);

/* Bytes of one population buffer (a checkpoint of the state). */
size_t tflbm_state_bytes(const tflbm_sim *sim);

/* (async) Copies the current populations into d_dst (tflbm_state_bytes bytes). */
int tflbm_state_save(const tflbm_sim *sim, void *d_dst, tflbm_stream_t stream);

/* (async) Replaces the current populations by d_src (written by
 * tflbm_state_save of a handle with the same parameters) and sets the step
 * counter to `step`.  The kappa field is kept. */
int tflbm_state_load(tflbm_sim *sim, const void *d_src, int64_t step, tflbm_stream_t stream);

/* ---- Reverse mode (the vector-Jacobian product of the step) ------------
 * The adjoint of n steps from f = E(h0) with respect to h0 and theta, for a
 * loss whose gradient with respect to the final height is given.  Use:
 *   seed with dL/dh_N; then for each step t = N-1 ... 0, in that order, call
 *   tflbm_adj_step with the capture of step t (the moments at the start of
 *   step t, written by tflbm_step_capture), or tflbm_adj_steps once per
 *   captured segment; then tflbm_adj_finish.
 * The adjoint state is stored in the working precision (FP64 for
 * TFLBM_FP64, FP32 otherwise); the kappa gradient accumulates in FP64. */

/* Bytes of one step's capture: h, h u_x, h u_y at the start of the step, in
 * the working type, laid out in records of the population records' columns
 * (internal layout, read only by tflbm_adj_step). */
size_t tflbm_capture_bytes(const tflbm_sim *sim);

/* (async) Like tflbm_step, and also writes the capture of step i
 * (0 <= i < nsteps) to d_capture + i * tflbm_capture_bytes. */
int tflbm_step_capture(tflbm_sim *sim, int64_t nsteps, void *d_capture, tflbm_stream_t stream);

/* Bytes of the adjoint workspace: two adjoint population buffers and the
 * FP64 kappa-gradient field. */
size_t tflbm_adj_bytes(const tflbm_sim *sim);

/* (async) Starts a reverse pass in d_adj (tflbm_adj_bytes bytes, 256-byte
 * aligned): the adjoint of the final populations is dL/dh_N(x) for every l,
 * and the kappa gradient is zeroed.  d_grad_h: [ny][nx] FP64.  TFLBM_EINVAL
 * for a handle with params.gamma_field = 1. */
int tflbm_adj_seed(tflbm_sim *sim, void *d_adj, const double *d_grad_h, tflbm_stream_t stream);

/* (async) Moves the adjoint from the end of step t to its start, using the
 * capture of step t (d_capture_t, tflbm_capture_bytes bytes), and adds the
 * step's contribution to the kappa gradient. */
int tflbm_adj_step(tflbm_sim *sim, void *d_adj, const void *d_capture_t, tflbm_stream_t stream);

/* (async) The reverse pass over one captured segment: tflbm_adj_step for
 * t = nsteps-1 down to 0 with the capture of step t at
 * d_capture + t * tflbm_capture_bytes (the layout tflbm_step_capture writes;
 * nsteps captures must be there).  On lattices that fill the GPU, two
 * steps run per pass over the lattice, the adjoint of step t feeding that of
 * step t-1 on chip, which halves the adjoint and kappa-gradient traffic; on
 * smaller ones the steps run singly.  The result is bit for bit that of the
 * single steps either way.  nsteps = 0 does nothing; EINVAL for nsteps < 0 or
 * a NULL pointer, ESTATE before tflbm_adj_seed. */
int tflbm_adj_steps(tflbm_sim *sim, void *d_adj, const void *d_capture, int64_t nsteps, tflbm_stream_t stream);

/* (async) dL/dh0 = sum_l lambda_l dE_l/dh0 and dL/dtheta = dL/dkappa dkappa/dtheta.
 * d_h0: the initial height used by tflbm_init; d_theta: its theta field, or
 * NULL if tflbm_init was given NULL (then *d_grad_theta still receives the
 * per-site gradient with respect to a theta field equal to theta0).
 * Outputs [ny][nx] FP64; either may be NULL. */
int tflbm_adj_finish(tflbm_sim *sim, const void *d_adj, const double *d_h0, const double *d_theta,
                     double *d_grad_h0, double *d_grad_theta, tflbm_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TFLBM_H */
