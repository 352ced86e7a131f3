/*
 * wave.h -- C ABI of the time-tiled acoustic-wave sweep for MI355X (gfx950).
 *
 * What is computed.  The time-stepped finite-difference sweep for
 *     m u_tt + damp u_t = lap u + q          (2D or 3D, space order 2..16)
 * under time-tiling: several time steps fused per tile (the paper's
 * contribution, implementation chapter, "Skewing" and "Time-tiling"), with
 * the fused-step count T and the halo ("skew") depth per fused step as run-time
 * parameters (parameterised tile sizes, Devito chapter, "Parameterisation").
 * The skew must be at least the stencil radius so/2 (background chapter,
 * "Validity of skewing factors"); smaller values are rejected.  Results of the
 * time-tiled sweep are bitwise identical to the untiled sweep (evaluation
 * chapter, "Functional correctness").
 *
 * The discretisation (the paper never prints it; see the library's design
 * notes for every reading taken): leapfrog in time, order-`so` central
 * differences in space with zero values outside the grid, centred damping
 * damp = m * sigma with sigma = sigma_max * sum_a (d_a/nbl)^2 inside an
 * absorbing layer nbl points wide at every face, sources injected and
 * receivers sampled by multilinear interpolation:
 *   u^{n+1} = [dt^2 (L u^n + sum_s w_s q_s^n) + 2 m u^n - (m - eta) u^{n-1}] / (m + eta),
 *   eta = damp dt / 2,   d_r^n = sum_p w_{r,p} u^{n+1}_p.
 * The adjoint is the same step run backwards in time; the gradient of
 * J = 1/2 sum_n |d^n - d_obs^n|^2 with respect to m is accumulated by the
 * imaging condition  g_p = -sum_j u^j_p ((1+st) mu^{j-1} - 2 mu^j + (1-st) mu^{j+1})_p,
 * st = sigma dt / 2.
 *
 * Memory.  The library never allocates device memory.  The caller provides a
 * persistent state buffer at wave_init (size from wave_state_bytes) and a
 * scratch buffer per call (size from wave_scratch_bytes); both are device
 * memory the caller owns and frees after wave_destroy.  All device pointers
 * are plain FP32 arrays, row-major [n0][n1][n2] (2D: [n0][n1]) with the last
 * axis of unit stride; axis 0 is the one streamed through registers.
 * Coordinates are host FP64 arrays [count][ndim], metres from grid node 0.
 *
 * Streams and errors.  Every call is asynchronous on the stream given to
 * wave_init (a hipStream_t passed as void*; NULL is the null stream) except
 * where noted.  Every call returns a wave_status; nothing throws.  A kernel
 * fault surfaces as WAVE_EHIP on a later call or synchronisation.  A context
 * is not thread-safe; separate contexts are independent.
 */
#ifndef WAVETT_WAVE_H
#define WAVETT_WAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WAVE_OK = 0,
  WAVE_EINVAL = -1,       /* bad argument (sizes, pointers, order, shape) */
  WAVE_ESKEW = -2,        /* skew < so/2: the fused tile would violate a dependence */
  WAVE_ECFL = -3,         /* dt above the stability limit of the scheme */
  WAVE_ENOMEM = -4,       /* state or scratch buffer smaller than required */
  WAVE_EHIP = -5,         /* HIP runtime error (message in wave_last_error) */
  WAVE_ESTATE = -6,       /* call sequence error (e.g. no checkpoints to reuse) */
  WAVE_EUNSUPPORTED = -7  /* tile depth / tile shape not built for this order */
} wave_status;

/* Problem and schedule description. */
typedef struct wave_desc {
  int32_t ndim;          /* 2 or 3 */
  int32_t space_order;   /* even, 2..16; stencil radius r = space_order/2 */
  int64_t shape[3];      /* computational grid (absorbing layer included), n0 n1 [n2] */
  double spacing[3];     /* metres per axis */
  double dt;             /* seconds */
  int32_t nbl;           /* absorbing-layer width in points; 0 = no damping */
  double sigma_max;      /* damping maximum in 1/s (ignored if nbl == 0) */
  int32_t time_tile;     /* T >= 1 time steps per time tile; -1 = untiled single-step
                            sweep (the reference schedule); 0 = default: 3D T = 3 on
                            32x128 tiles at radius 1, T = 2 on 32x128 tiles at radius 2;
                            2D T = 6 at radius 1, 4 at radius 2, 3 up to radius 4; untiled
                            otherwise (the measured best on MI355X; wave_autotune
                            refines by timing) */
  int32_t skew;          /* skewing factor: halo per fused step on the tiled axes (slab = 0)
                            or plane shift per step of the skewed schedule (slab > 0);
                            0 = r; must be >= r (background chapter, "Validity of skewing
                            factors") */
  int32_t tile[2];       /* register-tiled sweep (slab = 0, T >= 1): the extended tile
                            (b1 rows along axis 1, b2 columns along the unit-stride axis)
                            loaded by one workgroup, of which the inner (b1 - 2 skew T) x
                            (b2 - 2 skew T) are written (Devito chapter, "Parameterisation":
                            tile sizes as run-time parameters).  {0, 0} = auto: the first
                            entry of the table below that builds depth T at this order.  Must be an
                            entry of the table of built tiles (wave_tile_extent): 3D 64x64,
                            32x64, 32x128, 16x128; 2D 1x1024.  Others: WAVE_EUNSUPPORTED */
  int32_t slab;          /* > 0 (with T >= 1): the skewed schedule of the implementation
                            chapter ("Time-tiling"): each time tile advances the grid slab by
                            slab along axis 0, every slab all T steps (one single-step launch
                            each, its planes shifted by -skew per step) before the next, so
                            no point is computed twice and a slab's levels stay in the
                            last-level cache between its steps.  The value is the slab
                            thickness in planes (any; the tile size along axis 0).
                            0 = register-tiled or untiled sweep */
  int32_t zchunks;       /* segments of axis 0 per launch (of a slab, with slab > 0);
                            0 = auto (untiled 3D: about 32 workgroups per CU, segments of
                            at least max(16, 4r) planes; register-tiled 3D: the most
                            segments whose workgroups fit one per CU; time-tiled 2D:
                            about 16 per CU) */
} wave_desc;

typedef struct wave_ctx wave_ctx;

/* Bytes of the persistent device state for `d` (0 if d is invalid): four
 * time levels (two ping-pong pairs of the leapfrog scheme's two levels; the
 * paper's time buffer of the Devito chapter, "Time-buffering", holds the
 * dependence depth plus the time tile) and b = dt^2/m.  Host-only. */
size_t wave_state_bytes(const wave_desc* d);

/* Set up the operator of the paper's problem statement (Devito chapter: grid,
 * spacing, time step, space order, then the schedule parameters of
 * "Parameterisation"; the acoustic-wave operator of the evaluation chapter,
 * "Performance of the acoustic wave equation operator").
 * Validate `d`, build the schedule and the per-axis damping tables, and derive
 * b = dt^2/m from the model m_dev [N] (s^2/m^2, device, must stay > 0).  The
 * CFL check uses max velocity 1/sqrt(min m): this call synchronises the
 * stream once.  time_tile == 0 picks the default schedule (see wave_desc);
 * wave_autotune measures.  state_dev must hold wave_state_bytes(d) bytes.
 * Errors: WAVE_EINVAL, WAVE_ESKEW, WAVE_ECFL, WAVE_ENOMEM, WAVE_EUNSUPPORTED, WAVE_EHIP. */
wave_status wave_init(const wave_desc* d, const float* m_dev, void* state_dev, size_t state_bytes,
                      void* hip_stream, wave_ctx** out);

/* Replace the model m (the wave operator's coefficient field; evaluation
 * chapter, acoustic wave equation operator) of the same shape; re-checks the
 * CFL limit (synchronises).
 * Every entry must be a positive finite number (WAVE_EINVAL otherwise,
 * NaN included). */
wave_status wave_set_model(wave_ctx* ctx, const float* m_dev);

/* Change the schedule of an existing context (the paper's run-time time-tile
 * size, skewing factor and tile sizes; Devito chapter, "Parameterisation"):
 * T >= 1 or -1 (untiled), skew (0 = r), tile [2] (NULL or {0, 0} = auto),
 * slab and zchunks as in wave_desc.  Host-only.  Errors: WAVE_EINVAL,
 * WAVE_ESKEW, WAVE_EUNSUPPORTED (tile not built, depth above the tile's
 * limit, no core left); the schedule is then unchanged. */
wave_status wave_set_schedule(wave_ctx* ctx, int32_t time_tile, int32_t skew, const int32_t* tile,
                              int32_t slab, int32_t zchunks);

/* Read back the schedule in use (after autotuning): tile receives the
 * extended tile {b1, b2} of the register-tiled sweep ({0, 0} when the
 * schedule is untiled or skewed).  Any pointer may be NULL. */
wave_status wave_get_schedule(const wave_ctx* ctx, int32_t* time_tile, int32_t* skew, int32_t* tile,
                              int32_t* slab, int32_t* zchunks);

/* Memory plan of a call (the library allocates nothing; the caller's buffer
 * holds what the paper's generated code keeps in its time buffer and point
 * tables).  Host-only.
 * Scratch bytes needed by wave_forward (adjoint = 0), by wave_forward with
 * checkpoints followed by wave_adjoint_grad (adjoint = 1), or by one shot of
 * wave_batch with a gradient (adjoint = 2: also the residual traces) for nt
 * steps with nsrc sources and nrec receivers; ckpt_every = K > 0 keeps a
 * checkpoint of (u^{cK}, u^{cK-1}) for every segment.  On a diffusion
 * context: the scratch wave_autotune needs (2 N floats), whatever the
 * arguments. */
size_t wave_scratch_bytes(const wave_ctx* ctx, int32_t nt, int32_t nsrc, int32_t nrec, int32_t ckpt_every,
                          int32_t adjoint);

/* Forward modelling, nt steps: the time loop of the paper's operator under
 * the context's schedule (implementation chapter, "Time-tiling"; untiled,
 * register-tiled or skewed), with source injection and receiver sampling
 * inside the tiles (left to future work in the paper: implementation
 * chapter, the source and receiver loops; conclusion, future work).
 *   src_xyz  host [nsrc][ndim];  wavelet_dev device [nt][nsrc]  (q_s^n drives u^{n+1})
 *   rec_xyz  host [nrec][ndim];  rec_dev device [nt][nrec] out (d^n samples u^{n+1}) or NULL
 *   u_init_dev  device [2][N] = (u^0, u^{-1}) or NULL for zeros
 *   u_final_dev device [2][N] out = (u^{nt}, u^{nt-1}) or NULL
 *   ckpt_every  0: no checkpoints; K > 0: keep checkpoints in scratch so that a
 *               following wave_adjoint_grad(..., reuse = 1) can skip the forward
 *   scratch_dev / scratch_bytes  from wave_scratch_bytes(ctx, nt, nsrc, nrec, K, K > 0);
 *               with K > 0 and u_init_dev NULL, every wave_history_segment_bytes(ctx, K)
 *               beyond wave_scratch_bytes(ctx, nt, nsrc, nrec, K, 1) keeps one more
 *               segment's history for that adjoint (as in wave_adjoint_grad)
 * Points outside the grid contribute nothing (their corners are dropped). */
wave_status wave_forward(wave_ctx* ctx, int32_t nt,
                         int32_t nsrc, const double* src_xyz, const float* wavelet_dev,
                         int32_t nrec, const double* rec_xyz, float* rec_dev,
                         const float* u_init_dev, float* u_final_dev,
                         int32_t ckpt_every, void* scratch_dev, size_t scratch_bytes);

/* Adjoint sweep and gradient, zero initial state (not in the paper: the
 * discrete adjoint of the same leapfrog operator, run backwards in time under
 * the same schedules, with the imaging condition fused; every recomputed
 * forward segment and every adjoint step use the schedule of the context).
 *   resid_dev       device [nt][nrec]: dJ/dd (e.g. d - d_obs)
 *   grad_m_dev      device [N] out: dJ/dm
 *   grad_wavelet_dev device [nt][nsrc] out: dJ/dq, or NULL
 *   ckpt_every      K >= 1 (segment length of the checkpointed recompute; K >= nt
 *                   keeps the whole history)
 *   reuse           1: use the checkpoints of the immediately preceding
 *                   wave_forward on this context and scratch (same nt, K,
 *                   sources, receiver count and wavelet buffer, model unchanged since:
 *                   wave_set_model and every other sweep discard them; else
 *                   WAVE_ESTATE); the wavelet's contents must not have
 *                   changed either; 0: run that forward here.
 * Forward segments are recomputed from checkpoints with the time-tiled
 * kernel (storing their history), then swept backwards with the time-tiled
 * adjoint kernel that accumulates the imaging condition.
 *   scratch_dev / scratch_bytes  at least wave_scratch_bytes(ctx, nt, nsrc,
 *                   nrec, K, 1).  With reuse = 0, every further
 *                   wave_history_segment_bytes(ctx, K) keeps one more segment's
 *                   history (the last segments first) straight from the
 *                   forward, which then skips that segment's checkpoint and
 *                   the adjoint its recompute.  Every schedule writes those
 *                   levels (and the recomputed ones) out of place straight into
 *                   their history slots, so keeping them costs the forward no
 *                   extra bytes beyond a deep register tile's intermediate
 *                   levels.  The gradient is bitwise the same for any number
 *                   of kept segments. */
wave_status wave_adjoint_grad(wave_ctx* ctx, int32_t nt,
                              int32_t nsrc, const double* src_xyz, const float* wavelet_dev,
                              int32_t nrec, const double* rec_xyz, const float* resid_dev,
                              float* grad_m_dev, float* grad_wavelet_dev,
                              int32_t ckpt_every, int32_t reuse, void* scratch_dev, size_t scratch_bytes);

/* Host-only.  Bytes of one kept segment's history in wave_adjoint_grad's
 * scratch (K levels of N floats, aligned); 0 for a NULL or diffusion context
 * or K < 1. */
size_t wave_history_segment_bytes(const wave_ctx* ctx, int32_t ckpt_every);

/* Host-only.  Segments whose history the last wave_adjoint_grad on this
 * context kept from its forward (0 before any); -1 for a NULL context. */
int32_t wave_last_kept_segments(const wave_ctx* ctx);

/* Many independent shots advanced together, for example the sources of one
 * survey (the paper leaves multi-operator batching to future work; this is
 * the GPU form of running many small operators at full occupancy).  Every
 * shot is its own context (own grid, order, model, schedule); all contexts
 * share the stream of ctxs[0].  Per-shot arrays have length nshots:
 *   nsrc, src_xyz, wavelet_dev, nrec, rec_xyz   as in wave_forward
 *   rec_dev      device [nt][nrec] out: modelled traces
 *   grad_m_dev   NULL: forward only.  Otherwise device [N] out per shot: the
 *                gradient of J = 1/2 sum |rec - dobs|^2 with respect to m
 *                (forward with checkpoints every ckpt_every >= 1 steps, the
 *                residual, recompute, adjoint and imaging, as wave_adjoint_grad)
 *   dobs_dev     device [nt][nrec] observed traces (with grad_m_dev only)
 *   scratch_dev  device, scratch_bytes[i] >= wave_scratch_bytes(ctx_i, nt,
 *                nsrc_i, nrec_i, ckpt_every if gradient else 0, 2 if gradient else 0)
 * Each shot's operations are recorded and the pending sweeps of the shots
 * are merged in lockstep: one launch per group of shots with equal (radius,
 * depth, dim, tile shape, mode), at most 12 shots per launch, each workgroup
 * finding its shot from the launch arguments.  A gradient batch merges all
 * shots; a forward-only batch merges consecutive shots up to 96 MiB of
 * per-step working set and runs those groups one after another (cache
 * locality between steps).  In a forward-only batch the shots of each
 * stencil radius form an independent branch of the captured graph (a stream
 * each), so the launches of different orders run side by side; a gradient
 * batch keeps one branch (measured faster or level).  The environment variable
 * WAVE_BATCH_BRANCHES=0 or =1 forces one branch or one per radius.  The merged sequence is
 * captured into a HIP graph and launched; a later call with the same
 * arguments on contexts that no other call has touched since replays that
 * graph without recording again (device inputs may change in between).
 * Results are bitwise those of the per-shot calls.  Every shot's schedule
 * must be the untiled sweep, the skewed schedule, or a register-tiled depth
 * T <= 2 on the 64x64 or 32x64 tile (WAVE_EUNSUPPORTED otherwise); a
 * context may appear once; calls on the same contexts must not overlap.
 * Errors: WAVE_EINVAL (null arrays, duplicate context, different streams),
 * WAVE_ENOMEM (scratch too small), WAVE_EHIP; the message is on ctxs[0]. */
wave_status wave_batch(wave_ctx* const* ctxs, int32_t nshots, int32_t nt,
                       const int32_t* nsrc, const double* const* src_xyz, const float* const* wavelet_dev,
                       const int32_t* nrec, const double* const* rec_xyz, float* const* rec_dev,
                       const float* const* dobs_dev, float* const* grad_m_dev,
                       int32_t ckpt_every, void* const* scratch_dev, const size_t* scratch_bytes);

/* Autotune the schedule on this context's model by timing short trial
 * sweeps, as the paper's auto-tuner times candidate tile sizes
 * (implementation chapter, "Auto-tuning"; evaluation chapter, "Auto-tuner
 * iterations" and "Time-tiling parameters").  Minimum of `repeats` trials per
 * candidate.  Phase 1: the untiled sweep, every register tile of the table at
 * every built depth T <= max_T, and the skewed schedule at T = 2, 4, ... <=
 * max_T (16 if max_T = 0) on slabs of 32 and 64 planes, all at the default
 * number of axis-0 segments.  Phase 2: 1..32 axis-0 segments for the five
 * fastest and for the untiled sweep.  Phase 3: the skewing factor (r, a multiple of 4, 2r) of the best
 * register-tiled schedule, or the slab thickness and depth of the best skewed
 * one (the paper's skew experiment, "Effect of the skewing factor").  Keeps
 * the fastest; a time-tiled schedule replaces the untiled sweep only when
 * faster by more than 1 % (the trials' run-to-run spread), and among untiled
 * segment counts within 1 % of the fastest the largest is kept (the forward
 * trials rarely separate them, while the gradient's history and adjoint
 * sweeps of the same schedule run faster with more workgroups).  Synchronises;
 * needs scratch for `trial_steps` forward steps without sources
 * (wave_scratch_bytes(ctx, trial_steps, 0, 0, 0, 0)).  On a diffusion
 * context (diff_init) the trials are diff_forward calls from a zero field
 * between two levels in the scratch (2 N floats, also what
 * wave_scratch_bytes returns for such a context). */
wave_status wave_autotune(wave_ctx* ctx, int32_t trial_steps, int32_t repeats, int32_t max_T,
                          void* scratch_dev, size_t scratch_bytes, double* best_seconds_per_step);

/* The estimator-guided autotuner the paper proposes (evaluation chapter,
 * "Minimising runtime based on tile size choices" and "Further uses for an
 * arithmetic intensity estimator"; conclusion, future work): instead of
 * timing every candidate of phase 1, it times four anchors (the untiled
 * sweep, the shallowest and the deepest register tile of 32 x 64, one skewed
 * schedule), calibrates on them a model of every candidate's time -- the
 * larger of its memory side (compulsory bytes per point-update x the
 * workgroup's halo re-load factor x the ratio of the naive to the tight
 * intensity bound, over the bandwidth the untiled anchor achieved) and its
 * compute side (the redundant work of a register tile x the register
 * anchors' cost interpolated in T, or the single-step kernel's) -- and times only the
 * `keep` >= 1 candidates the model ranks fastest; phase 2 then covers the two
 * fastest and the untiled sweep, phase 3 as in wave_autotune.  *timed_trials (may be NULL) receives
 * the number of candidates timed.  Arguments and errors as wave_autotune. */
wave_status wave_autotune_guided(wave_ctx* ctx, int32_t trial_steps, int32_t repeats, int32_t max_T,
                                 int32_t keep, void* scratch_dev, size_t scratch_bytes,
                                 double* best_seconds_per_step, int32_t* timed_trials);

/* The autotuner with the operator's point sets, since the paper's auto-tuner
 * times the operator as it will run (implementation chapter, "Auto-tuning").
 * The trial forwards of wave_autotune (keep = 0) or wave_autotune_guided
 * (keep >= 1) carry the nsrc sources (a zero wavelet: their forcing lookups,
 * not their values, cost time) and the nrec receivers at src_xyz / rec_xyz
 * (host, [n][ndim] in the units of the spacing, as wave_forward).  Point
 * lookups run on the planes that hold points in every workgroup that
 * crosses them, so they cost a schedule with few long-running workgroups
 * more than one with many short ones: a 512-receiver line costs a one-wave
 * register-tiled sweep of 592^3 about 2 % per step, the untiled sweep 0.3 %.
 * Scratch: wave_autotune_scratch_bytes(ctx, trial_steps, nsrc, nrec)
 * (device).  A diffusion context takes no points (WAVE_EINVAL if nsrc or
 * nrec > 0).  Other arguments and errors as wave_autotune_guided; keep = 0
 * is accepted here and means exhaustive. */
wave_status wave_autotune_points(wave_ctx* ctx, int32_t trial_steps, int32_t repeats, int32_t max_T,
                                 int32_t keep, int32_t nsrc, const double* src_xyz, int32_t nrec,
                                 const double* rec_xyz, void* scratch_dev, size_t scratch_bytes,
                                 double* best_seconds_per_step, int32_t* timed_trials);

/* The autotuner for gradients (wave_adjoint_grad), since the paper's
 * auto-tuner times the operator as it will run (implementation chapter,
 * "Auto-tuning") and the adjoint's kernels hold more registers than the
 * forward's, so the forward's ranking does not carry over: first
 * wave_autotune_points (exhaustive) with these points, then trial gradients
 * of trial_steps steps with checkpoints every K (a zero wavelet and a zero
 * residual) for the forward's winner, the untiled sweep and the register
 * tiles of depth 2..min(4, max_T) on 32x64 and 32x128 (2D: 1x1024); the
 * fastest is kept, a time-tiled schedule only when more than 1 % faster than
 * the untiled sweep.  Synchronises.  *best_seconds_per_step: the kept
 * schedule's gradient trial per step; *timed_trials (may be NULL): forward
 * and gradient candidates timed.  Scratch: wave_autotune_gradient_scratch_bytes
 * (device).  Errors: WAVE_ESTATE (a diffusion context), WAVE_EINVAL,
 * WAVE_ENOMEM, WAVE_EHIP. */
wave_status wave_autotune_gradient(wave_ctx* ctx, int32_t trial_steps, int32_t repeats, int32_t max_T,
                                   int32_t ckpt_every, int32_t nsrc, const double* src_xyz, int32_t nrec,
                                   const double* rec_xyz, void* scratch_dev, size_t scratch_bytes,
                                   double* best_seconds_per_step, int32_t* timed_trials);

/* Scratch bytes wave_autotune_gradient needs (the larger of the forward
 * trials' and a trial gradient's with its outputs and zero inputs); 0 for a
 * null or diffusion context or invalid arguments.  Host-only. */
size_t wave_autotune_gradient_scratch_bytes(const wave_ctx* ctx, int32_t trial_steps, int32_t nsrc, int32_t nrec,
                                            int32_t ckpt_every);

/* Scratch bytes wave_autotune_points needs for these point counts (with
 * nsrc = nrec = 0 also what wave_autotune and wave_autotune_guided need);
 * 0 for a null context or invalid counts.  Host-only. */
size_t wave_autotune_scratch_bytes(const wave_ctx* ctx, int32_t trial_steps, int32_t nsrc, int32_t nrec);

/* Arithmetic-intensity estimators of the evaluation chapter ("Arithmetic
 * intensity under time-tiling").  Host-only, no device access.
 *   ai_space   AI of the space-tiled (untiled) sweep, flops per byte
 *   t_t        time-tile size
 *   ndim, D[], delta[], tile[]   extents, radii and tile sizes per spatial
 *              dimension, ordered d_1 (outermost tile loop) .. d_n
 *   omega      cache size in floats
 * wave_ai_naive returns t_t * ai_space; wave_ai_tight divides that by
 * 1 + |B| / prod D with |B| the union of re-loaded tile faces (face sizes
 * F_i multiplied by t_t) -- the tighter bound of the same section. */
double wave_ai_naive(double ai_space, int32_t t_t);
double wave_ai_tight(double ai_space, int32_t t_t, int32_t ndim, const double* D, const double* delta,
                     const double* tile, double omega);

/* Largest fused depth T of the register-tiled sweep built for this order,
 * dimension and extended tile {ey, ex} (an entry of wave_tile_extent's
 * table); 0 if none.  Bounded by the register file (every fused level keeps
 * a (so+1)-plane window per column) and by the core (ey - 2 r T >= 1).  The
 * skewed schedule (slab > 0) has no such bound.  Host-only. */
int32_t wave_tiled_max_depth(int32_t space_order, int32_t ndim, int32_t ey, int32_t ex);

/* Entry `index` (1, 2, ...) of the table of extended tiles built for the
 * register-tiled sweep in ndim dimensions (Devito chapter, "Parameterisation";
 * the run-time tile sizes are drawn from it): the rows ey along axis 1 and
 * columns ex along the unit-stride axis that one workgroup loads.  3D: 1 =
 * 64x64, 2 = 32x64, 3 = 32x128, 4 = 16x128; 2D: 1 = 1x1024.  Host-only.
 * Returns WAVE_EINVAL past the end of the table or for a bad ndim. */
wave_status wave_tile_extent(int32_t ndim, int32_t index, int32_t* ey, int32_t* ex);

/* The counts behind the roofline analysis of the evaluation chapter
 * ("Arithmetic intensity under time-tiling", compulsory memory traffic):
 * flops per point-update of the sweep (adds + multiplies, FMA = 2) for order
 * so in ndim dimensions, and compulsory HBM bytes per point-update of a
 * schedule of depth time_tile (T = -1 untiled; damping computed from
 * indices; the register-tiled and the skewed schedules move the same
 * compulsory bytes) for mode 0 (forward), 1 (forward storing the history,
 * +4 B), 2 (adjoint reading the history at every step and the gradient
 * once per window, updating it in registers across the window's stages:
 * +4 + 8/T B, i.e. (7 + T) 4 / T for T >= 2), 3 (explicit diffusion: read one level, write one level per
 * launch, 8/T B) or 4 (the two-level diffusion step: 12 B untiled, 16/T B
 * per time tile).  Host-only. */
double wave_flops_per_point(int32_t ndim, int32_t space_order, int32_t damped);
double wave_bytes_per_point(int32_t time_tile, int32_t mode);

/* ------------------------------------------------------------------------
 * Explicit diffusion: the Laplace-operator workload of the paper's evaluation
 * chapter (Evaluation, Performance of the Laplace operator: first order in
 * time, one time dependency).  The paper never prints
 * its equation; it is read as
 *     u^{n+1} = u^n + dt a (L u^n)
 * with the Laplacian, coefficients and zero ghosts of the wave sweep above
 * and a constant diffusivity a.  It runs on the same schedules (untiled
 * sweep or time-tiled with depth, skew, tile shape and axis-0 segments) and
 * kernels; the per-point update is u + lap with the weights scaled by
 * dt a / h_axis^2 (FP64 on the host, rounded once).  Every schedule gives the
 * same bits.  Layout as above (axis 0 streamed, last axis unit stride). */
typedef struct diff_desc {
  int32_t ndim;          /* 2 or 3 */
  int32_t space_order;   /* even, 2..16 */
  int64_t shape[3];      /* grid, n0 n1 [n2] */
  double spacing[3];     /* per axis */
  double dt;             /* time step */
  double alpha;          /* diffusivity a (> 0); units spacing^2 / time */
  int32_t time_tile;     /* -1: untiled sweep; T >= 1: fused steps per launch; 0: default
                            (3D: T = 4 at radius 1, T = 2 at radius 2, on 32x64 tiles;
                            at radii 3 and 4 the skewed schedule, T = 8 on slabs of 64
                            planes in 2 segments (grids deeper than 64 planes); 2D:
                            T = 4 up to radius 2, T = 2 up to radius 4; untiled
                            otherwise -- measured on MI355X) */
  int32_t skew;          /* 0 = r; must be >= r */
  int32_t tile[2];       /* as in wave_desc */
  int32_t slab;          /* as in wave_desc */
  int32_t zchunks;       /* as in wave_desc; 0 = auto (time-tiled: about 6 workgroups per CU
                            in 3D, 16 in 2D) */
  int32_t scheme;        /* 0: one time level, u^{n+1} = u^n + dt a L u^n (forward Euler);
                            1: two time levels (delta_t = 2; evaluation chapter, "Time-tiling
                            with larger time dependences"), the two-step Adams-Bashforth
                            rule u^{n+1} = u^n + dt a (3/2 L u^n - 1/2 L u^{n-1}) with
                            u^{-1} = u^0.  Scheme 1 runs the untiled sweep or the skewed
                            schedule (slab > 0; WAVE_EUNSUPPORTED for register tiles); its
                            default (time_tile = 0) is skewed, T = 16 on slabs of 64 planes,
                            up to radius 2 in 3D, untiled otherwise (measured); its stability limit
                            is half that of scheme 0 */
} diff_desc;

/* Flops per point-update of explicit diffusion (FMA = 2) for scheme 0 (one
 * level) or 1 (two levels: also forming 3/2 u^n - 1/2 u^{n-1}). Host-only. */
double diff_flops_per_point(int32_t ndim, int32_t space_order, int32_t scheme);

/* Bytes of device state for `d`: two levels of N floats (scheme 1: three)
 * (0 if d is invalid). */
size_t diff_state_bytes(const diff_desc* d);

/* Validate `d` (as wave_desc, plus alpha > 0 finite, scheme 0 or 1) and the
 * stability limit dt a sum_a rho / h_a^2 <= 2 (scheme 1: <= 1; rho as for
 * wave_init), and carve the state.
 * The context takes wave_set_schedule, wave_get_schedule, wave_autotune,
 * wave_scratch_bytes, wave_last_error and wave_destroy; the wave-equation
 * calls reject it with WAVE_ESTATE.
 * Errors: WAVE_EINVAL, WAVE_ESKEW, WAVE_ECFL, WAVE_ENOMEM, WAVE_EUNSUPPORTED. */
wave_status diff_init(const diff_desc* d, void* state_dev, size_t state_bytes, void* hip_stream,
                      wave_ctx** out);

/* nt steps from u0_dev [N] (device, read only) into u_out_dev [N] (device);
 * the two must not overlap each other or the context's state (WAVE_EINVAL).  Intermediate levels live in the state.  nt == 0
 * copies.  Asynchronous on the context's stream.  Errors: WAVE_EINVAL,
 * WAVE_ESTATE (not a diffusion context), WAVE_EUNSUPPORTED, WAVE_EHIP. */
wave_status diff_forward(wave_ctx* ctx, int32_t nt, const float* u0_dev, float* u_out_dev);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): wave_forward
 * without checkpoints and without a scratch argument.  Its point tables,
 * forcing table and sample buffer live in a static device array of
 * WAVE_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; the call allocates nothing.  The caller still
 * passes inputs and outputs (as in wave_forward; u_init_dev / u_final_dev may
 * be NULL).  All calls on one GPU share that GPU's array: calls that overlap
 * in time on one GPU (any contexts, any streams) race and give wrong results.
 * A call needing more scratch than the maximum (its size is
 * wave_scratch_bytes(ctx, nt, nsrc, nrec, 0, 0)) returns WAVE_ENOMEM and
 * launches nothing.  Other errors as wave_forward. */
#define WAVE_STATIC_SCRATCH_BYTES (32u << 20)
wave_status wave_forward_static(wave_ctx* ctx, int32_t nt,
                                int32_t nsrc, const double* src_xyz, const float* wavelet_dev,
                                int32_t nrec, const double* rec_xyz, float* rec_dev,
                                const float* u_init_dev, float* u_final_dev);

/* Library housekeeping (no passage of the paper): the text of a status, the
 * message of the last failed call on a context, and the release of a
 * context's host resources (the caller frees its device buffers after). */
const char* wave_strerror(wave_status s);
const char* wave_last_error(const wave_ctx* ctx);
void wave_destroy(wave_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* WAVETT_WAVE_H */
