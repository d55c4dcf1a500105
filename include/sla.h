/*
 * sla.h -- C ABI of the multi-stage semi-Lagrangian advection library (gfx950).
 *
 * The library advects passive scalars on periodic Cartesian grids with the
 * schemes of Cameron, Raynaud & Dormy, "Multi-stage high order semi-Lagrangian
 * schemes for incompressible flows in Cartesian geometries":
 *
 *   CIR  one call of the interpolation operator L_U (section 3, first
 *        equation; eq. CIR2D for the multilinear 2D/3D form),
 *   FEC  forward error correction, eq. intro:FEC (two calls),
 *   BEC  backward error correction, eq. intro:BEC (three calls),
 *   CEC  the third-order combination A*FEC + B*BEC of eq. intro:CEC with the
 *        weights of eq. intro:CECcoef, taken from U mod 1 at large Courant
 *        numbers (eq. intro:CECcoefSL) and applied one axis at a time
 *        (section 5, eqs. split:1 and split:2),
 *
 * and, as options, the third order under Strang's symmetric splitting
 * (SLA_CEC_STRANG) and FEC and BEC one axis at a time (SLA_FEC_SPLIT,
 * SLA_BEC_SPLIT), and the large-CFL weights read literally (SLA_CEC_LITERAL).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named phi, u, a, b, phis[k] are HIP device pointers on the
 *   context's device; every other pointer is host memory.  The caller owns
 *   all of them; the library never frees or keeps them past the call.
 * - A field is FP32, x fastest: cell (x, y, z) sits at x + nx*(y + ny*z).
 *   A velocity is ndim such planes back to back (u_x, u_y[, u_z]), the
 *   physical velocity; the Courant number of axis d is c_d = u_d*dt/dx_d,
 *   formed as one FP32 multiply by fl32(dt/dx_d).
 * - The departure point of node i along an axis is i - c: it lies between the
 *   anchor node i - s*n and the far node i - s*(n+1), with s = +1 if c >= 0
 *   else -1, n = floor(|c|), f = |c| - n.  Interpolation is p + f*(q - p).
 * - Boundaries are periodic on every axis.
 * - Calls are asynchronous on the context's stream unless stated; a device
 *   fault surfaces at a later synchronising call.
 * - Every function returns an sla_status (0 = success, negative = error) and
 *   never aborts; sla_last_error() gives the detail of the last failure.
 * - One context per host thread; calls on one context must not overlap.
 */
#ifndef SLA_H
#define SLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SLA_CIR = 0, /* L_U only: first order */
  SLA_FEC = 1, /* eq. intro:FEC, unsplit multilinear: second order */
  SLA_BEC = 2, /* eq. intro:BEC, unsplit multilinear: second order */
  SLA_CEC = 3, /* eqs. intro:CEC + intro:CECcoef(SL), split per axis: third order */
  /* the same sweeps under Strang's symmetric splitting (section 5): half a
     step along x (and y in 3D), a whole step along the last axis, then the
     half steps in reverse order; every step the same (no step0 dependence) */
  SLA_CEC_STRANG = 4,
  /* FEC and BEC split per axis (eqs. split:1-2 applied to eqs. intro:FEC and
     intro:BEC): one one-dimensional FEC or BEC sweep per axis, the order
     alternating like SLA_CEC's */
  SLA_FEC_SPLIT = 5,
  SLA_BEC_SPLIT = 6,
  /* the large-CFL weights of eq. intro:CECcoefSL read literally, per axis
     and order as SLA_CEC: A FEC + B BEC with 3A = 2 - 1/(|c| mod 1) and
     B = 1 - A, FEC's correction added at the arrival node.  Equal to SLA_CEC
     (up to rounding) while every |c| < 1; second order beyond, and not
     finite where |c| is a whole number (the formula divides by zero); near
     a whole number, rounding is amplified by |A|, about 1/(3 (|c| mod 1)).
     A comparison, not the third-order scheme. */
  SLA_CEC_LITERAL = 7
} sla_scheme;

typedef enum {
  SLA_OK = 0,
  SLA_EINVAL = -1,   /* bad argument: see sla_last_error() */
  SLA_ECOURANT = -2, /* floor(max |c|) + 1 exceeds SLA_MAX_REACH, or a kernel
                        met a Courant number beyond the bound it was given */
  SLA_EHIP = -3,     /* HIP runtime error */
  SLA_ENOMEM = -4,   /* device allocation failed */
  SLA_ENOMODEL = -5, /* learned correction called without usable weights */
  SLA_ECAPTURE = -6  /* the call would synchronise the stream or allocate while
                        the stream is being captured into a graph */
} sla_status;

/* Largest backtrace reach, in cells, the kernels are built for: every
 * |c_d| must be < SLA_MAX_REACH (so CFL < 4). */
#define SLA_MAX_REACH 4

/* A periodic grid.  ndim is 1, 2 or 3; n[d] >= 8 cells on each used axis and
 * n[d] = 1 on unused axes; n[0]*n[1]*n[2] < 2^31; dx[d] > 0 and finite. */
typedef struct {
  int32_t ndim;
  int32_t n[3];
  double dx[3];
} sla_grid;

typedef struct sla_ctx sla_ctx; /* opaque */

/* Create a context on HIP device `device` issuing work on `stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context. */
int sla_create(sla_ctx **out, int device, void *stream);
/* Release a context and the device memory it allocated.  NULL is ignored. */
void sla_destroy(sla_ctx *ctx);
/* Change the stream later calls are issued on. */
int sla_set_stream(sla_ctx *ctx, void *stream);
/* Static text for a status code. */
const char *sla_strerror(int status);
/* Detail of the last failure on this context (empty string if none).  The
 * pointer stays valid until the next call on the context. */
const char *sla_last_error(const sla_ctx *ctx);

/* Largest Courant number max_d max_cells |fl32(u_d * fl32(dt/dx_d))| of the
 * velocity `u` (ndim planes on `grid`), written to host *out.  Synchronises
 * the stream.  Returns SLA_EINVAL if u holds a NaN or an infinity. */
int sla_courant_max(sla_ctx *ctx, const sla_grid *grid, const float *u,
                    double dt, double *out);

/* Advance `phi` in place by `steps` time steps of `scheme` with the steady
 * velocity `u`, time step `dt` (any finite value; a negative dt advects
 * backwards).  The velocity is sampled at the arrival node and traced back
 * one explicit step (section 2: L_U[Phi](x) = Phi~(x - U dt)).
 *
 * step0 is the global index of the first step; for SLA_CEC (and the split
 * FEC and BEC) it fixes the sweep
 * order (x,y,z on even steps, z,y,x on odd steps), so a run split into
 * several calls matches one call when step0 is carried along.  SLA_CEC_STRANG
 * runs x/2, y/2, z, y/2, x/2 (2D: x/2, y, x/2; 1D: x) every step, each a
 * third-order sweep kernel (the x and y half steps in one kernel where the
 * fused x+y sweep applies); the half steps use the Courant number u * fl32(dt
 * / dx) / 2, exactly half the whole step's.
 *
 * courant_max: if > 0, a bound the caller guarantees on every |c_d|; the call
 * then does not read u to measure it.  If a kernel still meets a larger
 * Courant number it clamps the offset (the result is then wrong but every
 * access stays in bounds) and records SLA_ECOURANT for sla_check().
 * If <= 0 the call measures the bound itself (one extra read of u and one
 * stream synchronisation).
 *
 * steps == 0 is a successful no-op.  Work memory (one field) is allocated on
 * the context on first use and kept, unless the caller gave the context a
 * workspace (sla_set_workspace).  The result is in phi when the stream
 * reaches the end of the call.
 *
 * Graph capture: the call only launches kernels (and at most one device
 * copy) when courant_max > 0 and the work memory is large enough, so it can
 * be captured into a graph; while the stream is captured it returns
 * SLA_ECAPTURE instead of measuring the bound or allocating. */
int sla_advect(sla_ctx *ctx, const sla_grid *grid, float *phi, const float *u,
               double dt, int32_t scheme, int32_t steps, int64_t step0,
               double courant_max);

/* Largest grid, in cells, that sla_advect_noalloc takes (2^23: 32 MiB of
 * static device memory per device). */
#define SLA_NOALLOC_MAX_CELLS 8388608

/* sla_advect for callers that cannot allocate device memory: code being
 * captured into a graph, tight serving loops, hosts that forbid allocation.
 * Same arguments, checks and result (bit for bit) as sla_advect, but the work
 * field is a static device array of SLA_NOALLOC_MAX_CELLS FP32 values that
 * each device holds from the library's load to the end of the process; the
 * call never allocates, frees or creates anything, and ignores the context's
 * workspace and its timing (its launches are not timed).  A grid of more than
 * SLA_NOALLOC_MAX_CELLS cells returns SLA_EINVAL before any work.  With
 * courant_max > 0 the call only launches kernels (and at most one device
 * copy); with courant_max <= 0 it measures the bound (one stream
 * synchronisation; SLA_ECAPTURE while the stream is captured).
 * Every context on a device shares that device's array, and nothing of it
 * carries over between calls: calls on one device whose work overlaps in time
 * (other streams, other contexts, other host threads) race on it and must be
 * ordered by the caller. */
int sla_advect_noalloc(sla_ctx *ctx, const sla_grid *grid, float *phi, const float *u,
                       double dt, int32_t scheme, int32_t steps, int64_t step0,
                       double courant_max);

/* sla_advect on nscalars fields that share the velocity u: phis is a host
 * array of nscalars device fields, each advanced in place with the same
 * grid, dt, scheme and steps.  The Courant bound is measured (or taken from
 * courant_max) once for all of them.  Third-order steps of a 3D grid whose
 * Courant numbers are all below 1 run the fields four at a time (then two,
 * then one) through a fused kernel that loads the velocity once per tile for
 * all of them; each field of such a group takes its own work field (up to
 * four, see sla_workspace_size; a smaller caller workspace runs fewer at a
 * time).  Other cases run the fields one after another through one work
 * field.  Every field's result equals sla_advect on it, bit for bit. */
int sla_advect_multi(sla_ctx *ctx, const sla_grid *grid, int32_t nscalars, float *const *phis,
                     const float *u, double dt, int32_t scheme, int32_t steps, int64_t step0,
                     double courant_max);

/* Device bytes of work memory sla_advect and sla_advect_multi need on grid:
 * one FP32 field, or for SLA_CEC on a 3D grid min(nscalars, 4) fields (the
 * fields of a shared-velocity group each take one).  0 for an invalid grid
 * or scheme. */
size_t sla_workspace_size(const sla_grid *grid, int32_t scheme, int32_t nscalars);

/* Make the context use `bytes` of caller-owned device memory at dev_ptr as
 * its work memory instead of memory it allocates.  Later sla_advect and
 * sla_advect_multi calls then never allocate work memory: a call that needs
 * more than `bytes` (see sla_workspace_size) fails with SLA_EINVAL.  The
 * caller keeps the memory valid until it sets another workspace or destroys
 * the context; the library never frees it.  dev_ptr == NULL returns to
 * library-allocated work memory.  Synchronises the stream (earlier calls may
 * still use the old work memory). */
int sla_set_workspace(sla_ctx *ctx, void *dev_ptr, size_t bytes);

/* Context options. */
typedef enum {
  /* 1 (default): a 3D third-order step whose reach is 1 on every axis runs as
   * one fused kernel (all three sweeps, 20 B per cell of HBM traffic), on
   * grids of fewer than 2^30 cells or of 2^30 cells with ny >= 2 (others
   * run the sweeps).  0: every third-order step runs one sweep kernel per
   * axis.  Both paths perform the same FP32 operations per node. */
  SLA_OPT_FUSED = 0,
  /* Which implementation runs the fused step (same FP32 operations, same
   * results): 1 register segments, 2 streaming (direct global-to-LDS
   * loads), 4 window march (no LDS: x across lanes, 4-row segments of one
   * axis in registers, the third axis along the march), 6 window march with
   * 8-row segments, 7 window march whose workgroups (2 or 3 windows, 2 waves
   * each) share the segment halo rows through LDS, 8 the same with 16-row
   * groups of 12 waves (in march chunks, or persistent), 9 as 8 with the
   * inputs loaded two planes ahead, 10 and 11 as 8 and 9 with one window (4
   * waves) per workgroup, 12 and 13 with two, 14 a march along z on x
   * windows of 128 nodes aligned to 512-byte lines, two nodes per lane,
   * with 32-row groups of 8 waves (the window's x halo loaded apart, its
   * edge outputs computed by packed edge lanes; odd steps sweep z first
   * along the march; needs an even nx, else runs 8), 5 (default) the choice
   * sla_tune measured for the grid if the context has one, else the fastest
   * of these for each parity and grid size as measured from 256^3 to
   * 1024^3 (14 from 2^24 cells on with an even nx). */
  SLA_OPT_CEC3D_KERNEL = 1,
  /* How the sweeps of a third-order step that is not fused, and of the
   * split schemes (SLA_CEC_STRANG, SLA_FEC_SPLIT, SLA_BEC_SPLIT,
   * SLA_CEC_LITERAL), run (same FP32 operations, same results): 3 (default) the x and y sweeps in one kernel
   * (x then y on even steps, y then x on odd ones) with two nodes per lane
   * (128-node x windows marching along y) when nx is even and their reach
   * is at most 3, z by column walks, else as 2; 2 the x and y sweeps in
   * one kernel with 64-lane x windows when their reach is at most 2, else
   * as 1; 1 one kernel per axis, x in 64-lane windows, y and z by each
   * thread walking one column with its stencil in registers; 0 one kernel
   * per axis with LDS tiles.  1 to 3 need grids of fewer than 2^30 cells,
   * or of 2^30 cells with ny >= 2 (others run 0). */
  SLA_OPT_SWEEP_KERNEL = 2,
  /* How unsplit FEC and BEC steps run (same FP32 operations, same results):
   * 3 (default) on 3D grids at reach 1 (every |c| < 1; fewer than 2^30 cells
   * or 2^30 with ny >= 2), all calls of a step in one z-march whose stages
   * live in LDS rings (the field read once, written once), elsewhere as 2;
   * 0 all calls of a step in one kernel of LDS tiles; 1 one gather kernel
   * per call (FEC: 2, BEC: 3), the intermediates through the work field
   * (44 and 64 B per cell moved); 2 as 1. */
  SLA_OPT_EC_KERNEL = 3,
  /* Launch shape of the fused step (same results whatever the value): the
   * planes a workgroup marches (variants 1-7); for variants 8-13, > 0 the
   * persistent workgroups launched per compute unit, < 0 one workgroup per
   * chunk of -value planes; for variant 14, < 0 the chunk, else the longest
   * of 128, 64, 32 and 16 planes that still gives every compute unit a
   * workgroup; 0 (default): the implementation's own rule. */
  SLA_OPT_CEC3D_SHAPE = 4,
  /* How the learned step's correction runs (same results): 1 (default) a
   * march along z with each node's neighbourhood staged in LDS; 0 a gather
   * of the 27 values per node. */
  SLA_OPT_LEARNED_KERNEL = 5,
  /* The largest group of fields sla_advect_multi runs through one fused
   * kernel that reads the shared velocity once per tile for all of them
   * (third-order 3D steps at reach 1): 4 (default) or 2; 0 or 1: field after
   * field.  Same results. */
  SLA_OPT_SHARED_VELOCITY = 6,
  /* Launch shape of the unsplit FEC/BEC z-march (same results whatever the
   * value): < 0 one workgroup per chunk of -value planes of a group; > 0
   * that many persistent workgroups per CU (at most as many as fit), each
   * marching one range of the groups' planes laid end to end; 0 (default)
   * chunks whose count minimises rounds of workgroups x (planes per chunk +
   * pipeline fill). */
  SLA_OPT_EC_SHAPE = 7,
  /* Departure points of third-order steps (SLA_CEC): 0 (default) one explicit
   * step from the arrival node, x - c(x) (the paper's); 1 a midpoint
   * (second-order Runge-Kutta) backtrace, beyond the paper: along each axis
   * the calls of L_U depart from x - c(x - c(x)/2) and the call of L_{-U}
   * from x + c(x + c(x)/2), c interpolated linearly between nodes.  With 1,
   * third-order steps run one tile sweep per axis (no fused or marching
   * kernel) and sla_plan_create refuses the context; uniform velocities
   * give the default's results to rounding. */
  SLA_OPT_BACKTRACE = 8
} sla_option;
/* Set option `option` to `value`.  Returns SLA_EINVAL for an unknown option
 * or value. */
int sla_set_option(sla_ctx *ctx, int option, int64_t value);

/* Fused-step tuner.  Time every implementation of the fused third-order
 * step (SLA_OPT_CEC3D_KERNEL values and launch shapes) on `grid` with the
 * caller's field phi (read only; the launches write the context's work
 * memory) and velocity u, for each parity of the sweep order, and keep the
 * fastest per parity in the context: later third-order steps of this grid
 * with SLA_OPT_CEC3D_KERNEL = 5 (the default) use them.  Every choice gives
 * the same results.  If table_path is not NULL the choice is also written to
 * that text file (one line per grid: nx ny nz, then variant, shape and ms of
 * even and of odd steps; other grids' lines are kept).  The grid must be 3D
 * with every Courant number below 1 (SLA_ECOURANT otherwise).  Synchronises
 * the stream; allocates the work memory if the context has none. */
int sla_tune(sla_ctx *ctx, const sla_grid *grid, const float *phi, const float *u, double dt,
             const char *table_path);
/* Read a table that sla_tune wrote into the context (its grids' choices
 * replace any the context holds).  SLA_EINVAL for a missing file or a
 * malformed line. */
int sla_tune_load(sla_ctx *ctx, const char *table_path);
/* The context's tuned choice for a 3D grid: variants[2], shapes[2] and the
 * measured ms[2] (even, odd); any pointer may be NULL.  SLA_EINVAL if the
 * context has none for the grid. */
int sla_tune_info(const sla_ctx *ctx, const sla_grid *grid, int32_t *variants, int32_t *shapes,
                  double *ms);

/* Synchronise the context's stream and report a Courant overflow recorded by
 * a kernel since the previous sla_check() (then SLA_ECOURANT), or a HIP
 * error.  Clears the record. */
int sla_check(sla_ctx *ctx);

/* FP64 reductions of two FP32 arrays of `count` elements (section 4 rates
 * schemes by the norm of their difference to a reference).  Writes to the
 * host array out[5]:
 *   out[0] = sum (a-b)^2, out[1] = sum b^2, out[2] = max |a-b|,
 *   out[3] = sum a,       out[4] = sum b,
 * all accumulated in FP64 in a fixed order (bitwise reproducible for a given
 * count).  Synchronises the stream. */
int sla_norms(sla_ctx *ctx, int64_t count, const float *a, const float *b,
              double *out);

/* ------------------------------------------------------------------------
 * Batched third-order steps in one captured graph.
 *
 * A plan advances many independent problems by the same number of
 * third-order steps (eq. intro:CEC, split per axis as in section 5) with one
 * graph launch.  A problem is a 3D periodic grid with its own field, and
 * either its own velocity planes or a uniform velocity.  Problems whose
 * velocity pointer and grid are equal share the velocity: their tiles run
 * side by side on the same accelerator partition, so the shared velocity is
 * read from memory about once for all of them.  Each step launches one
 * persistent kernel over the tiles of all problems, except problems with
 * their own velocity planes and at least 2^24 cells: those fill the GPU
 * alone.  Such problems with the same velocity pointer, grid and time step
 * run up to four (the creating context's SLA_OPT_SHARED_VELOCITY) per launch
 * of the shared-velocity fused step, which loads the velocity once per tile
 * for all of them; the others take one launch of the fused third-order step
 * each (the creating context's SLA_OPT_CEC3D_KERNEL choice).  A result
 * equals sla_advect(..., SLA_CEC, ...) on that problem (with a uniform
 * velocity field for a uniform problem), bit for bit.
 * ---------------------------------------------------------------------- */
typedef struct {
  sla_grid grid;        /* 3D, as for sla_advect */
  float *phi;           /* device field, advanced in place */
  const float *u;       /* device velocity planes, or NULL for a uniform one */
  float u_uniform[3];   /* the uniform velocity (x, y, z) when u is NULL */
  double dt;            /* time step */
} sla_problem;

typedef struct sla_plan sla_plan; /* opaque; owns work memory and the graph */

/* Plan `steps` steps (global step indices step0 .. step0+steps-1) of the
 * nprob problems probs (host array, copied).  Every Courant number must be
 * below 1: courant_max > 0 is the caller's bound for all problems, else the
 * plan measures it.  If tune != 0 the plan times candidate launch shapes (y
 * extent of a tile, persistent grid size) on the problems (reading their
 * fields, writing only its own work memory) and keeps the fastest.  Work
 * memory: one field per problem.  The graph is built on a private stream.
 * Grids are 3D with at most 2^30 cells each, and ny >= 2 at 2^30 cells
 * (else SLA_EINVAL).
 * Synchronises the context's stream. */
int sla_plan_create(sla_ctx *ctx, sla_plan **out, int32_t nprob, const sla_problem *probs,
                    int32_t steps, int64_t step0, double courant_max, int32_t tune);
/* Launch the plan's graph on the context's stream (asynchronous). */
int sla_plan_run(sla_ctx *ctx, sla_plan *plan);
/* Chosen launch shape: y extent of a tile, workgroups of the persistent
 * kernel, its work items per step (problems launched on their own have
 * none), and the tuned time of one whole step in ms (0 if not tuned).  Any
 * pointer may be NULL. */
int sla_plan_info(const sla_plan *plan, int32_t *ychunk, int32_t *blocks, int32_t *items,
                  double *step_ms);
/* Release a plan.  NULL is ignored. */
void sla_plan_destroy(sla_plan *plan);

/* Advance nprob independent problems (host array) by `steps` steps of any
 * scheme; a problem with u == NULL has the uniform velocity u_uniform.
 * Third-order runs of 3D problems whose Courant numbers are all below 1 go
 * through a plan (sla_plan_create, no tuning) run once.  Otherwise each
 * problem runs as sla_advect would (courant_max as there); a uniform
 * velocity is first written into a temporary field of ndim planes that the
 * call allocates and frees.  Every result equals sla_advect on that problem
 * (with a uniform velocity field for a uniform problem), bit for bit.
 * Synchronises the stream when it used a plan or a temporary field. */
int sla_advect_batch(sla_ctx *ctx, int32_t nprob, const sla_problem *probs, int32_t scheme,
                     int32_t steps, int64_t step0, double courant_max);

/* ------------------------------------------------------------------------
 * Learned correction (not in the paper; an addition of this library).
 *
 * A per-node network predicts the correction that takes the CIR step to the
 * third-order step (eq. intro:CEC, split per axis as in section 5).  Inputs
 * of node i (SLA_MLP_INPUTS values, BF16): the 27 differences
 * Phi1[i+o] - Phi1[i] over the 3x3x3 neighbourhood (o = (dz,dy,dx), z
 * outermost, x innermost) divided by sigma = sqrt(sum d^2/27 + 1e-30), then
 * the node's Courant numbers c_x, c_y, c_z, then two zeros; Phi1 is the CIR
 * step.  Network: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2),
 * y = h2 w3 + b3 (30 -> 64 -> 64 -> 1), run on the matrix cores with BF16
 * weights and activations and FP32 accumulation.  Corrected value:
 * Phi1[i] + sigma * y, limited to [min, max] of the 27 values Phi1[i+o]
 * (the step cannot raise the maximum norm of the field, whatever the
 * network outputs).  Training target: (third-order step - Phi1) / sigma;
 * loss: mean squared error; optimiser: Adam on FP32 master weights.
 *
 * Parameter vector (FP32, SLA_MLP_PARAMS values): W1 (32 x 64 row-major,
 * [input][hidden]), b1 (64), W2 (64 x 64 row-major, [in][out]), b2 (64),
 * w3 (64), b3 (1).
 * ---------------------------------------------------------------------- */
#define SLA_MLP_INPUTS 32
#define SLA_MLP_HIDDEN 64
#define SLA_MLP_PARAMS 6337

typedef struct sla_model sla_model; /* opaque; owns its device memory */

/* Create a model on the context's device with all weights zero and no
 * trained Courant range (so sla_advect_learned treats it as untrained). */
int sla_model_create(sla_ctx *ctx, sla_model **out);
/* Release a model.  NULL is ignored. */
void sla_model_destroy(sla_model *model);
/* Load n = SLA_MLP_PARAMS FP32 weights from host memory and reset the
 * optimiser state.  Synchronises the stream. */
int sla_model_set_params(sla_ctx *ctx, sla_model *model, const float *params, int64_t n);
/* Copy the FP32 master weights to host memory.  Synchronises the stream. */
int sla_model_get_params(sla_ctx *ctx, const sla_model *model, float *params, int64_t n);
/* The same two calls under the names of a weight file's load and save. */
int sla_model_load(sla_ctx *ctx, sla_model *model, const float *params, int64_t n);
int sla_model_save(sla_ctx *ctx, const sla_model *model, float *params, int64_t n);
/* Declare the largest |c_d| the weights were trained for (> 0), or 0 for an
 * untrained model. */
int sla_model_set_courant_range(sla_model *model, double range);

/* Training pairs on a 3D grid: for each of the m nodes in cells (device,
 * linear indices x + nx*(y + ny*z)), write its features to feats (device,
 * m rows of SLA_MLP_INPUTS BF16 values), (phi_next - phi1)/sigma to target
 * and sigma to sigma (device FP32, m values).  phi1 is the CIR step of the
 * field, phi_next the step the network should reproduce, u/dt give the
 * Courant inputs. */
int sla_make_pairs(sla_ctx *ctx, const sla_grid *grid, const float *phi1,
                   const float *phi_next, const float *u, double dt,
                   const int32_t *cells, int64_t m, uint16_t *feats,
                   float *target, float *sigma);
/* Network output y for m feature rows (device) into y (device FP32). */
int sla_model_forward(sla_ctx *ctx, const sla_model *model, const uint16_t *feats,
                      int64_t m, float *y);
/* Gradient of the mean squared error over m rows w.r.t. every parameter,
 * into host grads[SLA_MLP_PARAMS]; the loss into host *loss.  Does not
 * update the model.  Synchronises the stream. */
int sla_model_grads(sla_ctx *ctx, sla_model *model, const uint16_t *feats,
                    const float *target, int64_t m, float *grads, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * mean squared error over m rows.  If loss is not NULL the loss before the
 * update is written there (and the stream synchronised). */
int sla_model_train_step(sla_ctx *ctx, sla_model *model, const uint16_t *feats,
                         const float *target, int64_t m, double lr, double *loss);
/* Advance a 3D field by `steps` learned steps (a CIR step plus the network's
 * correction).  The plain third-order scheme is the fallback: when the model
 * is untrained, or the Courant bound (measured as in sla_advect, or
 * courant_max if > 0) exceeds the model's trained range, the call runs
 * sla_advect(..., SLA_CEC, ...) instead if fell_back is not NULL (and sets
 * *fell_back = 1; otherwise 0), and returns SLA_ENOMODEL or SLA_ECOURANT if
 * fell_back is NULL. */
int sla_advect_learned(sla_ctx *ctx, const sla_model *model, const sla_grid *grid,
                       float *phi, const float *u, double dt, int32_t steps,
                       int64_t step0, double courant_max, int32_t *fell_back);

/* ------------------------------------------------------------------------
 * Per-kernel timing (for roofline measurements).
 * While enabled, every kernel launch of later calls on the context is
 * bracketed by HIP events recorded on the context's stream; durations are
 * accumulated per kernel kind.  Recording adds two event records per launch.
 * ---------------------------------------------------------------------- */
typedef enum {
  SLA_K_CIR = 0,     /* unsplit CIR step                      */
  SLA_K_FEC = 1,     /* unsplit FEC step (each of its launches) */
  SLA_K_BEC = 2,     /* unsplit BEC step (each of its launches) */
  SLA_K_SWEEP_X = 3, /* third-order sweep along x             */
  SLA_K_SWEEP_Y = 4, /* third-order sweep along y             */
  SLA_K_SWEEP_Z = 5, /* third-order sweep along z             */
  SLA_K_CEC3D = 6,   /* fused three-axis third-order step     */
  SLA_K_COPY = 7,    /* device-to-device copy of the result   */
  SLA_K_LEARNED = 8, /* learned correction on top of a CIR step */
  SLA_K_SWEEP_XY = 9, /* fused x and y third-order sweeps       */
  SLA_K_COUNT = 10
} sla_kernel_kind;

/* enable != 0: start recording (totals are cleared); 0: stop recording. */
int sla_timing(sla_ctx *ctx, int enable);
/* Synchronise the stream and write, per kernel kind, the number of launches
 * recorded and their summed duration in milliseconds to the host arrays
 * launches[SLA_K_COUNT] and ms[SLA_K_COUNT].  Totals keep accumulating until
 * the next sla_timing(ctx, 1). */
int sla_timing_read(sla_ctx *ctx, int64_t *launches, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* SLA_H */
