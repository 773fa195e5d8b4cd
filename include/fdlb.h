/*
 * fdlb.h -- C interface of the MI355X finite-difference lattice Boltzmann (FDLB) solver for
 * compressible flow at high Mach number: the model of Gan, Xu, Zhang, Yu and Li,
 * "Two-dimensional lattice Boltzmann model for compressible flows with high Mach number"
 * (arXiv:0801.4169).
 *
 * The problem statement follows the paper: a rectangular grid of nx x ny cells with spacing
 * dx, dy (Sec. 5), the Watari-Tsutahara velocity set with speeds v1..v4 (Sec. 2,
 * Eq. dvm_eq_1), the BGK relaxation time tau (Eq. bgk_eq), the time step dt and the
 * artificial-viscosity amplitude lambda (Sec. 3, Eq. add4), an initial field of density,
 * velocity and temperature, and a condition per side (Sec. 5.2: reflecting wall, outflow,
 * Dirichlet; periodic for the one-dimensional tubes of Sec. 5.1).  One call to
 * fdlb_step advances every distribution by Eq. (dis_eq1).
 *
 * Conventions
 *  - Host fields (rho, ux, uy, T) are float64 arrays of ny rows of nx values (x fastest).
 *  - Density is the particle number density n of Eq. (n_eq) (particle mass 1); T is
 *    theta = T/m of Sec. 2; the pressure is P = n T (Eq. p_eq).
 *  - Device memory is owned by the caller (for example a torch tensor) and borrowed for the
 *    lifetime of a context.  The library allocates only small descriptor, tile-table and
 *    reduction blocks of its own and frees them in fdlb_destroy.
 *  - All work is enqueued on the HIP stream given at creation (NULL = the null stream).
 *    Calls documented as "syncs" wait for that stream.
 *  - Every call returns an fdlb_status; nothing throws across this interface.  A context
 *    is not thread-safe; distinct contexts may be used from distinct threads.
 *  - The device keeps a sticky non-physical flag (n <= 0, T <= 0, a non-finite moment, or
 *    |u dt/dx| >= 1 in some cell after some step).  Calls that sync report it as
 *    FDLB_ENONPHYS; the state is still readable.
 */
#ifndef FDLB_H
#define FDLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdlb_ctx fdlb_ctx;

typedef enum {
    FDLB_OK = 0,
    FDLB_EINVAL = 1,   /* bad argument: sizes, non-positive dx/dt/tau, Courant number >= 1,
                          unpaired periodic sides, short buffer, wrong instance index */
    FDLB_ENOMEM = 2,   /* the library's own small allocation failed (hipErrorOutOfMemory) */
    FDLB_EDEVICE = 3,  /* a HIP call failed (the HIP error string is kept, fdlb_last_error) */
    FDLB_ENONPHYS = 4, /* the non-physical flag is set (see above) */
    FDLB_ESTATE = 5    /* call order: stepping or reading before a state was set */
} fdlb_status;

/* Storage and arithmetic of the distributions.
 *   FDLB_F64:     float64 storage and arithmetic.  The arithmetic follows one fixed
 *                 evaluation order without fused multiply-add, so it reproduces a plain
 *                 float64 evaluation of the same formulas bit for bit.
 *   FDLB_F32:     float32 storage of f; equilibrium and stencil in float32; the moments
 *                 (density, velocity, temperature, pressure) are accumulated in float64.
 *                 At high Mach number the f^eq values grow large and of both signs
 *                 (sum |f| / n ~ 1e3 at Mach 10, 1e4 at Mach 20), and rounding them to
 *                 float32 alone moves T by 0.7% (Mach 10) to 70% (Mach 20).
 *   FDLB_F32_DEV: deviation storage: per cell the moments M = (n, ux, uy, T) in float64
 *                 and g_q = f_q - f^eq_q(M) in float32.  Each step rebuilds f = f^eq(M) + g
 *                 in float64, applies Eq. (dis_eq1) in float64 and stores the new moments
 *                 and g relative to them; only the small deviation g is rounded to
 *                 float32.  Reported moments are M. */
typedef enum { FDLB_F64 = 0, FDLB_F32 = 1, FDLB_F32_DEV = 2 } fdlb_precision;

/* Side conditions (Sec. 5.2).  Sides are ordered x-, x+, y-, y+.
 *   PERIODIC : wrap around; both sides of an axis must be periodic together.
 *   OUTFLOW  : zero gradient, the ghost cells copy the edge cell ("supersonic outflow").
 *   DIRICHLET: the ghost cells hold f^eq of the side's (rho, ux, uy, T).
 *   WALL     : reflecting wall, the specular mirror of the cells inside about the cell
 *              face (the velocity component normal to the wall reversed).
 * A non-periodic side may have a lower segment with a condition of its own (the double
 * Mach reflection of Sec. 5.2.2: a wall that begins at x = 0.08; a top state that changes
 * at a point moving with the shock).  Ghost cells whose centre coordinate along the side
 * (x on the y sides, y on the x sides; cell i has centre (i + 1/2) dx) is below
 * split + split_rate * t take lo_kind and the lo state, where t = steps * dt and steps
 * counts the steps since the state was set (fdlb_set_clock changes it). */
typedef enum {
    FDLB_BC_PERIODIC = 0,
    FDLB_BC_OUTFLOW = 1,
    FDLB_BC_DIRICHLET = 2,
    FDLB_BC_WALL = 3
} fdlb_bc_kind;

typedef struct {
    int32_t kind;   /* fdlb_bc_kind */
    int32_t pad_;
    double rho, ux, uy, T; /* used by FDLB_BC_DIRICHLET only */
    int32_t lo_kind;       /* condition of the lower segment; FDLB_BC_PERIODIC (0): none */
    int32_t pad2_;
    double lo_rho, lo_ux, lo_uy, lo_T; /* the lower segment's Dirichlet state */
    double split, split_rate;          /* end of the lower segment: split + split_rate * t */
} fdlb_bc;

typedef struct {
    int32_t nx, ny;      /* cells; nx, ny >= 1, nx * ny <= 2^28, >= 2 across a wall; in
                            float64 also (nx rounded up to 32) * ny * 8 < 2^31 (a plane is
                            addressed with 32-bit byte offsets) */
    double dx, dy;       /* cell sizes, > 0 */
    double dt, tau;      /* time step and BGK relaxation time, > 0 (Eq. bgk_eq) */
    double lambda;       /* artificial-viscosity amplitude, >= 0 (Eq. add4) */
    double v[4];         /* speeds v1..v4 (Eq. dvm_eq_1); the paper uses 1, 1.92, 2.99, 4.49 */
    fdlb_bc bc[4];       /* x-, x+, y-, y+ */
    int32_t precision;   /* fdlb_precision */
    int32_t tile;        /* tile shape id (fdlb_tile_shapes); 0 = library default (measured) */
    int32_t lines;       /* terms of Eq. (dis_eq1) kept: bit 0..3 = lines I..IV (central
                            difference, Lax-Wendroff dissipation, dispersion, artificial
                            viscosity); 0 or 15 = the full scheme.  Sec. 4 and Fig. 3 study
                            the scheme with lines left out; the BGK term is always kept. */
    int32_t tblock;      /* time steps per pass over memory: 0 or 1 = one; 2 (FDLB_F64 only)
                            = tiles whose 16 x 8 cells and four cells around them lie inside
                            the grid take two steps per launch, keeping the intermediate step
                            in on-chip memory (the stencil reaches two cells per step); the
                            other tiles take single steps through a third buffer.  The
                            values are those of single steps bit for bit; the tile shape is
                            16 x 8 (shape id 8); the context borrows three buffers instead of
                            two. */
    int32_t theta_fixed; /* 0: theta of line IV from the switching function, Eq. (add4);
                            1: theta := theta_value in every cell and step.  Sec. 4 freezes
                            theta to linearise the scheme for its von Neumann analysis; with it
                            frozen, one step is linear in f around a uniform equilibrium and
                            its Fourier symbol is the matrix of Eq. (gi_j_eq).  A test knob. */
    int32_t pad_;
    double theta_value;  /* finite, >= 0; read when theta_fixed = 1 */
} fdlb_params;

/* Bytes of device memory a context for these parameters borrows (both ping-pong halves,
 * and the intermediate buffer when tblock = 2: 33 distribution planes, the moment and
 * pressure planes and the wall-pressure rows each).  0 if the parameters are invalid. */
size_t fdlb_required_bytes(const fdlb_params *p);

/* Creates a context.  `arena` is a device pointer to at least fdlb_required_bytes(p)
 * bytes, 256-byte aligned, owned by the caller and kept alive until fdlb_destroy.
 * `stream` is a hipStream_t (may be NULL).  The state is undefined until fdlb_set_state
 * or fdlb_set_f.  Errors: FDLB_EINVAL (parameters, Courant number max|v| dt/dx >= 1,
 * arena too small or misaligned), FDLB_ENOMEM, FDLB_EDEVICE. */
fdlb_status fdlb_create(const fdlb_params *p, void *stream, void *arena, size_t arena_bytes,
                        fdlb_ctx **out);

/* Sets every f to the equilibrium of Eq. (feq_eq) for the given host fields (each nx*ny
 * float64, row-major) and derives the pressure field.  Enqueued; the host arrays may be
 * reused when the call returns (they are copied to device first and the call syncs on
 * that copy).  Errors: FDLB_EINVAL (NULL field). */
fdlb_status fdlb_set_state(fdlb_ctx *c, const double *rho, const double *ux, const double *uy,
                           const double *T);

/* As fdlb_set_state, but `fields` is a device pointer to 4 * nx * ny float64 values:
 * rho, ux, uy, T planes, each row-major.  Asynchronous; the buffer must stay valid until
 * the stream reaches this point. */
fdlb_status fdlb_set_state_device(fdlb_ctx *c, const double *fields);

/* Advances nsteps >= 0 time steps of Eq. (dis_eq1) (asynchronous).  Each step is one
 * kernel launch over the grid; the launches are replayed from a captured HIP graph.
 * Errors: FDLB_ESTATE (no state yet), FDLB_EINVAL (nsteps < 0), FDLB_EDEVICE. */
fdlb_status fdlb_step(fdlb_ctx *c, int64_t nsteps);

/* Density, velocity and temperature (Eqs. n_eq, nu_eq, p_eq) of the current state into
 * host arrays of nx*ny float64 each.  Syncs.  Returns FDLB_ENONPHYS if the flag is set
 * (the fields are still written). */
fdlb_status fdlb_get_moments(fdlb_ctx *c, double *rho, double *ux, double *uy, double *T);

/* As fdlb_get_moments into a device buffer of 4 * nx * ny float64 (rho, ux, uy, T
 * planes).  Asynchronous; does not report the flag. */
fdlb_status fdlb_get_moments_device(fdlb_ctx *c, double *fields);

/* Checkpoint: the stored state.  FDLB_F64 / FDLB_F32: the 33 distribution planes as
 * 33 * ny * nx values of the storage type (float64 / float32), plane q = 0 (rest particle)
 * first, then q = 1 + 8 (k - 1) + (i - 1) for speed k and direction i pi/4.
 * FDLB_F32_DEV: the 33 planes of g (float32, same order), then the four float64 planes
 * n, ux, uy, T.  `bytes` must equal fdlb_f_bytes(c).  fdlb_get_f syncs; fdlb_set_f copies
 * then derives the pressure (and checks the state). */
size_t fdlb_f_bytes(const fdlb_ctx *c);
fdlb_status fdlb_get_f(fdlb_ctx *c, void *host, size_t bytes);
fdlb_status fdlb_set_f(fdlb_ctx *c, const void *host, size_t bytes);

/* Totals over the grid of n, n ux, n uy and the energy sum |v|^2 f / 2, and the sticky
 * non-physical flag (0/1).  Deterministic (fixed reduction order).  Syncs. */
fdlb_status fdlb_diag(fdlb_ctx *c, double sums[4], int32_t *nonphys);

/* As fdlb_diag, for callers that cannot allocate device memory (code under HIP graph
 * capture of their own work, tight serving loops, harnesses that forbid hipMalloc): the
 * reduction's partial totals and final sums go to a fixed scratch array compiled into the
 * library (2 MiB per GPU, held until the process ends) instead of the context's blocks.
 * The call itself allocates nothing.  Limit: the context's grids together may hold at
 * most 2^24 cells (2^16 blocks of 256); larger ones get FDLB_EINVAL with the sizes in
 * fdlb_last_error(c).  Same totals, bit for bit, as fdlb_diag.  All contexts on one GPU
 * share that GPU's scratch: calls that overlap in time on one GPU (other host threads,
 * other streams) race and must be serialised by the caller.  Syncs the context's stream. */
fdlb_status fdlb_diag_noalloc(fdlb_ctx *c, double sums[4], int32_t *nonphys);

/* Steps taken since the last state was set. */
int64_t fdlb_steps_done(const fdlb_ctx *c);

/* Sets the step count that times the moving side segments (t = steps * dt) and
 * fdlb_steps_done, for example to resume a checkpoint taken after `steps` steps.  Setting
 * a state resets it to 0.  Enqueued. */
fdlb_status fdlb_set_clock(fdlb_ctx *c, int64_t steps);

void fdlb_destroy(fdlb_ctx *c);
const char *fdlb_strerror(fdlb_status s);
/* The HIP error behind the last FDLB_EDEVICE (or FDLB_ENOMEM) of context c; with c = NULL,
 * that of the calling thread's last failed fdlb_create / fdlb_batch_create ("" after a
 * successful one).  The string stays valid until the next call on the same context
 * (thread). */
const char *fdlb_last_error(const fdlb_ctx *c);

/* Tile shapes the step kernel is built for: writes up to `cap` (tx, ty) pairs and returns
 * how many exist.  Shape id s (1-based) in fdlb_params.tile selects pair s - 1. */
int32_t fdlb_tile_shapes(int32_t *tx_ty, int32_t cap);

/* Tiling of the step launch: tile shape id (1-based, see fdlb_tile_shapes) and the width,
 * in tiles, of the column groups the tiles are dispatched in (row by row inside a group;
 * wider groups stream longer rows, narrower ones keep halo rows in L2).  Results do not
 * depend on the tiling; only the speed does.  Syncs. */
fdlb_status fdlb_set_tiling(fdlb_ctx *c, int32_t shape_id, int32_t group);
fdlb_status fdlb_get_tiling(const fdlb_ctx *c, int32_t *shape_id, int32_t *group);

/* Autotuner: times `trial_steps` steps for every (shape, group) candidate on the current
 * state and keeps the fastest.  NULL / 0-length lists mean all shapes and groups
 * {1, 4, 8, 16, 32}.  The trial steps do not advance the state (they read the current
 * buffers and overwrite the spare ones).  best_ms (may be NULL) receives the best time per
 * step.  Requires a state (FDLB_ESTATE).  Syncs. */
fdlb_status fdlb_autotune(fdlb_ctx *c, int32_t trial_steps, const int32_t *shape_ids, int32_t nshapes,
                          const int32_t *groups, int32_t ngroups, float *best_ms);

/* Measurement: the step is one launch per tile kind (0 interior tiles, 1 tiles spanning a
 * periodic height of one tile, 2 tiles touching a side; with tblock = 2 also 3, the
 * two-step tiles, whose launch takes two steps).  fdlb_tile_cells gives the grid
 * cells a kind covers; fdlb_time_kernel times `launches` launches of one kind (-1: the
 * whole step, `launches` steps; with tblock = 2 they run as two-step passes and the time
 * is per step) with HIP events on the context's stream, without advancing the state (like
 * the autotuner's trial steps).  Syncs. */
int64_t fdlb_tile_cells(const fdlb_ctx *c, int32_t kind);
fdlb_status fdlb_time_kernel(fdlb_ctx *c, int32_t kind, int32_t launches, float *ms_per_launch);
/* The practical bandwidth ceiling of the interior kernel: times `launches` launches of a
 * plain copy of every stored distribution plane (33 planes; the g planes in deviation
 * storage) over the interior tiles, from the current half to the other, with the step's
 * tile shape, dispatch order and stores, but no halo, no moment planes and no arithmetic.
 * The state is not advanced (the other half is overwritten, as by the autotuner's trial
 * steps).  FDLB_EINVAL without interior tiles; requires a state (FDLB_ESTATE).  Syncs. */
fdlb_status fdlb_copy_ceiling(fdlb_ctx *c, int32_t launches, float *ms_per_launch);

/* ---- Stability sweep (Sec. 4) --------------------------------------------------------- */
/* A uniform equilibrium and the scheme's parameters for the von Neumann analysis of Sec. 4:
 * one step of Eq. (dis_eq1) multiplies a Fourier mode exp(i phi x / dx) along x of the 33
 * perturbation amplitudes by the amplification matrix of Eq. (gi_j_eq),
 *   G(phi) = (1 - dt/tau + lines I-IV at phi) I + (dt/tau) d f^eq / d f,
 * with the Jacobian of Eq. (pian_fki_eq) taken in closed form and the switching function
 * of line IV frozen at `theta` (Eq. add4 gives zero on a uniform state).  `lines` selects
 * lines I..IV of Eq. (dis_eq1) as bits 0..3 (15: the full scheme), as in Figs. 2-6. */
typedef struct {
    double rho, ux, uy, T;   /* the uniform state */
    double dx, dt, tau;      /* > 0 */
    double theta;            /* frozen switching function of line IV */
    double v[4];             /* speeds v1..v4, distinct and > 0 */
    int32_t lines;           /* 0..15 */
    int32_t pad_;
} fdlb_vn_case;

/* Spectral radius max |omega| of G(phi_p) for every case c and phase p, computed on the GPU
 * in double-double arithmetic (about 32 significant digits: these matrices are strongly
 * non-normal at high Mach number, and float64 eigenvalues can be wrong in the second digit),
 * by a Householder reduction to Hessenberg form and the shifted QR algorithm, one
 * wavefront per matrix.  `cases`: ncases host structs; `phis`: nphi host phases (radians);
 * `radius`: host output of ncases * nphi values, case-major (NaN where the iteration did
 * not converge).  Allocates and frees its own device buffers and syncs `stream` (NULL: the
 * null stream).  Errors: FDLB_EINVAL (sizes, a non-positive rho, T, dx, dt, tau or speed,
 * equal speeds, lines outside 0..15, more than 2^24 matrices), FDLB_ENOMEM, FDLB_EDEVICE. */
fdlb_status fdlb_vn_sweep(const fdlb_vn_case *cases, int32_t ncases, const double *phis, int32_t nphi,
                          double *radius, void *stream);
/* The matrix G(phi) itself for one case: 33 x 33 row-major entries of four float64 each
 * (real part as a double-double hi, lo, then the imaginary part hi, lo) into `matrix`
 * (4 * 33 * 33 host doubles).  Same errors as fdlb_vn_sweep.  Syncs. */
fdlb_status fdlb_vn_matrix(const fdlb_vn_case *c, double phi, double *matrix, void *stream);

/* ---- Batched ensembles ------------------------------------------------------------- */
/* k independent problems of possibly different size and parameters advanced together:
 * every step is one launch over the tiles of all instances.  All instances must share
 * the precision and the tile shape.  `arena` holds fdlb_batch_required_bytes bytes.
 * fdlb_step, fdlb_diag (totals over all instances), fdlb_steps_done and fdlb_destroy
 * accept batch contexts. */
size_t fdlb_batch_required_bytes(int32_t k, const fdlb_params *p);
fdlb_status fdlb_batch_create(int32_t k, const fdlb_params *p, void *stream, void *arena,
                              size_t arena_bytes, fdlb_ctx **out);
/* Instance i (0 <= i < k).  set_state marks the batch as set once every instance has
 * been set at least once.  The instances share one step clock and one non-physical flag,
 * so once the batch has stepped, fdlb_batch_set_state returns FDLB_ESTATE (create a new
 * batch to restart it). */
fdlb_status fdlb_batch_set_state(fdlb_ctx *c, int32_t i, const double *rho, const double *ux,
                                 const double *uy, const double *T);
fdlb_status fdlb_batch_get_moments(fdlb_ctx *c, int32_t i, double *rho, double *ux, double *uy,
                                   double *T);
/* nsteps steps of every instance (Eq. dis_eq1), enqueued: the same as fdlb_step on a batch
 * context, under the batch family's name.  FDLB_ESTATE before every instance has a state. */
fdlb_status fdlb_batch_step(fdlb_ctx *c, int64_t nsteps);

#ifdef __cplusplus
}
#endif

#endif /* FDLB_H */
