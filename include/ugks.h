/*
 * ugks.h -- C ABI of the MI355X (gfx950) memory-saving UGKS library.
 *
 * One handle advances one flow case of the unified gas-kinetic scheme on an
 * unstructured mesh, as set out in Y. Zhang, Y. Wei, W. Long, K. Xu,
 * "An efficiency and memory-saving programming paradigm for the unified
 * gas-kinetic scheme" (arXiv:2412.06546):
 *   - model: BGK-Shakhov equation reduced to h = int f dxi and
 *     b = int xi^2 f dxi (Sections 2.1-2.2, Eq. BGKReduce);
 *   - discretisation: finite volumes in physical space, a weighted point set
 *     in velocity space (Section 2.3, Eqs. BGKdis, microscopicFlux,
 *     macroscopicUpdata, macroscopicFlux);
 *   - interface flux from the integral solution (Section 2.4,
 *     Eq. fullSolution), ghost-cell far field and Maxwellian isothermal wall
 *     (Section 2.5, Eq. maxWalldes), trapezoid source (Section 2.6);
 *   - the two-stage update of f (Section 3.2, Eqs. microS1 and microS2) and
 *     the step order of Algorithm 1.
 * Only f (h and b, or h alone in 3D) is stored per (cell, velocity); slopes
 * and residuals of f live in registers for the duration of one step.
 *
 * Units: the gas constant is R = 1/2, so lambda = 1/(2 R T) = 1/T and
 * p = rho T / 2.  The gas is monatomic (no internal degrees of freedom):
 * in 2D the reduced distributions are h and b (one internal velocity
 * component), in 3D only h.
 *
 * Conventions shared by all entry points:
 *   - Every pointer argument is a HOST pointer unless stated otherwise.
 *   - Inputs are read during the call only and copied to device memory; the
 *     handle owns every device allocation, and ugks_destroy frees them.
 *   - Status codes: 0 = success, negative = UGKS_ERR_*; no C++ exception
 *     crosses the ABI.  ugks_last_error() returns the text of the last
 *     failure on that handle (or, when the handle is NULL, of the last
 *     failed ugks_create / ugks_batch_create of the calling thread).
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 *     Distinct handles may be used from distinct threads.
 *   - All work of a handle is queued on the HIP stream given at creation;
 *     entry points that return host data synchronise that stream.
 */
#ifndef UGKS_H
#define UGKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UGKS_OK 0
#define UGKS_ERR_ARG (-1)         /* invalid argument: sizes, pointers, mesh topology */
#define UGKS_ERR_ALLOC (-2)       /* device or host allocation failed */
#define UGKS_ERR_HIP (-3)         /* a HIP runtime call or kernel launch failed */
#define UGKS_ERR_NONPHYSICAL (-4) /* rho <= 0, T <= 0 or a non-finite value appeared */
#define UGKS_ERR_STATE (-5)       /* call not valid in the handle's current state */

/* face boundary types */
#define UGKS_BC_INTERIOR 0 /* interior or periodic face: two cells */
#define UGKS_BC_INFLOW 1   /* far field, ghost = bc_prim[face_bc_id] */
#define UGKS_BC_OUTFLOW 2  /* far field, ghost = the interior cell's state */
#define UGKS_BC_WALL 3     /* Maxwellian isothermal wall (U_w, T_w) = bc_prim[face_bc_id] */

/* f storage precision; every macroscopic quantity, every coefficient and all
 * arithmetic on f are FP64 (f is widened on load and rounded on store).
 * UGKS_BF16 rounds to nearest (ties to even) from FP64 and flushes values
 * below the FP32 normal range (1.18e-38) to zero. */
#define UGKS_F64 0
#define UGKS_F32 1
#define UGKS_BF16 2

/* Physical mesh (Section 2.3): finite volumes Omega_i with faces S_ij. */
typedef struct {
    int dim;                     /* 2 or 3 */
    int n_cells, n_faces;
    const double *cell_volume;   /* [n_cells] |Omega_i| (area in 2D) */
    const double *cell_centroid; /* [n_cells][dim] */
    const int *face_cells;       /* [n_faces][2]: left, right; right = -1 on a boundary */
    const double *face_normal;   /* [n_faces][dim] unit, from left to right (outward on a boundary) */
    const double *face_area;     /* [n_faces] S_ij (length in 2D) */
    const double *face_centroid; /* [n_faces][dim], in the left cell's frame */
    const double *face_shift;    /* [n_faces][dim] or NULL: added to the right cell's centroid
                                    to place its periodic image next to the left cell */
    const int *face_bc;          /* [n_faces] UGKS_BC_*, or NULL for all interior */
    const int *face_bc_id;       /* [n_faces] row of ugks_gas_t.bc_prim, or NULL for 0 */
} ugks_mesh_t;

/* Discrete velocity space (Section 2.3): points u_k with weights V_k, so that
 * int Q du = sum_k Q_k V_k -- a Cartesian grid with trapezoid weights, or an
 * unstructured velocity mesh (cell centres, cell volumes as weights).  When
 * the points take at most 1023 distinct values per axis (Cartesian, octree
 * or ball-restricted sets) the Gaussians are tabulated per axis in LDS
 * (ugks_is_tensor_grid); otherwise they are evaluated directly. */
typedef struct {
    int dim;           /* must equal the mesh's */
    int n_vel;
    const double *u;   /* [n_vel][dim] */
    const double *w;   /* [n_vel] V_k */
} ugks_vgrid_t;

/* Gas and scheme parameters. */
typedef struct {
    double Pr;          /* Prandtl number of the Shakhov model (1 = BGK) */
    double omega;       /* viscosity exponent: mu = mu_ref T^omega, tau = mu / p */
    double mu_ref;      /* viscosity at T = 1 */
    double cfl;         /* CFL number of the time step */
    double dt_override; /* > 0: use this time step instead of the CFL one */
    double limiter_k;   /* Venkatakrishnan constant K: eps^2 = (K |Omega_i|^(1/dim))^3 */
    int limiter;        /* 0 none (unlimited least squares), 1 Venkatakrishnan */
    int fstore;         /* UGKS_F64, UGKS_F32 or UGKS_BF16 storage of f */
    int n_bc;
    const double *bc_prim; /* [n_bc][dim+2]: (rho, U, T); walls use (U_w, T_w) */
    int mem_mode;       /* UGKS_MEM_TWO_BUFFERS or UGKS_MEM_IN_PLACE (below) */
    int chunk;          /* in-place mode: velocities per chunk, 0 = UGKS_DEFAULT_CHUNK */
    int sweep;          /* UGKS_SWEEP_AUTO, _GATHER, _PUSH or _PUSH_UNORDERED (below) */
} ugks_gas_t;

/* How the per-velocity sweep (the velocity loop of Algorithm 1) evaluates the
 * face fluxes.
 * UGKS_SWEEP_PUSH: every face flux once per velocity, by the face's upwind
 * cell with its own limited slope; the cells are coloured so that no two
 * cells of a colour are neighbours or share one, one launch per colour adds
 * each flux to the stage-1 values of both of its cells (the second f buffer
 * holds them; in the in-place mode a ring of one velocity chunk does, chunk
 * after chunk), and a final kernel forms W^{n+1}, q^{n+1} and stage 2.
 * Takes BF16 f only when asked for explicitly: its stage-1 sums (the second
 * buffer, or the ring in place) are then FP32, 2 more bytes per value than
 * the gather sweep keeps, and such a handle cannot be batched.
 * UGKS_SWEEP_PUSH_UNORDERED: the push sweep with every cell in one launch,
 * in stored (space-filling-curve) order, so that neighbours run close
 * together and their f and stage-1 values are found in cache.  Several
 * workgroups may then add to one stage-1 value at once; the hardware adds
 * are atomic, so the sum is complete, but its order, and so its rounding,
 * can differ from run to run: results agree with the other sweeps to
 * rounding, not bit for bit, and a restart from a checkpoint is not
 * bitwise.  Same storage rules as UGKS_SWEEP_PUSH; never chosen
 * automatically.
 * UGKS_SWEEP_GATHER: one workgroup per cell evaluates every face of its cell,
 * rebuilding the upwind neighbour's limited slope where needed (each
 * interior face twice); BF16 f (unless a push is asked for) and batched
 * steps use it.
 * UGKS_SWEEP_AUTO (0): push for FP64 and FP32 f, except 2D with FP64 f in
 * two buffers (there gathering measured faster on MI355X); gather for BF16
 * f.  All give the same results up to the order of sums (BF16 f: and the
 * precision of the stage-1 sums); ugks_sweep_kind tells which a handle
 * uses. */
#define UGKS_SWEEP_AUTO 0
#define UGKS_SWEEP_GATHER 1
#define UGKS_SWEEP_PUSH 2
#define UGKS_SWEEP_PUSH_UNORDERED 3

/* Storage of f.  UGKS_MEM_TWO_BUFFERS: f^n is read from one buffer and
 * f^{n+1} written to the other (2 f of memory, the second in FP32 when BF16
 * f takes the push sweep, as is the ring in place; the fastest form).
 * UGKS_MEM_IN_PLACE: one buffer, updated in place as in the paper's
 * two-stage form (Section 3.2): the velocities are swept in chunks, the
 * stage-1 values of a chunk wait in a ring of n_cells x n_comp x chunk
 * values until no cell reads that chunk's f^n any more, and stage 2 is
 * applied in place; memory 1 f + the ring + a few doubles per cell (the
 * chunks' moment sums and the wall densities).  Both forms give the same
 * results up to the order of the sums over velocities.  In-place handles
 * cannot be batched (ugks_batch_step); with the gather sweep they keep no
 * copy of the f that started a step (ugks_wall_flux and ugks_surface return
 * UGKS_ERR_STATE), the push sweep records the wall flux during the step. */
#define UGKS_MEM_TWO_BUFFERS 0
#define UGKS_MEM_IN_PLACE 1
/* Velocities per chunk when gas.chunk is 0 (capped at n_vel).  Every chunk
 * launch repeats the per-cell set-up, so fewer, larger chunks are faster and
 * cost a larger ring (n_cells x n_comp x chunk values of f). */
#define UGKS_DEFAULT_CHUNK 1024

typedef struct ugks ugks_t;

/* Create a case: the discretised problem of Section 2.3 (finite volumes and
 * a discrete velocity set) with the gas of Sections 2.1-2.2.
 * prim0 [n_cells][dim+2] holds the initial (rho, U, T) of
 * each cell; f^0 is the discrete Maxwellian of it, and W^0 and q^0 are the
 * discrete moments of f^0.  stream is a hipStream_t (NULL = default stream).
 * The time step is fixed at creation (the velocity grid does not change):
 * dt = cfl * min over cells and velocities of
 *      |Omega_i| / sum_faces S max(0, u_k . n_outward).
 * Limits: at most 16,000,000 cells and 16,384 velocities (UGKS_ERR_ARG).
 * The inputs are checked on the host before any device call; UGKS_ERR_ARG
 * names the first offending item: empty mesh or velocity set, a velocity
 * that is not finite or whose weight is not positive, dim not 2 or
 * 3, a face whose cell index is out of range or whose boundary type does
 * not match its cells, a non-positive area or volume, a normal that is not
 * a unit vector (|n|^2 off 1 by 1e-6 or more), a non-finite centroid or
 * periodic shift, a cell with fewer than dim + 1 or more than 4 (2D) / 6
 * (3D) faces, a non-positive initial density or temperature, a storage type
 * or gas constant out of range.
 * Returns UGKS_OK and *out, or an error code (*out = NULL). */
int ugks_create(const ugks_mesh_t *mesh, const ugks_vgrid_t *vgrid, const ugks_gas_t *gas,
                const double *prim0, void *stream, ugks_t **out);

/* Advance nsteps time steps (Algorithm 1 each, Section 3.2).  residual_out
 * (nullable, [dim+2]) receives the L2 norm over cells of W^{n+1} - W^n of
 * the last step, per conservative component, W^{n+1} from
 * Eq. macroscopicUpdata (the steady-state measure of a run to convergence).  Returns UGKS_ERR_NONPHYSICAL if a cell
 * lost positivity or finiteness (checked once at the end of the call). */
int ugks_step(ugks_t *h, int nsteps, double *residual_out);

/* Asynchronous stepping, for serving several cases at once on different
 * streams (each step is Algorithm 1, Section 3.2; the paper's concern with
 * the memory of many large cases is Sections 3.2 and 4.3).
 * ugks_step_async enqueues nsteps steps (as ugks_step) plus the
 * copies of the non-physical flag and of the last step's residual into
 * handle-owned pinned host memory, and returns without waiting.  Only one
 * batch may be outstanding per handle (UGKS_ERR_STATE otherwise).
 * ugks_poll sets *done = 0 while the batch runs; once it has finished it
 * sets *done = 1, writes residual_out (nullable, [dim+2]) and returns
 * UGKS_ERR_NONPHYSICAL if a cell lost positivity or finiteness. */
int ugks_step_async(ugks_t *h, int nsteps);
int ugks_poll(ugks_t *h, int *done, double *residual_out);

/* Batched stepping (continuous batching of many cases on one GPU; each
 * step is Algorithm 1 of Section 3.2 for every case): the
 * steps of several handles run in the same launches -- one grid per kernel
 * holds the cells (or faces) of every case end to end, each workgroup finds
 * its case from a table of per-case offsets -- so small cases fill the GPU
 * together and the launch count does not grow with the number of cases.
 * ugks_batch_create makes a batch object for up to max_cases handles on
 * `stream` (a hipStream_t).  ugks_batch_step enqueues nsteps steps of every
 * handle in hs[0..n) and returns at once; each handle is then pending as
 * after ugks_step_async (ugks_poll gives its residual and non-physical
 * flag).  All handles must have been created on the batch's stream, have
 * the same dimension, and have nothing outstanding (UGKS_ERR_ARG /
 * UGKS_ERR_STATE otherwise; the text from ugks_batch_last_error).  A case's
 * results are bitwise those of stepping it alone.  Handles may be created
 * and destroyed between calls; only the handles passed in are touched. */
typedef struct ugks_batch ugks_batch_t;
int ugks_batch_create(int max_cases, void *stream, ugks_batch_t **out);
int ugks_batch_step(ugks_batch_t *b, ugks_t *const *hs, int n, int nsteps);
const char *ugks_batch_last_error(const ugks_batch_t *b);
void ugks_batch_destroy(ugks_batch_t *b);

/* For callers that cannot allocate device or host memory at step time --
 * code being captured into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc: the batched step of ugks_batch_step without a batch
 * object.  It calls no hipMalloc, hipFree, hipHostMalloc or other
 * allocating routine: the batch descriptors and offset tables go into a
 * fixed device array of the library (about 17 KB per GPU, kept until the
 * process ends), whose address is looked up once per device when the first
 * handle is created on it.  hs[0..n) as for ugks_batch_step, all created on
 * `stream` (a hipStream_t) with that stream's device current; at most
 * UGKS_STATIC_BATCH_MAX cases (UGKS_ERR_ARG beyond, text from
 * ugks_batch_last_error(NULL)).  The descriptors are copied to the device
 * and the call waits for that copy (the host layout lives on its stack),
 * then enqueues the steps and returns; each handle is pending as after
 * ugks_batch_step.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (from several threads) race and must be
 * serialised by the caller.  Results are bitwise those of ugks_batch_step. */
#define UGKS_STATIC_BATCH_MAX 64
int ugks_batch_step_static(ugks_t *const *hs, int n, int nsteps, void *stream);

/* Device bytes ugks_create would allocate for these inputs (host-side
 * computation, no GPU needed): admission control against an HBM budget
 * (the memory of f per cell and velocity dominates, as in the accounting of
 * Section 4.3).
 * Returns 0 for invalid arguments. */
size_t ugks_footprint_estimate(const ugks_mesh_t *mesh, const ugks_vgrid_t *vgrid, const ugks_gas_t *gas);

/* Copy the conservative variables W [n_cells][dim+2] = (rho, rho U, rho E)
 * (the moments of f with psi = (1, u, (|u|^2 + |xi|^2)/2), Section 2.1) and
 * the heat flux q [n_cells][dim] (nullable; the Shakhov heat flux of
 * Section 2.1, carried from step to step as in Algorithm 1's first step) to host
 * memory. */
int ugks_macros(ugks_t *h, double *W_out, double *q_out);

/* Copy f to host memory as FP64 [n_cells][n_comp][n_vel]: the reduced
 * distributions of Section 2.2 at the discrete velocities of Section 2.3
 * (n_comp = 2 in 2D: h then b; 1 in 3D). */
int ugks_get_f(ugks_t *h, double *f_out);

/* Replace f with a host array laid out as in ugks_get_f; W and q become its
 * discrete moments (Sections 2.1 and 2.3: checkpoint restart or a
 * non-equilibrium start), and a
 * non-physical flag left by an earlier step is cleared. */
int ugks_set_f(ugks_t *h, const double *f_in);

/* Checkpoint and restart, exact: the state blob holds what Algorithm 1
 * carries from one step to the next (Section 3.2: f, the conservative
 * variables W and the heat flux q), f in its
 * storage precision and the library's order, and the step count.
 * ugks_state_bytes gives its size; ugks_get_state writes it to a host
 * buffer of at least that size; ugks_set_state restores it into a handle
 * created from the same inputs (sizes, storage and the library's cell and
 * velocity orders are checked: UGKS_ERR_ARG otherwise), after which the
 * steps continue bit for bit as the saved run would have (with
 * UGKS_SWEEP_PUSH_UNORDERED, to rounding: its sums have no fixed order).  Unlike
 * ugks_set_f, W and q are restored, not recomputed as moments of f.  The
 * blob is in host byte order. */
size_t ugks_state_bytes(const ugks_t *h);
int ugks_get_state(ugks_t *h, void *buf, size_t bytes);
int ugks_set_state(ugks_t *h, const void *buf, size_t bytes);

/* Time step of Algorithm 1's first step (from the CFL condition, fixed for the run),
 * or -1 for a NULL handle. */
double ugks_dt(const ugks_t *h);
/* Stored reduced distributions per (cell, velocity) (Section 2.2): 2 (h, b)
 * in 2D, 1 (h) in 3D. */
int ugks_n_comp(const ugks_t *h);
/* Steps of Algorithm 1 taken since creation (or restored by a state). */
long ugks_step_count(const ugks_t *h);
/* Device bytes owned by the handle (the memory accounting of Section 4.3). */
size_t ugks_footprint_bytes(const ugks_t *h);
/* 1 if the Gaussians over the velocity set of Section 2.3 are tabulated per
 * axis (few distinct coordinate values per axis), 0 if evaluated directly. */
int ugks_is_tensor_grid(const ugks_t *h);
/* UGKS_SWEEP_PUSH, UGKS_SWEEP_PUSH_UNORDERED or UGKS_SWEEP_GATHER: how the
 * handle's steps evaluate the face fluxes in the velocity loop of Algorithm 1 (batched steps
 * always gather); -1 for a NULL handle. */
int ugks_sweep_kind(const ugks_t *h);
/* The number of colour classes (launches per step, or per velocity chunk in
 * place) into which the push sweep splits the face-flux loop of Algorithm 1
 * (its velocity loop): cells of one class share no neighbour and are not neighbours; 1 for
 * the unordered push (one class of all cells), 0 when the handle gathers, -1
 * for a NULL handle. */
int ugks_sweep_colours(const ugks_t *h);

/* Timing of the step's kernels with HIP events on the handle's stream (the
 * per-step wall time the paper reports in Table UGKSeff).
 * ugks_profile(h, 1) resets the counters and records events around every
 * launch from then on (0 stops).  ugks_profile_read gives ms_out[0] = total
 * milliseconds in the sweep (the velocity loop of Algorithm 1 and the
 * updates after it: every kernel of it, e.g. the push sweep's wall, push
 * and final launches), ms_out[1] = total in the two prologue kernels (macro
 * gradients and interface equilibria, the steps of Algorithm 1 before its
 * velocity loop), and the number of steps timed. */
int ugks_profile(ugks_t *h, int enable);
int ugks_profile_read(const ugks_t *h, double *ms_out, long *launches);

/* Surface quantities (Section 2.5).  ugks_n_wall_faces gives the number of
 * faces of type UGKS_BC_WALL.  ugks_wall_flux writes out [n_wall][dim+2]:
 * for every wall face, in increasing (caller's) face index, the macroscopic
 * flux through the face during the last step, per unit area and per unit
 * time -- mass (zero up to round-off: rho_w is chosen so), momentum F_m
 * [dim], energy -- the moments (1, u, (|u|^2 h + b)/2) of u_n times the time
 * integral of the wall distribution (outgoing: the limited reconstruction
 * of the interior f transported freely; incoming: the wall Maxwellian of
 * density rho_w).  n is the face normal (out of the gas, into the wall):
 * surface pressure p_w = F_m . n, shear stress |F_m - p_w n|, heat flux =
 * the energy component.  The push sweep records it during the step; after a
 * gather step it is recomputed from the f that started the step (kept in
 * the second f buffer).  UGKS_ERR_STATE if no step ran since creation or
 * ugks_set_f, while asynchronous steps are outstanding, or after an
 * in-place gather step (which keeps no copy of that f). */
int ugks_n_wall_faces(const ugks_t *h);
int ugks_wall_flux(ugks_t *h, double *out);

/* Surface coefficients of every wall face in the last step (Section 2.5 for
 * the wall flux and the surface pressure, shear stress and heat flux;
 * Section 4.1 for the coefficients).  out [n_wall][6], wall faces in
 * increasing (caller's) face index as in ugks_wall_flux:
 *   p_w = F_m . n, sigma_w = |F_m - p_w n|, q_w = energy flux,
 *   Cp = p_w / d, Ct = sigma_w / d, Ch = q_w / (d u_inf),
 * with F the wall flux per unit area and time of ugks_wall_flux, n the
 * face normal (out of the gas) and d = rho_inf u_inf^2 / 2.  All computed on
 * the device.  rho_inf and u_inf must be positive and finite (UGKS_ERR_ARG);
 * same state conditions as ugks_wall_flux (UGKS_ERR_STATE). */
int ugks_surface(ugks_t *h, double rho_inf, double u_inf, double *out);

/* The library stores the velocity set of Section 2.3 in its own order (by
 * direction, so that the lanes of a wavefront agree on upwind sides).  perm_out [n_vel] receives,
 * for each stored position, the caller's velocity index.  ugks_get_f and
 * ugks_set_f use the caller's order. */
int ugks_velocity_order(const ugks_t *h, int *perm_out);

/* The library stores the cells of the mesh (Section 2.3) in its own order
 * too: along a Morton (Z-order)
 * curve through the cell centroids, so that consecutive stored cells -- the
 * workgroups that share one XCD's L2 cache -- are mesh neighbours whatever
 * the caller's numbering.  perm_out [n_cells] receives, for each stored
 * position, the caller's cell index.  Every entry point that takes or
 * returns per-cell host data (prim0, ugks_macros, ugks_get_f, ugks_set_f,
 * the cell named by an error) uses the caller's numbering. */
int ugks_cell_order(const ugks_t *h, int *perm_out);

/* Device pointer of the current f, the reduced distributions of Section 2.2
 * (for zero-copy inspection):
 * [n_cells][n_comp][n_vel] in the storage precision, the library's cell
 * order (ugks_cell_order) and velocity order (ugks_velocity_order); valid
 * until the next ugks_step or ugks_destroy. */
const void *ugks_device_f(const ugks_t *h);

/* Free the handle and all its device memory (ownership as stated at the top
 * of this file); NULL is ignored. */
void ugks_destroy(ugks_t *h);
/* Text of the last failure on h (NULL: of the last failed ugks_create or
 * ugks_batch_create of the calling thread); valid until the next call on h. */
const char *ugks_last_error(const ugks_t *h);

#ifdef __cplusplus
}
#endif
#endif
